// Workgroup-level exact arithmetic on little-endian 32-bit-limb numbers.
//
// One workgroup of T threads (T/64 wavefronts) owns one multi-precision
// instance.  Operands live in LDS (or are read straight from global memory
// through a view); every primitive below is called by all T threads with the
// same (uniform) arguments, begins with a workgroup barrier so that it sees
// every earlier write, and leaves its results unsynchronised (the next
// primitive's opening barrier publishes them).
//
// Building blocks of the paper's data-parallel division (Sec. 3):
//   reduce_max / prec / cmp  -- the less-than and precision operators
//   addsub                   -- map-scan-map carry/borrow propagation
//                               (Sec. 3.2), here as a per-thread sequential
//                               chunk plus a carry-lookahead scan over the
//                               thread summaries built from wave ballots
//   mul                      -- classical convolution (Sec. 3.3), one wave
//                               per 256-column strip, 96-bit column sums
//   shortdiv                 -- division by a single limb (Alg. 1 special
//                               case "v < B")
// The primitives header (mp_prims_hip.hpp) must be included first.
#pragma once

#include <stdint.h>

namespace mp {

constexpr int kRCol = 4;                 // product columns per lane
constexpr int kStrip = kLanes * kRCol;   // product columns per wave pass
constexpr int kPad = kStrip + 8;         // zero guard on both sides of a staged window operand
constexpr int kCMax = 17;                // most limbs one thread handles in a linear operation

// control block at the start of the instance's LDS (32-bit words)
constexpr int kCtlRed = 0;       // 3 x 16 per-wave reduction slots
constexpr int kCtlScan = 48;     // 16 x (generate, propagate) wave summaries
constexpr int kCtlPrec = 80;     // 16 per-wave result-precision slots of the last addsub
constexpr int kCtlStrip = 96;    // 2 words per strip carry, up to 72 strips
constexpr int kCtlBcast = 240;   // 16 broadcast scalars
constexpr int kCtlWords = 256;
constexpr int kMaxStrips = 72;

MP_DEV int round4(int x) { return (x + 3) & ~3; }
MP_DEV int imin(int a, int b) { return a < b ? a : b; }
MP_DEV int imax(int a, int b) { return a > b ? a : b; }

// ------------------------------------------------------------------ views

// limb k of a number stored at p[0..len) placed at offset `off`: p[k - off]
// inside the stored range, zero elsewhere.  off > 0 multiplies by B^off,
// off < 0 takes the whole shift by -off limbs (floor).
struct Span {
    const uint32_t *p;
    int off;
    int len;
    MP_DEV uint32_t operator()(int k) const
    {
        unsigned i = (unsigned)(k - off);
        return i < (unsigned)len ? p[i] : 0u;
    }
};

struct Zero {
    MP_DEV uint32_t operator()(int) const { return 0u; }
};

// a one-limb number x
struct Limb0 {
    uint32_t x;
    MP_DEV uint32_t operator()(int k) const { return k == 0 ? x : 0u; }
};

// B^e
struct PowB {
    int e;
    MP_DEV uint32_t operator()(int k) const { return k == e ? 1u : 0u; }
};

// strip carries of a product: carry e_s (64-bit) enters at column (s+1)*kStrip
struct StripCarries {
    const uint32_t *sc;
    int nstrips;
    MP_DEV uint32_t operator()(int k) const
    {
        int s = (k / kStrip) - 1, o = k % kStrip;
        if (s < 0 || s >= nstrips || o > 1) return 0u;
        return sc[2 * s + o];
    }
};

// writes limb k to p[k - off] when that index lies in [0, len)
struct Store {
    uint32_t *p;
    int off;
    int len;
    MP_DEV void operator()(int k, uint32_t x) const
    {
        unsigned i = (unsigned)(k - off);
        if (i < (unsigned)len) p[i] = x;
    }
};

struct Discard {
    MP_DEV void operator()(int, uint32_t) const {}
};

// ------------------------------------------------------------- reductions

MP_DEV uint32_t wave_max(uint32_t x)
{
#pragma unroll
    for (int m = 1; m < kLanes; m <<= 1) {
        uint32_t y = shfl_xor(x, m);
        x = x > y ? x : y;
    }
    return x;
}

// maximum of one value per thread over the workgroup (same on every thread)
template <int T>
MP_DEV uint32_t wg_max(uint32_t *ctl, uint32_t x)
{
    constexpr int W = T / kLanes;
    x = wave_max(x);
    if (lane() == 0) ctl[kCtlRed + tid() / kLanes] = x;
    sync();
    uint32_t r = 0;
#pragma unroll
    for (int w = 0; w < W; w++) {
        uint32_t y = ctl[kCtlRed + w];
        r = r > y ? r : y;
    }
    return uniform(r);
}

// element-wise maxima of N values per thread over the workgroup (N <= 3)
template <int T, int N>
MP_DEV void wg_max_n(uint32_t *ctl, uint32_t (&x)[N])
{
    constexpr int W = T / kLanes;
    const int w = uniform(tid() / kLanes);
#pragma unroll
    for (int i = 0; i < N; i++) {
        const uint32_t m = wave_max(x[i]);
        if (lane() == 0) ctl[kCtlRed + 16 * i + w] = m;
    }
    sync();
#pragma unroll
    for (int i = 0; i < N; i++) {
        uint32_t r = 0;
#pragma unroll
        for (int v = 0; v < W; v++) {
            const uint32_t y = ctl[kCtlRed + 16 * i + v];
            r = r > y ? r : y;
        }
        x[i] = uniform(r);
    }
}

// max over k in [0, n) of f(k)  (f(k) >= 0)
template <int T, class F>
MP_DEV int reduce_max(uint32_t *ctl, int n, const F &f)
{
    sync();
    uint32_t m = 0;
    for (int k = tid(); k < n; k += T) {
        uint32_t y = f(k);
        m = m > y ? m : y;
    }
    return (int)wg_max<T>(ctl, m);
}

// number of significant limbs of x over [0, n)
template <int T, class FX>
MP_DEV int prec(uint32_t *ctl, int n, const FX &x)
{
    return reduce_max<T>(ctl, n, [&](int k) -> uint32_t { return x(k) ? (uint32_t)(k + 1) : 0u; });
}

// sign of x - y over limbs [0, n): -1, 0, 1
template <int T, class FX, class FY>
MP_DEV int cmp(uint32_t *ctl, int n, const FX &x, const FY &y)
{
    int top = reduce_max<T>(ctl, n, [&](int k) -> uint32_t { return x(k) != y(k) ? (uint32_t)(k + 1) : 0u; });
    if (top == 0) return 0;
    return x(top - 1) < y(top - 1) ? -1 : 1;
}

// ------------------------------------------------------- add / subtract

// z = x + y + cin (sub = false) or z = x - y - cin (sub = true) over limbs
// [0, n); out(k, z_k) for every k.  Returns the carry (borrow) out of limb
// n-1, identical on every thread.  n <= T * kCMax.
//
// Thread t owns the contiguous limbs [t*C, t*C + C).  It adds its chunk with
// carry-in 0, giving a generate bit g (carry out) and a propagate bit p (all
// result limbs 0xFFFFFFFF for add, 0 for sub); g and p are never both set.
// The carries into the threads follow from a carry-lookahead scan: inside a
// wave, with G = ballot(g), P = ballot(p), X = G | P, the carries into the
// lanes are the bits of (X + G + cin) ^ X ^ G (binary addition realises
// c_{i+1} = g_i | (p_i & c_i)); across the <= 16 waves the per-wave
// (generate, propagate) pairs are combined in LDS.  Inputs are read before
// the internal barrier and outputs written after it, so out may overwrite
// the storage x or y read from.  The precision of z (1 + index of its top
// nonzero limb, 0 for zero) is left in per-wave slots for read_prec.
template <int T, int CM, class FX, class FY, class FO>
MP_DEV uint32_t addsub_chunk(uint32_t *ctl, int n, int C, bool sub, uint32_t cin,
                             const FX &x, const FY &y, const FO &out)
{
    constexpr int W = T / kLanes;
    const int k0 = tid() * C;
    uint32_t z[CM];
    uint32_t c = 0;
    bool prop = true;
#pragma unroll
    for (int j = 0; j < CM; j++) {
        const int k = k0 + j;
        if (j < C && k < n) {
            const uint32_t a = x(k), b = y(k);
            if (!sub) {
                uint64_t s = (uint64_t)a + b + c;
                z[j] = (uint32_t)s;
                c = (uint32_t)(s >> 32);
                prop = prop && (z[j] == 0xFFFFFFFFu);
            } else {
                uint64_t d = (uint64_t)a - b - c;
                z[j] = (uint32_t)d;
                c = (uint32_t)(d >> 63);
                prop = prop && (z[j] == 0u);
            }
        }
    }
    const uint64_t G = ballot(c != 0), P = ballot(prop), X = G | P;
    const uint64_t s0 = X + G;
    const int w = uniform(tid() / kLanes);
    if (lane() == 0) {
        ctl[kCtlScan + 2 * w] = s0 < X ? 1u : 0u;      // wave generates
        ctl[kCtlScan + 2 * w + 1] = (~P == 0) ? 1u : 0u;  // wave propagates
    }
    sync();
    // scan of the wave summaries: carry into this wave, and out of the number
    uint32_t cin_w = cin, cout = cin;
#pragma unroll
    for (int v = 0; v < W; v++) {
        if (v == w) cin_w = cout;
        cout = ctl[kCtlScan + 2 * v] | (ctl[kCtlScan + 2 * v + 1] & cout);
    }
    const uint64_t cm = (X + G + (uint64_t)cin_w) ^ X ^ G;
    uint32_t ci = (uint32_t)(cm >> lane()) & 1u;
    uint32_t top = 0;
#pragma unroll
    for (int j = 0; j < CM; j++) {
        const int k = k0 + j;
        if (j < C && k < n) {
            if (!sub) {
                z[j] += ci;
                ci &= (z[j] == 0u) ? 1u : 0u;
            } else {
                const uint32_t o = z[j];
                z[j] -= ci;
                ci &= (o == 0u) ? 1u : 0u;
            }
            out(k, z[j]);
            top = z[j] ? (uint32_t)(k + 1) : top;
        }
    }
    // chunks ascend with the lane, so the wave's top is the top of its highest nonzero lane
    const uint64_t nzl = ballot(top != 0);
    const uint32_t wtop = nzl ? readlane(top, 63 - __builtin_clzll(nzl)) : 0u;
    if (lane() == 0) ctl[kCtlPrec + w] = wtop;
    return cout;
}

// precision of the result of the last addsub (reads the per-wave slots after a
// barrier); `off` converts to the coordinates of a Store with that offset
template <int T>
MP_DEV int read_prec(uint32_t *ctl, int off = 0)
{
    constexpr int W = T / kLanes;
    sync();
    uint32_t r = 0;
#pragma unroll
    for (int v = 0; v < W; v++) {
        const uint32_t y = ctl[kCtlPrec + v];
        r = r > y ? r : y;
    }
    const int p = (int)uniform(r) - off;
    return p > 0 ? p : 0;
}

template <int T, class FX, class FY, class FO>
MP_DEV uint32_t addsub(uint32_t *ctl, int n, bool sub, uint32_t cin,
                       const FX &x, const FY &y, const FO &out)
{
    sync();
    // odd chunk length: lanes then touch LDS with an odd word stride (no bank conflicts)
    const int C = ((n + T - 1) / T) | 1;
    if (C == 1) return addsub_chunk<T, 1>(ctl, n, C, sub, cin, x, y, out);
    if (C == 3) return addsub_chunk<T, 3>(ctl, n, C, sub, cin, x, y, out);
    if (C <= 7) return addsub_chunk<T, 7>(ctl, n, C, sub, cin, x, y, out);
    return addsub_chunk<T, kCMax>(ctl, n, C, sub, cin, x, y, out);
}

// dst[k] = src(k) for k in [0, n), zero for k in [n, clear)
template <int T, class FS>
MP_DEV void copy(uint32_t *dst, int n, int clear, const FS &src)
{
    sync();
    const int e = imax(n, clear);
    for (int k = tid(); k < e; k += T) dst[k] = k < n ? src(k) : 0u;
}

// ------------------------------------------------------------- multiply

// p[0, ncols) = (a * b) mod B^ncols, ncols <= na + nb (ncols = na + nb is the
// full product); returns the precision of the result.  `a` (na limbs, any LDS position, readable up to 3 limbs past
// its end) is the row operand, read with wave-uniform addresses; `bw` points
// at limb 0 of the window operand (nb limbs) staged in LDS with kPad zero
// limbs on both sides, 16-byte aligned.  The shorter operand should be the
// rows: the waste of a strip is then only the triangles at the ramps.
//
// Column strips of kStrip columns are dealt to the waves; lane l of the wave
// owns kRCol consecutive columns and keeps their 96-bit sums in registers
// while it walks the rows in blocks of 4 (the load-balanced classical
// schedule of Sec. 3.3 becomes a row walk per strip: one window load and 16
// limb products per lane per block).  The strip's sums are turned into limbs
// in-wave (lane-local carry, neighbour carry by shuffle, lookahead by
// ballot); the carry leaving each strip is added by one final addsub pass.
template <int T>
MP_DEV int mul(uint32_t *ctl, uint32_t *p, int ncols,
               const uint32_t *a, int na, const uint32_t *bw, int nb)
{
    constexpr int W = T / kLanes;
    sync();
    if (na == 0 || nb == 0 || ncols <= 0) {
        for (int k = tid(); k < ncols; k += T) p[k] = 0u;
        return 0;
    }
    const int nstrips = (ncols + kStrip - 1) / kStrip;
    const int w = uniform(tid() / kLanes), l = lane();
    for (int s = w; s < nstrips; s += W) {
        const int K0 = s * kStrip, k0 = K0 + l * kRCol;
        const int ilo = imax(0, K0 - nb + 1) & ~3;
        const int ihi = imin(na, imin(K0 + kStrip, ncols));
        uint64_t lo[4] = {0, 0, 0, 0};
        uint32_t hi[4] = {0, 0, 0, 0};
        if (ilo < ihi) {
            // column k0+r, row i+t takes window limb k0 + r - i - t; per block
            // of rows i..i+3 the lane needs window limbs k0-i-3 .. k0-i+3
            const uint32_t *wp = bw + (k0 - ilo);
            const uint32_t *ap = a + ilo;
            int nblk = (ihi - ilo) >> 2;
            for (; nblk >= 2; nblk -= 2) {
                const Limb4 w0 = load4(wp), w1 = load4(wp - 4), w2 = load4(wp - 8);
                const uint32_t a0 = ap[0], a1 = ap[1], a2 = ap[2], a3 = ap[3];
                const uint32_t a4 = ap[4], a5 = ap[5], a6 = ap[6], a7 = ap[7];
                mac4(lo, hi, a0, w0.x, w0.y, w0.z, w0.w);
                mac4(lo, hi, a1, w1.w, w0.x, w0.y, w0.z);
                mac4(lo, hi, a2, w1.z, w1.w, w0.x, w0.y);
                mac4(lo, hi, a3, w1.y, w1.z, w1.w, w0.x);
                mac4(lo, hi, a4, w1.x, w1.y, w1.z, w1.w);
                mac4(lo, hi, a5, w2.w, w1.x, w1.y, w1.z);
                mac4(lo, hi, a6, w2.z, w2.w, w1.x, w1.y);
                mac4(lo, hi, a7, w2.y, w2.z, w2.w, w1.x);
                keep(w2.x);   // keeps the third window load one aligned 16-byte read
                wp -= 8;
                ap += 8;
            }
            const int rem = (ihi - ilo) - ((ihi - ilo) & ~7);   // rows left: 0..7
            if (rem > 0) {
                // last rows: those at or past ihi (<= na) read as zero
                const int i = ihi - rem;
                const Limb4 w0 = load4(wp), w1 = load4(wp - 4), w2 = load4(wp - 8);
                const uint32_t a0 = ap[0];
                const uint32_t a1 = i + 1 < ihi ? ap[1] : 0u, a2 = i + 2 < ihi ? ap[2] : 0u;
                const uint32_t a3 = i + 3 < ihi ? ap[3] : 0u, a4 = i + 4 < ihi ? ap[4] : 0u;
                const uint32_t a5 = i + 5 < ihi ? ap[5] : 0u, a6 = i + 6 < ihi ? ap[6] : 0u;
                mac4(lo, hi, a0, w0.x, w0.y, w0.z, w0.w);
                mac4(lo, hi, a1, w1.w, w0.x, w0.y, w0.z);
                mac4(lo, hi, a2, w1.z, w1.w, w0.x, w0.y);
                mac4(lo, hi, a3, w1.y, w1.z, w1.w, w0.x);
                if (rem > 4) {
                    mac4(lo, hi, a4, w1.x, w1.y, w1.z, w1.w);
                    mac4(lo, hi, a5, w2.w, w1.x, w1.y, w1.z);
                    mac4(lo, hi, a6, w2.z, w2.w, w1.x, w1.y);
                }
            }
        }
        // lane-local carry: z = column sums as limbs, c = carry into column k0+4
        uint32_t z[4];
        uint64_t c = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint64_t t = lo[r] + c;
            const uint32_t kap = t < c ? 1u : 0u;
            z[r] = (uint32_t)t;
            c = ((uint64_t)(hi[r] + kap) << 32) | (t >> 32);
        }
        // add the carry of the lane below (< 2^46), leaving a 1-bit carry g
        const uint64_t cp = ((uint64_t)shfl_up1((uint32_t)(c >> 32)) << 32) | shfl_up1((uint32_t)c);
        uint64_t acc = (uint64_t)z[0] + (uint32_t)cp;
        z[0] = (uint32_t)acc;
        acc = (acc >> 32) + (cp >> 32) + z[1];
        z[1] = (uint32_t)acc;
        acc = (acc >> 32) + z[2];
        z[2] = (uint32_t)acc;
        acc = (acc >> 32) + z[3];
        z[3] = (uint32_t)acc;
        const bool g = (acc >> 32) != 0;
        const bool pr = (z[0] & z[1] & z[2] & z[3]) == 0xFFFFFFFFu;
        const uint64_t G = ballot(g), P = ballot(pr), X = G | P;
        const uint64_t sum = X + G;
        uint32_t ci = (uint32_t)(((sum ^ X ^ G) >> l) & 1u);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            z[r] += ci;
            ci &= (z[r] == 0u) ? 1u : 0u;
        }
        if (k0 + 3 < ncols) {
            store4(p + k0, z[0], z[1], z[2], z[3]);
        } else {
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (k0 + r < ncols) p[k0 + r] = z[r];
        }
        if (l == kLanes - 1) {
            const uint64_t e = c + (sum < X ? 1u : 0u);
            ctl[kCtlStrip + 2 * s] = (uint32_t)e;
            ctl[kCtlStrip + 2 * s + 1] = (uint32_t)(e >> 32);
        }
    }
    // add the strip carries; the product fits ncols limbs (or is taken mod B^ncols)
    addsub<T>(ctl, ncols, false, 0u, Span{p, 0, ncols}, StripCarries{ctl + kCtlStrip, nstrips},
              Store{p, 0, ncols});
    return read_prec<T>(ctl);
}

// --------------------------------------------------------- short division

// quotient of the n-limb number d (a view) by the single limb dv > 0:
// qout(k, limb) for k in [0, n); returns the remainder (same on all threads).
// Thread t divides the chunk [t*C, t*C + C): pass 1 reduces each chunk mod dv,
// one thread chains the chunk remainders from the top (R_t-1 = R_t * B^C +
// rem_t mod dv), pass 2 divides each chunk starting from its incoming R.
// `scratch` holds 2*T words.
template <int T, class FD, class FO>
MP_DEV uint32_t shortdiv(uint32_t *ctl, uint32_t *scratch, int n, const FD &d, uint32_t dv, const FO &qout)
{
    sync();
    const int C = imax((n + T - 1) / T, imin(n, 64));
    const int nch = (n + C - 1) / C;
    const int t = tid(), k0 = t * C;
    if (t < nch) {
        uint64_t r = 0;
        for (int j = C - 1; j >= 0; j--) {
            const int k = k0 + j;
            const uint32_t x = k < n ? d(k) : 0u;
            r = ((r << 32) | x) % dv;
        }
        scratch[t] = (uint32_t)r;
    }
    sync();
    if (t == 0) {
        uint64_t beta = 1;
        for (int j = 0; j < C; j++) beta = (beta << 32) % dv;   // B^C mod dv
        uint64_t R = 0;
        for (int c = nch - 1; c >= 0; c--) {
            scratch[T + c] = (uint32_t)R;
            R = ((R * beta) % dv + scratch[c]) % dv;
        }
        ctl[kCtlBcast] = (uint32_t)R;
    }
    sync();
    if (t < nch) {
        uint64_t R = scratch[T + t];
        for (int j = C - 1; j >= 0; j--) {
            const int k = k0 + j;
            if (k < n) {
                const uint64_t num = (R << 32) | d(k);
                qout(k, (uint32_t)(num / dv));
                R = num % dv;
            }
        }
    }
    return ctl[kCtlBcast];
}

}  // namespace mp
