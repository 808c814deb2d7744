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
constexpr int kHeadMaxLimbs = 9 * kLanes;   // longest operand of a one-wave addsub (9 limbs per lane)

// control block at the start of the instance's LDS (32-bit words)
constexpr int kCtlRed = 0;       // 3 x 16 per-wave reduction slots
constexpr int kCtlSticky = 32;   // 16 per-wave sticky flags of an addsub (the third reduction row)
constexpr int kCtlScan = 48;     // 16 x (generate, propagate) wave summaries
constexpr int kCtlPrec = 80;     // 16 per-wave result-precision slots of the last addsub
constexpr int kCtlStrip = 96;    // 2 words per strip carry, up to 72 strips
constexpr int kCtlBcast = 240;   // 16 broadcast scalars
constexpr int kCtlWords = 256;
constexpr int kMaxStrips = 72;
constexpr int kHeadStrips = 4;  // strips of a head's products (one wave, short operands)
constexpr int kHeadCtlWords = kCtlStrip + 2 * kHeadStrips;   // a head's control block (no broadcast slots)

// barrier of the T threads working on an instance: the workgroup, or (T = 64)
// a single wave, which needs no hardware barrier
template <int T>
MP_DEV void bar()
{
    if constexpr (T > kLanes) sync();
    else wave_sync();
}

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

// strip carries of a product: carry e_s (64-bit) enters at column
// (s+1)*width - off
struct StripCarries {
    const uint32_t *sc;
    int nstrips;
    int off;
    int width;
    MP_DEV uint32_t operator()(int k) const
    {
        const int kk = k + off;
        int s = (kk / width) - 1, o = kk % width;
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

MP_DEV uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }

// maximum of x over the wave (the same value on every lane): pairs, quads,
// half rows and rows by DPP permutations, then row 1 and 3 take the row below
// (row_bcast:15) and rows 2 and 3 take lane 31 (row_bcast:31), so lane 63
// holds the maximum of all 64 lanes
MP_DEV uint32_t wave_max(uint32_t x)
{
    x = umax(x, dpp<kDppQuadSwap1>(x));
    x = umax(x, dpp<kDppQuadSwap2>(x));
    x = umax(x, dpp<kDppRowHalfMirror>(x));
    x = umax(x, dpp<kDppRowMirror>(x));
    x = umax(x, dpp<kDppRowBcast15, 0xA>(x));
    x = umax(x, dpp<kDppRowBcast31, 0xC>(x));
    return readlane(x, kLanes - 1);
}

// maximum of one value per thread over the workgroup (same on every thread)
template <int T>
MP_DEV uint32_t wg_max(uint32_t *ctl, uint32_t x)
{
    constexpr int W = T / kLanes;
    x = wave_max(x);
    if constexpr (W == 1) return uniform(x);
    if (lane() == 0) ctl[kCtlRed + tid<T>() / kLanes] = x;
    bar<T>();
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
    const int w = uniform(tid<T>() / kLanes);
#pragma unroll
    for (int i = 0; i < N; i++) {
        const uint32_t m = wave_max(x[i]);
        if (lane() == 0) ctl[kCtlRed + 16 * i + w] = m;
    }
    bar<T>();
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

// max over k in [0, n) of f(k)  (f(k) >= 0).  Four independent reads per
// step, so their latencies overlap.
template <int T, class F>
MP_DEV int reduce_max(uint32_t *ctl, int n, const F &f)
{
    bar<T>();
    uint32_t m = 0;
    int k = tid<T>();
    for (; k + 3 * T < n; k += 4 * T) {
        const uint32_t y0 = f(k), y1 = f(k + T), y2 = f(k + 2 * T), y3 = f(k + 3 * T);
        m = umax(m, umax(umax(y0, y1), umax(y2, y3)));
    }
    for (; k < n; k += T) m = umax(m, f(k));
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
template <int T, int CM, class FX, class FY, class FO, class FS>
MP_DEV uint32_t addsub_chunk(uint32_t *ctl, int n, int C, bool sub, uint32_t cin,
                             const FX &x, const FY &y, const FO &out, const FS &stk, int scan)
{
    constexpr int W = T / kLanes;
    constexpr bool kPre = CM <= 9;   // short chunks: all reads first, so their latencies overlap
    constexpr int CP = kPre ? CM : 1;
    const int k0 = tid<T>() * C;
    uint32_t z[CM], av[CP], bv[CP];
    uint32_t c = 0;
    bool prop = true;
    const bool sk = stk.any(tid<T>());   // this thread's part of the sticky carry-in
    if (kPre) {
#pragma unroll
        for (int j = 0; j < CP; j++) {
            const int k = k0 + j;
            const bool in = j < C && k < n;
            av[j] = in ? x(k) : 0u;
            bv[j] = in ? y(k) : 0u;
        }
    }
#pragma unroll
    for (int j = 0; j < CM; j++) {
        const int k = k0 + j;
        if (j < C && k < n) {
            const uint32_t a = kPre ? av[j < CP ? j : 0] : x(k), b = kPre ? bv[j < CP ? j : 0] : y(k);
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
    const int w = uniform(tid<T>() / kLanes);
    const uint64_t SK = FS::kActive ? ballot(sk) : 0;
    uint32_t cin_w = cin, cout = cin;
    if constexpr (W == 1) {
        // one wave: its own summary is the whole scan
        if (FS::kActive && SK) cin = cin_w = 1u;
        cout = (s0 < X ? 1u : 0u) | ((~P == 0 ? 1u : 0u) & cin);
    } else {
        if (lane() == 0) {
            ctl[scan + 2 * w] = s0 < X ? 1u : 0u;      // wave generates
            ctl[scan + 2 * w + 1] = (~P == 0) ? 1u : 0u;  // wave propagates
            if (FS::kActive) ctl[kCtlSticky + w] = SK ? 1u : 0u;
        }
        bar<T>();
        if constexpr (FS::kActive) {
#pragma unroll
            for (int v = 0; v < W; v++) cin |= ctl[kCtlSticky + v];
            cin_w = cout = cin;
        }
        // scan of the wave summaries: carry into this wave, and out of the number
#pragma unroll
        for (int v = 0; v < W; v++) {
            if (v == w) cin_w = cout;
            cout = ctl[scan + 2 * v] | (ctl[scan + 2 * v + 1] & cout);
        }
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
    bar<T>();
    uint32_t r = 0;
#pragma unroll
    for (int v = 0; v < W; v++) {
        const uint32_t y = ctl[kCtlPrec + v];
        r = r > y ? r : y;
    }
    const int p = (int)uniform(r) - off;
    return p > 0 ? p : 0;
}

// no sticky carry-in
struct NoSticky {
    static constexpr bool kActive = false;
    MP_DEV bool any(int) const { return false; }
};

// sticky carry-in: 1 when any limb p[j], j in [0, n), is nonzero (the threads
// each test a strided share before the carry scan)
template <int T>
struct StickyAny {
    static constexpr bool kActive = true;
    const uint32_t *p;
    int n;
    MP_DEV bool any(int t) const
    {
        bool r = false;
        for (int j = t; j < n; j += T) r = r || p[j] != 0u;
        return r;
    }
};

// addsub without its leading barrier, for a caller that has just passed one
// and touched nothing since that addsub reads or writes.  `scan` is the
// control slot range of the wave summaries (2 words per wave): kCtlScan, or
// kCtlRed for a second addsub that follows the first without a barrier (its
// summaries must not overwrite those the first is still reading).
template <int T, class FX, class FY, class FO, class FS = NoSticky>
MP_DEV uint32_t addsub_nb(uint32_t *ctl, int n, bool sub, uint32_t cin,
                          const FX &x, const FY &y, const FO &out, const FS &stk = FS{}, int scan = kCtlScan)
{
    // odd chunk length: lanes then touch LDS with an odd word stride (no bank conflicts)
    const int C = ((n + T - 1) / T) | 1;
    if (C == 1) return addsub_chunk<T, 1>(ctl, n, C, sub, cin, x, y, out, stk, scan);
    if (C == 3) return addsub_chunk<T, 3>(ctl, n, C, sub, cin, x, y, out, stk, scan);
    if (C <= 5) return addsub_chunk<T, 5>(ctl, n, C, sub, cin, x, y, out, stk, scan);
    // a single wave (a head) handles at most kHeadMaxLimbs limbs per operation
    if constexpr (T == kLanes) {
        return addsub_chunk<T, 9>(ctl, n, C, sub, cin, x, y, out, stk, scan);
    } else {
        if (C <= 9) return addsub_chunk<T, 9>(ctl, n, C, sub, cin, x, y, out, stk, scan);
        return addsub_chunk<T, kCMax>(ctl, n, C, sub, cin, x, y, out, stk, scan);
    }
}

template <int T, class FX, class FY, class FO, class FS = NoSticky>
MP_DEV uint32_t addsub(uint32_t *ctl, int n, bool sub, uint32_t cin,
                       const FX &x, const FY &y, const FO &out, const FS &stk = FS{})
{
    bar<T>();
    return addsub_nb<T>(ctl, n, sub, cin, x, y, out, stk);
}

// dst[k] = src(k) for k in [0, n), zero for k in [n, clear)
template <int T, class FS>
MP_DEV void copy(uint32_t *dst, int n, int clear, const FS &src)
{
    bar<T>();
    const int e = imax(n, clear);
    int k = tid<T>();
    for (; k + 3 * T < e; k += 4 * T) {
        const uint32_t y0 = k < n ? src(k) : 0u, y1 = k + T < n ? src(k + T) : 0u;
        const uint32_t y2 = k + 2 * T < n ? src(k + 2 * T) : 0u, y3 = k + 3 * T < n ? src(k + 3 * T) : 0u;
        dst[k] = y0;
        dst[k + T] = y1;
        dst[k + 2 * T] = y2;
        dst[k + 3 * T] = y3;
    }
    for (; k < e; k += T) dst[k] = k < n ? src(k) : 0u;
}

// ------------------------------------------------------------- multiply

// Turns the 96-bit column sums lo/hi of strip s (first column K0; lane l
// holds columns K0 + 4l .. K0 + 4l + 3) into limbs: lane-local carry, the
// neighbour's carry by shuffle, then a carry-lookahead over the wave from
// ballots.  The limbs of columns in [c0, ncols) go to p (c0 a multiple of 4);
// the carry leaving the strip goes to the strip carry slot s (added to the
// next strip by the final addsub).
MP_DEV void strip_resolve(uint32_t *ctl, int s, int K0, const uint64_t (&lo)[4], const uint32_t (&hi)[4],
                          uint32_t *p, int c0, int ncols)
{
    const int l = lane();
    const int k0 = K0 + l * kRCol;
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
    if (k0 >= c0) {
        if (k0 + 3 < ncols) {
            store4(p + k0, z[0], z[1], z[2], z[3]);
        } else {
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (k0 + r < ncols) p[k0 + r] = z[r];
        }
    }
    if (l == kLanes - 1) {
        const uint64_t e = c + (sum < X ? 1u : 0u);
        ctl[kCtlStrip + 2 * s] = (uint32_t)e;
        ctl[kCtlStrip + 2 * s + 1] = (uint32_t)(e >> 32);
    }
}


// p[c0, ncols) += the strip carries (strip s, based at column base, passes
// its carry to column base + (s+1) kStrip), mod B^(ncols - c0); returns the
// precision as mul's (or -1 without want_prec, saving a barrier)
template <int T>
MP_DEV int add_strip_carries(uint32_t *ctl, uint32_t *p, int c0, int ncols, int nstrips, int base, bool want_prec,
                             int width = kStrip)
{
    const int n = ncols - c0;
    addsub<T>(ctl, n, false, 0u, Span{p + c0, 0, n}, StripCarries{ctl + kCtlStrip, nstrips, c0 - base, width},
              Store{p + c0, 0, n});
    if (!want_prec) return -1;
    const int e = read_prec<T>(ctl);
    return e ? e + c0 : 0;
}

// First column of the lowest strip.  A product kept only mod B^ncols (c0 = 0,
// ncols short of the full width) ends its top strip at ncols (rounded up to 8
// limbs) so that the partial strip is the lowest one, which has the fewest
// products; other products start at c0, leaving the cheap top strip partial.
MP_DEV int strip_base(int c0, int ncols, int nfull, int nstrips, int width = kStrip)
{
    return (c0 == 0 && ncols < nfull) ? ((ncols + 7) & ~7) - nstrips * width : c0;
}

// p[c0, ncols) = the columns c0 .. ncols-1 of a * b, ncols <= na + nb (with
// c0 = 0 and ncols = na + nb, the full product): every limb product of those
// columns with all carries between them, and no carry from below c0, so
// limbs [c0, ncols) hold floor(T / B^c0) mod B^(ncols-c0) for T = the sum of
// the products in columns >= c0.  c0 is a multiple of 8; p below c0 is not
// written.  Returns the precision of the result (c0 + the precision of the
// stored limbs, or 0 when they are all zero).  `a` (na limbs, any LDS position, readable up to 3 limbs past
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
               const uint32_t *a, int na, const uint32_t *bw, int nb, int c0 = 0, bool want_prec = true)
{
    constexpr int W = T / kLanes;
    bar<T>();
    if (na == 0 || nb == 0 || ncols <= c0) {
        for (int k = c0 + tid<T>(); k < ncols; k += T) p[k] = 0u;
        return 0;
    }
    const int nstrips = (ncols - c0 + kStrip - 1) / kStrip;
    const int base = strip_base(c0, ncols, na + nb, nstrips);
    const int w = uniform(tid<T>() / kLanes), l = lane();
    for (int s = w; s < nstrips; s += W) {
        const int K0 = base + s * kStrip, k0 = K0 + l * kRCol;
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
        strip_resolve(ctl, s, K0, lo, hi, p, c0, ncols);
    }
    MP_PT(4);
    return add_strip_carries<T>(ctl, p, c0, ncols, nstrips, base, want_prec);
}

// The same product for a single wave, one column per lane: for short
// operands, where most lanes of a 256-column strip would be idle.  The wave
// walks strips of 64 columns from the bottom; lane l of strip s sums column
// K0 + l over the rows in four independent 96-bit accumulators (rows i, i+1,
// i+2, i+3), reading window limb k - i of each row.  The column sums
// S_l = s0 + s1 B + s2 B^2 become limbs as t_l = s0_l + s1_(l-1) + s2_(l-2)
// (neighbour values by DPP lane shifts) plus, in lanes 0 and 1, the carry E
// of the strip below; then y_l = lo(t_l) + hi(t_(l-1)) has a one-bit carry,
// resolved by the ballot lookahead.  The carry leaving the strip (into its
// next two columns) is kept in scalar registers for the next strip, so no
// pass over the stored limbs follows; the top strip's carry lies above
// ncols and is dropped.
template <int T>
MP_DEV int mul1(uint32_t *ctl, uint32_t *p, int ncols, const uint32_t *a, int na, const uint32_t *bw, int nb, int c0,
                bool want_prec)
{
    static_assert(T == kLanes, "mul1 is the single-wave product");
    (void)ctl;
    wave_sync();
    if (na == 0 || nb == 0 || ncols <= c0) {
        for (int k = c0 + lane(); k < ncols; k += kLanes) p[k] = 0u;
        return 0;
    }
    const int nstrips = (ncols - c0 + kLanes - 1) / kLanes;
    const int base = strip_base(c0, ncols, na + nb, nstrips, kLanes);
    const int l = lane();
    uint64_t E = 0;        // carry into columns K0, K0 + 1 of the current strip
    int top = 0;           // 1 + highest nonzero stored column
    for (int s = 0; s < nstrips; s++) {
        const int K0 = base + s * kLanes, k = K0 + l;
        const int ilo = imax(0, K0 - nb + 1);
        const int ihi = imin(na, imin(K0 + kLanes, ncols));
        uint64_t lo[4] = {0, 0, 0, 0};
        uint32_t hi[4] = {0, 0, 0, 0};
        const uint32_t *wp = bw + k;
        int i = ilo;
        for (; i + 3 < ihi; i += 4) {
            const uint32_t w0 = wp[-i], w1 = wp[-i - 1], w2 = wp[-i - 2], w3 = wp[-i - 3];
            mac4x(lo, hi, a[i], w0, a[i + 1], w1, a[i + 2], w2, a[i + 3], w3);
        }
        if (i < ihi) {
            const uint32_t a1 = i + 1 < ihi ? a[i + 1] : 0u, a2 = i + 2 < ihi ? a[i + 2] : 0u;
            mac4x(lo, hi, a[i], wp[-i], a1, wp[-i - 1], a2, wp[-i - 2], 0u, 0u);
        }
        // the four partial sums of column k, added exactly (each below 2^(64 + 7))
        uint64_t sl = lo[0];
        uint32_t sh = hi[0];
#pragma unroll
        for (int r = 1; r < 4; r++) {
            const uint64_t t = sl + lo[r];
            sh += hi[r] + (t < sl ? 1u : 0u);
            sl = t;
        }
        // limbs: t = s0 + s1 of the lane below + s2 of the lane two below (+ E at the bottom)
        const uint32_t s1m = shfl_up1((uint32_t)(sl >> 32)), s2m = shfl_up2(sh);
        const uint32_t e = l == 0 ? (uint32_t)E : l == 1 ? (uint32_t)(E >> 32) : 0u;
        const uint64_t t = (uint64_t)(uint32_t)sl + s1m + s2m + e;     // < 4 B
        const uint32_t cm = shfl_up1((uint32_t)(t >> 32));                // 0..3 from the lane below
        const uint64_t y = (uint64_t)(uint32_t)t + cm;
        uint32_t z = (uint32_t)y;
        const bool g = (y >> 32) != 0, pr = z == 0xFFFFFFFFu;
        const uint64_t G = ballot(g), P = ballot(pr), X = G | P;
        const uint64_t sum = X + G;
        z += (uint32_t)(((sum ^ X ^ G) >> l) & 1u);
        const bool st = k >= c0 && k < ncols;
        if (st) p[k] = z;
        const uint64_t nz = ballot(st && z != 0u);
        if (nz) top = K0 + kLanes - __builtin_clzll(nz);
        // carry into the next strip: what lanes 62 and 63 pass upward plus the lookahead's carry out
        const uint32_t s2_62 = readlane(sh, 62), s2_63 = readlane(sh, 63);
        const uint32_t s1_63 = readlane((uint32_t)(sl >> 32), 63), c_63 = readlane((uint32_t)(t >> 32), 63);
        E = (uint64_t)s1_63 + s2_62 + c_63 + (sum < X ? 1u : 0u) + ((uint64_t)s2_63 << 32);
    }
    return want_prec ? top : -1;
}

// ---------------------------------------------------- matrix-core product
//
// Exact products on the int8 matrix cores.  A number is rewritten in radix 256
// with balanced digits in [-128, 127]:  x = sum d_i 256^i.  Adding 0x80 to
// every byte and carrying (x + 0x8080...80) makes the carry into byte i exactly
// [b_i + c_i >= 128], so the digit bytes are (x + 0x8080...80) XOR 0x8080...80
// limb by limb, and the carry out of the top limb is one more digit (0 or 1).
// For balanced digits the byte-column sums M_k = sum_{i+j=k} d_i e_j are exact
// int32 values (|M_k| < 2^29 up to 8192-limb operands), and
// x*y = sum_k M_k 256^k.
//
// Strip s of the product (limb columns 256s .. 256s+255 = byte columns
// 1024s .. 1024s+1023) is one 32x32 matrix-core tile accumulated over the
// diagonals d:  D[t][n] += sum_r X_d[t][r] Y_d[r][n]  with
//   X_d[t][r] = e_(32d + t - r)            (Toeplitz slice of the short operand)
//   Y_d[r][n] = d_(32(32s + n - d) + r)   (32 consecutive 32-byte blocks of the long one)
// so D[t][n] = M_(32(32s + n) + t).  X is read from the byte-reversed digits of
// the short operand (16 bytes per lane at any byte offset: 5 words and four
// byte aligns); Y is one aligned 16-byte load per lane.  The accumulator of
// lane (n, h) ends up holding the four byte sums of limb columns
// 8n + 2q + h (q = 0..3) of the strip.
//
// X_d depends on d only, so a wave that owns two adjacent strips loads each
// X_d once for both (the diagonal ranges of strips s and s+1 overlap in all
// but 32 diagonals at each end).  The long operand's digits are held in two
// planes of 16-byte half-blocks (plane h holds bytes 16h .. 16h+15 of every
// 32-byte block), so the lanes of either half-wave read 32 consecutive
// 16-byte chunks of one plane: the Y load has no bank conflicts.

// (limb k of x) + 0x80808080 for k < n: the radix-256 balancing addend
struct Bal80 {
    int n;
    MP_DEV uint32_t operator()(int k) const { return k < n ? 0x80808080u : 0u; }
};

constexpr int kYPadBlk = 31;   // zero blocks each digit plane needs on each side
constexpr int kXPad = 16;      // zero words the reversed short operand needs on each side

// words from the start of plane 0 to the start of plane 1 for an ny-limb long operand
MP_DEV int mfma_plane(int ny) { return 4 * (((ny + 8) >> 3) + kYPadBlk); }
// one past the last word of the planes that can be nonzero
MP_DEV int mfma_ext(int ny) { return mfma_plane(ny) + 4 * ((ny + 8) >> 3); }

// word of the planes holding limb k: block k / 8, plane (k / 4) % 2, word k % 4
MP_DEV int plane_word(int k, int ly) { return ((k >> 1) & ~3) + (k & 3) + ((k >> 2) & 1) * ly; }

// balanced digit limbs in the two planes: limb k, k in [0, n]
struct StoreBal {
    uint32_t *p;
    int n, ly;
    MP_DEV void operator()(int k, uint32_t z) const { p[plane_word(k, ly)] = k < n ? z ^ 0x80808080u : z; }
};

// balanced digit limbs byte-reversed: dst[n - k] = bytes of limb k reversed
struct StoreBalRev {
    uint32_t *p;
    int n;
    MP_DEV void operator()(int k, uint32_t z) const { p[n - k] = bswap(k < n ? z ^ 0x80808080u : z); }
};

// Balanced digits of the long operand (ny limbs) into the planes at yb and of
// the short operand (nx limbs) byte-reversed into xr[0 .. nx].  Plane 0 holds
// blocks [0, nb) at yb[0, 4 nb), nb = (ny + 8) / 8, plane 1 the same at
// yb + mfma_plane(ny); each plane has kYPadBlk zero blocks on both sides (the
// pad below plane 0 must already be zero; the rest up to mfma_ext(ny), and
// the words from there up to yclear, are written here).  xr gets kXPad zero
// words on both sides.  The short operand must not live in xr's padded range
// unless it is exactly the limbs the conversion reads first (the reads all
// precede the writes inside addsub).
//
// One barrier orders every earlier use of yb and xr before this; the two
// conversions then follow each other without one (they read only x and y,
// write disjoint digits, and keep their wave summaries in separate slots).
//
// With x_ready the short operand's digits are already in xr (the same number
// converted by an earlier call) and only the long operand is converted.
template <int T, class FY, class FX>
MP_DEV void mfma_operands(uint32_t *ctl, const FY &y, int ny, uint32_t *yb, int yclear,
                          const FX &x, int nx, uint32_t *xr, bool x_ready = false)
{
    bar<T>();
    const int nb = (ny + 8) >> 3, ly = mfma_plane(ny);
    // the top block's limbs past the digits, the pad above plane 0 (= the pad
    // below plane 1), the pad above plane 1 and what lies above it up to yclear
    for (int k = ny + 1 + tid<T>(); k < 8 * nb; k += T) yb[plane_word(k, ly)] = 0u;
    for (int k = tid<T>(); k < 4 * kYPadBlk; k += T) yb[4 * nb + k] = 0u;
    const int hiend = imax(ly + 4 * nb + 4 * kYPadBlk, yclear);
    for (int k = ly + 4 * nb + tid<T>(); k < hiend; k += T) yb[k] = 0u;
    addsub_nb<T>(ctl, ny + 1, false, 0u, y, Bal80{ny}, StoreBal{yb, ny, ly});
    if (x_ready) return;
    addsub_nb<T>(ctl, nx + 1, false, 0u, x, Bal80{nx}, StoreBalRev{xr, nx}, NoSticky{}, kCtlRed);
    // every read of x happened before addsub's internal barrier, and the pads
    // are disjoint from the digits written: no barrier needed here
    for (int k = tid<T>(); k < 2 * kXPad; k += T) {
        if (k < kXPad) xr[k - kXPad] = 0u;
        else xr[nx + 1 + k - kXPad] = 0u;
    }
}

// X_d of this lane: 16 bytes of the reversed short digits from word xp on,
// shifted by sft bytes (five words read, four byte aligns)
struct XRaw {
    uint32_t w0, w1, w2, w3, w4;
};
struct XFrag {
    uint32_t a, b, c, d;
};

MP_DEV XRaw xraw(const uint32_t *xp) { return XRaw{xp[0], xp[1], xp[2], xp[3], xp[4]}; }
MP_DEV XFrag xfrag(const XRaw &r, uint32_t sft)
{
    return XFrag{alignbyte(r.w1, r.w0, sft), alignbyte(r.w2, r.w1, sft), alignbyte(r.w3, r.w2, sft),
                 alignbyte(r.w4, r.w3, sft)};
}

// Scheduling of one diagonal step: its LDS reads first (all in flight
// together), then the vector ALU work (byte aligns, addresses), then the
// matrix-core products; without this the scheduler of a kernel near its
// register limit interleaves them and pays one LDS round trip per product.
MP_DEV void sched_loads_first()
{
    __builtin_amdgcn_sched_group_barrier(0x100, 32, 0);   // DS reads
    __builtin_amdgcn_sched_group_barrier(0x002, 32, 0);   // VALU
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);    // MFMA
}

MP_DEV MfmaAcc mfma_x(MfmaAcc acc, const XFrag &x, const Limb4 &y)
{
    return mfma_i8(acc, x.a, x.b, x.c, x.d, y.x, y.y, y.z, y.w);
}

// The limbs of strip s (its accumulator acc) into p, its carry into the strip slot
MP_DEV void mfma_strip_out(uint32_t *ctl, const MfmaAcc &acc, int s, int base, uint32_t *p, int c0, int ncols)
{
    const int l = lane(), t = l & 31, h = l >> 5;
    // limb columns 8t + 2q + h of the strip, biased to be non-negative: column
    // base gets 2^56, every other column 2^56 - 2^24 (the biases telescope to
    // 2^24 B^ncols, i.e. to 0 mod B^ncols)
    uint32_t tl[4], th[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t m = (int64_t)mfma_get(acc, 4 * q) + (int64_t)mfma_get(acc, 4 * q + 1) * 256 +
                          (int64_t)mfma_get(acc, 4 * q + 2) * 65536 + (int64_t)mfma_get(acc, 4 * q + 3) * 16777216;
        const int col = s * kStrip + 8 * t + 2 * q + h;   // relative to base
        const uint64_t v = (uint64_t)(m + (col == 0 ? ((int64_t)1 << 56) : ((int64_t)1 << 56) - ((int64_t)1 << 24)));
        tl[q] = (uint32_t)v;
        th[q] = (uint32_t)(v >> 32);
    }
    // regroup: lane l takes columns 4l .. 4l+3; column 4l + j sits in lane
    // (l >> 1) + 32 (j & 1), slot q = 2 (l & 1) + (j >> 1)
    uint64_t lo[4];
    const uint32_t hi[4] = {0u, 0u, 0u, 0u};
    const int par = l & 1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int src = (l >> 1) + 32 * (j & 1);
        const uint32_t al = shfl(tl[j >> 1], src), ah = shfl(th[j >> 1], src);
        const uint32_t bl = shfl(tl[2 + (j >> 1)], src), bh = shfl(th[2 + (j >> 1)], src);
        lo[j] = par ? (((uint64_t)bh << 32) | bl) : (((uint64_t)ah << 32) | al);
    }
    strip_resolve(ctl, s, base + s * kStrip, lo, hi, p, c0, ncols);
}

// p[c0, ncols) = the columns c0 .. ncols-1 of x * y (as mul, c0 a multiple
// of 8) from the digits prepared by mfma_operands (yb: the planes of the ny+1
// digit limbs of the long operand, xr: nx+1 reversed limbs of the short);
// returns the precision of the result.  With c0 > 0 the columns are those of
// the balanced radix-256 digit products, T = sum of M_k 256^k over byte
// columns k >= 4 c0, which differs from the limb-product sum by less than
// 2^16 c0 B^c0 in either direction.
//
// A wave takes two of its strips sa < sb at a time: diagonals only sa
// reaches, then those both reach (one X_d, two Y loads, two products), then
// those only sb reaches.  With at least two pairs of adjacent strips per wave
// the pairs are (2q, 2q + 1), dealt round robin (pair q to wave q mod W);
// otherwise wave w keeps strips w, w + W, w + 2W, ... and pairs them in that
// order (strips W apart share the diagonals where their ranges overlap).
template <int T>
MP_DEV int mul_mfma(uint32_t *ctl, uint32_t *p, int ncols, const uint32_t *yb, int ny,
                    const uint32_t *xr, int nx, int c0 = 0, bool want_prec = true)
{
    constexpr int W = T / kLanes;
    bar<T>();
    if (ncols <= c0) return 0;
    const int nstrips = (ncols - c0 + kStrip - 1) / kStrip;
    const int base = strip_base(c0, ncols, nx + ny, nstrips);
    const int w = uniform(tid<T>() / kLanes), l = lane();
    const int t = l & 31, h = l >> 5;
    const int nyblk = (ny + 1 + 7) >> 3;          // 32-byte blocks of the long digits
    const int R0 = 4 * (nx + 1) - 1;              // reversed byte x holds digit R0 - x
    const int dmax = (4 * (nx + 1) + 30) >> 5;    // last diagonal touching the short digits
    // Row t, half h of X_d starts at reversed byte R0 - 32 d - t + 16 h: word
    // (ox >> 2) - 8 d with the same byte shift ox & 3 for every d.  Y_d of a
    // strip whose first block is S0 is block S0 + t - d of plane h.
    const int ox = R0 - t + 16 * h;
    const uint32_t sft = (uint32_t)ox & 3u;
    const uint32_t *x0 = xr + (ox >> 2);
    const uint32_t *y0 = yb + h * mfma_plane(ny) + 4 * t;
    // strips sa and (if sb < nstrips) sb > sa.  Where one strip runs alone,
    // a step keeps four diagonals' operands in flight and chains their
    // products on the strip's accumulator (the other accumulator is not yet
    // or no longer live there, which leaves the registers for the operands);
    // where both run, a step is one diagonal whose X fragment feeds both.
    auto step = [&](int sa, int sb) {
        const bool two = sb < nstrips;
        const int SA = 32 * sa + (base >> 3), SB = 32 * sb + (base >> 3);   // first 8-limb blocks
        const int dloA = uniform(imax(0, SA - nyblk + 1)), dhiA = uniform(imin(dmax, SA + 31));
        const int dloB = two ? uniform(imax(0, SB - nyblk + 1)) : dhiA + 1;
        const int dhiB = two ? uniform(imin(dmax, SB + 31)) : dhiA;
        // diagonal d: X_d from x0 - 8 d, Y_d of strip sa from yA - 4 d, of sb from yB - 4 d
        const uint32_t *yA = y0 + 4 * SA, *yB = y0 + 4 * SB;
        MfmaAcc accA = mfma_zero(), accB = mfma_zero();
        int d = dloA;
        // strip sa alone: four diagonals' operands in flight per step, one
        // accumulator (its chain of products costs about what the LDS round
        // trip of the next step does)
        const int eA = imin(dhiA, dloB - 1);
        // (one wave alone on an instance, a head, keeps one diagonal per step:
        // its registers hold the vector-ALU product's state too)
        for (; T > kLanes && d + 3 <= eA; d += 4) {
            const XRaw r0 = xraw(x0 - 8 * d), r1 = xraw(x0 - 8 * d - 8);
            const XRaw r2 = xraw(x0 - 8 * d - 16), r3 = xraw(x0 - 8 * d - 24);
            const Limb4 y0v = load4(yA - 4 * d), y1v = load4(yA - 4 * d - 4);
            const Limb4 y2v = load4(yA - 4 * d - 8), y3v = load4(yA - 4 * d - 12);
            accA = mfma_x(accA, xfrag(r0, sft), y0v);
            accA = mfma_x(accA, xfrag(r1, sft), y1v);
            accA = mfma_x(accA, xfrag(r2, sft), y2v);
            accA = mfma_x(accA, xfrag(r3, sft), y3v);
            sched_loads_first();
        }
        for (; d <= eA; d++) {
            const XRaw r0 = xraw(x0 - 8 * d);
            const Limb4 y0v = load4(yA - 4 * d);
            accA = mfma_x(accA, xfrag(r0, sft), y0v);
            sched_loads_first();
        }
        // both strips: one diagonal per step (its two products are independent)
        for (; d <= dhiA; d++) {
            const XRaw r0 = xraw(x0 - 8 * d);
            const Limb4 ya0 = load4(yA - 4 * d), yb0 = load4(yB - 4 * d);
            const XFrag xf = xfrag(r0, sft);
            accA = mfma_x(accA, xf, ya0);
            accB = mfma_x(accB, xf, yb0);
            sched_loads_first();
        }
        mfma_strip_out(ctl, accA, sa, base, p, c0, ncols);
        if (!two) return;
        // strip sb alone (from dloB on, if strip sa ended before it began)
        d = imax(d, dloB);
        for (; T > kLanes && d + 3 <= dhiB; d += 4) {
            const XRaw r0 = xraw(x0 - 8 * d), r1 = xraw(x0 - 8 * d - 8);
            const XRaw r2 = xraw(x0 - 8 * d - 16), r3 = xraw(x0 - 8 * d - 24);
            const Limb4 y0v = load4(yB - 4 * d), y1v = load4(yB - 4 * d - 4);
            const Limb4 y2v = load4(yB - 4 * d - 8), y3v = load4(yB - 4 * d - 12);
            accB = mfma_x(accB, xfrag(r0, sft), y0v);
            accB = mfma_x(accB, xfrag(r1, sft), y1v);
            accB = mfma_x(accB, xfrag(r2, sft), y2v);
            accB = mfma_x(accB, xfrag(r3, sft), y3v);
            sched_loads_first();
        }
        for (; d <= dhiB; d++) {
            const XRaw r0 = xraw(x0 - 8 * d);
            const Limb4 y0v = load4(yB - 4 * d);
            accB = mfma_x(accB, xfrag(r0, sft), y0v);
            sched_loads_first();
        }
        mfma_strip_out(ctl, accB, sb, base, p, c0, ncols);
    };
    const int npairs = (nstrips + 1) >> 1;
    if constexpr (T == kLanes) {
        for (int s = 0; s < nstrips; s++) step(s, nstrips);   // one accumulator live at a time
    } else if (npairs >= 2 * W) {
        for (int q = w; q < npairs; q += W) step(2 * q, 2 * q + 1);
    } else {
        for (int s = w; s < nstrips; s += 2 * W) step(s, s + W);
    }
    MP_STAMP(10);   // the first wave's strips done
    MP_PT(4);
    return add_strip_carries<T>(ctl, p, c0, ncols, nstrips, base, want_prec);
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
    bar<T>();
    const int C = imax((n + T - 1) / T, imin(n, 64));
    const int nch = (n + C - 1) / C;
    const int t = tid<T>(), k0 = t * C;
    if (t < nch) {
        uint64_t r = 0;
        for (int j = C - 1; j >= 0; j--) {
            const int k = k0 + j;
            const uint32_t x = k < n ? d(k) : 0u;
            r = ((r << 32) | x) % dv;
        }
        scratch[t] = (uint32_t)r;
    }
    bar<T>();
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
    bar<T>();
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
