// One multi-precision product, shifted inverse or division per workgroup.
//
// The division is the paper's shifted-inverse method:
//   Alg. 1 (Shinv): special cases, 2-limb initial approximation
//                   w = floor(B^3 / (v_{k-1} + v_k B)), then Refine: Newton
//                   steps with shorter iterates (l doubling) and divisor
//                   prefixes (v >> s limbs), 2 guard limbs.
//   Alg. 1 (Step):  w' = shift_m(w) +- shift_{2m-H}(w * x), the negative
//                   branch rounded toward -infinity.
//   Alg. 2 (PowDiff): (sign, |B^h - v w|) from the full product, or from the
//                   low L limbs of v w (the close product).
//   Alg. 3 (Div):   q = shift_{-h}(u * shinv_h(v)), m = v q, then quotient
//                   corrections.
// All numbers are little-endian base B = 2^32 limbs; h, k, l, m, s, g count
// limbs.  Readings taken where the printed algorithms are silent or garbled:
//   * the Refine loop runs 2 + ceil(log2(h-k-1)) times, 2 times when
//     h-k-1 <= 1;
//   * Step's rounding test looks at the h-2m (not 2m-h) low limbs of w*x;
//   * PowDiff's sign is 1 iff B^h - v*w >= 0;
//   * the computed inverse can be floor(B^h/v) - 1 as well as + 1, and the
//     clipped products below move it by at most one more unit either way, so
//     the division corrects q0 by up to four subtractions and five additions
//     of v (q - 4 <= q0 <= q + 3 is what the bound allows; one more step
//     each way is a safety margin that reports INTERNAL instead of a wrong
//     answer), and the stand-alone shinv ends with an exact fix-up.
//
// Two kernels share the work of one instance.  The head (one wave per
// instance, many instances per compute unit) computes the initial
// approximation and the early Refine iterations, whose operands are short;
// it leaves their state in a record at the start of the instance's own output
// row (q for a division, w for a shifted inverse).  The body (one workgroup
// per instance) picks the record up and runs the remaining iterations and
// the quotient and remainder products.  Without a record the body runs every
// step itself.
#pragma once

#include <stdint.h>

#include "launch.hpp"

namespace mp {

enum : int32_t { kInstOk = 0, kInstDivZero = 1, kInstQWidth = 2, kInstInternal = 3 };

#define MP_HD __host__ __device__ __forceinline__

MP_HD constexpr int r4(int x) { return (x + 3) & ~3; }
MP_HD constexpr int hmax(int a, int b) { return a > b ? a : b; }

// LDS layout of one division / shifted-inverse instance with h = prec(u)
// (or the shinv precision) and k = prec(v) - 1, in 32-bit words.  Capacities
// bound every intermediate of the method: w <= h-k+4 limbs, x <= k+8,
// shinv <= h-k+1.  R holds the reversed digits of the shorter operand of a
// matrix-core product (up to h/2 + 15 limbs); the window area SB doubles as
// the long operand's digits.  P holds the columns a product forms, from its
// first formed column on: PowDiff's close product (L <= k + 7 columns), the
// Step's w x from column sh - 2 up (about m + 16 columns: within max(k, d) + 9
// over a scan of random and structured operands of up to 700 limbs), u * shinv
// from column h - 9 up (at most h - k + 11), the low k + 2 columns of v q0
// and shinv's fix-up product (k + 4); every use is guarded.
struct Plan {
    int capV, capW, capX, capR, capSB, capP;
    int offV, offW, offX, offR, offSB, offP;   // offR: word 0 of the reversed digits, offSB: limb 0 of the window
    int vbase;                                 // index of the divisor limb stored at offV (limbs below are not held)
    int capY;          // longest operand whose matrix-core digit planes (with their zero pads) fit the window area
    int sbLo, sbHi;    // the window area is SB[-sbLo, sbHi), kept zero where nothing is staged
    int total;
};

MP_HD constexpr Plan plan_div(int h, int k)
{
    Plan p{};
    p.vbase = 0;
    const int d = h - k;
    p.capV = r4(k + 1);
    p.capW = r4(d + 8);
    p.capX = r4(k + 12);
    p.capR = r4(h / 2 + 16);
    p.capSB = r4(hmax(hmax(h, k + 12), d + 8) + 4);
    p.capP = r4(hmax(k, d) + 24);
    p.offV = kCtlWords;
    p.offW = p.offV + p.capV;
    p.offX = p.offW + p.capW;
    p.offR = p.offX + p.capX + kXPad;
    p.offSB = p.offR + p.capR + kXPad + kPad;
    p.offP = p.offSB + p.capSB + kPad;
    p.total = p.offP + p.capP + 4;
    p.capY = 1 << 30;   // kPad covers the planes of any operand the window holds
    p.sbLo = kPad;
    p.sbHi = p.capSB + kPad;
    return p;
}

// LDS layout of one wave's head (the Refine iterations whose iterate has fewer
// than `limit` limbs, so l <= limit - 4): a short control block (a head's
// products have at most kHeadStrips strips and it broadcasts nothing through
// LDS), the divisor limbs [vbase, k] it reads (v' = v >> s has at most 2l + 2
// limbs), the iterate (at most 2l + 2 limbs after the last of these
// iterations), PowDiff's residual (at most 3l + 3 limbs, B^h' minus a
// product), the reversed digits of a matrix-core product's shorter operand
// (the iterate, at most l + 4 limbs), the window operand with its zero
// guards, and products (w * x: at most 4l + 9 limbs).  Every use is guarded;
// an iteration that would overrun returns false and the body does it instead.
// The window's guards cover both product engines: the one-wave VALU product
// reads strip [K0, K0 + 64) with rows [ilo, ihi) within 65 limbs below the
// window and 63 above it; the matrix-core digit planes of a long operand of
// up to capY = 2 limit + 8 limbs (v' and PowDiff's residual in the
// iterations a head runs) need 4 kYPadBlk zero words below the window and
// reach 8 ((capY + 8) / 8) + 8 kYPadBlk words above its start (a longer
// operand takes the VALU product).  Sized so that 16 heads share a compute
// unit's LDS up to the largest limit.
constexpr int kHeadMaxLimit = 140;   // largest small_limit: every head operand then fits kHeadMaxLimbs
constexpr int kHeadPad = kLanes + 8; // zero guard on both sides of a head's VALU window operand
// (the longest one-wave linear operation of a head is bounded by capP, capX or
// capW + l, all below 4 * limit + 8 limbs)
static_assert(4 * kHeadMaxLimit + 8 <= kHeadMaxLimbs, "head operands must fit one wave's addsub");
static_assert(4 * kHeadMaxLimit + 8 <= kHeadStrips * kStrip, "a head's products must fit its strip slots");

MP_HD constexpr Plan plan_head(int limit, int vbase)
{
    Plan p{};
    const int L = limit < 4 ? 4 : limit > kHeadMaxLimit ? kHeadMaxLimit : limit;
    p.vbase = vbase;
    p.capV = r4(2 * L);
    p.capW = r4(2 * L + 8);
    p.capX = r4(3 * L + 8);
    p.capR = r4(L + 4);
    p.capSB = r4(3 * L + 8);
    p.capP = r4(4 * L + 8);
    p.capY = 2 * L + 8;
    p.sbLo = hmax(kHeadPad, 4 * kYPadBlk);
    p.sbHi = hmax(p.capSB + kHeadPad, 8 * ((p.capY + 8) >> 3) + 8 * kYPadBlk);
    p.offV = kHeadCtlWords;
    p.offW = p.offV + p.capV;
    p.offX = p.offW + p.capW;
    p.offR = p.offX + p.capX + kXPad;
    p.offSB = p.offR + p.capR + kXPad + p.sbLo;
    p.offP = p.offSB + p.sbHi;
    p.total = p.offP + p.capP + 4;
    return p;
}

// Record of the head in the instance's output row (32-bit words):
//   [0] kRecValid, or 0 when the body is to do every step itself
//   [1] Refine iterations done   [2] l   [3] we   [4] nw   [5] h   [6] k
//   [kRecHdr, kRecHdr + we) the limbs of the iterate W
constexpr uint32_t kRecValid = 0x52454331u;
constexpr int kRecHdr = 8;
constexpr int kHeadWaves = 4;   // head instances (waves) per workgroup
static_assert(16 * plan_head(kHeadMaxLimit, 0).total * 4 <= 160 * 1024, "16 heads must share a compute unit's LDS");

// words needed by the single-limb-divisor path (quotient + chunk scratch)
MP_HD int plan_short_words(int n, int T) { return kCtlWords + 2 * T + r4(n + 1) + 4; }

// LDS words for a batch whose dividends have at most nu limbs and divisors at
// most nv limbs (every (h, k) an instance can reach)
MP_HD int div_lds_words(int nu, int nv, int T)
{
    int best = plan_short_words(nu, T);
    const int kmax = (nv < nu ? nv : nu) - 1;
    for (int k = 1; k <= kmax; k++) best = hmax(best, plan_div(nu, k).total);
    return best;
}

MP_HD int mul_lds_words(int na, int nb)
{
    const int lo = na < nb ? na : nb, hi = na < nb ? nb : na;
    return kCtlWords + kXPad + r4(lo + 1) + kXPad + 4 + kPad + r4(hi + 1) + kPad + r4(na + nb) + 4;
}

// ------------------------------------------------------------------ helpers

// p[c0, ncols) = columns c0 .. ncols-1 of x*y (c0 = 0: x*y mod B^ncols; see
// mul and mul_mfma for c0 > 0, a multiple of 8); returns the precision of the
// result.  Long enough products run on the matrix cores (long operand's
// digits in sb, short operand's reversed digits in xr, which holds xrcap
// limbs); the rest walk the rows on the VALU with the longer operand staged in
// sb as window.
//
// MF = false builds the vector-ALU path only (for code that never has an
// operand long enough for the matrix cores).
template <int T, bool MF, class FL, class FS>
MP_DEV int product_views(uint32_t *ctl, uint32_t *p, int ncols, const FL &lng, int nl, const uint32_t *lng_lds,
                         const FS &sht, int ns, const uint32_t *sht_lds, uint32_t *sb, int &sbext,
                         uint32_t *xr, int xrcap, int mfma_min, int c0 = 0, bool want_prec = true,
                         bool sht_ready = false)
{
    MP_PT_BEGIN(ns, nl, ncols, c0);
    int r;
    if constexpr (MF) {
        if (ns >= mfma_min && ns + 1 <= xrcap) {
            mfma_operands<T>(ctl, lng, nl, sb, sbext, sht, ns, xr, sht_ready);
            MP_PT(3);
            sbext = mfma_ext(nl);
            r = mul_mfma<T>(ctl, p, ncols, sb, nl, xr, ns, c0, want_prec);
            MP_PT_END();
            return r;
        }
    }
    copy<T>(sb, nl, sbext, lng);
    MP_PT(3);
    sbext = nl;
    if constexpr (T == kLanes) r = mul1<T>(ctl, p, ncols, sht_lds, ns, sb, nl, c0, want_prec);
    else r = mul<T>(ctl, p, ncols, sht_lds, ns, sb, nl, c0, want_prec);
    MP_PT_END();
    return r;
}

template <int T, bool MF = true>
MP_DEV int product(uint32_t *ctl, uint32_t *p, int ncols, const uint32_t *x, int nx,
                   const uint32_t *y, int ny, uint32_t *sb, int &sbext, uint32_t *xr, int xrcap, int mfma_min,
                   int c0 = 0, bool want_prec = true, bool sht_ready = false)
{
    const uint32_t *sht = nx >= ny ? y : x, *lng = nx >= ny ? x : y;
    const int ns = nx >= ny ? ny : nx, nl = nx >= ny ? nx : ny;
    return product_views<T, MF>(ctl, p, ncols, Span{lng, 0, nl}, nl, lng, Span{sht, 0, ns}, ns, sht, sb, sbext,
                                xr, xrcap, mfma_min, c0, want_prec, sht_ready);
}

// dst[0, n) = src limbs [0, e) zero-padded, where e = prec(src) must be <= n;
// returns false (and stores nothing) when the value needs more than n limbs
template <int T, class FS>
MP_DEV bool store_fit(uint32_t *ctl, uint32_t *dst, int n, int ext, const FS &src)
{
    const int e = prec<T>(ctl, ext, src);
    if (e > n) return false;
    int i = tid<T>();
    for (; i + 3 * T < n; i += 4 * T) {
        const uint32_t y0 = i < e ? src(i) : 0u, y1 = i + T < e ? src(i + T) : 0u;
        const uint32_t y2 = i + 2 * T < e ? src(i + 2 * T) : 0u, y3 = i + 3 * T < e ? src(i + 3 * T) : 0u;
        dst[i] = y0;
        dst[i + T] = y1;
        dst[i + 2 * T] = y2;
        dst[i + 3 * T] = y3;
    }
    for (; i < n; i += T) dst[i] = i < e ? src(i) : 0u;
    return true;
}

template <int T>
MP_DEV void store_zero(uint32_t *dst, int n)
{
    for (int i = tid<T>(); i < n; i += T) dst[i] = 0u;
}

// ------------------------------------------------------- Alg. 1 Refine

// (trace build: sub-steps of two of a head's iterations, i = 3 in slots 5-7
// and i = 6 in slots 8-10: PowDiff's product, its residual, Step's product)
#define MP_HEAD_SUB(i, k)                                       \
    do {                                                        \
        if constexpr (T == kLanes) {                            \
            if ((i) == 3) MP_WSTAMP(5 + (k));                   \
            else if ((i) == 6) MP_WSTAMP(8 + (k));              \
        }                                                       \
    } while (0)

// Iteration i of the Refine loop (Alg. 1): PowDiff, then Step, updating the
// iterate W (nonzero limbs inside [0, we), precision nw) and l.  Run by T
// threads (the workgroup, or one wave in a head); MF as for product_views.
template <int T, bool MF = true>
MP_DEV bool refine_iter(uint32_t *ctl, const Plan &pl, const Knobs &kn, uint32_t *lds, int h, int k, int i, int &l,
                        int &we, int &nw, int &sbext)
{
    uint32_t *V = lds + pl.offV, *W = lds + pl.offW, *X = lds + pl.offX;
    uint32_t *SB = lds + pl.offSB, *P = lds + pl.offP, *XR = lds + pl.offR;
    const int g = 2, d = h - k;
    const int m = imin(d + 1 - l, l);
    const int s = imax(0, k - 2 * l + 1 - g);
    const int H = k + l + m - s + g;
    if (s < pl.vbase) return false;      // (a head holds only the limbs its iterations read)
    const uint32_t *vp = V + (s - pl.vbase);   // divisor prefix shift_{-s}(v)
    const int nvp = k + 1 - s;
    const int hp = H - m, lp = l - g;   // PowDiff(v', w, H - m, l - g)
    const int L = nvp + nw - lp + 1;
    // a product goes to the matrix cores only if its longer operand's digit
    // planes fit the window area
    const int mm_pd = imax(nvp, nw) <= pl.capY ? kn.mfma_min : (1 << 30);
    bool sign;
    int nx;
    if (L >= hp) {                      // full product, compare with B^hp
        const int np0 = nvp + nw;
        if (np0 > pl.capP) return false;
        const int np = product<T, MF>(ctl, P, np0, vp, nvp, W, nw, SB, sbext, XR, pl.capR, mm_pd);
        MP_HEAD_SUB(i, 0);
        if (np <= hp) {                 // P < B^hp: x = B^hp - P
            if (hp > pl.capX) return false;
            sign = true;
            addsub<T>(ctl, hp, true, 0u, Zero{}, Span{P, 0, np}, Store{X, 0, hp});
        } else {                        // x = P - B^hp
            if (np > pl.capX) return false;
            sign = false;
            addsub<T>(ctl, np, true, 0u, Span{P, 0, np}, PowB{hp}, Store{X, 0, np});
        }
        nx = read_prec<T>(ctl);
    } else {                            // close product: P = v'w mod B^L
        if (L > pl.capP || L > pl.capX) return false;
        const int np = product<T, MF>(ctl, P, L, vp, nvp, W, nw, SB, sbext, XR, pl.capR, mm_pd);
        MP_STAMP(11);   // (trace build: sub-steps of the latest iteration)
        MP_HEAD_SUB(i, 0);
        if (np == 0) {                  // v'w = B^hp exactly
            sign = true;
            nx = 0;
        } else if (np < L) {            // top limb 0: v'w = B^hp + P
            sign = false;
            nx = np;
            copy<T>(X, np, 0, Span{P, 0, np});
        } else {                        // v'w = B^hp - (B^L - P)
            sign = true;
            addsub<T>(ctl, L, true, 0u, Zero{}, Span{P, 0, L}, Store{X, 0, L});
            nx = read_prec<T>(ctl);
        }
    }
    // Step: res = shift_m(w) +- shift_{2m-H}(w x); then w = shift_{-post}(res).
    // When nw + nx <= sh, w x < B^sh: the shifted product is 0 and, in the
    // negative branch, its nonzero low part borrows one; no product is formed.
    // Otherwise only the columns of w x from cs = sh - 2 (rounded down to a
    // multiple of 8) up are formed: the columns below change the shifted
    // product by less than one unit of the iterate's last guard limb, and the
    // sticky bit of the negative branch is taken from the formed columns below
    // sh.  The matrix-core digits can make the dropped part negative (less
    // than 2^17 cs B^cs in size), so the formed sum T may exceed w x: one more
    // column holds T < 2 B^(nw+nx), and w x >= B^(nw+nx-2) >= B^(sh-1) keeps
    // T > 0.
    MP_HEAD_SUB(i, 1);
    const int sh = H - 2 * m;
    const int post = i < 2 ? m : 1;
    int nt = 0, cs = 0;
    uint32_t below = 0;   // borrow of a product that lies wholly below sh
    if (nx && nw + nx <= sh) {
        below = sign ? 0u : 1u;
    } else if (nx) {
        nt = nw + nx;
        cs = imax(sh - 2, 0) & ~7;
        if (cs) nt += 1;
        if (nt - cs > pl.capP) return false;
        // w is the shorter operand of both products on the matrix cores: its
        // digits from PowDiff's product are still in XR
        const bool w_ready = MF && nvp >= nw && nw < nx && nw >= mm_pd && nw + 1 <= pl.capR;
        const int mm_st = imax(nw, nx) <= pl.capY ? kn.mfma_min : (1 << 30);
        MP_STAMP(12);
        // column c of the product goes to P[c - cs]
        product<T, MF>(ctl, P - cs, nt, W, nw, X, nx, SB, sbext, XR, pl.capR, mm_st, cs, false, w_ready);
        MP_STAMP(13);
    }
    MP_HEAD_SUB(i, 2);
    // the sticky borrow of the negative branch (any nonzero formed column
    // below sh) is found by the Step's own addsub before its carry scan
    const int stop = !sign && nt > cs ? imin(sh, nt) - cs : 0;
    const int nres = imax(nw + m, nt - sh) + 1;
    if (nres - post > pl.capW) return false;
    const uint32_t co = addsub<T>(ctl, nres, !sign, below, Span{W, m, nw}, Span{P, cs - sh, imax(nt - cs, 0)},
                                  Store{W, post, pl.capW}, StickyAny<T>{P, stop});
    if (!sign && co) return false;
    we = nres - post;
    nw = read_prec<T>(ctl, post);
    if (i >= 2) l = l + m - 1;
    return true;
}

// ------------------------------------------------ one-wave tiny iterations
//
// A Refine iteration whose operands, products and result all fit 64 limbs,
// run by one wave with limb j of every intermediate in lane j: the same
// arithmetic as refine_iter (the same products, the same clipping of the Step
// product at cs, the same sticky borrow), with every carry resolved by the
// ballot lookahead in registers instead of a pass through LDS.  Only the
// divisor prefix and the iterate are read from LDS and only the new iterate is
// written back.

// the carry (or borrow) into each lane of a one-limb-per-lane addition
// (subtraction) whose lanes generate g and propagate p, with carry-in cin;
// cout gets the carry out of lane 63
MP_DEV uint32_t lane_carry_in(bool g, bool p, uint32_t cin, uint32_t &cout)
{
    const uint64_t G = ballot(g), P = ballot(p), X = G | P;
    const uint64_t s0 = X + G;
    cout = (s0 < X ? 1u : 0u) | ((~P == 0 ? 1u : 0u) & cin);
    const uint64_t cm = (X + G + (uint64_t)cin) ^ X ^ G;
    return (uint32_t)(cm >> lane()) & 1u;
}

// a - b - bin in lanes [0, n) (zero above); bout: the borrow out of lane n - 1
MP_DEV uint32_t lane_sub(uint32_t a, uint32_t b, int n, uint32_t bin, uint32_t &bout)
{
    const bool in = lane() < n;
    const uint32_t d = in ? a - b : 0u;
    const uint32_t bi = lane_carry_in(in && a < b, !in || d == 0u, bin, bout);
    return in ? d - bi : 0u;
}

// a + b + cin in lanes [0, n) (zero above); cout: the carry out of lane n - 1
MP_DEV uint32_t lane_add(uint32_t a, uint32_t b, int n, uint32_t cin, uint32_t &cout)
{
    const bool in = lane() < n;
    const uint64_t s = (uint64_t)a + b;
    const uint32_t z = in ? (uint32_t)s : 0u;
    const uint32_t ci = lane_carry_in(in && (s >> 32) != 0, !in || z == 0xFFFFFFFFu, cin, cout);
    return in ? z + ci : 0u;
}

// 1 + the highest lane holding a nonzero limb (0 when none)
MP_DEV int lane_prec(uint32_t z)
{
    const uint64_t m = ballot(z != 0u);
    return m ? 64 - __builtin_clzll(m) : 0;
}

// column K0 + lane of a * b with the carries between columns K0 .. K0 + 63
// and none from below K0: rows a_i (i < na) from rowf(i) (wave-uniform i),
// window limbs b_j (j < nb) from LDS, read per lane with a range mask
template <class FR>
MP_DEV uint32_t lane_mul(const FR &rowf, int na, const uint32_t *b, int nb, int K0)
{
    const int l = lane(), k = K0 + l;
    const int ilo = imax(0, K0 - nb + 1), ihi = imin(na, K0 + kLanes);
    uint64_t lo[4] = {0, 0, 0, 0};
    uint32_t hi[4] = {0, 0, 0, 0};
    for (int i = ilo; i < ihi; i += 4) {
        uint32_t a[4], w[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            a[j] = i + j < ihi ? rowf(i + j) : 0u;
            const int c = k - i - j;
            w[j] = (unsigned)c < (unsigned)nb ? b[c] : 0u;
        }
        mac4x(lo, hi, a[0], w[0], a[1], w[1], a[2], w[2], a[3], w[3]);
    }
    uint64_t sl = lo[0];
    uint32_t sh = hi[0];
#pragma unroll
    for (int r = 1; r < 4; r++) {
        const uint64_t t = sl + lo[r];
        sh += hi[r] + (t < sl ? 1u : 0u);
        sl = t;
    }
    // S = s0 + s1 B + s2 B^2 per column: t = s0 + s1 of the lane below + s2 of the lane two below
    const uint32_t s1m = shfl_up1((uint32_t)(sl >> 32)), s2m = shfl_up2(sh);
    const uint64_t t = (uint64_t)(uint32_t)sl + s1m + s2m;
    const uint32_t cm = shfl_up1((uint32_t)(t >> 32));
    const uint64_t y = (uint64_t)(uint32_t)t + cm;
    uint32_t top_carry;   // leaves column K0 + 63: above every column a caller keeps
    const uint32_t z = (uint32_t)y;
    return z + lane_carry_in((y >> 32) != 0, z == 0xFFFFFFFFu, 0u, top_carry);
}

struct LdsRows {
    const uint32_t *p;
    MP_DEV uint32_t operator()(int i) const { return p[i]; }
};
struct LaneRows {
    uint32_t x;
    MP_DEV uint32_t operator()(int i) const { return readlane(x, i); }
};

// whether Refine iteration i (with l, nw, we) fits one limb per lane throughout
MP_DEV bool iter_fits_wave(const Plan &pl, int h, int k, int l, int nw, int we)
{
    const int g = 2, d = h - k;
    const int m = imin(d + 1 - l, l);
    const int s = imax(0, k - 2 * l + 1 - g);
    const int H = k + l + m - s + g;
    const int nvp = k + 1 - s;
    const int hp = H - m, lp = l - g;
    const int L = nvp + nw - lp + 1;
    const int ncA = L >= hp ? nvp + nw : L;
    const int nxmax = imax(ncA, hp);
    const int sh = H - 2 * m;
    const int cs = imax(sh - 2, 0) & ~7;
    return s >= pl.vbase && ncA <= kLanes && hp <= kLanes && nw + nxmax + 1 - cs <= kLanes &&
           imax(nw + m, nw + nxmax + 1 - sh) + 1 <= kLanes && we <= kLanes;
}

// Refine iteration i (as refine_iter) by one wave in registers, for an
// iteration that iter_fits_wave accepts
MP_DEV bool refine_iter_wave(const Plan &pl, uint32_t *lds, int h, int k, int i, int &l, int &we, int &nw)
{
    uint32_t *V = lds + pl.offV, *W = lds + pl.offW;
    const int g = 2, d = h - k;
    const int m = imin(d + 1 - l, l);
    const int s = imax(0, k - 2 * l + 1 - g);
    const int H = k + l + m - s + g;
    const int nvp = k + 1 - s;
    const int hp = H - m, lp = l - g;
    const int L = nvp + nw - lp + 1;
    const bool full = L >= hp;
    const int ncA = full ? nvp + nw : L;          // columns PowDiff forms
    const int sh = H - 2 * m;
    const int cs = imax(sh - 2, 0) & ~7;
    const int post = i < 2 ? m : 1;
    const uint32_t *vp = V + (s - pl.vbase);
    wave_sync();
    const int ln = lane();
    // PowDiff: P = v' w (all columns, or mod B^L), then x = |v' w - B^hp|
    uint32_t P = lane_mul(LdsRows{W}, nw, vp, nvp, 0);
    if (ln >= ncA) P = 0u;
    const int np = lane_prec(P);
    bool sign;
    uint32_t x, bo;
    if (full) {
        if (np <= hp) {                 // x = B^hp - P
            sign = true;
            x = lane_sub(0u, P, hp, 0u, bo);
        } else {                        // x = P - B^hp
            sign = false;
            x = lane_sub(P, ln == hp ? 1u : 0u, np, 0u, bo);
        }
    } else if (np == 0) {               // v'w = B^hp exactly
        sign = true;
        x = 0u;
    } else if (np < L) {                // v'w = B^hp + P
        sign = false;
        x = P;
    } else {                            // v'w = B^hp - (B^L - P)
        sign = true;
        x = lane_sub(0u, P, L, 0u, bo);
    }
    const int nx = lane_prec(x);
    // Step: res = shift_m(w) +- shift_{2m-H}(w x), formed from column cs up
    int nt = 0, cse = 0;
    uint32_t below = 0, Ps = 0u;
    if (nx && nw + nx <= sh) {
        below = sign ? 0u : 1u;
    } else if (nx) {
        nt = nw + nx;
        cse = cs;
        if (cse) nt += 1;
        Ps = lane_mul(LaneRows{x}, nx, W, nw, cse);
        if (ln >= nt - cse) Ps = 0u;
    }
    const int stop = !sign && nt > cse ? imin(sh, nt) - cse : 0;
    const bool sticky = ballot(ln < stop && Ps != 0u) != 0;
    const int nres = imax(nw + m, nt - sh) + 1;
    if (nres - post > pl.capW) return false;
    const uint32_t wk = (unsigned)(ln - m) < (unsigned)nw ? W[ln - m] : 0u;
    const int src = ln + sh - cse;   // column ln + sh of w x, at lane src of Ps
    const uint32_t yk = shfl(Ps, src < kLanes ? src : 0);
    const uint32_t y = (src < kLanes && src < nt - cse) ? yk : 0u;
    const uint32_t cin = sticky ? 1u : below;
    uint32_t co;
    const uint32_t res = sign ? lane_add(wk, y, nres, cin, co) : lane_sub(wk, y, nres, cin, co);
    if (!sign && co) return false;
    wave_sync();
    if (ln >= post && ln < nres) W[ln - post] = res;
    we = nres - post;
    nw = imax(lane_prec(res) - post, 0);
    if (i >= 2) l = l + m - 1;
    return true;
}

MP_HD int refine_iters(int d)   // Alg. 1's iteration count for h - k = d >= 1
{
    int r = 0;
    while (d - 1 > 1 && (1 << r) < d - 1) r++;
    return 2 + r;
}

// l at the start of Refine iteration i (d = h - k)
MP_HD int refine_l(int d, int i)
{
    int l = 2;
    for (int j = 2; j < i; j++) l = l + (d + 1 - l < l ? d + 1 - l : l) - 1;
    return l;
}

// number of leading Refine iterations whose iterate (l + g + 1 limbs) is
// shorter than `limit` limbs
MP_HD int small_iters(int d, int limit)
{
    const int iters = refine_iters(d);
    int n = 0;
    while (n < iters && refine_l(d, n) + 3 < limit) n++;
    return n;
}

// floor(B^3 / V) for B <= V < B^2, by one wave (every lane gets the result):
// the quotient is B^2 when V = B and below B^2 otherwise.  Its bits are found
// six at a time from the top: in each round lane j tests whether the bits
// known so far followed by j (and zeros below) times V is at most B^3; the
// lanes that pass are 0 .. J (the product grows with j), so J is the next six
// bits.  Ten rounds of six bits and one of four: exact integer arithmetic, no
// division.
MP_DEV void inv96_wave(uint64_t V, uint64_t &q, uint32_t &q64)
{
    q = 0;
    q64 = 0;
    if (V == (1ull << 32)) {
        q64 = 1;
        return;
    }
    const unsigned __int128 B3 = ((unsigned __int128)1) << 96;
    const uint64_t j = (uint64_t)lane();
    for (int sh = 58; sh >= 0; sh -= 6) {
        const uint64_t c = q | (j << (sh < 4 ? 0 : sh));
        const bool ok = (sh >= 4 || j < 16) && (unsigned __int128)c * V <= B3;
        const uint64_t m = ballot(ok);
        q |= (uint64_t)(63 - __builtin_clzll(m)) << (sh < 4 ? 0 : sh);
        if (sh < 4) break;
        if (sh == 4) sh = 6;   // the last round takes bits 3 .. 0
    }
}

// Alg. 1's initial approximation w = shift_g(floor(B^3 / V)), V = v_{k-1} + v_k B:
// w0 <= B^2 has 3 limbs (65 bits when V = B).  vtop points at v_{k-1}, v_k.
// Computed by the first wave of the T threads.
template <int T>
MP_DEV void refine_init(uint32_t *ctl, const uint32_t *vtop, uint32_t *W, int &we, int &nw)
{
    bar<T>();
    if (T == kLanes || tid<T>() < kLanes) {
        const uint64_t Vt = ((uint64_t)vtop[1] << 32) | vtop[0];
        uint64_t w0;
        uint32_t w64;
        inv96_wave(Vt, w0, w64);
        const uint32_t code = w64 ? 5u : (w0 >> 32) ? 4u : 3u;
        if (lane() == 0) {
            W[0] = 0u;
            W[1] = 0u;
            W[2] = (uint32_t)w0;
            W[3] = (uint32_t)(w0 >> 32);
            W[4] = w64;
            if constexpr (T > kLanes) ctl[kCtlBcast + 1] = code;
        }
        if constexpr (T == kLanes) nw = (int)uniform(code);
    }
    bar<T>();
    if constexpr (T > kLanes) nw = (int)uniform(ctl[kCtlBcast + 1]);
    we = 5;
}

// the same for one wave (a head) from V = v_{k-1} + v_k B held in registers
MP_DEV void head_init(uint64_t Vt, uint32_t *W, int &we, int &nw)
{
    uint64_t w0;
    uint32_t w64;
    inv96_wave(Vt, w0, w64);
    if (lane() == 0) {
        W[0] = 0u;
        W[1] = 0u;
        W[2] = (uint32_t)w0;
        W[3] = (uint32_t)(w0 >> 32);
        W[4] = w64;
    }
    nw = (int)uniform(w64 ? 5u : (w0 >> 32) ? 4u : 3u);
    we = 5;
}

// Initial approximation and the Refine loop for B^k <= v < B^(k+1), k >= 1,
// h - k >= 1, B < v <= B^h / 2, v not a power of B.  v is in V (k+1 limbs),
// W and the window area are zero.  With a valid head record `rec` (in global
// memory) the iterations it covers are taken from it instead.  On return the
// shifted inverse is the limbs of W above `shf`; W's nonzero limbs lie inside
// [0, we) and nw = prec(W).  Returns false if a capacity guard trips or a
// Step result turns negative (never expected).
template <int T>
MP_DEV bool refine(uint32_t *ctl, const Plan &pl, const Knobs &kn, uint32_t *lds, int h, int k, int &we, int &nw,
                   int &shf, int &sbext, const uint32_t *rec)
{
    uint32_t *V = lds + pl.offV, *W = lds + pl.offW;
    const int d = h - k;
    const int iters = refine_iters(d);
    int l = 2, i = 0;
    if (rec) {
        i = (int)uniform(rec[1]);
        l = (int)uniform(rec[2]);
        we = (int)uniform(rec[3]);
        nw = (int)uniform(rec[4]);
        if (we > pl.capW) return false;
        copy<T>(W, we, 0, Span{rec + kRecHdr, 0, we});
    } else {
        refine_init<T>(ctl, V + k - 1, W, we, nw);
    }
    MP_STAMP(3);
    MP_STAMP(4);
    for (; i < iters; i++) {
        if (!refine_iter<T>(ctl, pl, kn, lds, h, k, i, l, we, nw, sbext)) return false;
        MP_STAMP(16 + (i & 15));
    }
    shf = d < 2 ? 4 - d : 2;
    return true;
}

// ------------------------------------------------------------------- head

// number of significant limbs of x[0, n) (global memory), by one wave from the top
MP_DEV int wave_prec(const uint32_t *x, int n)
{
    for (int top = n; top > 0; top -= kLanes) {
        const int i = top - kLanes + lane();
        const uint64_t m = ballot(i >= 0 && x[i] != 0u);
        if (m) return top - kLanes + 64 - __builtin_clzll(m);
    }
    return 0;
}

// index of the lowest nonzero limb of x[0, n) (n when there is none), by one wave
MP_DEV int wave_low(const uint32_t *x, int n)
{
    for (int base = 0; base < n; base += kLanes) {
        const int i = base + lane();
        const uint64_t m = ballot(i < n && x[i] != 0u);
        if (m) return base + __builtin_ctzll(m);
    }
    return n;
}

// The head of one instance with h, k = prec(v) - 1 and vlow (index of v's
// lowest nonzero limb), by one wave in its own LDS area (plan_head words):
// for the general case with h - k >= 2 and v not a power of B, Alg. 1's
// initial approximation and its Refine iterations while the iterate is
// shorter than kn.small_limit limbs, recorded in rec[0, nrec); otherwise (or
// when the state does not fit) rec[0] = 0.  With have_top, vtop holds
// v_{k-1} + v_k B (read by the caller), else they are read here.
MP_DEV void head_refine(uint32_t *lds, int h, int k, int vlow, const uint32_t *v, uint64_t vtop, bool have_top,
                        uint32_t *rec, int nrec, const Knobs &kn)
{
    constexpr int T = kLanes;
    uint32_t *ctl = lds;
    const int d = h - k, g = 2;
    bool go = k >= 1 && d >= 2;
    uint64_t Vt = vtop;
    if (go && !have_top) Vt = ((uint64_t)v[k] << 32) | v[k - 1];
    if (go) go = !(vlow == k && (uint32_t)(Vt >> 32) == 1u);
    const int ns = go ? small_iters(d, kn.small_limit) : 0;
    const int vbase = ns ? imax(0, k - 2 * refine_l(d, ns - 1) + 1 - g) : 0;
    const Plan pl = plan_head(kn.small_limit, vbase);
    if (ns == 0 || k + 1 - vbase > pl.capV) {
        if (lane() == 0) rec[0] = 0u;
        return;
    }
    uint32_t *V = lds + pl.offV, *W = lds + pl.offW, *SB = lds + pl.offSB;
    // the divisor limbs [vbase, k] (at most capV <= 5 T): every read in flight
    // at once; the LDS areas are zeroed and the initial approximation (from
    // the top limbs in registers) computed while they arrive, then they are
    // stored
    int we = 0, nw = 0, sbext = 0, l = 2;
    {
        static_assert(r4(2 * kHeadMaxLimit) <= 5 * T, "a head stages its divisor limbs in one round");
        const int nvs = k + 1 - vbase;
        uint32_t a[5];
#pragma unroll
        for (int j = 0; j < 5; j++) a[j] = lane() + j * T < nvs ? v[vbase + lane() + j * T] : 0u;
        for (int i = lane(); i < pl.capW; i += T) W[i] = 0u;
        for (int i = lane() - pl.sbLo; i < pl.sbHi; i += T) SB[i] = 0u;
        wave_sync();
        head_init(Vt, W, we, nw);
#pragma unroll
        for (int j = 0; j < 5; j++)
            if (lane() + j * T < nvs) V[lane() + j * T] = a[j];
    }
    MP_WSTAMP(2);   // (trace build: staging and the initial approximation)
    MP_WSTAMP(3);
    bool ok = true;
    int i = 0;
    // the first iterations in registers, one limb per lane; the rest as in the body
    for (; i < ns && ok && iter_fits_wave(pl, h, k, l, nw, we); i++) {
        ok = refine_iter_wave(pl, lds, h, k, i, l, we, nw);
        MP_WSTAMP(16 + (i & 15));
    }
    for (; i < ns && ok; i++) {
        ok = refine_iter<T>(ctl, pl, kn, lds, h, k, i, l, we, nw, sbext);
        MP_WSTAMP(16 + (i & 15));
    }
    ok = ok && kRecHdr + we <= nrec;
    wave_sync();
    if (!ok) {
        if (lane() == 0) rec[0] = 0u;
        return;
    }
    for (int i = lane(); i < we; i += T) rec[kRecHdr + i] = W[i];
    if (lane() == 0) {
        rec[1] = (uint32_t)ns;
        rec[2] = (uint32_t)l;
        rec[3] = (uint32_t)we;
        rec[4] = (uint32_t)nw;
        rec[5] = (uint32_t)h;
        rec[6] = (uint32_t)k;
        rec[7] = 0u;
        rec[0] = kRecValid;
    }
    MP_WSTAMP(4);
    MP_WRSTAMP(15);   // (trace build: real time at the end and the start of a head)
}

// prec(x[0, n)) when x[0, n) is nonzero below its top 64 limbs or in them:
// the ballot of the top chunk m (read by the caller) decides it, else the
// scan goes on downwards
MP_DEV int wave_prec_from(const uint32_t *x, int n, uint64_t m)
{
    if (m) return n - kLanes + 64 - __builtin_clzll(m);
    return n > kLanes ? wave_prec(x, n - kLanes) : 0;
}

// k = prec(v) - 1 and the index of v's lowest nonzero limb, by one wave
// from the ballots of v's top 64 limbs (mv) and bottom 64 limbs (mb), read
// by the caller; a chunk of 64 zero limbs sends the scan on
MP_DEV void wave_vshape(const uint32_t *v, int nv, uint64_t mv, uint64_t mb, int &k, int &vlow)
{
    k = wave_prec_from(v, nv, mv) - 1;
    vlow = mb ? __builtin_ctzll(mb) : wave_low(v, k + 1);
}

// v_{k-1} + v_k B from the registers of v's top 64 limbs (lane j holds limb
// nv - 64 + j), when both limbs lie in that chunk
MP_DEV bool wave_vtop(uint32_t vt, int nv, int k, uint64_t &V)
{
    const int j = k - (nv - kLanes);   // lane of v_k
    if (k < 1 || j < 1 || j >= kLanes) return false;
    V = ((uint64_t)readlane(vt, j) << 32) | readlane(vt, j - 1);
    return true;
}

// the head of a division (h = prec(u), k = prec(v) - 1): the top 64 limbs of
// u and of v and the bottom 64 of v are read together, which settles both
// precisions and v's lowest nonzero limb in one round trip unless a number
// has 64 zero limbs at that end
MP_DEV void head_divrem(uint32_t *lds, const uint32_t *u, int nu, const uint32_t *v, int nv, uint32_t *rec, int nrec,
                        const Knobs &kn)
{
    MP_WSTAMP(0);
    MP_WRSTAMP(14);
    const int iu = nu - kLanes + lane(), iv = nv - kLanes + lane(), il = lane();
    const uint32_t ut = iu >= 0 ? u[iu] : 0u, vt = iv >= 0 ? v[iv] : 0u, vb = il < nv ? v[il] : 0u;
    const uint64_t mu = ballot(ut != 0u), mv = ballot(vt != 0u), mb = ballot(vb != 0u);
    const int h = wave_prec_from(u, nu, mu);
    int k, vlow;
    wave_vshape(v, nv, mv, mb, k, vlow);
    uint64_t vtop = 0;
    const bool top = wave_vtop(vt, nv, k, vtop);
    MP_WSTAMP(1);
    head_refine(lds, h, k, vlow, v, vtop, top, rec, nrec, kn);
}

// the head of a shifted inverse floor(B^h / v)
MP_DEV void head_shinv(uint32_t *lds, int h, const uint32_t *v, int nv, uint32_t *rec, int nrec, const Knobs &kn)
{
    const int iv = nv - kLanes + lane(), il = lane();
    const uint32_t vt = iv >= 0 ? v[iv] : 0u, vb = il < nv ? v[il] : 0u;
    int k, vlow;
    wave_vshape(v, nv, ballot(vt != 0u), ballot(vb != 0u), k, vlow);
    uint64_t vtop = 0;
    const bool top = wave_vtop(vt, nv, k, vtop);
    head_refine(lds, h, k, vlow, v, vtop, top, rec, nrec, kn);
}

// a head record for (h, k) in the output row rec[0, nrec), or nullptr when rec
// is absent or holds none (a valid record always fits its row)
template <int T>
MP_DEV const uint32_t *head_record(const uint32_t *rec, int nrec, int h, int k)
{
    if (!rec || nrec < kRecHdr) return nullptr;
    if (uniform(rec[0]) != kRecValid) return nullptr;
    return (int)uniform(rec[5]) == h && (int)uniform(rec[6]) == k ? rec : nullptr;
}

// ------------------------------------------------------------ instances

// c = a * b  (c has na + nb limbs)
template <int T>
MP_DEV void mul_instance(uint32_t *lds, const uint32_t *a, int na, const uint32_t *b, int nb, uint32_t *c,
                         const Knobs &kn)
{
    uint32_t *ctl = lds;
    const int nlo = na < nb ? na : nb, nhi = na < nb ? nb : na;
    const uint32_t *sht = na < nb ? a : b, *lng = na < nb ? b : a;
    uint32_t *A = lds + kCtlWords + kXPad;          // short operand (rows, or reversed digits)
    uint32_t *SBbase = A + r4(nlo + 1) + kXPad + 4;
    uint32_t *SB = SBbase + kPad;                   // long operand (window, or digits)
    uint32_t *P = SB + r4(nhi + 1) + kPad;
    int np;
    MP_RSTAMP(6);
    MP_STAMP(0);
    if (nlo >= kn.mfma_min) {
        copy<T>(SBbase, 0, 2 * kPad + r4(nhi + 1), Zero{});
        MP_STAMP(1);
        mfma_operands<T>(ctl, Span{lng, 0, nhi}, nhi, SB, 0, Span{sht, 0, nlo}, nlo, A);
        MP_STAMP(2);
        np = mul_mfma<T>(ctl, P, na + nb, SB, nhi, A, nlo, 0, false);
        MP_STAMP(3);
    } else {
        copy<T>(A, nlo, r4(nlo) + 4, Span{sht, 0, nlo});
        copy<T>(SBbase, kPad + nhi, 2 * kPad + r4(nhi), Span{lng, kPad, nhi});
        np = mul<T>(ctl, P, na + nb, A, nlo, SB, nhi, 0, false);
    }
    (void)np;
    bar<T>();
    MP_STAMP(4);
    for (int i = tid<T>(); i < na + nb; i += T) c[i] = P[i];
    MP_STAMP(5);
    MP_RSTAMP(7);
}

// w = floor(B^h / v), exactly (nw limbs).  rec: the head's record (at w), or
// nullptr when no head ran
template <int T>
MP_DEV void shinv_instance(uint32_t *lds, const uint32_t *v, int nv, int h, uint32_t *w, int nw,
                           int32_t *status, const Knobs &kn, const uint32_t *rec)
{
    uint32_t *ctl = lds;
    const Span Vg{v, 0, nv};
    int32_t st = kInstOk;
    const int nvv = prec<T>(ctl, nv, Vg);
    if (nvv == 0) {
        store_zero<T>(w, nw);
        if (status && tid<T>() == 0) *status = kInstDivZero;
        return;
    }
    const int k = nvv - 1;
    const int lowz = prec<T>(ctl, k, Vg) == 0;   // limbs below k all zero
    const uint32_t vk = v[k];
    bool ok = true;
    if (k == 0) {                                 // v < B: B^h quo v by short division
        uint32_t *scratch = lds + kCtlWords, *Q = scratch + 2 * T;
        shortdiv<T>(ctl, scratch, h + 1, PowB{h}, vk, Store{Q, 0, h + 1});
        ok = store_fit<T>(ctl, w, nw, h + 1, Span{Q, 0, h + 1});
    } else if (k > h || (k == h && !(lowz && vk == 1u))) {   // v > B^h
        store_zero<T>(w, nw);
    } else if (k == h ||                                      // v = B^h
               (k == h - 1 && (vk > 0x80000000u || (vk == 0x80000000u && !lowz)))) {  // 2v > B^h
        ok = nw >= 1;
        if (ok)
            for (int i = tid<T>(); i < nw; i += T) w[i] = i == 0 ? 1u : 0u;
    } else if (lowz && vk == 1u) {                            // v = B^k: B^(h-k)
        ok = nw > h - k;
        if (ok) {
            const int e = h - k;
            for (int i = tid<T>(); i < nw; i += T) w[i] = i == e ? 1u : 0u;
        }
    } else {
        const Plan pl = plan_div(h, k);
        uint32_t *V = lds + pl.offV, *W = lds + pl.offW, *X = lds + pl.offX;
        uint32_t *SB = lds + pl.offSB, *P = lds + pl.offP, *XR = lds + pl.offR;
        copy<T>(V, k + 1, 0, Vg);
        copy<T>(W, 0, pl.capW, Zero{});
        copy<T>(SB - kPad, 0, pl.capSB + 2 * kPad, Zero{});
        int we = 0, nwi = 0, shf = 0, sbext = 0;
        if (!refine<T>(ctl, pl, kn, lds, h, k, we, nwi, shf, sbext, head_record<T>(rec, nw, h, k))) {
            st = kInstInternal;
        } else {
            // exact fix-up: D = B^h - v s with s within two of floor(B^h/v), so
            // -2v <= D < 3v.  D is formed as a signed Lr-limb number (Lr = k+3
            // when h >= k+3: B^h vanishes mod B^Lr and |D| < B^Lr / 2), then
            // moved into [0, v) by whole multiples of v.
            uint32_t *S = W + shf;
            int se = imax(we - shf, 0);
            const int ns = imax(nwi - shf, 0);
            const int d = h - k;
            const int full = k + 1 + ns;
            const int Lr = d >= 3 ? k + 3 : imax(full, h + 1) + 1;
            const int pc = imin(Lr, full);
            product<T>(ctl, P, pc, V, k + 1, S, ns, SB, sbext, XR, pl.capR, kn.mfma_min, 0, false);
            addsub<T>(ctl, Lr, true, 0u, PowB{h}, Span{P, 0, pc}, Store{X, 0, Lr});
            uint32_t *R = X, *R2 = P;
            int adj = 0;
            bool good = true;
            for (int it = 0; good; it++) {         // D < 0: s too large
                bar<T>();
                if (!(R[Lr - 1] >> 31)) break;
                if (it == 4) { good = false; break; }
                addsub<T>(ctl, Lr, false, 0u, Span{R, 0, Lr}, Span{V, 0, k + 1}, Store{R, 0, Lr});
                adj -= 1;
            }
            for (int it = 0; good; it++) {         // D >= v: s too small
                if (addsub<T>(ctl, Lr, true, 0u, Span{R, 0, Lr}, Span{V, 0, k + 1}, Store{R2, 0, Lr})) break;
                if (it == 5) { good = false; break; }
                uint32_t *t = R;
                R = R2;
                R2 = t;
                adj += 1;
            }
            if (good && adj != 0) {
                addsub<T>(ctl, se + 1, adj < 0, 0u, Span{S, 0, se}, Limb0{(uint32_t)(adj < 0 ? -adj : adj)},
                          Store{S, 0, se + 1});
                se += 1;
            }
            if (!good) st = kInstInternal;
            if (good) ok = store_fit<T>(ctl, w, nw, se, Span{S, 0, se});
        }
    }
    if (st == kInstOk && !ok) st = kInstQWidth;
    if (st != kInstOk) {
        bar<T>();
        store_zero<T>(w, nw);
    }
    if (status && tid<T>() == 0) *status = st;
}

// (q, r) with u = q v + r, 0 <= r < v  (q: nq limbs, r: nv limbs).  rec: the
// head's record (at q), or nullptr when no head ran
template <int T>
MP_DEV void divrem_instance(uint32_t *lds, const uint32_t *u, int nu, const uint32_t *v, int nv,
                            uint32_t *q, int nq, uint32_t *r, int32_t *status, const Knobs &kn,
                            const uint32_t *rec)
{
    uint32_t *ctl = lds;
    const Span Ug{u, 0, nu}, Vg{v, 0, nv};
    int32_t st = kInstOk;
    bool ok = true;
    // one pass over u and v: prec(u), prec(v), and the lowest nonzero limb of v
    uint32_t red[3] = {0u, 0u, 0u};
    bar<T>();
    MP_RSTAMP(14);
    MP_PT_RESET();
    MP_STAMP(0);
    {
        // eight limbs of u and of v per thread and step, all read before use;
        // v's limbs below nu also go to LDS right after the control block, where
        // the divisor lives in every path that uses it (the allocation always
        // holds kCtlWords + nu words)
        uint32_t *V0 = lds + kCtlWords;
        const int nm = nu > nv ? nu : nv, nvs = nu < nv ? nu : nv;
        for (int i0 = tid<T>(); i0 < nm; i0 += 8 * T) {
            uint32_t ua[8], va[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int i = i0 + j * T;
                ua[j] = i < nu ? u[i] : 0u;
                va[j] = i < nv ? v[i] : 0u;
            }
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int i = i0 + j * T;
                if (i < nvs) V0[i] = va[j];
                if (ua[j]) red[0] = (uint32_t)(i + 1);
                if (va[j]) {
                    red[1] = (uint32_t)(i + 1);
                    red[2] = red[2] ? red[2] : (uint32_t)(nv - i);
                }
            }
        }
    }
    wg_max_n<T, 3>(ctl, red);
    MP_STAMP(1);
    const int h = (int)red[0], nvv = (int)red[1], vlow = nv - (int)red[2];
    if (nvv == 0) {
        store_zero<T>(q, nq);
        store_zero<T>(r, nv);
        if (status && tid<T>() == 0) *status = kInstDivZero;
        return;
    }
    const int c0 = h < nvv ? -1 : (h > nvv ? 1 : cmp<T>(ctl, h, Ug, Vg));
    const int k = nvv - 1;
    if (c0 < 0) {                                 // u < v: (0, u)
        store_zero<T>(q, nq);
        for (int i = tid<T>(); i < nv; i += T) r[i] = i < h ? u[i] : 0u;
        if (status && tid<T>() == 0) *status = kInstOk;
        return;
    }
    const uint32_t vk = lds[kCtlWords + k];      // k < nvv <= h <= nu: stored by the first pass
    const bool lowz = vlow == k;                  // v = v_k B^k
    if (k == 0) {                                 // single-limb divisor: short division of u
        uint32_t *scratch = lds + kCtlWords, *Q = scratch + 2 * T;
        const uint32_t rem = shortdiv<T>(ctl, scratch, h, Ug, vk, Store{Q, 0, h});
        ok = store_fit<T>(ctl, q, nq, h, Span{Q, 0, h});
        if (ok)
            for (int i = tid<T>(); i < nv; i += T) r[i] = i == 0 ? rem : 0u;
    } else if (lowz && vk == 1u) {                // v = B^k: shinv = B^(h-k), q = u >> k
        ok = store_fit<T>(ctl, q, nq, h - k, Span{u, -k, h});
        if (ok)
            for (int i = tid<T>(); i < nv; i += T) r[i] = i < k ? u[i] : 0u;
    } else {
        const Plan pl = plan_div(h, k);
        uint32_t *V = lds + pl.offV, *W = lds + pl.offW, *X = lds + pl.offX;
        uint32_t *SB = lds + pl.offSB, *P = lds + pl.offP, *XR = lds + pl.offR;
        // V = v (already there); W, X, R and the window staging area (with its guards) = 0
        copy<T>(V + k + 1, 0, pl.offP - pl.offV - k - 1, Zero{});
        MP_STAMP(2);
        int we = 0, nw = 0, shf = 0, sbext = 0;
        bool good = true;
        if (k == h - 1 && (vk > 0x80000000u || (vk == 0x80000000u && !lowz))) {
            bar<T>();                               // 2v > B^h: shinv = 1
            if (tid<T>() == 0) W[0] = 1u;
            we = 1;
            nw = 1;
            shf = 0;
        } else {
            good = refine<T>(ctl, pl, kn, lds, h, k, we, nw, shf, sbext, head_record<T>(rec, nq, h, k));
        }
        if (good) {
            // q0 = shift_{-h}(u * s)
            const uint32_t *S = W + shf;
            const int ns = imax(nw - shf, 0);
            good = ns <= h;
            if (good) {
                // only the columns from c0 = h - 2 (rounded down to a multiple of 8)
                // up: the products below c0 sum to less than B^h, so the top
                // limbs are floor(u s / B^h) or one less (one more on the matrix
                // cores, whose digit products below c0 may be negative)
                const int c0 = imax(h - 2, 0) & ~7;
                good = h + ns - c0 <= pl.capP;
            }
            if (good) {
                // column c of the product goes to P[c - c0]
                const int c0 = imax(h - 2, 0) & ~7;
                const int np = product_views<T, true>(ctl, P - c0, h + ns, Ug, h, nullptr, Span{S, 0, ns}, ns, S, SB,
                                                      sbext, XR, pl.capR, kn.mfma_min, c0);
                MP_STAMP(5);
                const int nq0 = imax(np - h, 0);
                copy<T>(W, nq0, we, Span{P, c0 - h, h + ns - c0});
                we = nq0;
                // With s within two of the shifted inverse (the Step products
                // are clipped too), q - 4 <= q0 <= q + 3 and r0 = u - v q0 lies
                // in [-3v, 5v): |r0| < B^(k+2) / 2, so r0 is exact as a signed
                // (k+2)-limb number and only the low k+2 limbs of m = v q0 are
                // needed.  The loops below allow one more step each way.
                const int rl = k + 2;
                product<T>(ctl, P, rl, W, nq0, V, k + 1, SB, sbext, XR, pl.capR, kn.mfma_min, 0, false);
                MP_STAMP(6);
                uint32_t *R = SB, *R2 = X;
                int delta = 0;
                addsub<T>(ctl, rl, true, 0u, Ug, Span{P, 0, rl}, Store{R, 0, rl});
                // r0 < 0 (top bit of the signed value): add v until it is not
                for (int it = 0; good; it++) {
                    bar<T>();
                    if (!(R[rl - 1] >> 31)) break;
                    if (it == 4) { good = false; break; }
                    addsub<T>(ctl, rl, false, 0u, Span{R, 0, rl}, Span{V, 0, k + 1}, Store{R, 0, rl});
                    delta -= 1;
                }
                // now 0 <= r < 6v
                for (int it = 0; good; it++) {
                    if (addsub<T>(ctl, rl, true, 0u, Span{R, 0, rl}, Span{V, 0, k + 1}, Store{R2, 0, rl}))
                        break;                    // r < v
                    if (it == 5) { good = false; break; }
                    uint32_t *t = R;
                    R = R2;
                    R2 = t;
                    delta += 1;
                }
                if (good && delta != 0) {
                    addsub<T>(ctl, we + 1, delta < 0, 0u, Span{W, 0, we}, Limb0{(uint32_t)(delta < 0 ? -delta : delta)},
                              Store{W, 0, we + 1});
                    we += 1;
                }
                MP_STAMP(7);
                if (good) {
                    ok = store_fit<T>(ctl, q, nq, we, Span{W, 0, we});
                    if (ok)
                        for (int i = tid<T>(); i < nv; i += T) r[i] = i < k + 1 ? R[i] : 0u;
                }
            }
        }
        if (!good) st = kInstInternal;
    }
    if (st == kInstOk && !ok) st = kInstQWidth;
    if (st != kInstOk) {
        bar<T>();
        store_zero<T>(q, nq);
        store_zero<T>(r, nv);
    }
    if (status && tid<T>() == 0) *status = st;
    MP_STAMP(8);
    MP_RSTAMP(15);
}

}  // namespace mp
