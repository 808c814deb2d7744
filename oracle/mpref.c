/*
 * Oracle for batched multi-precision division -- TEST INFRASTRUCTURE ONLY.
 * (Only tests, the smoke check and the benchmark's CPU-baseline leg use it.)
 *
 * Every routine computes the plain definition of its result:
 *   - ref_mul:    schoolbook (operand-scanning) product, 64-bit intermediates.
 *   - ref_divrem: Knuth, TAOCP Vol. 2, Sec. 4.3.1, Algorithm D, with base
 *                 B = 2^32 (the quotient/remainder of the paper's Alg. 3
 *                 problem statement: u = q*v + r, 0 <= r < v).
 *   - ref_shinv:  shinv_h(v) = floor(B^h / v) from Definition 1 (Sec. 2.1),
 *                 computed by running ref_divrem on the number B^h.
 * Nothing here follows the paper's Newton method; the method reaches these
 * same unique results, so the definitions are the oracle.
 */
#include "mpref.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* number of significant limbs (0 for the number zero) */
static int32_t ref_prec(const uint32_t *x, int32_t n)
{
    while (n > 0 && x[n - 1] == 0) n--;
    return n;
}

/* three-way compare of two n-limb numbers */
static int ref_cmp(const uint32_t *x, const uint32_t *y, int32_t n)
{
    for (int32_t i = n - 1; i >= 0; i--) {
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    }
    return 0;
}

static int ref_clz32(uint32_t x)
{
    int n = 0;
    while (!(x & 0x80000000u)) { x <<= 1; n++; }
    return n;
}

void ref_mul(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb, uint32_t *c)
{
    memset(c, 0, sizeof(uint32_t) * (size_t)(na + nb));
    for (int32_t i = 0; i < na; i++) {
        uint64_t carry = 0;
        for (int32_t j = 0; j < nb; j++) {
            /* a_i*b_j + c_{i+j} + carry <= (B-1)^2 + 2(B-1) = B^2 - 1 */
            uint64_t t = (uint64_t)a[i] * b[j] + c[i + j] + carry;
            c[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        c[i + nb] = (uint32_t)carry;
    }
}

/*
 * Knuth Algorithm D on significant lengths m = prec(u) >= n = prec(v) >= 2.
 * qt receives m-n+1 quotient limbs, rt receives n remainder limbs.
 */
static void knuth_d(const uint32_t *u, int32_t m, const uint32_t *v, int32_t n,
                    uint32_t *qt, uint32_t *rt)
{
    const uint64_t B = (uint64_t)1 << 32;
    uint32_t *vn = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *un = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m + 1));

    /* D1: normalize so that the top limb of v has its high bit set */
    int s = ref_clz32(v[n - 1]);
    if (s == 0) {
        memcpy(vn, v, sizeof(uint32_t) * (size_t)n);
        memcpy(un, u, sizeof(uint32_t) * (size_t)m);
        un[m] = 0;
    } else {
        for (int32_t i = n - 1; i > 0; i--) vn[i] = (v[i] << s) | (v[i - 1] >> (32 - s));
        vn[0] = v[0] << s;
        un[m] = u[m - 1] >> (32 - s);
        for (int32_t i = m - 1; i > 0; i--) un[i] = (u[i] << s) | (u[i - 1] >> (32 - s));
        un[0] = u[0] << s;
    }

    /* D2..D7: one quotient limb per position, most significant first */
    for (int32_t j = m - n; j >= 0; j--) {
        /* D3: estimate qhat from the top two limbs of the current remainder */
        uint64_t num = ((uint64_t)un[j + n] << 32) | un[j + n - 1];
        uint64_t qhat = num / vn[n - 1];
        uint64_t rhat = num % vn[n - 1];
        while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
            qhat--;
            rhat += vn[n - 1];
            if (rhat >= B) break;
        }
        /* D4: multiply and subtract qhat*vn from un[j .. j+n] */
        uint64_t carry = 0, borrow = 0;
        for (int32_t i = 0; i < n; i++) {
            uint64_t p = qhat * vn[i] + carry;
            carry = p >> 32;
            uint64_t d = (uint64_t)un[i + j] - (p & 0xffffffffu) - borrow;
            un[i + j] = (uint32_t)d;
            borrow = (d >> 32) ? 1 : 0;
        }
        uint64_t d = (uint64_t)un[j + n] - carry - borrow;
        un[j + n] = (uint32_t)d;
        /* D5/D6: the estimate was one too large: add v back */
        if (d >> 32) {
            qhat--;
            uint64_t c = 0;
            for (int32_t i = 0; i < n; i++) {
                uint64_t t = (uint64_t)un[i + j] + vn[i] + c;
                un[i + j] = (uint32_t)t;
                c = t >> 32;
            }
            un[j + n] += (uint32_t)c;
        }
        qt[j] = (uint32_t)qhat;
    }

    /* D8: unnormalize the remainder */
    if (s == 0) {
        memcpy(rt, un, sizeof(uint32_t) * (size_t)n);
    } else {
        for (int32_t i = 0; i < n; i++) rt[i] = (un[i] >> s) | (un[i + 1] << (32 - s));
    }
    free(vn);
    free(un);
}

int32_t ref_divrem(const uint32_t *u, int32_t nu, const uint32_t *v, int32_t nv,
                   uint32_t *q, int32_t nq, uint32_t *r, int32_t nr)
{
    memset(q, 0, sizeof(uint32_t) * (size_t)nq);
    memset(r, 0, sizeof(uint32_t) * (size_t)nr);
    int32_t m = ref_prec(u, nu), n = ref_prec(v, nv);
    if (n == 0) return REF_DIVZERO;

    if (m < n || (m == n && ref_cmp(u, v, n) < 0)) {
        /* u < v: quotient 0, remainder u */
        if (m > nr) return REF_QWIDTH;
        memcpy(r, u, sizeof(uint32_t) * (size_t)m);
        return REF_OK;
    }

    int32_t nqt = m - n + 1;
    uint32_t *qt = (uint32_t *)calloc((size_t)nqt, sizeof(uint32_t));
    uint32_t *rt = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
    if (n == 1) {
        /* short division by a single limb */
        uint64_t rem = 0, d = v[0];
        for (int32_t i = m - 1; i >= 0; i--) {
            uint64_t t = (rem << 32) | u[i];
            qt[i] = (uint32_t)(t / d);
            rem = t % d;
        }
        rt[0] = (uint32_t)rem;
    } else {
        knuth_d(u, m, v, n, qt, rt);
    }

    int32_t st = REF_OK;
    if (ref_prec(qt, nqt) > nq || ref_prec(rt, n) > nr) {
        st = REF_QWIDTH;
    } else {
        int32_t cq = nqt < nq ? nqt : nq, cr = n < nr ? n : nr;
        memcpy(q, qt, sizeof(uint32_t) * (size_t)cq);
        memcpy(r, rt, sizeof(uint32_t) * (size_t)cr);
    }
    free(qt);
    free(rt);
    return st;
}

int32_t ref_shinv(const uint32_t *v, int32_t nv, int32_t h, uint32_t *w, int32_t nw)
{
    /* B^h as an (h+1)-limb number, then plain long division */
    uint32_t *bh = (uint32_t *)calloc((size_t)h + 1, sizeof(uint32_t));
    bh[h] = 1;
    uint32_t *rem = (uint32_t *)calloc((size_t)(nv > 0 ? nv : 1), sizeof(uint32_t));
    int32_t st = ref_divrem(bh, h + 1, v, nv, w, nw, rem, nv);
    free(bh);
    free(rem);
    return st;
}

static int32_t ref_threads(int32_t nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int32_t ref_mul_batch(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb,
                      uint32_t *c, int32_t batch, int32_t nthreads)
{
    int32_t nt = ref_threads(nthreads);
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int32_t j = 0; j < batch; j++)
        ref_mul(a + (size_t)j * na, na, b + (size_t)j * nb, nb, c + (size_t)j * (na + nb));
    return nt;
}

int32_t ref_divrem_batch(const uint32_t *u, int32_t nu, const uint32_t *v, int32_t nv,
                         uint32_t *q, int32_t nq, uint32_t *r, int32_t nr,
                         int32_t *status, int32_t batch, int32_t nthreads)
{
    int32_t nt = ref_threads(nthreads);
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int32_t j = 0; j < batch; j++) {
        int32_t st = ref_divrem(u + (size_t)j * nu, nu, v + (size_t)j * nv, nv,
                                q + (size_t)j * nq, nq, r + (size_t)j * nr, nr);
        if (status) status[j] = st;
    }
    return nt;
}

int32_t ref_shinv_batch(const uint32_t *v, int32_t nv, int32_t h, uint32_t *w, int32_t nw,
                        int32_t *status, int32_t batch, int32_t nthreads)
{
    int32_t nt = ref_threads(nthreads);
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int32_t j = 0; j < batch; j++) {
        int32_t st = ref_shinv(v + (size_t)j * nv, nv, h, w + (size_t)j * nw, nw);
        if (status) status[j] = st;
    }
    return nt;
}
