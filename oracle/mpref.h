/*
 * Oracle for batched multi-precision division -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct CPU reference for what the GPU path computes.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the GPU path.
 *
 * Numbers are little-endian arrays of 32-bit limbs (base B = 2^32): limb i
 * has weight B^i.  Leading zero limbs are allowed in every input.
 *
 *   ref_mul     c = a * b                      (the paper's Mult; Alg. 2/3)
 *   ref_divrem  (q, r), u = q*v + r, 0<=r<v    (problem statement of Alg. 3)
 *   ref_shinv   floor(B^h / v)                 (Definition 1, shinv_h)
 *
 * Division is Knuth's Algorithm D (TAOCP Vol. 2, Sec. 4.3.1); the shifted
 * inverse is computed by its definition: the same long division applied to
 * the (h+1)-limb number B^h.
 */
#ifndef MPREF_H
#define MPREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { REF_OK = 0, REF_DIVZERO = 1, REF_QWIDTH = 2 };

/* c[0 .. na+nb) = a[0..na) * b[0..nb).  c must not alias a or b. */
void ref_mul(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb, uint32_t *c);

/* q[0..nq), r[0..nr) zero-padded.  Returns REF_DIVZERO (v = 0) or REF_QWIDTH
 * (quotient needs more than nq limbs, or remainder more than nr) with q and r
 * zeroed, else REF_OK. */
int32_t ref_divrem(const uint32_t *u, int32_t nu, const uint32_t *v, int32_t nv,
                   uint32_t *q, int32_t nq, uint32_t *r, int32_t nr);

/* w[0..nw) = floor(B^h / v), h >= 0.  Same error codes as ref_divrem. */
int32_t ref_shinv(const uint32_t *v, int32_t nv, int32_t h, uint32_t *w, int32_t nw);

/* Batched forms: instance j of an L-limb operand starts at p + j*L.  They run
 * the single-instance routines over instances with an OpenMP parallel loop on
 * `nthreads` threads (<= 0: the OpenMP default) and return the thread count
 * actually used. */
int32_t ref_mul_batch(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb,
                      uint32_t *c, int32_t batch, int32_t nthreads);
int32_t ref_divrem_batch(const uint32_t *u, int32_t nu, const uint32_t *v, int32_t nv,
                         uint32_t *q, int32_t nq, uint32_t *r, int32_t nr,
                         int32_t *status, int32_t batch, int32_t nthreads);
int32_t ref_shinv_batch(const uint32_t *v, int32_t nv, int32_t h, uint32_t *w, int32_t nw,
                        int32_t *status, int32_t batch, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
