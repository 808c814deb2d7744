/*
 * Pin of the oracle against native 128-bit integer division (compiler
 * runtime), independent of the oracle's code.  Operands of up to 4 limbs:
 *   - exhaustive over limbs drawn from an edge-value set (all 7^4 values of
 *     u and v, including every precision 0..4 through the zero limb),
 *   - random pairs of random precision,
 *   - shinv_h(v) = floor(B^h / v) for h = 0..3 (B^3 < 2^128),
 *   - products of 2-limb operands.
 * Usage: pin_int128 [quick]   Exit status 0 iff every case matches.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "mpref.h"

typedef unsigned __int128 u128;

static const uint32_t EDGE[7] = {0u, 1u, 2u, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFEu, 0xFFFFFFFFu};

static u128 val(const uint32_t *x)
{
    return (u128)x[0] | ((u128)x[1] << 32) | ((u128)x[2] << 64) | ((u128)x[3] << 96);
}

static uint64_t rng_state = 0x1234567887654321ull;
static uint64_t next64(void) /* splitmix64 */
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static long failures = 0, checked = 0;

static void check_div(const uint32_t *u, const uint32_t *v)
{
    uint32_t q[4], r[4];
    int32_t st = ref_divrem(u, 4, v, 4, q, 4, r, 4);
    u128 U = val(u), V = val(v);
    checked++;
    if (V == 0) {
        if (st != REF_DIVZERO) { failures++; }
        return;
    }
    if (st != REF_OK || val(q) != U / V || val(r) != U % V) {
        if (failures < 10)
            fprintf(stderr, "divrem mismatch u=%08x%08x%08x%08x v=%08x%08x%08x%08x\n",
                    u[3], u[2], u[1], u[0], v[3], v[2], v[1], v[0]);
        failures++;
    }
}

static void check_mul(const uint32_t *a, const uint32_t *b)
{
    uint32_t c[4];
    ref_mul(a, 2, b, 2, c);
    checked++;
    u128 A = (u128)a[0] | ((u128)a[1] << 32), Bv = (u128)b[0] | ((u128)b[1] << 32);
    if (val(c) != A * Bv) {
        if (failures < 10) fprintf(stderr, "mul mismatch a=%08x%08x b=%08x%08x\n", a[1], a[0], b[1], b[0]);
        failures++;
    }
}

static void check_shinv(const uint32_t *v, int h)
{
    uint32_t w[4];
    int32_t st = ref_shinv(v, 4, h, w, 4);
    u128 V = val(v);
    checked++;
    if (V == 0) { if (st != REF_DIVZERO) failures++; return; }
    u128 Bh = (u128)1 << (32 * h);
    if (st != REF_OK || val(w) != Bh / V) {
        if (failures < 10)
            fprintf(stderr, "shinv mismatch h=%d v=%08x%08x%08x%08x\n", h, v[3], v[2], v[1], v[0]);
        failures++;
    }
}

int main(int argc, char **argv)
{
    int quick = argc > 1 && strcmp(argv[1], "quick") == 0;
    uint32_t u[4], v[4];
    if (!quick) {
        for (int a = 0; a < 2401; a++) {
            for (int i = 0, t = a; i < 4; i++, t /= 7) u[i] = EDGE[t % 7];
            for (int b = 0; b < 2401; b++) {
                for (int i = 0, t = b; i < 4; i++, t /= 7) v[i] = EDGE[t % 7];
                check_div(u, v);
            }
            for (int h = 0; h <= 3; h++) check_shinv(u, h);
            for (int b = 0; b < 49; b++) {
                uint32_t x[2] = {EDGE[b % 7], EDGE[b / 7]};
                check_mul(u, x);
            }
            if (failures) break;
        }
    }
    long nrand = quick ? 200000 : 2000000;
    for (long n = 0; n < nrand && failures == 0; n++) {
        int pu = (int)(next64() % 5), pv = (int)(next64() % 5);
        memset(u, 0, sizeof u);
        memset(v, 0, sizeof v);
        for (int i = 0; i < pu; i++) u[i] = (uint32_t)(next64() >> 32);
        for (int i = 0; i < pv; i++) v[i] = (uint32_t)(next64() >> 32);
        /* bias towards near-equal tops, where quotient-digit estimates are tight */
        if (pu && pv && (next64() & 3) == 0) v[pv - 1] = u[pu - 1] - (uint32_t)(next64() & 1);
        check_div(u, v);
        if ((n & 15) == 0) check_shinv(v, (int)(next64() % 4));
        if ((n & 15) == 1) check_mul(u, v);
    }
    printf("checked %ld failures %ld\n", checked, failures);
    return failures ? 1 : 0;
}
