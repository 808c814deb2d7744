// Issue-rate probe for the integer instructions the limb products can use.
//
// Every lane runs `iters` blocks of 8 independent dependency chains of one
// instruction sequence (inline asm, so the sequence is exactly what is
// timed); enough workgroups are launched to give every SIMD of every CU
// several waves.  The host times the launch with HIP events and reports
// lane-operations per second, which calibrates the integer-multiply roofline:
//   0  v_mad_u64_u32               (32x32->64 multiply-add, one limb product)
//   1  v_mad_u64_u32 + v_addc_co   (the 96-bit column accumulate of the product kernel)
//   2  v_mul_lo_u32 + v_mul_hi_u32 (a limb product as two 32-bit halves)
//   3  v_add_u32                   (full-rate reference: lanes x clock)
//   4  v_mul_u32_u24               (24-bit multiply)
//   5  v_addc_co_u32_e64           (carry fold from an SGPR pair, VOP3)
//   6  v_addc_co_u32_e32           (carry fold through VCC, VOP2)
//   7  v_add3_u32
//   8  v_lshl_add_u64              (64-bit add)
//   9  v_cndmask_b32_e64
//  10  v_mad_u64_u32 + v_add_u32   (multiply plus an independent 32-bit add)
//  11  v_dot4_u32_u8               (four 8x8-bit products summed)
//  12  v_mfma_i32_32x32x32_i8      (counted in 32x32x32 multiply-accumulates per lane-op / 64)
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef int mp_i32x16 __attribute__((ext_vector_type(16)));
typedef int mp_i32x4 __attribute__((ext_vector_type(4)));

namespace {

template <int V>
__global__ __launch_bounds__(256) void k_probe(uint32_t *out, int iters, uint32_t seed)
{
    const uint32_t t = threadIdx.x + blockIdx.x * 256u + seed;
    const uint32_t a = t * 2654435761u | 1u;
    uint64_t acc[8];
    uint32_t hi[8];
    mp_i32x16 macc[4] = {};
#pragma unroll
    for (int r = 0; r < 8; r++) {
        acc[r] = t + r;
        hi[r] = r;
    }
    for (int i = 0; i < iters; i++) {
        if constexpr (V == 0) {
#pragma unroll
            for (int r = 0; r < 8; r++) {
                uint64_t c;
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[r]), "=s"(c) : "v"(a), "v"(hi[r]));
            }
        } else if constexpr (V == 1) {
            uint64_t c0, c1, c2, c3;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                asm volatile(
                    "v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
                    "v_mad_u64_u32 %1, %9, %12, %13, %1\n\t"
                    "v_mad_u64_u32 %2, %10, %12, %13, %2\n\t"
                    "v_mad_u64_u32 %3, %11, %12, %13, %3\n\t"
                    "v_addc_co_u32_e64 %4, %8, 0, %4, %8\n\t"
                    "v_addc_co_u32_e64 %5, %9, 0, %5, %9\n\t"
                    "v_addc_co_u32_e64 %6, %10, 0, %6, %10\n\t"
                    "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
                    : "+v"(acc[4 * h]), "+v"(acc[4 * h + 1]), "+v"(acc[4 * h + 2]), "+v"(acc[4 * h + 3]),
                      "+v"(hi[4 * h]), "+v"(hi[4 * h + 1]), "+v"(hi[4 * h + 2]), "+v"(hi[4 * h + 3]),
                      "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3)
                    : "v"(a), "v"(t));
            }
        } else if constexpr (V == 2) {
#pragma unroll
            for (int r = 0; r < 8; r++) {
                uint32_t lo = (uint32_t)acc[r];
                asm volatile("v_mul_lo_u32 %0, %2, %0\n\tv_mul_hi_u32 %1, %2, %1" : "+v"(lo), "+v"(hi[r]) : "v"(a));
                acc[r] = lo;
            }
        } else if constexpr (V == 3) {
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_add_u32 %0, %1, %0" : "+v"(hi[r]) : "v"(a));
        } else if constexpr (V == 4) {
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_mul_u32_u24 %0, %1, %0" : "+v"(hi[r]) : "v"(a));
        } else if constexpr (V == 5) {
            uint64_t c;
            asm volatile("v_cmp_lt_u32_e64 %0, %1, %2" : "=s"(c) : "v"(a), "v"(t));
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(hi[r]), "+s"(c));
        } else if constexpr (V == 6) {
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_addc_co_u32_e32 %0, vcc, 0, %0, vcc" : "+v"(hi[r]) : : "vcc");
        } else if constexpr (V == 7) {
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_add3_u32 %0, %1, %0, %2" : "+v"(hi[r]) : "v"(a), "v"(t));
        } else if constexpr (V == 8) {
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(acc[r]) : "v"(acc[(r + 1) & 7]));
        } else if constexpr (V == 9) {
            uint64_t c;
            asm volatile("v_cmp_lt_u32_e64 %0, %1, %2" : "=s"(c) : "v"(a), "v"(t));
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(hi[r]) : "v"(a), "s"(c));
        } else if constexpr (V == 10) {
            uint32_t b = t;
#pragma unroll
            for (int r = 0; r < 8; r++) {
                uint64_t c;
                asm volatile("v_mad_u64_u32 %0, %1, %3, %4, %0\n\tv_add_u32 %2, %3, %2"
                             : "+v"(acc[r]), "=s"(c), "+v"(b) : "v"(a), "v"(hi[r]));
            }
            hi[0] ^= b;
        } else if constexpr (V == 11) {
#pragma unroll
            for (int r = 0; r < 8; r++) asm volatile("v_dot4_u32_u8 %0, %1, %2, %0" : "+v"(hi[r]) : "v"(a), "v"(t));
        } else {
            mp_i32x4 x = {(int)a, (int)t, (int)(a ^ t), (int)(a + t)};
#pragma unroll
            for (int r = 0; r < 2; r++) {
                macc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, x, macc[0], 0, 0, 0);
                macc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, x, macc[1], 0, 0, 0);
                macc[2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, x, macc[2], 0, 0, 0);
                macc[3] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, x, macc[3], 0, 0, 0);
            }
        }
    }
    if constexpr (V == 12) {
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int e = 0; e < 16; e++) hi[r] ^= (uint32_t)macc[r][e];
    }
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < 8; r++) s ^= (uint32_t)acc[r] ^ (uint32_t)(acc[r] >> 32) ^ hi[r];
    out[threadIdx.x + blockIdx.x * 256u] = s;
}

}  // namespace

// Runs probe `variant` (0..12) with `iters` blocks per lane over `blocks`
// workgroups of 256 threads (`scratch` holds blocks*256 words of device
// memory).  Writes the kernel time in ms and the number of timed
// instruction-sequence executions (lane count x iters x 8).  0 on success.
extern "C" int mp_probe_rate(int variant, int iters, int blocks, uint32_t *scratch, float *ms, double *lane_ops)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    if (hipEventRecord(e0, 0) != hipSuccess) return 1;
    switch (variant) {
    case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 4: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 5: hipLaunchKernelGGL(k_probe<5>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 6: hipLaunchKernelGGL(k_probe<6>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 7: hipLaunchKernelGGL(k_probe<7>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 8: hipLaunchKernelGGL(k_probe<8>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 9: hipLaunchKernelGGL(k_probe<9>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 10: hipLaunchKernelGGL(k_probe<10>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 11: hipLaunchKernelGGL(k_probe<11>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    case 12: hipLaunchKernelGGL(k_probe<12>, dim3(blocks), dim3(256), 0, 0, scratch, iters, 1u); break;
    default: return 2;
    }
    if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 3;
    const bool timed = hipEventElapsedTime(ms, e0, e1) == hipSuccess;
    *lane_ops = (double)blocks * 256.0 * (double)iters * 8.0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return timed && hipGetLastError() == hipSuccess ? 0 : 4;
}
