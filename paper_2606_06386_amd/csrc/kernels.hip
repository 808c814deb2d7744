// Division kernels and their launchers.
//
// One workgroup per instance (or, for the persistent ragged kernels, per
// instance taken from a work queue).  The workgroup size follows the operand
// width so that every linear pass handles at most 16 limbs per thread:
//   width <= 2048 limbs -> 256 threads, <= 4096 -> 512, <= 8192 -> 1024.
// All operands and intermediates of an instance live in dynamic LDS laid out
// by plan_div (about 4h + 800 words: 36 KB at 2^16 bits, 134 KB at 2^18).
//
// A division or shifted inverse may run in two launches: the head kernels
// (four waves per workgroup, one instance per wave) compute the initial
// approximation and the Refine iterations with short operands and leave a
// record in each instance's output row; the body kernels pick it up.
//
// The build compiles this file once per kernel family and workgroup size
// (MP_KFAMILY: 0 product, 1 shifted inverse, 2 division, 3 ragged division,
// 4 heads; MP_KT: threads), each object holding one explicit instantiation
// of a launcher, so the translation units compile in parallel.
#include "mp_prims_hip.hpp"
#include "mp_core.hpp"
#include "mp_div.hpp"

namespace mp {

// Division kernels ask the compiler for at most 128 registers per lane (four
// waves per SIMD: four 256-thread workgroups per compute unit at 2^16 bits).
// MP_BODY_WAVES=5 builds the 256-thread kernels for five (96 registers, a few
// spills; the LDS plan at 2^16 bits also allows five): measured slower, as the
// instances then contend for the same units.
#ifndef MP_BODY_WAVES
#define MP_BODY_WAVES 4
#endif
#define MP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(T == 256 ? MP_BODY_WAVES : 4, 8)))
// heads: four waves per SIMD (16 per compute unit, which is also what their LDS allows)
#define MP_HEAD_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4, 8)))

// Workspace of a ragged batch (int32): [0, 4) instances per class, [4, 8)
// queue heads, then one list of instance indices per class, each `count` long.
constexpr int kClasses = 4;
constexpr int kWsHeader = 16;

MP_DEV int64_t uniform64(int64_t x)
{
    const uint32_t lo = uniform((uint32_t)x), hi = uniform((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int T>
__global__ __launch_bounds__(T) void k_mul(const uint32_t *a, int na, const uint32_t *b, int nb, uint32_t *c,
                                           Knobs kn)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mul_instance<T>(lds, a + j * na, na, b + j * nb, nb, c + j * (size_t)(na + nb), kn);
}

template <int T>
__global__ __launch_bounds__(T) MP_OCCUPANCY void k_shinv(const uint32_t *v, int nv, int h, uint32_t *w, int nw,
                                                          int32_t *status, Knobs kn, int head)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    uint32_t *wj = w + j * nw;
    shinv_instance<T>(lds, v + j * nv, nv, h, wj, nw, status ? status + j : nullptr, kn, head ? wj : nullptr);
}

template <int T>
__global__ __launch_bounds__(T) MP_OCCUPANCY void k_divrem(const uint32_t *u, int nu, const uint32_t *v, int nv,
                                                           uint32_t *q, int nq, uint32_t *r, int32_t *status,
                                                           Knobs kn, int head)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    uint32_t *qj = q + j * nq;
    divrem_instance<T>(lds, u + j * nu, nu, v + j * nv, nv, qj, nq, r + j * nv, status ? status + j : nullptr, kn,
                       head ? qj : nullptr);
}

// persistent workgroups of one class: take the next instance of the class's
// queue until it is empty
template <int T>
__global__ __launch_bounds__(T) MP_OCCUPANCY void k_ragged(const uint32_t *up, const uint32_t *vp,
                                                           const mp_desc_t *desc, uint32_t *qp, uint32_t *rp,
                                                           int32_t *status, int32_t *ws, int cls, int count, Knobs kn,
                                                           int head)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const int n = ws[cls];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) lds[kCtlBcast + 2] = (uint32_t)atomicAdd(&ws[kClasses + cls], 1);
        __syncthreads();
        // every value below is the same on all lanes: keep it in scalar registers
        const int idx = uniform((int)lds[kCtlBcast + 2]);
        if (idx >= n) break;
        const int j = uniform(ws[kWsHeader + (size_t)cls * count + idx]);
        const mp_desc_t &d = desc[j];
        const int64_t uo = uniform64(d.u_off), vo = uniform64(d.v_off), qo = uniform64(d.q_off),
                      ro = uniform64(d.r_off);
        const int nu = uniform(d.nu), nv = uniform(d.nv), nq = uniform(d.nq);
        divrem_instance<T>(lds, up + uo, nu, vp + vo, nv, qp + qo, nq, rp + ro, status + j, kn,
                           head ? qp + qo : nullptr);
    }
}

template <int T>
hipError_t launch_mul(int grid, size_t lds, hipStream_t st, const uint32_t *a, int na, const uint32_t *b, int nb,
                      uint32_t *c, Knobs kn)
{
    if (!lds_attr(reinterpret_cast<const void *>(k_mul<T>), lds)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mul<T>, dim3(grid), dim3(T), lds, st, a, na, b, nb, c, kn);
    return hipGetLastError();
}

template <int T>
hipError_t launch_shinv(int grid, size_t lds, hipStream_t st, const uint32_t *v, int nv, int h, uint32_t *w, int nw,
                        int32_t *status, Knobs kn, int head)
{
    if (!lds_attr(reinterpret_cast<const void *>(k_shinv<T>), lds)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_shinv<T>, dim3(grid), dim3(T), lds, st, v, nv, h, w, nw, status, kn, head);
    return hipGetLastError();
}

template <int T>
hipError_t launch_divrem(int grid, size_t lds, hipStream_t st, const uint32_t *u, int nu, const uint32_t *v, int nv,
                         uint32_t *q, int nq, uint32_t *r, int32_t *status, Knobs kn, int head)
{
    if (!lds_attr(reinterpret_cast<const void *>(k_divrem<T>), lds)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_divrem<T>, dim3(grid), dim3(T), lds, st, u, nu, v, nv, q, nq, r, status, kn, head);
    return hipGetLastError();
}

template <int T>
hipError_t launch_ragged(int grid, size_t lds, hipStream_t st, const uint32_t *up, const uint32_t *vp,
                         const mp_desc_t *desc, uint32_t *qp, uint32_t *rp, int32_t *status, int32_t *ws, int cls,
                         int count, Knobs kn, int head)
{
    if (!lds_attr(reinterpret_cast<const void *>(k_ragged<T>), lds)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ragged<T>, dim3(grid), dim3(T), lds, st, up, vp, desc, qp, rp, status, ws, cls, count, kn,
                       head);
    return hipGetLastError();
}

#if defined(MP_KFAMILY) && MP_KFAMILY == 4
// heads (not templates: compiled in their own translation unit only)

// Heads: wave w of workgroup b owns instance b * kHeadWaves + w and the
// `words` LDS words at lds + w * words (no workgroup barrier anywhere).
__global__ __launch_bounds__(kLanes * kHeadWaves) MP_HEAD_OCCUPANCY void k_head_divrem(const uint32_t *u, int nu, const uint32_t *v,
                                                                      int nv, uint32_t *q, int nq, int batch,
                                                                      int words, Knobs kn)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const int w = (int)(threadIdx.x / kLanes);
    const size_t j = (size_t)blockIdx.x * kHeadWaves + w;
    if (j >= (size_t)batch) return;
    head_divrem(lds + w * words, u + j * nu, nu, v + j * nv, nv, q + j * nq, nq, kn);
}

__global__ __launch_bounds__(kLanes * kHeadWaves) MP_HEAD_OCCUPANCY void k_head_shinv(const uint32_t *v, int nv, int h, uint32_t *w,
                                                                     int nw, int batch, int words, Knobs kn)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const int wv = (int)(threadIdx.x / kLanes);
    const size_t j = (size_t)blockIdx.x * kHeadWaves + wv;
    if (j >= (size_t)batch) return;
    head_shinv(lds + wv * words, h, v + j * nv, nv, w + j * nw, nw, kn);
}

// heads of a ragged batch: wave g takes the g-th valid instance of the class
// lists (the preparation kernel's buckets, in class order)
__global__ __launch_bounds__(kLanes * kHeadWaves) MP_HEAD_OCCUPANCY void k_head_ragged(const uint32_t *up, const uint32_t *vp,
                                                                      const mp_desc_t *desc, uint32_t *qp,
                                                                      const int32_t *ws, int count, int words,
                                                                      Knobs kn)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const int w = (int)(threadIdx.x / kLanes);
    int idx = (int)blockIdx.x * kHeadWaves + w, c = 0;
    while (c < kClasses && idx >= ws[c]) idx -= ws[c++];
    if (c == kClasses) return;
    const int j = uniform(ws[kWsHeader + (size_t)c * count + idx]);
    const mp_desc_t &d = desc[j];
    const int64_t uo = uniform64(d.u_off), vo = uniform64(d.v_off), qo = uniform64(d.q_off);
    const int nu = uniform(d.nu), nv = uniform(d.nv), nq = uniform(d.nq);
    head_divrem(lds + w * words, up + uo, nu, vp + vo, nv, qp + qo, nq, kn);
}

// LDS words of one head wave for the current knobs
int head_words(const Knobs &kn) { return plan_head(kn.small_limit, 0).total; }

hipError_t launch_head_divrem(hipStream_t st, const uint32_t *u, int nu, const uint32_t *v, int nv, uint32_t *q,
                              int nq, int batch, Knobs kn)
{
    const int words = head_words(kn);
    const size_t lds = (size_t)words * 4 * kHeadWaves;
    if (!lds_attr(reinterpret_cast<const void *>(k_head_divrem), lds)) return hipErrorInvalidValue;
    const int grid = (batch + kHeadWaves - 1) / kHeadWaves;
    hipLaunchKernelGGL(k_head_divrem, dim3(grid), dim3(kLanes * kHeadWaves), lds, st, u, nu, v, nv, q, nq, batch,
                       words, kn);
    return hipGetLastError();
}

hipError_t launch_head_shinv(hipStream_t st, const uint32_t *v, int nv, int h, uint32_t *w, int nw, int batch,
                             Knobs kn)
{
    const int words = head_words(kn);
    const size_t lds = (size_t)words * 4 * kHeadWaves;
    if (!lds_attr(reinterpret_cast<const void *>(k_head_shinv), lds)) return hipErrorInvalidValue;
    const int grid = (batch + kHeadWaves - 1) / kHeadWaves;
    hipLaunchKernelGGL(k_head_shinv, dim3(grid), dim3(kLanes * kHeadWaves), lds, st, v, nv, h, w, nw, batch, words,
                       kn);
    return hipGetLastError();
}

hipError_t launch_head_ragged(hipStream_t st, const uint32_t *up, const uint32_t *vp, const mp_desc_t *desc,
                              uint32_t *qp, const int32_t *ws, int count, Knobs kn)
{
    const int words = head_words(kn);
    const size_t lds = (size_t)words * 4 * kHeadWaves;
    if (!lds_attr(reinterpret_cast<const void *>(k_head_ragged), lds)) return hipErrorInvalidValue;
    const int grid = (count + kHeadWaves - 1) / kHeadWaves;
    hipLaunchKernelGGL(k_head_ragged, dim3(grid), dim3(kLanes * kHeadWaves), lds, st, up, vp, desc, qp, ws, count,
                       words, kn);
    return hipGetLastError();
}

#endif

#if defined(MP_KFAMILY) && defined(MP_KT)
#if MP_KFAMILY == 0
template hipError_t launch_mul<MP_KT>(int, size_t, hipStream_t, const uint32_t *, int, const uint32_t *, int,
                                      uint32_t *, Knobs);
#elif MP_KFAMILY == 1
template hipError_t launch_shinv<MP_KT>(int, size_t, hipStream_t, const uint32_t *, int, int, uint32_t *, int,
                                        int32_t *, Knobs, int);
#elif MP_KFAMILY == 2
template hipError_t launch_divrem<MP_KT>(int, size_t, hipStream_t, const uint32_t *, int, const uint32_t *, int,
                                         uint32_t *, int, uint32_t *, int32_t *, Knobs, int);
#elif MP_KFAMILY == 3
template hipError_t launch_ragged<MP_KT>(int, size_t, hipStream_t, const uint32_t *, const uint32_t *,
                                         const mp_desc_t *, uint32_t *, uint32_t *, int32_t *, int32_t *, int, int,
                                         Knobs, int);
#endif
#endif

}  // namespace mp

#if defined(MP_PHASE_TRACE) && MP_KFAMILY == 4
// copies the head stamps of the first `waves` instances (32 per instance) to host memory
extern "C" int mp_trace_read_head(uint64_t *dst, int waves)
{
    return (int)hipMemcpyFromSymbol(dst, HIP_SYMBOL(mp_trace_buf), (size_t)waves * 32 * sizeof(uint64_t), 0,
                                    hipMemcpyDeviceToHost);
}
#endif

#if defined(MP_PHASE_TRACE) && MP_KFAMILY == 0 && MP_KT == 256
// copies the stamps of the first `blocks` product workgroups (32 per workgroup) to host memory
extern "C" int mp_trace_read_mul(uint64_t *dst, int blocks)
{
    return (int)hipMemcpyFromSymbol(dst, HIP_SYMBOL(mp_trace_buf), (size_t)blocks * 32 * sizeof(uint64_t), 0,
                                    hipMemcpyDeviceToHost);
}
#endif

#if defined(MP_PHASE_TRACE) && MP_KFAMILY == 2 && MP_KT == 256
// copies the stamps of the first `blocks` workgroups (32 per workgroup) to host memory
extern "C" int mp_trace_read_divrem(uint64_t *dst, int blocks)
{
    return (int)hipMemcpyFromSymbol(dst, HIP_SYMBOL(mp_trace_buf), (size_t)blocks * 32 * sizeof(uint64_t), 0,
                                    hipMemcpyDeviceToHost);
}
// copies the product records of the first `blocks` workgroups (48 x 6 words each)
extern "C" int mp_trace_read_products(uint64_t *dst, int blocks)
{
    return (int)hipMemcpyFromSymbol(dst, HIP_SYMBOL(mp_ptrace_buf), (size_t)blocks * 48 * 6 * sizeof(uint64_t), 0,
                                    hipMemcpyDeviceToHost);
}
#endif
