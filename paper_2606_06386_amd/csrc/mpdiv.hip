// Kernels and C ABI of libmpdiv (see include/mpdiv.h).
//
// One workgroup per instance.  The workgroup size follows the operand width
// so that every linear pass handles at most 16 limbs per thread:
//   width <= 2048 limbs -> 256 threads, <= 4096 -> 512, <= 8192 -> 1024.
// All operands and intermediates of an instance live in dynamic LDS laid out
// by plan_div (about 4h + 800 words: 36 KB at 2^16 bits, 134 KB at 2^18).
#include "mp_prims_hip.hpp"
#include "mp_core.hpp"
#include "mp_div.hpp"

#include "../../include/mpdiv.h"

#include <mutex>
#include <string.h>

namespace {

constexpr int kMaxLimbs = 8192;

// Division kernels ask the compiler for at most 128 registers per lane, so
// that four waves share each SIMD: four 256-thread workgroups per compute
// unit at 2^16 bits, where the LDS plan also allows four.
#define MP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4, 8)))
constexpr int kLdsWords = 160 * 1024 / 4;   // gfx950: 160 KB of LDS per workgroup

template <int T>
__global__ __launch_bounds__(T) void k_mul(const uint32_t *a, int na, const uint32_t *b, int nb, uint32_t *c)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mp::mul_instance<T>(lds, a + j * na, na, b + j * nb, nb, c + j * (size_t)(na + nb));
}

template <int T>
__global__ __launch_bounds__(T) MP_OCCUPANCY void k_shinv(const uint32_t *v, int nv, int h, uint32_t *w, int nw,
                                             int32_t *status)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mp::shinv_instance<T>(lds, v + j * nv, nv, h, w + j * nw, nw, status ? status + j : nullptr);
}

template <int T>
__global__ __launch_bounds__(T) MP_OCCUPANCY void k_divrem(const uint32_t *u, int nu, const uint32_t *v, int nv,
                                              uint32_t *q, int nq, uint32_t *r, int32_t *status)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mp::divrem_instance<T>(lds, u + j * nu, nu, v + j * nv, nv, q + j * nq, nq, r + j * nv,
                           status ? status + j : nullptr);
}

// ------------------------------------------------------------ ragged batches
//
// Workspace (int32): [0, 4) instances per class, [4, 8) queue heads, then one
// list of instance indices per class, each `count` long.
constexpr int kClasses = 4;
constexpr int kClassWidth[kClasses] = {1024, 2048, 4096, 8192};
constexpr int kWsHeader = 16;

__device__ __forceinline__ int width_class(int nu)
{
    return nu <= 1024 ? 0 : nu <= 2048 ? 1 : nu <= 4096 ? 2 : 3;
}

// one workgroup: validate descriptors and bucket instance indices by class
__global__ __launch_bounds__(1024) void k_ragged_prep(const mp_desc_t *desc, int count, int64_t lu, int64_t lv,
                                                      int64_t lq, int64_t lr, int32_t *status, int32_t *ws)
{
    __shared__ int cnt[kClasses];
    if (threadIdx.x < kClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < count; j += blockDim.x) {
        const mp_desc_t d = desc[j];
        const bool ok = d.nu >= 1 && d.nu <= kMaxLimbs && d.nv >= 1 && d.nv <= kMaxLimbs && d.nq >= 1 &&
                        d.u_off >= 0 && d.v_off >= 0 && d.q_off >= 0 && d.r_off >= 0 &&
                        d.u_off <= lu - d.nu && d.v_off <= lv - d.nv && d.q_off <= lq - d.nq &&
                        d.r_off <= lr - d.nv;   // (no overflow: widths are small, offsets >= 0)
        if (!ok) {
            status[j] = MP_INST_BADDESC;
            continue;
        }
        const int c = width_class(d.nu);
        const int slot = atomicAdd(&cnt[c], 1);
        ws[kWsHeader + (size_t)c * count + slot] = j;
    }
    __syncthreads();
    if (threadIdx.x < kClasses) {
        ws[threadIdx.x] = cnt[threadIdx.x];
        ws[kClasses + threadIdx.x] = 0;
    }
}

__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    const uint32_t lo = mp::uniform((uint32_t)x), hi = mp::uniform((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// persistent workgroups of one class: take the next instance of the class's
// queue until it is empty
template <int T>
__global__ __launch_bounds__(T) MP_OCCUPANCY void k_ragged(const uint32_t *up, const uint32_t *vp, const mp_desc_t *desc,
                                              uint32_t *qp, uint32_t *rp, int32_t *status, int32_t *ws, int cls,
                                              int count)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const int n = ws[cls];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) lds[mp::kCtlBcast + 2] = (uint32_t)atomicAdd(&ws[kClasses + cls], 1);
        __syncthreads();
        // every value below is the same on all lanes: keep it in scalar registers
        const int idx = mp::uniform((int)lds[mp::kCtlBcast + 2]);
        if (idx >= n) break;
        const int j = mp::uniform(ws[kWsHeader + (size_t)cls * count + idx]);
        const mp_desc_t &d = desc[j];
        const int64_t uo = uniform64(d.u_off), vo = uniform64(d.v_off), qo = uniform64(d.q_off),
                      ro = uniform64(d.r_off);
        const int nu = mp::uniform(d.nu), nv = mp::uniform(d.nv), nq = mp::uniform(d.nq);
        mp::divrem_instance<T>(lds, up + uo, nu, vp + vo, nv, qp + qo, nq, rp + ro, status + j);
    }
}

struct RaggedConfig {
    int threads[kClasses] = {256, 256, 512, 1024};
    int wgs_per_cu[kClasses] = {6, 3, 2, 1};
};
RaggedConfig g_ragged;
std::mutex g_ragged_mu;

int threads_for(int width)
{
    return width <= 2048 ? 256 : width <= 4096 ? 512 : 1024;
}

// the current device is gfx950 (checked once per device)
bool device_ok()
{
    static int checked[64];   // 0 unknown, 1 ok, 2 not usable
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    if (checked[dev] == 0) {
        hipDeviceProp_t prop;
        bool ok = hipGetDeviceProperties(&prop, dev) == hipSuccess &&
                  strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        checked[dev] = ok ? 1 : 2;
    }
    return checked[dev] == 1;
}

mp_status_t finish_launch()
{
    return hipGetLastError() == hipSuccess ? MP_OK : MP_ERR_LAUNCH;
}

// raise a kernel's dynamic LDS limit to at least `bytes` on the current
// device; the attribute is set only when it grows, so repeated launches (and
// launches under stream capture) make no further runtime call
template <typename Kern>
bool set_lds(Kern kernel, size_t bytes)
{
    struct Entry {
        const void *fn;
        int dev;
        size_t bytes;
    };
    static Entry seen[256];
    static int nseen;
    static std::mutex mu;
    const void *fn = reinterpret_cast<const void *>(kernel);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lock(mu);
    Entry *e = nullptr;
    for (int i = 0; i < nseen; i++)
        if (seen[i].fn == fn && seen[i].dev == dev) e = &seen[i];
    if (e && e->bytes >= bytes) return true;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return false;
    if (!e && nseen < 256) e = &seen[nseen++];
    if (e) *e = Entry{fn, dev, bytes};
    return true;
}

}  // namespace

extern "C" {

const char *mp_status_str(mp_status_t s)
{
    switch (s) {
    case MP_OK: return "MP_OK";
    case MP_ERR_ARG: return "MP_ERR_ARG: invalid argument";
    case MP_ERR_SIZE: return "MP_ERR_SIZE: operand wider than mp_max_limbs()";
    case MP_ERR_LAUNCH: return "MP_ERR_LAUNCH: kernel launch failed";
    case MP_ERR_DEVICE: return "MP_ERR_DEVICE: no usable gfx950 device";
    }
    return "unknown mp_status_t";
}

int32_t mp_max_limbs(void) { return kMaxLimbs; }

mp_status_t mp_mul_batch(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb,
                         uint32_t *c, int32_t batch, void *stream)
{
    if (!a || !b || !c || na <= 0 || nb <= 0 || batch < 0) return MP_ERR_ARG;
    if (na > kMaxLimbs || nb > kMaxLimbs) return MP_ERR_SIZE;
    if (batch == 0) return MP_OK;
    if (!device_ok()) return MP_ERR_DEVICE;
    const int words = mp::mul_lds_words(na, nb);
    if (words > kLdsWords) return MP_ERR_SIZE;
    const size_t bytes = (size_t)words * 4;
    hipStream_t st = (hipStream_t)stream;
    switch (threads_for((na + nb + 1) / 2)) {
    case 256:
        if (!set_lds(k_mul<256>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_mul<256>, dim3(batch), dim3(256), bytes, st, a, na, b, nb, c);
        break;
    case 512:
        if (!set_lds(k_mul<512>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_mul<512>, dim3(batch), dim3(512), bytes, st, a, na, b, nb, c);
        break;
    default:
        if (!set_lds(k_mul<1024>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_mul<1024>, dim3(batch), dim3(1024), bytes, st, a, na, b, nb, c);
        break;
    }
    return finish_launch();
}

mp_status_t mp_shinv_batch(const uint32_t *v, int32_t nv, int32_t h, uint32_t *w, int32_t nw,
                           int32_t *inst_status, int32_t batch, void *stream)
{
    if (!v || !w || nv <= 0 || nw <= 0 || h < 0 || batch < 0) return MP_ERR_ARG;
    if (nv > kMaxLimbs || h > kMaxLimbs) return MP_ERR_SIZE;
    if (batch == 0) return MP_OK;
    if (!device_ok()) return MP_ERR_DEVICE;
    const int T = threads_for(h > 0 ? h : 1);
    int words = mp::plan_short_words(h + 1, T);
    const int kmax = (nv < h ? nv : h) - 1;
    for (int k = 1; k <= kmax; k++) words = mp::hmax(words, mp::plan_div(h, k).total);
    if (words > kLdsWords) return MP_ERR_SIZE;
    const size_t bytes = (size_t)words * 4;
    hipStream_t st = (hipStream_t)stream;
    switch (T) {
    case 256:
        if (!set_lds(k_shinv<256>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_shinv<256>, dim3(batch), dim3(256), bytes, st, v, nv, h, w, nw, inst_status);
        break;
    case 512:
        if (!set_lds(k_shinv<512>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_shinv<512>, dim3(batch), dim3(512), bytes, st, v, nv, h, w, nw, inst_status);
        break;
    default:
        if (!set_lds(k_shinv<1024>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_shinv<1024>, dim3(batch), dim3(1024), bytes, st, v, nv, h, w, nw, inst_status);
        break;
    }
    return finish_launch();
}

mp_status_t mp_divrem_batch(const uint32_t *u, int32_t nu, const uint32_t *v, int32_t nv,
                            uint32_t *q, int32_t nq, uint32_t *r, int32_t *inst_status,
                            int32_t batch, void *stream)
{
    if (!u || !v || !q || !r || nu <= 0 || nv <= 0 || nq <= 0 || batch < 0) return MP_ERR_ARG;
    if (nu > kMaxLimbs || nv > kMaxLimbs) return MP_ERR_SIZE;
    if (batch == 0) return MP_OK;
    if (!device_ok()) return MP_ERR_DEVICE;
    const int T = threads_for(nu);
    const int words = mp::div_lds_words(nu, nv, T);
    if (words > kLdsWords) return MP_ERR_SIZE;
    const size_t bytes = (size_t)words * 4;
    hipStream_t st = (hipStream_t)stream;
    switch (T) {
    case 256:
        if (!set_lds(k_divrem<256>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_divrem<256>, dim3(batch), dim3(256), bytes, st, u, nu, v, nv, q, nq, r, inst_status);
        break;
    case 512:
        if (!set_lds(k_divrem<512>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_divrem<512>, dim3(batch), dim3(512), bytes, st, u, nu, v, nv, q, nq, r, inst_status);
        break;
    default:
        if (!set_lds(k_divrem<1024>, bytes)) return MP_ERR_LAUNCH;
        hipLaunchKernelGGL(k_divrem<1024>, dim3(batch), dim3(1024), bytes, st, u, nu, v, nv, q, nq, r, inst_status);
        break;
    }
    return finish_launch();
}

int64_t mp_ragged_workspace_bytes(int32_t count)
{
    return count < 0 ? 0 : (int64_t)4 * (kWsHeader + (int64_t)kClasses * count);
}

mp_status_t mp_ragged_config(int32_t cls, int32_t threads, int32_t wgs_per_cu)
{
    if (cls < 0 || cls >= kClasses || wgs_per_cu < 1 || wgs_per_cu > 8) return MP_ERR_ARG;
    if (threads != 256 && threads != 512 && threads != 1024) return MP_ERR_ARG;
    if (threads * 8 < kClassWidth[cls]) return MP_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_ragged_mu);
    g_ragged.threads[cls] = threads;
    g_ragged.wgs_per_cu[cls] = wgs_per_cu;
    return MP_OK;
}

mp_status_t mp_divrem_ragged(const uint32_t *u_pool, int64_t u_limbs, const uint32_t *v_pool, int64_t v_limbs,
                             const mp_desc_t *desc, uint32_t *q_pool, int64_t q_limbs, uint32_t *r_pool,
                             int64_t r_limbs, int32_t *inst_status, int32_t count, void *workspace,
                             void *stream)
{
    if (!u_pool || !v_pool || !desc || !q_pool || !r_pool || !inst_status || !workspace || count < 0)
        return MP_ERR_ARG;
    if (u_limbs < 0 || v_limbs < 0 || q_limbs < 0 || r_limbs < 0) return MP_ERR_ARG;
    if (count == 0) return MP_OK;
    if (!device_ok()) return MP_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_ragged_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MP_ERR_DEVICE;
    // per-device fork streams and events (default priority), made once
    static hipStream_t fork[64][kClasses];
    static hipEvent_t ev_fork[64], ev_join[64][kClasses];
    static int cus[64];
    if (cus[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MP_ERR_DEVICE;
        for (int c = 0; c < kClasses; c++) {
            if (hipStreamCreateWithFlags(&fork[dev][c], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev_join[dev][c], hipEventDisableTiming) != hipSuccess)
                return MP_ERR_LAUNCH;
        }
        if (hipEventCreateWithFlags(&ev_fork[dev], hipEventDisableTiming) != hipSuccess) return MP_ERR_LAUNCH;
        cus[dev] = prop.multiProcessorCount;
    }
    hipStream_t st = (hipStream_t)stream;
    int32_t *ws = (int32_t *)workspace;
    hipLaunchKernelGGL(k_ragged_prep, dim3(1), dim3(1024), 0, st, desc, count, u_limbs, v_limbs, q_limbs,
                       r_limbs, inst_status, ws);
    if (hipGetLastError() != hipSuccess || hipEventRecord(ev_fork[dev], st) != hipSuccess) return MP_ERR_LAUNCH;
    for (int c = 0; c < kClasses; c++) {
        hipStream_t fs = fork[dev][c];
        if (hipStreamWaitEvent(fs, ev_fork[dev], 0) != hipSuccess) return MP_ERR_LAUNCH;
        const int T = g_ragged.threads[c];
        // LDS of the class's widest instance (a scan over every divisor length: computed once)
        static size_t lds_bytes[kClasses][3];
        const int ti = T == 256 ? 0 : T == 512 ? 1 : 2;
        if (lds_bytes[c][ti] == 0) lds_bytes[c][ti] = (size_t)mp::div_lds_words(kClassWidth[c], kClassWidth[c], T) * 4;
        const size_t bytes = lds_bytes[c][ti];
        if (bytes > (size_t)kLdsWords * 4) return MP_ERR_SIZE;
        const int fit = (int)(((size_t)kLdsWords * 4) / bytes);
        const int wpc = g_ragged.wgs_per_cu[c] < fit ? g_ragged.wgs_per_cu[c] : fit;
        const dim3 grid(cus[dev] * wpc);
        switch (T) {
        case 256:
            if (!set_lds(k_ragged<256>, bytes)) return MP_ERR_LAUNCH;
            hipLaunchKernelGGL(k_ragged<256>, grid, dim3(256), bytes, fs, u_pool, v_pool, desc, q_pool, r_pool,
                               inst_status, ws, c, count);
            break;
        case 512:
            if (!set_lds(k_ragged<512>, bytes)) return MP_ERR_LAUNCH;
            hipLaunchKernelGGL(k_ragged<512>, grid, dim3(512), bytes, fs, u_pool, v_pool, desc, q_pool, r_pool,
                               inst_status, ws, c, count);
            break;
        default:
            if (!set_lds(k_ragged<1024>, bytes)) return MP_ERR_LAUNCH;
            hipLaunchKernelGGL(k_ragged<1024>, grid, dim3(1024), bytes, fs, u_pool, v_pool, desc, q_pool, r_pool,
                               inst_status, ws, c, count);
            break;
        }
        if (hipGetLastError() != hipSuccess || hipEventRecord(ev_join[dev][c], fs) != hipSuccess ||
            hipStreamWaitEvent(st, ev_join[dev][c], 0) != hipSuccess)
            return MP_ERR_LAUNCH;
    }
    return MP_OK;
}

}  // extern "C"
