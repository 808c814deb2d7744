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

#include <string.h>

namespace {

constexpr int kMaxLimbs = 8192;
constexpr int kLdsWords = 160 * 1024 / 4;   // gfx950: 160 KB of LDS per workgroup

template <int T>
__global__ __launch_bounds__(T) void k_mul(const uint32_t *a, int na, const uint32_t *b, int nb, uint32_t *c)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mp::mul_instance<T>(lds, a + j * na, na, b + j * nb, nb, c + j * (size_t)(na + nb));
}

template <int T>
__global__ __launch_bounds__(T) void k_shinv(const uint32_t *v, int nv, int h, uint32_t *w, int nw,
                                             int32_t *status)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mp::shinv_instance<T>(lds, v + j * nv, nv, h, w + j * nw, nw, status ? status + j : nullptr);
}

template <int T>
__global__ __launch_bounds__(T) void k_divrem(const uint32_t *u, int nu, const uint32_t *v, int nv,
                                              uint32_t *q, int nq, uint32_t *r, int32_t *status)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const size_t j = blockIdx.x;
    mp::divrem_instance<T>(lds, u + j * nu, nu, v + j * nv, nv, q + j * nq, nq, r + j * nv,
                           status ? status + j : nullptr);
}

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

template <typename Kern>
bool set_lds(Kern kernel, size_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
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

}  // extern "C"
