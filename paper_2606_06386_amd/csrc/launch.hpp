// Host-side launchers of the division kernels (defined in kernels.hip, one
// translation unit per kernel family and workgroup size so that they compile
// in parallel) and the tuning knobs every division kernel receives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpdiv.h"

namespace mp {

// Run-time tuning knobs of the division kernels (kernel arguments, so a
// change applies to the next launch without a rebuild):
//   mfma_min     products whose shorter operand has at least this many limbs
//                run on the int8 matrix cores, shorter ones on the vector ALU;
//   small_limit  Refine iterations whose iterate (l + g + 1 limbs) is shorter
//                than this run in the head kernels (one wave per instance);
//                0 runs every step in the body kernels.
struct Knobs {
    int32_t mfma_min;
    int32_t small_limit;
};

// sets a kernel's dynamic-LDS limit to at least `bytes` on the current device
// (cached: no runtime call once the limit is high enough)
bool lds_attr(const void *kernel, size_t bytes);

template <int T>
hipError_t launch_mul(int grid, size_t lds, hipStream_t st, const uint32_t *a, int na, const uint32_t *b, int nb,
                      uint32_t *c, Knobs kn);

// body kernels: head != 0 when a head kernel ran before on the same stream
template <int T>
hipError_t launch_shinv(int grid, size_t lds, hipStream_t st, const uint32_t *v, int nv, int h, uint32_t *w, int nw,
                        int32_t *status, Knobs kn, int head);

template <int T>
hipError_t launch_divrem(int grid, size_t lds, hipStream_t st, const uint32_t *u, int nu, const uint32_t *v, int nv,
                         uint32_t *q, int nq, uint32_t *r, int32_t *status, Knobs kn, int head);

template <int T>
hipError_t launch_ragged(int grid, size_t lds, hipStream_t st, const uint32_t *up, const uint32_t *vp,
                         const mp_desc_t *desc, uint32_t *qp, uint32_t *rp, int32_t *status, int32_t *ws, int cls,
                         int count, Knobs kn, int head);

// head kernels (kn.small_limit > 0): records in the q (w) rows of the instances
hipError_t launch_head_divrem(hipStream_t st, const uint32_t *u, int nu, const uint32_t *v, int nv, uint32_t *q,
                              int nq, int batch, Knobs kn);
hipError_t launch_head_shinv(hipStream_t st, const uint32_t *v, int nv, int h, uint32_t *w, int nw, int batch,
                             Knobs kn);
hipError_t launch_head_ragged(hipStream_t st, const uint32_t *up, const uint32_t *vp, const mp_desc_t *desc,
                              uint32_t *qp, const int32_t *ws, int count, Knobs kn);

}  // namespace mp
