// Workgroup and wavefront primitives for gfx950 (CDNA4, wave64).
//
// The multi-precision code in mp_core.hpp / mp_div.hpp is written against
// exactly this small set of operations: thread index, workgroup barrier,
// wave ballot / shuffles, a wave-uniform broadcast, and the 4x4 block of
// 32x32->64-bit multiply-accumulates that dominates every product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MP_DEV __device__ __forceinline__

// Phase tracing (a diagnostic build option, off by default): with
// MP_PHASE_TRACE defined, MP_STAMP(id) records the shader clock of
// workgroup thread 0 in slot id (< 32) of the workgroup's row of
// mp_trace_buf (one per translation unit, for up to 8192 workgroups).
#ifdef MP_PHASE_TRACE
static __device__ uint64_t mp_trace_buf[8192 * 32];
#define MP_STAMP(id)                                                                                          \
    do {                                                                                                      \
        if (threadIdx.x == 0 && blockIdx.x < 8192) mp_trace_buf[(size_t)blockIdx.x * 32 + (id)] = __builtin_readcyclecounter(); \
    } while (0)
// MP_RSTAMP(id): the constant-rate (100 MHz) real-time counter instead, which
// gives the shader clock rate of the run against the cycle stamps
#define MP_RSTAMP(id)                                                                                         \
    do {                                                                                                      \
        if (threadIdx.x == 0 && blockIdx.x < 8192) mp_trace_buf[(size_t)blockIdx.x * 32 + (id)] = __builtin_amdgcn_s_memrealtime(); \
    } while (0)
// MP_WSTAMP(id): the same for lane 0 of each wave, in the row of the wave's
// global index (heads: one instance per wave)
#define MP_WSTAMP(id)                                                                                          \
    do {                                                                                                       \
        const size_t wv_ = (size_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;                          \
        if ((threadIdx.x & 63) == 0 && wv_ < 8192) mp_trace_buf[wv_ * 32 + (id)] = __builtin_readcyclecounter(); \
    } while (0)
// MP_WRSTAMP(id): the real-time counter for lane 0 of each wave (heads)
#define MP_WRSTAMP(id)                                                                                         \
    do {                                                                                                       \
        const size_t wv_ = (size_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;                          \
        if ((threadIdx.x & 63) == 0 && wv_ < 8192) mp_trace_buf[wv_ * 32 + (id)] = __builtin_amdgcn_s_memrealtime(); \
    } while (0)
// Product trace: for each product an instance forms (up to 48), thread 0
// records its shape and the shader clock at its start, after the digit
// conversion (or window copy), after the first wave's strips and at its end,
// in 6 words of the workgroup's row of mp_ptrace_buf.  The running count
// lives in LDS, touched by thread 0 only.
static __device__ uint64_t mp_ptrace_buf[8192 * 48 * 6];
__device__ __forceinline__ int &mp_ptrace_count()
{
    __shared__ int n;
    return n;
}
#define MP_PT_RESET()                                                    \
    do {                                                                 \
        if (threadIdx.x == 0) mp_ptrace_count() = 0;                     \
    } while (0)
#define MP_PT_BEGIN(nx, ny, ncols, c0)                                                                       \
    do {                                                                                                     \
        const int n_ = mp_ptrace_count();                                                                    \
        if (threadIdx.x == 0 && blockIdx.x < 8192 && n_ < 48) {                                             \
            uint64_t *r_ = mp_ptrace_buf + ((size_t)blockIdx.x * 48 + n_) * 6;                               \
            r_[0] = (uint64_t)(uint32_t)(nx) | ((uint64_t)(uint32_t)(ny) << 32);                             \
            r_[1] = (uint64_t)(uint32_t)(ncols) | ((uint64_t)(uint32_t)(c0) << 32);                          \
            r_[2] = __builtin_readcyclecounter();                                                            \
        }                                                                                                    \
    } while (0)
#define MP_PT(slot)                                                                                          \
    do {                                                                                                     \
        const int n_ = mp_ptrace_count();                                                                    \
        if (threadIdx.x == 0 && blockIdx.x < 8192 && n_ < 48)                                               \
            mp_ptrace_buf[((size_t)blockIdx.x * 48 + n_) * 6 + (slot)] = __builtin_readcyclecounter();      \
    } while (0)
#define MP_PT_END()                                                                                          \
    do {                                                                                                     \
        MP_PT(5);                                                                                            \
        if (threadIdx.x == 0) mp_ptrace_count() += 1;                                                        \
    } while (0)
#else
#define MP_PT_RESET() \
    do {              \
    } while (0)
#define MP_PT_BEGIN(nx, ny, ncols, c0) \
    do {                               \
    } while (0)
#define MP_PT(slot) \
    do {            \
    } while (0)
#define MP_PT_END() \
    do {            \
    } while (0)
#define MP_STAMP(id) \
    do {             \
    } while (0)
#define MP_WSTAMP(id) \
    do {              \
    } while (0)
#define MP_RSTAMP(id) \
    do {              \
    } while (0)
#define MP_WRSTAMP(id) \
    do {               \
    } while (0)
#endif

namespace mp {

constexpr int kLanes = 64;  // CDNA wavefront width

MP_DEV int lane() { return (int)(threadIdx.x & (kLanes - 1)); }
// index of the calling thread among the T threads working on one instance:
// the workgroup's thread index, or the lane when a single wave owns the
// instance (that wave may be any wave of its workgroup)
template <int T>
MP_DEV int tid()
{
    if constexpr (T == kLanes) return lane();
    else return (int)threadIdx.x;
}
MP_DEV void sync() { __syncthreads(); }
// orders this wave's LDS accesses before and after it (a wave runs in
// lockstep and the LDS serves one wave's requests in order; only the
// compiler must not move accesses across)
MP_DEV void wave_sync() { asm volatile("" ::: "memory"); }
MP_DEV uint64_t ballot(bool p) { return __ballot(p); }

// DPP controls (GFX9 data-parallel primitives: a VALU source operand read
// from another lane of the same wave, no LDS round trip)
constexpr int kDppQuadSwap1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kDppWaveShr1 = 0x138;      // lane i reads lane i - 1
constexpr int kDppRowMirror = 0x140;     // lane i of a 16-lane row reads lane 15 - i
constexpr int kDppRowHalfMirror = 0x141; // lane i of an 8-lane half row reads lane 7 - i
constexpr int kDppRowBcast15 = 0x142;    // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143;    // lane 31 to rows 2 and 3

// x of the lane the DPP control selects; lanes without a source (and rows
// outside row_mask) receive 0
template <int CTRL, int ROWS = 0xF>
MP_DEV uint32_t dpp(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, false);
}

// value held by lane-1 (lane 0 receives 0)
MP_DEV uint32_t shfl_up1(uint32_t x) { return dpp<kDppWaveShr1>(x); }

// value held by lane-2 (lanes 0 and 1 receive 0)
MP_DEV uint32_t shfl_up2(uint32_t x) { return dpp<kDppWaveShr1>(dpp<kDppWaveShr1>(x)); }

MP_DEV uint32_t shfl_xor(uint32_t x, int m) { return __shfl_xor(x, m); }

// value of x in lane src (src may differ per lane)
MP_DEV uint32_t shfl(uint32_t x, int src) { return __shfl(x, src); }

// value of x in lane l (l wave-uniform)
MP_DEV uint32_t readlane(uint32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }

// a value every lane of the wave already agrees on, moved to a scalar register
MP_DEV uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
MP_DEV int uniform(int x) { return (int)__builtin_amdgcn_readfirstlane((uint32_t)x); }

// acc[r] += a * b[r] for r = 0..3, each acc a 96-bit column sum held as a
// 64-bit low part and a 32-bit high part.  v_mad_u64_u32 forms a*b + lo with
// the carry out in an SGPR pair; v_addc folds the carry into hi.  On gfx950 a
// VALU carry write needs two wait states before a VALU reads it; the three
// independent multiplies placed between each write and its read provide them.
MP_DEV void mac4(uint64_t (&lo)[4], uint32_t (&hi)[4], uint32_t a,
                 uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3)
{
    uint64_t c0, c1, c2, c3;
    asm volatile(
        "v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
        "v_mad_u64_u32 %1, %9, %12, %14, %1\n\t"
        "v_mad_u64_u32 %2, %10, %12, %15, %2\n\t"
        "v_mad_u64_u32 %3, %11, %12, %16, %3\n\t"
        "v_addc_co_u32_e64 %4, %8, 0, %4, %8\n\t"
        "v_addc_co_u32_e64 %5, %9, 0, %5, %9\n\t"
        "v_addc_co_u32_e64 %6, %10, 0, %6, %10\n\t"
        "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
        : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]),
          "+v"(hi[0]), "+v"(hi[1]), "+v"(hi[2]), "+v"(hi[3]),
          "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3)
        : "v"(a), "v"(b0), "v"(b1), "v"(b2), "v"(b3));
}

// acc[r] += a_r * b_r for r = 0..3 (four independent 96-bit column sums, as
// mac4 but with a different multiplier per sum; the same wait-state spacing)
MP_DEV void mac4x(uint64_t (&lo)[4], uint32_t (&hi)[4], uint32_t a0, uint32_t b0, uint32_t a1, uint32_t b1,
                  uint32_t a2, uint32_t b2, uint32_t a3, uint32_t b3)
{
    uint64_t c0, c1, c2, c3;
    asm volatile(
        "v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
        "v_mad_u64_u32 %1, %9, %14, %15, %1\n\t"
        "v_mad_u64_u32 %2, %10, %16, %17, %2\n\t"
        "v_mad_u64_u32 %3, %11, %18, %19, %3\n\t"
        "v_addc_co_u32_e64 %4, %8, 0, %4, %8\n\t"
        "v_addc_co_u32_e64 %5, %9, 0, %5, %9\n\t"
        "v_addc_co_u32_e64 %6, %10, 0, %6, %10\n\t"
        "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
        : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]),
          "+v"(hi[0]), "+v"(hi[1]), "+v"(hi[2]), "+v"(hi[3]),
          "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3)
        : "v"(a0), "v"(b0), "v"(a1), "v"(b1), "v"(a2), "v"(b2), "v"(a3), "v"(b3));
}

// bytes [sel, sel + 4) of the 8-byte value hi:lo (sel in 0..3)
MP_DEV uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t sel) { return __builtin_amdgcn_alignbyte(hi, lo, sel); }

MP_DEV uint32_t bswap(uint32_t x) { return __builtin_bswap32(x); }

// ---------------------------------------------------------- int8 matrix core
// v_mfma_i32_32x32x32_i8: D[32x32] += X[32x32] * Y[32x32], int8 inputs, int32
// sums.  Lane l supplies X row l%32 and Y column l%32, each as 16 bytes
// (k = 16*(l/32) + byte index, the same k order for X and Y), and receives
// D[8*(v/4) + 4*(l/32) + v%4][l%32] in accumulator element v.
typedef int MfmaFrag __attribute__((ext_vector_type(4)));
typedef int MfmaAcc __attribute__((ext_vector_type(16)));

MP_DEV MfmaAcc mfma_zero() { return MfmaAcc{}; }
MP_DEV MfmaAcc mfma_i8(MfmaAcc acc, uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                       uint32_t y0, uint32_t y1, uint32_t y2, uint32_t y3)
{
    const MfmaFrag x = {(int)x0, (int)x1, (int)x2, (int)x3}, y = {(int)y0, (int)y1, (int)y2, (int)y3};
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(x, y, acc, 0, 0, 0);
}
MP_DEV int mfma_get(const MfmaAcc &acc, int v) { return acc[v]; }
MP_DEV MfmaAcc mfma_add(MfmaAcc a, MfmaAcc b) { return a + b; }

// marks a value as used without emitting any instruction
MP_DEV void keep(uint32_t x) { asm volatile("" : : "v"(x)); }

// 16-byte vector load and store of four limbs; p must be 16-byte aligned
struct Limb4 {
    uint32_t x, y, z, w;
};

MP_DEV Limb4 load4(const uint32_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(__builtin_assume_aligned(p, 16));
    return Limb4{v.x, v.y, v.z, v.w};
}

MP_DEV void store4(uint32_t *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    *reinterpret_cast<uint4 *>(__builtin_assume_aligned(p, 16)) = make_uint4(a, b, c, d);
}

}  // namespace mp
