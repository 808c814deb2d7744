// C ABI of libmpdiv (see include/mpdiv.h): argument checks, launch
// configuration and the ragged-batch preparation kernel.  The division
// kernels themselves are in kernels.hip.
#include "mp_prims_hip.hpp"
#include "mp_core.hpp"
#include "mp_div.hpp"
#include "launch.hpp"

#include "../../include/mpdiv.h"

#include <atomic>
#include <mutex>
#include <string.h>

namespace {

constexpr int kMaxLimbs = 8192;
constexpr int kLdsWords = 160 * 1024 / 4;   // gfx950: 160 KB of LDS per workgroup

// run-time knobs (mp_set_knob)
std::atomic<int32_t> g_mfma_min{64}, g_small_limit{MP_SMALL_LIMIT_AUTO};

// Head limits of the automatic setting.  The head runs every instance of a
// batch at once (one wave each), the bodies in rounds of workgroups; moving
// the Refine iteration whose iterate is ~130 limbs into the head costs its
// latency once and saves it in every body round, so it pays from two rounds
// on.
constexpr int kSmallOneRound = 96, kSmallRounds = 136;
static_assert(kSmallRounds <= mp::kHeadMaxLimit, "automatic head limit out of range");

int device_cus();

// the knobs of a launch whose body workgroups of T threads use `bytes` of LDS,
// for `count` instances (the automatic head limit resolved)
mp::Knobs knobs_for(int T, size_t bytes, int64_t count)
{
    int sl = g_small_limit.load();
    if (sl == MP_SMALL_LIMIT_AUTO) {
        const int cus = device_cus();
        int per_cu = 16 / (T / 64);                 // four waves per SIMD
        const int by_lds = bytes ? (int)(160 * 1024 / bytes) : per_cu;
        per_cu = per_cu < by_lds ? per_cu : by_lds;
        const int64_t slots = (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
        sl = count > slots ? kSmallRounds : kSmallOneRound;
    }
    return mp::Knobs{g_mfma_min.load(), sl};
}

// a head kernel runs first when it has iterations to do and an output row can
// hold a record with at least a few limbs (rows too short get none and the
// body does every step)
int use_head(const mp::Knobs &kn, int row) { return kn.small_limit > 0 && row >= mp::kRecHdr + 8; }

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

}  // namespace

// raise a kernel's dynamic LDS limit to at least `bytes` on the current
// device; the attribute is set only when it grows, so repeated launches (and
// launches under stream capture) make no further runtime call
bool mp::lds_attr(const void *fn, size_t bytes)
{
    struct Entry {
        const void *fn;
        int dev;
        size_t bytes;
    };
    static Entry seen[256];
    static int nseen;
    static std::mutex mu;
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

namespace {

mp_status_t status_of(hipError_t e) { return e == hipSuccess ? MP_OK : MP_ERR_LAUNCH; }

// compute units of the current device (queried once per device)
int device_cus()
{
    static int cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cus[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
        cus[dev] = prop.multiProcessorCount;
    }
    return cus[dev];
}

// The work queue of mp_divrem_ragged_static: a library-owned array of one
// ragged workspace for MP_STATIC_MAX_COUNT instances (1 MiB), one copy per
// GPU, kept until the process ends.  Host code never uses the array's name as
// an address: static_scratch() returns this device's copy's address, fetched
// once per device with that device current.
static __device__ __align__(256) int32_t scratch[kWsHeader + kClasses * MP_STATIC_MAX_COUNT];

int32_t *static_scratch()
{
    static void *ptr[64];
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        ptr[dev] = p;
    }
    return (int32_t *)ptr[dev];
}

// fork streams and events of the concurrent class kernels
struct Forks {
    hipStream_t fs[kClasses];
    hipEvent_t ev_fork, ev_join[kClasses];
};

// The launches of one ragged batch: descriptor check and bucketing, heads,
// then one persistent kernel per width class, each on its own fork stream
// joined back into st (all on st, one after another, when fk is null).  The
// preparation kernel sets every counter of the workspace, so it needs no
// clearing.  Called with g_ragged_mu held.
mp_status_t ragged_launch(const uint32_t *u_pool, int64_t u_limbs, const uint32_t *v_pool, int64_t v_limbs,
                          const mp_desc_t *desc, uint32_t *q_pool, int64_t q_limbs, uint32_t *r_pool,
                          int64_t r_limbs, int32_t *inst_status, int32_t count, int32_t *ws, hipStream_t st,
                          const Forks *fk)
{
    const int cus = device_cus();
    if (cus <= 0) return MP_ERR_DEVICE;
    // (the automatic head limit counts rounds of the narrowest class's workgroups)
    static const size_t narrow_bytes = (size_t)mp::div_lds_words(kClassWidth[0], kClassWidth[0], 256) * 4;
    const mp::Knobs kn = knobs_for(256, narrow_bytes, count);
    hipLaunchKernelGGL(k_ragged_prep, dim3(1), dim3(1024), 0, st, desc, count, u_limbs, v_limbs, q_limbs,
                       r_limbs, inst_status, ws);
    if (hipGetLastError() != hipSuccess) return MP_ERR_LAUNCH;
    const int head = kn.small_limit > 0;
    if (head && mp::launch_head_ragged(st, u_pool, v_pool, desc, q_pool, ws, count, kn) != hipSuccess)
        return MP_ERR_LAUNCH;
    if (fk && hipEventRecord(fk->ev_fork, st) != hipSuccess) return MP_ERR_LAUNCH;
    for (int c = 0; c < kClasses; c++) {
        hipStream_t fs = fk ? fk->fs[c] : st;
        if (fk && hipStreamWaitEvent(fs, fk->ev_fork, 0) != hipSuccess) return MP_ERR_LAUNCH;
        const int T = g_ragged.threads[c];
        // LDS of the class's widest instance (a scan over every divisor length: computed once)
        static size_t lds_bytes[kClasses][3];
        const int ti = T == 256 ? 0 : T == 512 ? 1 : 2;
        if (lds_bytes[c][ti] == 0) lds_bytes[c][ti] = (size_t)mp::div_lds_words(kClassWidth[c], kClassWidth[c], T) * 4;
        const size_t bytes = lds_bytes[c][ti];
        if (bytes > (size_t)kLdsWords * 4) return MP_ERR_SIZE;
        const int fit = (int)(((size_t)kLdsWords * 4) / bytes);
        const int wpc = g_ragged.wgs_per_cu[c] < fit ? g_ragged.wgs_per_cu[c] : fit;
        const int grid = cus * wpc;
        hipError_t e;
        switch (T) {
        case 256:
            e = mp::launch_ragged<256>(grid, bytes, fs, u_pool, v_pool, desc, q_pool, r_pool, inst_status, ws, c,
                                       count, kn, head);
            break;
        case 512:
            e = mp::launch_ragged<512>(grid, bytes, fs, u_pool, v_pool, desc, q_pool, r_pool, inst_status, ws, c,
                                       count, kn, head);
            break;
        default:
            e = mp::launch_ragged<1024>(grid, bytes, fs, u_pool, v_pool, desc, q_pool, r_pool, inst_status, ws, c,
                                        count, kn, head);
            break;
        }
        if (e != hipSuccess) return MP_ERR_LAUNCH;
        if (fk && (hipEventRecord(fk->ev_join[c], fs) != hipSuccess ||
                   hipStreamWaitEvent(st, fk->ev_join[c], 0) != hipSuccess))
            return MP_ERR_LAUNCH;
    }
    return MP_OK;
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
    case MP_ERR_COUNT: return "MP_ERR_COUNT: count exceeds MP_STATIC_MAX_COUNT (the static work queue's size)";
    }
    return "unknown mp_status_t";
}

int32_t mp_max_limbs(void) { return kMaxLimbs; }

mp_status_t mp_set_knob(int32_t knob, int32_t value)
{
    switch (knob) {
    case MP_KNOB_MFMA_MIN:
        if (value < 1) return MP_ERR_ARG;
        g_mfma_min.store(value);
        return MP_OK;
    case MP_KNOB_SMALL_LIMIT:
        if (value != MP_SMALL_LIMIT_AUTO && (value < 0 || value > mp::kHeadMaxLimit)) return MP_ERR_ARG;
        g_small_limit.store(value);
        return MP_OK;
    }
    return MP_ERR_ARG;
}

int32_t mp_get_knob(int32_t knob)
{
    switch (knob) {
    case MP_KNOB_MFMA_MIN: return g_mfma_min.load();
    case MP_KNOB_SMALL_LIMIT: return g_small_limit.load();
    }
    return -1;
}

int64_t mp_lds_bytes(int32_t op, int32_t n1, int32_t n2)
{
    if (n1 <= 0 || n2 <= 0 || n1 > kMaxLimbs || n2 > kMaxLimbs) return -1;
    switch (op) {
    case MP_OP_MUL: return (int64_t)4 * mp::mul_lds_words(n1, n2);
    case MP_OP_DIVREM: return (int64_t)4 * mp::div_lds_words(n1, n2, threads_for(n1));
    case MP_OP_SHINV: {
        const int T = threads_for(n2);
        int words = mp::plan_short_words(n2 + 1, T);
        const int kmax = (n1 < n2 ? n1 : n2) - 1;
        for (int k = 1; k <= kmax; k++) words = mp::hmax(words, mp::plan_div(n2, k).total);
        return (int64_t)4 * words;
    }
    }
    return -1;
}

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
    const mp::Knobs kn = knobs_for(threads_for((na + nb + 1) / 2), bytes, batch);
    switch (threads_for((na + nb + 1) / 2)) {
    case 256: return status_of(mp::launch_mul<256>(batch, bytes, st, a, na, b, nb, c, kn));
    case 512: return status_of(mp::launch_mul<512>(batch, bytes, st, a, na, b, nb, c, kn));
    default: return status_of(mp::launch_mul<1024>(batch, bytes, st, a, na, b, nb, c, kn));
    }
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
    const mp::Knobs kn = knobs_for(T, bytes, batch);
    const int head = use_head(kn, nw);
    if (head && mp::launch_head_shinv(st, v, nv, h, w, nw, batch, kn) != hipSuccess) return MP_ERR_LAUNCH;
    switch (T) {
    case 256: return status_of(mp::launch_shinv<256>(batch, bytes, st, v, nv, h, w, nw, inst_status, kn, head));
    case 512: return status_of(mp::launch_shinv<512>(batch, bytes, st, v, nv, h, w, nw, inst_status, kn, head));
    default: return status_of(mp::launch_shinv<1024>(batch, bytes, st, v, nv, h, w, nw, inst_status, kn, head));
    }
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
    const mp::Knobs kn = knobs_for(T, bytes, batch);
    const int head = use_head(kn, nq);
    if (head && mp::launch_head_divrem(st, u, nu, v, nv, q, nq, batch, kn) != hipSuccess) return MP_ERR_LAUNCH;
    switch (T) {
    case 256:
        return status_of(mp::launch_divrem<256>(batch, bytes, st, u, nu, v, nv, q, nq, r, inst_status, kn, head));
    case 512:
        return status_of(mp::launch_divrem<512>(batch, bytes, st, u, nu, v, nv, q, nq, r, inst_status, kn, head));
    default:
        return status_of(mp::launch_divrem<1024>(batch, bytes, st, u, nu, v, nv, q, nq, r, inst_status, kn, head));
    }
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
    // fork streams and events (default priority), one set per caller stream
    // (up to kForkSets per device, made on first use), so batches launched on
    // different streams run their class kernels side by side; further caller
    // streams share the last set (correct, only serialised)
    constexpr int kForkSets = 8;
    static Forks forks[64][kForkSets];
    static hipStream_t owner[64][kForkSets];
    static int nsets[64];
    hipStream_t st = (hipStream_t)stream;
    int f = 0;
    while (f < nsets[dev] && owner[dev][f] != st) f++;
    if (f == nsets[dev]) {
        // no set for this stream yet: none is made while the stream is being
        // captured into a graph (the kernels then run in order on it)
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess) return MP_ERR_LAUNCH;
        if (cap != hipStreamCaptureStatusNone)
            return ragged_launch(u_pool, u_limbs, v_pool, v_limbs, desc, q_pool, q_limbs, r_pool, r_limbs,
                                 inst_status, count, (int32_t *)workspace, st, nullptr);
        if (f == kForkSets) {
            f = kForkSets - 1;
        } else {
            Forks &fk = forks[dev][f];
            for (int c = 0; c < kClasses; c++) {
                if (hipStreamCreateWithFlags(&fk.fs[c], hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreateWithFlags(&fk.ev_join[c], hipEventDisableTiming) != hipSuccess)
                    return MP_ERR_LAUNCH;
            }
            if (hipEventCreateWithFlags(&fk.ev_fork, hipEventDisableTiming) != hipSuccess) return MP_ERR_LAUNCH;
            owner[dev][f] = st;
            nsets[dev] = f + 1;
        }
    }
    return ragged_launch(u_pool, u_limbs, v_pool, v_limbs, desc, q_pool, q_limbs, r_pool, r_limbs, inst_status,
                         count, (int32_t *)workspace, st, &forks[dev][f]);
}

mp_status_t mp_divrem_ragged_static(const uint32_t *u_pool, int64_t u_limbs, const uint32_t *v_pool,
                                    int64_t v_limbs, const mp_desc_t *desc, uint32_t *q_pool, int64_t q_limbs,
                                    uint32_t *r_pool, int64_t r_limbs, int32_t *inst_status, int32_t count,
                                    void *stream)
{
    if (!u_pool || !v_pool || !desc || !q_pool || !r_pool || !inst_status || count < 0) return MP_ERR_ARG;
    if (u_limbs < 0 || v_limbs < 0 || q_limbs < 0 || r_limbs < 0) return MP_ERR_ARG;
    if (count > MP_STATIC_MAX_COUNT) return MP_ERR_COUNT;
    if (count == 0) return MP_OK;
    if (!device_ok()) return MP_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_ragged_mu);
    int32_t *ws = static_scratch();
    if (!ws) return MP_ERR_DEVICE;
    return ragged_launch(u_pool, u_limbs, v_pool, v_limbs, desc, q_pool, q_limbs, r_pool, r_limbs, inst_status,
                         count, ws, (hipStream_t)stream, nullptr);
}

}  // extern "C"
