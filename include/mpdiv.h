/*
 * mpdiv.h -- batched exact multi-precision integer division on MI355X (gfx950).
 *
 * The library computes, for many independent instances at once, the
 * operations of the shifted-inverse division method of Marchioro, Raahauge,
 * Lovenskjold, Oancea and Watt, "On GPU Implementation for Multi-Precision
 * Integer Division" (Watt's whole-shifted-inverse Newton iteration):
 *
 *   mp_mul_batch     c = a * b                     (the method's Mult; Alg. 2, 3)
 *   mp_shinv_batch   w = shinv_h(v) = floor(B^h/v) (Definition 1; Alg. 1)
 *   mp_divrem_batch  (q, r): u = q*v + r, 0<=r<v   (Alg. 3 with Thm. 2's correction)
 *
 * Representation: base B = 2^32.  A number is a little-endian array of
 * uint32_t limbs; limb i has weight B^i.  Leading zero limbs are allowed in
 * every input (each instance's effective precision is found on the device).
 * A batch of L-limb operands is dense and row-major: instance j starts at
 * p + (size_t)j * L.
 *
 * Memory: every data pointer is a DEVICE pointer (for example a torch tensor's
 * data_ptr()).  The library never allocates, frees or keeps caller memory.
 * Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL is
 * the default stream); the caller synchronises before reading results.  Calls
 * on one stream are ordered; outputs must not overlap inputs.
 *
 * Errors: argument errors are detected on the host and returned before
 * anything is launched; a failed launch returns MP_ERR_LAUNCH.  Per-instance
 * outcomes are written to inst_status[j] (may be NULL):
 *   MP_INST_OK        result written;
 *   MP_INST_DIVZERO   v = 0: every output limb of the instance is 0;
 *   MP_INST_QWIDTH    the quotient (or shifted inverse) needs more limbs than
 *                     the output width: every output limb of the instance is 0;
 *   MP_INST_INTERNAL  an internal bound of the method was exceeded (not
 *                     expected for any input): outputs are 0.
 */
#ifndef MPDIV_H
#define MPDIV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MP_OK = 0,          /* launched (or nothing to do: batch == 0) */
    MP_ERR_ARG = 1,     /* null pointer, non-positive width, negative batch */
    MP_ERR_SIZE = 2,    /* an operand width exceeds mp_max_limbs() */
    MP_ERR_LAUNCH = 3,  /* the HIP launch failed */
    MP_ERR_DEVICE = 4,  /* no usable gfx950 device */
    MP_ERR_COUNT = 5    /* mp_divrem_ragged_static: count > MP_STATIC_MAX_COUNT */
} mp_status_t;

enum { MP_INST_OK = 0, MP_INST_DIVZERO = 1, MP_INST_QWIDTH = 2, MP_INST_INTERNAL = 3, MP_INST_BADDESC = 4 };

/*
 * c = a * b for each instance: the classical (schoolbook) product, the
 * multiplication the method is parameterised by (Sec. 3.3).
 *   a: batch x na limbs, b: batch x nb limbs, c: batch x (na + nb) limbs.
 *   1 <= na, nb <= mp_max_limbs().
 */
mp_status_t mp_mul_batch(const uint32_t *a, int32_t na, const uint32_t *b, int32_t nb,
                         uint32_t *c, int32_t batch, void *stream);

/*
 * w = floor(B^h / v) for each instance, exactly (Definition 1, computed by
 * Alg. 1 and corrected to the exact value).
 *   v: batch x nv limbs (1 <= nv <= mp_max_limbs()), h: 0 <= h <= mp_max_limbs(),
 *   w: batch x nw limbs, zero-padded; nw >= h - prec(v) + 2 always suffices
 *   (h + 1 for any v).
 *   inst_status: batch int32 or NULL.
 */
mp_status_t mp_shinv_batch(const uint32_t *v, int32_t nv, int32_t h, uint32_t *w, int32_t nw,
                           int32_t *inst_status, int32_t batch, void *stream);

/*
 * Quotient and remainder of u by v for each instance (Alg. 3: the quotient
 * q0 from the top limbs of u times the shifted inverse of v, then
 * corrections.  Theorem 2's range for q0, widened by the clipped products,
 * is q - 4 <= q0 <= q + 3, so the remainder u - v q0 reaches [0, v) after at
 * most three additions or four subtractions of v; one more of each is
 * allowed, and an instance needing more reports MP_INST_INTERNAL instead of
 * a wrong result).
 *   u: batch x nu limbs, v: batch x nv limbs, 1 <= nu, nv <= mp_max_limbs();
 *   q: batch x nq limbs, zero-padded; nq >= nu - prec(v) + 1 suffices (nu always);
 *   r: batch x nv limbs, zero-padded;
 *   inst_status: batch int32 or NULL.
 * u = 0 gives (0, 0); u < v gives (0, u).
 */
mp_status_t mp_divrem_batch(const uint32_t *u, int32_t nu, const uint32_t *v, int32_t nv,
                            uint32_t *q, int32_t nq, uint32_t *r, int32_t *inst_status,
                            int32_t batch, void *stream);

/*
 * One division of a ragged (mixed-precision) batch: widths in limbs and limb
 * offsets into packed pools.  u = u_pool[u_off .. u_off+nu), v = v_pool[v_off ..
 * v_off+nv), q = q_pool[q_off .. q_off+nq), r = r_pool[r_off .. r_off+nv).
 */
typedef struct {
    int64_t u_off, v_off, q_off, r_off;
    int32_t nu, nv, nq, reserved;
} mp_desc_t;

/*
 * Quotients and remainders of a batch of divisions of uneven precisions in one
 * launch sequence (Alg. 3 per instance, as mp_divrem_batch).  On the device,
 * instances are bucketed by dividend width into the classes <= 1024, <= 2048,
 * <= 4096 and <= 8192 limbs; each class runs one persistent kernel whose
 * workgroups take instances from a per-class work queue, the class kernels
 * running concurrently.  Nothing is synchronised with the host, so the
 * sequence can be captured into a hipGraph and replayed.
 *   desc:      count descriptors (device memory);
 *   *_limbs:   sizes of the four pools; a descriptor whose ranges leave its
 *              pool or whose widths are outside [1, mp_max_limbs()] gets
 *              MP_INST_BADDESC and its outputs are not written;
 *   workspace: device memory of mp_ragged_workspace_bytes(count) bytes, owned
 *              by the caller, not shared by concurrent calls;
 *   inst_status: count int32 (required).
 * Widths and offsets are checked on the device; null pointers and count < 0 on
 * the host.  The class kernels run on library-owned fork streams joined back
 * into `stream`; each caller stream (up to eight per device) gets its own set,
 * so batches launched on different streams overlap on the device.  A stream
 * first seen while it is being captured into a graph gets no set: the class
 * kernels then run one after another on it (call once outside capture first
 * to capture the concurrent form).
 */
mp_status_t mp_divrem_ragged(const uint32_t *u_pool, int64_t u_limbs, const uint32_t *v_pool, int64_t v_limbs,
                             const mp_desc_t *desc, uint32_t *q_pool, int64_t q_limbs, uint32_t *r_pool,
                             int64_t r_limbs, int32_t *inst_status, int32_t count, void *workspace,
                             void *stream);

/* bytes of workspace mp_divrem_ragged needs for count instances */
int64_t mp_ragged_workspace_bytes(int32_t count);

/*
 * mp_divrem_ragged without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and per-instance status as mp_divrem_ragged.  The
 * work queue lives in a static array of the library, one per GPU (1 MiB,
 * held until the process ends), so count must not exceed
 * MP_STATIC_MAX_COUNT (else MP_ERR_COUNT, nothing launched).  The call
 * allocates nothing and creates no stream or event: all its kernels run on
 * `stream`, one after another.  Every call on a GPU shares that GPU's array:
 * calls that may overlap on one GPU (different streams, concurrent graph
 * replays) race and must be serialised by the caller.
 */
#define MP_STATIC_MAX_COUNT 65536
mp_status_t mp_divrem_ragged_static(const uint32_t *u_pool, int64_t u_limbs, const uint32_t *v_pool,
                                    int64_t v_limbs, const mp_desc_t *desc, uint32_t *q_pool, int64_t q_limbs,
                                    uint32_t *r_pool, int64_t r_limbs, int32_t *inst_status, int32_t count,
                                    void *stream);

/*
 * Launch configuration of width class cls (0..3) for mp_divrem_ragged:
 * threads per workgroup (256, 512 or 1024, at least width/8) and persistent
 * workgroups per compute unit (1..8).  Returns MP_ERR_ARG for an invalid
 * choice.  The defaults come from the library's tuned table.
 */
mp_status_t mp_ragged_config(int32_t cls, int32_t threads, int32_t wgs_per_cu);

/*
 * Run-time tuning knobs of the division kernels (process-wide; a change
 * applies to launches made after it).  Every setting gives the same results
 * bit for bit; only the speed differs.
 *   MP_KNOB_MFMA_MIN     products whose shorter operand has at least this many
 *                        limbs (>= 1) run on the int8 matrix cores as exact
 *                        balanced radix-256 digit products; shorter ones on the
 *                        vector ALU (32x32->64-bit multiply-adds).  Default 64.
 *   MP_KNOB_SMALL_LIMIT  Alg. 1's initial approximation and the Refine
 *                        iterations whose iterate has fewer than this many
 *                        limbs (0..140) run in a separate head launch, one wave
 *                        per instance, before the per-instance workgroups do
 *                        the rest; the head leaves its state in the first
 *                        limbs of the instance's q (mp_shinv_batch: w) row,
 *                        which the final result then overwrites.  0 (or an
 *                        output row shorter than 16 limbs) runs every step in
 *                        the per-instance workgroups.  MP_SMALL_LIMIT_AUTO
 *                        (the default) chooses per launch: 136 when the batch
 *                        needs more than one round of per-instance workgroups
 *                        on the device (the head runs all instances at once,
 *                        so its longer iterations are paid once and saved in
 *                        every round), 96 otherwise.
 * mp_set_knob returns MP_ERR_ARG for an unknown knob or a value out of range;
 * mp_get_knob returns the current value (-1 for an unknown knob).
 */
enum { MP_KNOB_MFMA_MIN = 0, MP_KNOB_SMALL_LIMIT = 1 };
/* MP_KNOB_SMALL_LIMIT value: chosen per launch (see above) */
#define MP_SMALL_LIMIT_AUTO (-2)
mp_status_t mp_set_knob(int32_t knob, int32_t value);
int32_t mp_get_knob(int32_t knob);

/*
 * Dynamic LDS bytes per workgroup that a launch needs (host-side query, no
 * device call): MP_OP_MUL with (na, nb), MP_OP_DIVREM with (nu, nv),
 * MP_OP_SHINV with (nv, h).  Returns -1 for an unknown op or a width outside
 * [1, mp_max_limbs()].  A launch whose figure exceeds the 160 KB of one
 * gfx950 workgroup returns MP_ERR_SIZE.
 */
enum { MP_OP_MUL = 0, MP_OP_DIVREM = 1, MP_OP_SHINV = 2 };
int64_t mp_lds_bytes(int32_t op, int32_t n1, int32_t n2);

/* human-readable name of a status code (static storage) */
const char *mp_status_str(mp_status_t s);

/* largest operand width in limbs any entry point accepts (8192 = 2^18 bits) */
int32_t mp_max_limbs(void);

#ifdef __cplusplus
}
#endif

#endif /* MPDIV_H */
