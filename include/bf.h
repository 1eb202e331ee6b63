/*
 * bf.h -- batched beamforming R = W x S on AMD Instinct MI355X (gfx950).
 *
 * The operation (Section III of the paper, beamforming paragraph and its
 * equation): many products R = W x S, where W is a precoding matrix that
 * stays constant while S changes.  W has one row per antenna (64, the
 * 4 x 8 x 2 transceiver array of Section II) and f columns, one per
 * parallel flow; S has f rows and b = 60 columns, one per resource
 * element; f is fixed within a product and ranges from 0 to 36.  Entries
 * are complex.  For f = 0 the product is the empty sum: R is all zeros.
 *
 * Data layout (all pointers are plain host or device addresses):
 *   complex numbers are complex64: two floats (re, im), interleaved;
 *   W pool  host, complex64 [n_w][64][f_max], row-major; item t uses the
 *           leading f_t columns of entry w_t (row stride f_max);
 *   S_t     device, complex64 [f_t][60], row-major, 8-byte aligned
 *           (16-byte alignment takes the faster load path);
 *   R_t     device, complex64 [64][60], row-major, 8-byte aligned; fully
 *           overwritten (zeros when f_t = 0).
 *
 * Streams: every `hip_stream` argument is a hipStream_t passed as void*
 * (NULL = the default stream).  Device work is asynchronous and ordered on
 * that stream; host arrays passed in are copied before the call returns.
 *
 * Errors: calls return a bf_status.  Arguments are checked before any
 * device work is enqueued, all-or-nothing: if any item is invalid nothing
 * is launched and BF_ERR_INVALID is returned.  A failing HIP call gives
 * BF_ERR_DEVICE.  bf_last_error() returns a thread-local description of
 * the most recent failure on the calling thread.  No C++ exception
 * crosses this interface.  S and R of one call must not overlap
 * (undefined, not checked).
 */
#ifndef BF_H
#define BF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BF_M 64    /* antennas: rows of W and R (Section II, III) */
#define BF_B 60    /* resource elements: columns of S and R (Section III) */
#define BF_FMAX 36 /* largest number of flows (Section III) */

typedef enum {
    BF_OK = 0,
    BF_ERR_INVALID = -1,     /* bad argument; nothing was launched */
    BF_ERR_OOM = -2,         /* device or pinned host allocation failed */
    BF_ERR_DEVICE = -3,      /* a HIP runtime call failed */
    BF_ERR_BUSY = -4,        /* serving: submission queue full */
    BF_ERR_TIMEOUT = -5,     /* serving: poll or drain timed out */
    BF_ERR_UNSUPPORTED = -6  /* precision form not prepared by the plan */
} bf_status;

/* Arithmetic forms of the contraction.  All read complex64 S and write
 * complex64 R with FP32 accumulation.
 *   BF_FP32    FP32 operands on the FP32 matrix cores.
 *   BF_FP16,   operands rounded to FP16 / BF16 (S scaled per product by a
 *   BF_BF16    power of two first; exact and undone on output).
 *   BF_FP16X2, 2-term split: x = hi + lo, products hi*hi + hi*lo + lo*hi
 *   BF_BF16X2  accumulated in FP32, recovering close to FP32 accuracy. */
typedef enum { BF_FP32 = 0, BF_FP16 = 1, BF_BF16 = 2, BF_FP16X2 = 3, BF_BF16X2 = 4 } bf_prec;
#define BF_PREC_BIT(p) (1u << (unsigned)(p))
#define BF_PREC_ALL 0x1Fu

typedef struct bf_plan_s *bf_plan;
typedef struct bf_graph_s *bf_graph;

/* ---- plan: the resident W pool --------------------------------------
 * W is constant across many products (Section III), so its preparation
 * happens once here and is not part of bf_apply: the pool is copied to
 * the current device and rearranged into the operand layout of each
 * precision form in prec_mask (BF_PREC_BIT(...) bits; 0 means FP32 only).
 *   out       receives the plan handle
 *   w_pool    host complex64 [n_w][64][f_max]; may be freed on return
 *   n_w       number of pool entries, >= 1
 *   f_max     columns per entry, 0..36
 *   hip_stream stream for the upload; the call synchronises it before
 *             returning, so the plan is ready on any stream.
 * Errors: BF_ERR_INVALID (null pointers, n_w < 1, f_max outside 0..36,
 * unknown mask bits), BF_ERR_OOM, BF_ERR_DEVICE. */
bf_status bf_plan_create(bf_plan *out, const void *w_pool, int32_t n_w, int32_t f_max,
                         uint32_t prec_mask, void *hip_stream);

/* Releases the plan after waiting for every launch that uses it. */
bf_status bf_plan_destroy(bf_plan plan);

/* Plan facts: number of entries, f_max, prepared precision mask. */
bf_status bf_plan_info(bf_plan plan, int32_t *n_w, int32_t *f_max, uint32_t *prec_mask);

/* ---- apply: one batch of products ------------------------------------
 * For t in [0, batch): R[t] = W_pool[w_ids[t]][:, :f[t]] x S[t].
 *   w_ids, f  host int32 [batch]
 *   S, R      host arrays [batch] of device pointers (S[t] may be NULL
 *             when f[t] == 0)
 *   prec      precision form; must be prepared by the plan
 * The descriptors are copied to the device on hip_stream and one kernel
 * launch processes the whole batch; the call returns without waiting.
 * S must stay unmodified and R untouched until that stream work is done.
 * batch == 0 is a no-op.  Errors: BF_ERR_INVALID (names the first bad
 * item), BF_ERR_UNSUPPORTED, BF_ERR_OOM, BF_ERR_DEVICE. */
bf_status bf_apply(bf_plan plan, int32_t batch, const int32_t *w_ids, const int32_t *f,
                   const void *const *S, void *const *R, bf_prec prec, void *hip_stream);

/* Same products for the common case of one S buffer and one R buffer:
 * S[t] = S_base + s_off[t] complex elements (host int64 [batch]),
 * R[t] = R_base + t * 64 * 60 complex elements. */
bf_status bf_apply_packed(bf_plan plan, int32_t batch, const int32_t *w_ids, const int32_t *f,
                          const void *S_base, const int64_t *s_off, void *R_base,
                          bf_prec prec, void *hip_stream);

/* Host-only argument check used by bf_apply (no device access):
 * returns BF_OK or BF_ERR_INVALID with bf_last_error() naming the first
 * offending item.  n_w and f_max describe the pool. */
bf_status bf_check_batch(int32_t n_w, int32_t f_max, int32_t batch, const int32_t *w_ids,
                         const int32_t *f, const void *const *S, void *const *R);

/* ---- graph: a fixed batch replayed many times ------------------------
 * A 5G slot loop often repeats the same set of products over the same
 * (double-buffered) S and R buffers.  bf_graph_create validates the batch
 * once, uploads its descriptors (ordered longest-first for balance) to
 * device memory owned by the graph, and captures the persistent kernel
 * into a hipGraph; bf_graph_launch replays it on any stream with no host
 * work besides the launch.  Arguments as for bf_apply. */
bf_status bf_graph_create(bf_graph *out, bf_plan plan, int32_t batch, const int32_t *w_ids,
                          const int32_t *f, const void *const *S, void *const *R,
                          bf_prec prec, void *hip_stream);
bf_status bf_graph_launch(bf_graph graph, void *hip_stream);
bf_status bf_graph_destroy(bf_graph graph);

/* ---- kernel variants and tuning --------------------------------------
 * A variant fixes how the batch is spread over the chip: work
 * distribution (one product per workgroup, or persistent workgroups that
 * claim products from an atomic counter), workgroups per CU and product
 * order.  bf_autotune times every candidate on the given batch and stores
 * the fastest for (prec, f bucket) in the plan; bf_apply uses it from
 * then on.  The table can be saved to and loaded from a text file. */
typedef struct {
    int32_t schedule;      /* 0: one product per workgroup; 1: persistent, atomic claim;
                              2: persistent, static share per XCD, next S prefetched */
    int32_t wg_per_cu;     /* persistent grid = wg_per_cu * CU count (ignored for 0) */
    int32_t order;         /* 0: as given; 1: longest f first, then by W id */
    int32_t reserved;
} bf_variant;

bf_status bf_set_variant(bf_plan plan, bf_prec prec, int32_t f_bucket, const bf_variant *v);
bf_status bf_get_variant(bf_plan plan, bf_prec prec, int32_t f_bucket, bf_variant *v);
/* f_bucket of a batch: its largest f divided by 9, i.e. 0..4. */
int32_t bf_f_bucket(int32_t f);
bf_status bf_autotune(bf_plan plan, int32_t batch, const int32_t *w_ids, const int32_t *f,
                      const void *const *S, void *const *R, bf_prec prec, int32_t reps,
                      void *hip_stream, bf_variant *best, float *best_us);
bf_status bf_tune_save(bf_plan plan, const char *path);
bf_status bf_tune_load(bf_plan plan, const char *path);

/* ---- diagnostics ------------------------------------------------------ */
const char *bf_status_str(bf_status s);
const char *bf_last_error(void);
/* Fills up to 64 bytes with the library's build tag (gfx target, flags). */
const char *bf_build_info(void);
/* Number of compute units of the current device, or a bf_status. */
int32_t bf_device_cu_count(void);

#ifdef __cplusplus
}
#endif

#endif /* BF_H */
