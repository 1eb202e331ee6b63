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
 *   R_t     device, complex64 [64][60], row-major, 16-byte aligned (R is
 *           written with 16-byte stores); fully overwritten (zeros when
 *           f_t = 0).
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
 *   BF_FP32    FP32 operands on the FP32 matrix cores, four real products
 *              per complex product.
 *   BF_FP32_3M FP32 operands, three real products per complex product
 *              (Gauss): Re = Wr Sr - Wi Si, Im = (Wr + Wi)(Sr + Si) - Wr Sr
 *              - Wi Si, with Wr + Wi formed by one FP32 add.  A quarter
 *              fewer matrix-core steps; rounding differs from BF_FP32 (for
 *              example an identity W no longer returns S bit for bit) but
 *              stays within the FP32 error bar.
 *   BF_FP16,   operands rounded to FP16 / BF16 (S scaled per product by a
 *   BF_BF16    power of two first; exact and undone on output).
 *   BF_FP16X2, 2-term split: x = hi + lo, products hi*hi + hi*lo + lo*hi
 *   BF_BF16X2  accumulated in FP32, recovering close to FP32 accuracy. */
typedef enum {
    BF_FP32 = 0, BF_FP16 = 1, BF_BF16 = 2, BF_FP16X2 = 3, BF_BF16X2 = 4, BF_FP32_3M = 5
} bf_prec;
#define BF_PREC_BIT(p) (1u << (unsigned)(p))
#define BF_PREC_ALL 0x3Fu

typedef struct bf_plan_s *bf_plan;
typedef struct bf_graph_s *bf_graph;
typedef struct bf_server_s *bf_server;
typedef struct bf_filter_s *bf_filter;

/* ---- plan: the resident W pool --------------------------------------
 * W is constant across many products (Section III), so its preparation
 * happens once here and is not part of bf_apply: the pool is copied to
 * the current device and rearranged into the operand layout of each
 * precision form in prec_mask (BF_PREC_BIT(...) bits; 0 means FP32 only).
 * Each layout has two slots per entry (see bf_plan_update); per slot and
 * entry at f_max = 36 the FP32 form takes 36,864 bytes and the
 * three-product layout 36,864 (built for BF_FP32 as well, whose 16 x 16
 * kernels read it), the 16-bit forms 20,480 (plain) plus 10,240 per part
 * of the compact layout.
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

/* Replaces pool entry w_id.  Section III has W constant while S changes;
 * in a running base station it stays constant only until the precoder is
 * recomputed, and this swaps one entry without re-planning.
 *   w          host complex64 [64][f_max], row-major; may be freed on return
 *   hip_stream the caller's stream, which is made to wait for the update
 * Every entry has two device slots in each prepared layout.  The new W is
 * written into the slot not in use, on a stream of the plan's own, and
 * becomes current when the call returns.  Then:
 *   - bf_apply / bf_apply_packed calls and server launches issued after
 *     this call read the new W; they wait on the device (on whatever
 *     stream they run) for the update to finish.
 *   - launches issued before it read the old W and are neither waited for
 *     nor disturbed.
 *   - the next update of the same entry rewrites the old slot only after
 *     every launch issued before this call has finished (device-side wait
 *     on the plan's stream; the host does not block).
 * Graphs keep the slots current at bf_graph_create: re-create a graph after
 * updating an entry it uses, and do not keep launching a graph created
 * before an update once the same entry is updated again.
 * Updates of one plan run one after another; the call blocks only while a
 * previous update's W is still being uploaded.
 * Errors: BF_ERR_INVALID (null plan or w, w_id outside [0, n_w)), BF_ERR_OOM,
 * BF_ERR_DEVICE.  With f_max = 0 there is nothing to replace and the call
 * only checks its arguments. */
bf_status bf_plan_update(bf_plan plan, int32_t w_id, const void *w, void *hip_stream);

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

/* bf_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, checks, products and results as bf_apply, for at most
 * BF_NOALLOC_MAX_ITEMS products (more: BF_ERR_INVALID, nothing launched).
 * The call allocates nothing: the descriptor block of the launch (the
 * counters of the persistent kernels, which start at zero each call, the
 * sink and the items) is written into a fixed array of the library
 * (about 520 KB, held on each device it is used on until the process
 * ends), uploaded on hip_stream from pinned host memory the plan reserved
 * when it was created.  Every call on one device shares that array and it
 * keeps the last call's contents: calls on different streams whose device
 * work overlaps race on it (calls on one stream are ordered).  The
 * current device must be the plan's (else BF_ERR_INVALID).  The tuning
 * table's product orders (order 1 and 2) are not applied; every product's
 * result is the same as in any order. */
#define BF_NOALLOC_MAX_ITEMS 16384
bf_status bf_apply_noalloc(bf_plan plan, int32_t batch, const int32_t *w_ids, const int32_t *f,
                           const void *const *S, void *const *R, bf_prec prec, void *hip_stream);

/* Same products for the common case of one S buffer and one R buffer:
 * S[t] = S_base + s_off[t] complex elements (host int64 [batch]),
 * R[t] = R_base + t * 64 * 60 complex elements (R_base 16-byte aligned). */
bf_status bf_apply_packed(bf_plan plan, int32_t batch, const int32_t *w_ids, const int32_t *f,
                          const void *S_base, const int64_t *s_off, void *R_base,
                          bf_prec prec, void *hip_stream);

/* Host-only argument check used by bf_apply (no device access):
 * returns BF_OK or BF_ERR_INVALID with bf_last_error() naming the first
 * offending item.  n_w and f_max describe the pool. */
bf_status bf_check_batch(int32_t n_w, int32_t f_max, int32_t batch, const int32_t *w_ids,
                         const int32_t *f, const void *const *S, void *const *R);

/* ---- environment ------------------------------------------------------
 * Read by bf_plan_create for the plan it makes:
 *   BF_FORCE_VARIANT=s:w:o:t  every launch of the plan (bf_apply*, graphs,
 *       the serving loop) uses bf_variant {s, w, o, t} instead of its tuning
 *       table, except bf_autotune's own trials; an out-of-range value is
 *       reported on stderr and ignored.
 *   BF_AUTOTUNE_CACHE=path    the plan loads this tuning database (as
 *       bf_tune_load) when the file exists, and bf_autotune saves the plan's
 *       table to it (as bf_tune_save) after each tuning.
 *   BF_LOG=1                  one stderr line ("[bf] ...") per plan, per
 *       tuning result, and per launch configuration (form, variant, schedule,
 *       grid) the first time the plan launches it.
 * The library also marks its host-side phases (plan creation, apply calls,
 * serving launches, tuning, graph creation, pool updates) as roctx ranges,
 * which rocprofv3 --marker-trace records. */

/* ---- kernel timing ----------------------------------------------------
 * With start and stop set (hipEvent_t, created by the caller with timing
 * enabled), the apply kernel that each later bf_apply, bf_apply_packed,
 * bf_apply_noalloc or bf_graph_launch call on this plan launches records
 * start when it begins executing and stop when it ends
 * (hipExtLaunchKernel), so that hipEventElapsedTime(start, stop) gives the
 * duration of that kernel alone: neither the descriptor upload nor the gap
 * the queue leaves between two launches.  Each launch overwrites the pair;
 * set a new pair before each call to time a sequence.  NULL, NULL switches
 * it off (the default).  Errors: BF_ERR_INVALID for a null plan or for
 * only one of the two events. */
bf_status bf_plan_set_kernel_events(bf_plan plan, void *start, void *stop);

/* ---- graph: a fixed batch replayed many times ------------------------
 * A 5G slot loop often repeats the same set of products over the same
 * (double-buffered) S and R buffers.  bf_graph_create validates the batch
 * once, uploads its descriptors (in the order the plan's variant for this
 * batch asks for) to device memory owned by the graph and fixes the launch
 * configuration; bf_graph_launch replays it on any stream as one kernel
 * launch, with no upload and no event (it may itself be captured into the
 * caller's hipGraph).  Replays of one graph must not
 * overlap (one stream, or ordered by the caller): the persistent claim
 * schedule re-arms its counter at the end of each replay.  Arguments as
 * for bf_apply. */
bf_status bf_graph_create(bf_graph *out, bf_plan plan, int32_t batch, const int32_t *w_ids,
                          const int32_t *f, const void *const *S, void *const *R,
                          bf_prec prec, void *hip_stream);
bf_status bf_graph_launch(bf_graph graph, void *hip_stream);
bf_status bf_graph_destroy(bf_graph graph);

/* ---- kernel variants and tuning --------------------------------------
 * A variant fixes how the batch is spread over the chip and how R leaves
 * it: work distribution (one product per workgroup, persistent workgroups
 * claiming products from an atomic counter, or persistent workgroups with
 * a static share that prefetch the next S), workgroups per CU, product
 * order, and the R store path.  bf_autotune times every candidate on the
 * given batch (the mean duration of reps launches of its kernel, from the
 * start and end events the kernel records itself: host packing, upload and
 * the queue's gaps are not timed) and stores the fastest for (prec, f
 * bucket) in the plan, with that duration in microseconds (*best_us);
 * bf_apply uses it from then on.  The trials launch the same batch again
 * and again: where its S is small enough for the device's memory-side
 * cache (256 MB on MI355X) to keep between launches, they time S read from
 * that cache, which can favour other variants than S read from HBM does
 * (tune on a batch whose S exceeds it, or on several, for streaming use).
 * The table can be saved to and loaded from a text file. */
typedef struct {
    int32_t schedule;      /* 0: one product per workgroup; 1: persistent, atomic claim;
                              2: persistent, static share per XCD, next S prefetched;
                              3: persistent, wave-specialised (matrix-core waves and
                              data-movement waves); needs every S 16-byte aligned
                              (other batches run schedule 0 for the three-product
                              form, 2 otherwise); for the 16-bit forms also one f
                              for every product of the batch (batches of mixed f
                              run schedule 2, and bf_autotune does not try 3 on
                              them); there the matrix-core waves also stage W */
    int32_t wg_per_cu;     /* persistent grid = wg_per_cu * CU count (ignored for 0) */
    int32_t order;         /* 0: as given; 1: longest f first, then by W id;
                              2: grouped by W id modulo 8 (each of the 8 XCDs
                              then works on an eighth of the pool), caller order
                              within a group; 3: grouped by W id modulo 8 and
                              by W id within a group, and on schedule 3 dealt
                              to the workgroups in contiguous blocks, so that
                              a workgroup's consecutive products mostly share
                              their W (the kernels that copy W themselves,
                              store 8 and 9, then copy it once per run);
                              4: grouped by W id modulo 8 and on schedule 3
                              dealt so that the workgroups' summed f match
                              (longest first, alternating directions, each
                              workgroup starting its list at a different
                              point), else as 2; bf_apply_noalloc keeps the
                              caller's order */
    int32_t store;         /* schedules 0 and 2: 0 = lanes write their accumulators
                              directly, 1 = each wave stages its 16 rows of R in LDS
                              and writes them as contiguous 16-byte stores;
                              schedule 3 (always staged): producer waves per
                              workgroup and products prefetched in their
                              registers, 0 = (4, 1), 1 = (8, 1), 2 = (8, 2),
                              3 = (8, 3), 4 = (12, 1), 5 = (12, 2); the
                              three-product form uses at most 8 producers; the
                              FP32 forms with 6 = (8, 1) or 7 = (8, 2) run 8
                              matrix-core waves on 16 x 16 tiles instead of 4
                              on 32 x 32, and with 8 = (8, 2) the same with the
                              matrix-core waves copying W into LDS by direct
                              global-to-LDS loads, the producers moving S and
                              R only, 9 = 8 with the producers also copying S
                              that way into three LDS buffers (6 to 9 read as
                              0 for the 16-bit forms); the
                              16-bit forms prefetch at least 2 products, and 3
                              only with 8 producers */
} bf_variant;

bf_status bf_set_variant(bf_plan plan, bf_prec prec, int32_t f_bucket, const bf_variant *v);
bf_status bf_get_variant(bf_plan plan, bf_prec prec, int32_t f_bucket, bf_variant *v);
/* Bucket of f: f / 9, i.e. 0..4.  A batch uses the bucket of its mean f
 * (rounded to nearest). */
int32_t bf_f_bucket(int32_t f);
bf_status bf_autotune(bf_plan plan, int32_t batch, const int32_t *w_ids, const int32_t *f,
                      const void *const *S, void *const *R, bf_prec prec, int32_t reps,
                      void *hip_stream, bf_variant *best, float *best_us);
/* The tuning table as a database in the manner of the optimizer tool of
 * Section IV, which picks the most efficient version of a building block for
 * a given matrix size and target architecture.  Key: (architecture, CU
 * count, precision form, f bucket); value: the variant and its measured
 * kernel time in microseconds (0 for untuned defaults).  Text lines
 *   arch cus prec bucket schedule wg_per_cu order store us
 * e.g. "gfx950 256 5 4 3 0 0 1 177.20"; '#' starts a comment.
 * bf_tune_save writes this device's entries, keeping the file's entries of
 * other architectures or CU counts.  bf_tune_load applies the entries of
 * this device's architecture and CU count (lines of the older form
 * "prec bucket schedule wg_per_cu order store" apply to any device) and
 * ignores the rest.  Errors: BF_ERR_INVALID (null arguments, unreadable or
 * malformed file: nothing is applied). */
bf_status bf_tune_save(bf_plan plan, const char *path);
bf_status bf_tune_load(bf_plan plan, const char *path);
/* The variant the plan uses for batches of precision form prec and mean f
 * (0..36), and its recorded time (0: default, not measured). */
bf_status bf_tune_query(bf_plan plan, bf_prec prec, int32_t f, bf_variant *v, float *tuned_us);

/* ---- serving: continuous batching of arriving requests ----------------
 * The pipeline of Section II runs its stages continuously on arriving
 * signal; this is the request loop for the beamforming stage.  A request
 * is (W id, f, n_s S blocks contiguous at S, n_s R blocks contiguous at
 * R); the W pool stays resident in the plan.  bf_submit enqueues it and
 * returns a ticket at once.  A batcher thread admits queued requests in
 * arrival order while the S + R bytes of admitted, unfinished requests
 * stay within hbm_budget_bytes, and packs the admitted requests into one
 * launch whenever one of n_streams device streams is free; a launch is
 * closed early when the running throughput estimate says a larger one
 * would finish after its oldest member's deadline.  A completion thread
 * reports each finished request through bf_poll and returns its bytes to
 * the budget.  Requests that arrive while earlier launches run join the
 * next launch, so device work of consecutive launches overlaps across
 * the streams.  Results are the same as for bf_apply on each request
 * alone: every product is computed independently, with the same kernels. */
typedef struct {
    uint64_t hbm_budget_bytes;  /* bound on S+R bytes of admitted, unfinished requests */
    int64_t deadline_us;        /* per-request deadline after t_arrival (<= 0: none) */
    int32_t n_streams;          /* device streams used round-robin, 1..8 */
    int32_t max_batch_items;    /* upper bound on S blocks per launch */
    int32_t queue_capacity;     /* submission queue slots (power of two) */
    int32_t prec;               /* bf_prec used for every launch */
} bf_server_cfg;

typedef struct {
    int32_t w_id;
    int32_t f;
    int32_t n_s;            /* number of S blocks, >= 1 */
    int32_t reserved;
    const void *S;          /* device, n_s contiguous f x 60 complex64 blocks */
    void *R;                /* device, n_s contiguous 64 x 60 complex64 blocks,
                               16-byte aligned */
    uint64_t tag;           /* opaque, returned in the completion */
    int64_t t_arrival_ns;   /* CLOCK_MONOTONIC arrival time (0: taken at submit) */
} bf_request;

typedef struct {
    uint64_t ticket;
    uint64_t tag;
    int32_t status;          /* BF_OK or a bf_status */
    int32_t deadline_missed; /* 1 if t_done > t_arrival + deadline */
    int64_t t_arrival_ns;
    int64_t t_submit_ns;     /* when bf_submit accepted it */
    int64_t t_launch_ns;     /* when its launch was enqueued */
    int64_t t_done_ns;       /* when its completion was observed */
} bf_completion;

typedef struct {
    uint64_t submitted, admitted, completed, refused, launches, deadline_misses;
    uint64_t inflight_bytes, peak_inflight_bytes, queued;
    uint64_t launch_host_ns;  /* host time the batcher spent packing and
                                 enqueueing launches, summed over them */
} bf_server_stats;

/* cfg may be NULL for defaults: 16 GiB budget, no deadline, 2 streams,
 * 16384 items per launch, 65536 queue slots, FP32.  The plan must outlive
 * the server and must have the precision form prepared.  Errors:
 * BF_ERR_INVALID, BF_ERR_UNSUPPORTED, BF_ERR_OOM, BF_ERR_DEVICE. */
bf_status bf_server_create(bf_server *out, bf_plan plan, const bf_server_cfg *cfg);
/* Enqueue one request.  BF_ERR_INVALID for a bad request (also one larger
 * than the whole budget), BF_ERR_BUSY if the queue is full.  One thread
 * at a time may submit to a server. */
bf_status bf_submit(bf_server server, const bf_request *req, uint64_t *ticket);
/* Enqueue reqs[0 .. n) as bf_submit would one by one, with one hand-over
 * to the batcher for all of them (requests that arrive together, such as
 * one slot's, cost a few tens of nanoseconds each this way).  Every
 * request is checked first: on a bad one (BF_ERR_INVALID, naming its
 * index) nothing is queued.  Then as many as the queue has room for are
 * queued, in order, with consecutive tickets from *first_ticket (may be
 * NULL); returns that count (0 .. n: fewer than n when the queue filled;
 * resubmit the rest) or a bf_status.  Same threading rule as bf_submit. */
int32_t bf_submit_batch(bf_server server, const bf_request *reqs, int32_t n, uint64_t *first_ticket);
/* Copy up to max completions into out, waiting up to timeout_us for the
 * first (0: no wait, < 0: forever).  Returns the count (>= 0) or a
 * bf_status (BF_ERR_TIMEOUT when nothing completed in time).  May be
 * called from a thread other than the submitter. */
int32_t bf_poll(bf_server server, bf_completion *out, int32_t max, int64_t timeout_us);
bf_status bf_server_stats_get(bf_server server, bf_server_stats *out);
/* Drains every submitted request, then stops the threads and frees.
 * Completions not yet polled are discarded. */
bf_status bf_server_destroy(bf_server server);
/* CLOCK_MONOTONIC in nanoseconds (the clock of t_arrival_ns and t_done_ns). */
int64_t bf_now_ns(void);

/* ---- filter stage -------------------------------------------------------
 * The pipeline's other stage of Section III: a block s of 2048 complex
 * samples is filtered as IFFT(MULT(FFT(s))), MULT being pointwise
 * multiplication by H, the 2048-point FFT of the filter sequence h
 * zero-padded to 2048 (so y is the circular convolution of s with h).
 * Conventions: FFT(x)[k] = sum_n x[n] exp(-2 pi i k n / 2048); the inverse
 * carries 1/2048.  Arithmetic is FP32 with twiddles rounded once from FP64.
 *
 * bf_filter_create: h host complex64 [n_taps], 1 <= n_taps <= 2048, may be
 * freed on return; H is computed on the device with the filter's own
 * transform; the call synchronises hip_stream.  Errors: BF_ERR_INVALID
 * (null pointers, n_taps out of range), BF_ERR_OOM, BF_ERR_DEVICE. */
bf_status bf_filter_create(bf_filter *out, const void *h, int32_t n_taps, void *hip_stream);
/* Filters `batch` blocks: x and y device complex64 [batch][2048], 8-byte
 * aligned; y may be the same buffer as x (in place) but must not overlap it
 * otherwise.  Asynchronous, ordered on hip_stream; batch = 0 does nothing.
 * Errors: BF_ERR_INVALID (null filter or buffers, batch < 0, misalignment,
 * partial overlap), BF_ERR_DEVICE. */
bf_status bf_filter_apply(bf_filter flt, int32_t batch, const void *x, void *y, void *hip_stream);
/* Copies H (complex64 [2048]) to host memory. */
bf_status bf_filter_spectrum(bf_filter flt, void *H_out);
/* Releases the filter after the device has finished all work. */
bf_status bf_filter_destroy(bf_filter flt);

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
