/* bf_serve_host.h - host-only executor of libbf's serving loop.
 *
 * The serving loop of include/bf.h (the request loop of the pipeline's
 * beamforming stage, which runs continuously on arriving signal, Section II)
 * is built from a device-independent core: submission ring, admission by an
 * HBM budget, batching onto streams, completion reporting.  This library
 * links that same core to a null device instead of HIP, so the loop can run
 * and be checked, also under ThreadSanitizer, on a machine without a GPU:
 *
 *   - launches compute nothing; each one is logged (stream, requests,
 *     blocks, bytes, times, tickets) and, if asked, writes a mark into the
 *     R memory of every S block it covers, so that the pointers the loop
 *     derives for each block can be checked;
 *   - a launch finishes by a cost model (a fixed time per launch plus its
 *     S + R bytes at a given rate, in order per stream) or only when the
 *     caller says so (bfh_device_complete);
 *   - the clock is CLOCK_MONOTONIC or a value the caller sets;
 *   - a chosen launch can be made to fail, as a device error would.
 *
 * The bfh_server_* calls behave as bf_server_* of include/bf.h (same
 * request, completion and statistics types, same errors) except that
 * BF_ERR_UNSUPPORTED never occurs (there is no plan) and the pool bounds
 * n_w and f_max are given directly.  S and R are host memory here; R must
 * be writable when marks are on, and S readable at its first and last
 * element.  The library also exports bf_status_str and bf_last_error.
 * Threading is that of the bf_server_* calls; every bfh_device_* call is
 * safe from any thread.
 */
#ifndef BF_SERVE_HOST_H
#define BF_SERVE_HOST_H

#include <stdint.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfh_device_s *bfh_device;
typedef struct bfh_server_s *bfh_server;

typedef struct {
    int32_t manual_clock;     /* 1: the clock is the value set by bfh_clock_set (starts at 1 s);
                                 0: CLOCK_MONOTONIC */
    int32_t manual_complete;  /* 1: launches finish only through bfh_device_complete;
                                 0: by the cost model below */
    int64_t launch_ns;        /* cost model: time per launch */
    double bytes_per_ns;      /* cost model: S + R bytes per ns (<= 0: no byte cost) */
    int32_t write_marks;      /* 1: every launch writes marks into R (see bfh_mark) */
    int32_t reserved;
} bfh_device_cfg;

/* Marks a launch writes for each S block (S, R, w_id, f) when write_marks
 * is on, as complex64 values of R (host memory):
 *   R[0]      = (w_id, f)
 *   R[1]      = S[0]          (first element of the block; (0, 0) when f = 0)
 *   R[2]      = S[60 f - 1]   (last element of the block; (0, 0) when f = 0)
 *   R[3839]   = (w_id, f)     (last element of the 64 x 60 block)
 * Nothing else of R is written. */

typedef struct {
    int32_t stream;
    int32_t n_reqs;
    int32_t n_items;          /* S blocks */
    int32_t status;           /* BF_OK, or the status it failed with */
    uint64_t bytes;           /* S + R bytes of its requests */
    int64_t t_launch_ns;      /* device clock when enqueued */
    int64_t t_end_ns;         /* cost model: when it finishes; manual: when completed (0 before) */
    uint64_t first_ticket;
} bfh_launch_rec;

/* cfg may be NULL: monotonic clock, cost model of 5 us per launch and
 * 5000 bytes per ns, no marks.  Errors: BF_ERR_INVALID, BF_ERR_OOM. */
bf_status bfh_device_create(bfh_device *out, const bfh_device_cfg *cfg);
/* The device must not be in use by a server. */
bf_status bfh_device_destroy(bfh_device dev);
/* Manual clock only (ignored otherwise). */
void bfh_clock_set(bfh_device dev, int64_t t_ns);
int64_t bfh_clock_now(bfh_device dev);
/* Manual completion: finishes the oldest `count` unfinished launches of
 * `stream` with `status` (BF_OK, or an error such as BF_ERR_DEVICE).
 * Returns how many were finished. */
int32_t bfh_device_complete(bfh_device dev, int32_t stream, int32_t count, int32_t status);
/* The launch with 0-based index `index` (in launch order since the device
 * was created) fails when enqueued, with `status`.  BF_ERR_INVALID for a
 * negative index or a status >= 0. */
bf_status bfh_device_fail_launch(bfh_device dev, int64_t index, int32_t status);
/* Copies up to max launch records (oldest first) into out; returns the
 * number of launches so far. */
int64_t bfh_device_launches(bfh_device dev, bfh_launch_rec *out, int64_t max);
/* Tickets of the requests of launch k, in launch order; returns their count
 * (or BF_ERR_INVALID for an unknown k). */
int64_t bfh_device_launch_tickets(bfh_device dev, int64_t k, uint64_t *out, int64_t max);
/* Launches enqueued on `stream` (all streams for -1) that have not finished. */
int32_t bfh_device_unfinished(bfh_device dev, int32_t stream);
/* Largest number of launches that were unfinished at one time. */
int32_t bfh_device_peak_unfinished(bfh_device dev);

bf_status bfh_server_create(bfh_server *out, bfh_device dev, const bf_server_cfg *cfg, int32_t n_w,
                            int32_t f_max);
bf_status bfh_submit(bfh_server server, const bf_request *req, uint64_t *ticket);
int32_t bfh_submit_batch(bfh_server server, const bf_request *reqs, int32_t n, uint64_t *first_ticket);
int32_t bfh_poll(bfh_server server, bf_completion *out, int32_t max, int64_t timeout_us);
bf_status bfh_server_stats_get(bfh_server server, bf_server_stats *out);
bf_status bfh_server_destroy(bfh_server server);

#ifdef __cplusplus
}
#endif

#endif /* BF_SERVE_HOST_H */
