// Load generator for the serving loop of libbf (benchmark helper, not part
// of the beamforming path): replays a schedule of requests against a
// bf_server from one native thread while another drains completions.
#include <stdint.h>
#include <stdio.h>

#include <atomic>
#include <thread>

#include "bf.h"

extern "C" {

/* Submits reqs[i] at t_start + t_offset_ns[i] (t_offset_ns non-decreasing;
 * busy-waits for each), retrying while the submission queue is full, and
 * collects every completion.  reqs[i].t_arrival_ns is set to the scheduled
 * time, so latency is measured from the schedule, not from the submit.
 * done[i] receives the completion of reqs[i] (matched by tag = i).
 *   progress_every  > 0: a line on stderr each time that many more
 *                   completions have arrived (label names the run)
 *   stall_ms        > 0: give up when requests are outstanding and no
 *                   completion has arrived for that long; returns
 *                   BF_ERR_TIMEOUT (the server still holds the requests)
 *   submit_ns       if not null: the nanoseconds spent inside bf_submit and
 *                   bf_submit_batch calls (accepted and refused), summed
 * Requests with equal offsets are submitted together (bf_submit_batch,
 * up to 4096 a call), others one by one (bf_submit).
 * Returns the number of BF_ERR_BUSY retries (>= 0), or a bf_status. */
int64_t bf_loadgen_replay(bf_server s, bf_request *reqs, const int64_t *t_offset_ns, int64_t n,
                          bf_completion *done, int64_t progress_every, int64_t stall_ms,
                          const char *label, int64_t *submit_ns)
{
    if (!s || (n > 0 && (!reqs || !t_offset_ns || !done)) || n < 0)
        return BF_ERR_INVALID;
    const char *name = label ? label : "replay";
    std::atomic<int64_t> received{0};
    std::atomic<int64_t> submitted{0};
    std::atomic<int> poll_error{0};
    std::atomic<bool> stop{false};
    const int64_t t_begin = bf_now_ns();
    std::thread poller([&] {
        bf_completion buf[256];
        int64_t next_report = progress_every > 0 ? progress_every : n + 1;
        int64_t last_seen = bf_now_ns();
        while (received.load() < n && !stop.load()) {
            const int32_t k = bf_poll(s, buf, 256, 1000);
            const int64_t now = bf_now_ns();
            if (k == BF_ERR_TIMEOUT) {
                if (stall_ms > 0 && submitted.load() > received.load() &&
                    now - last_seen > stall_ms * 1000000) {
                    fprintf(stderr, "[loadgen %s] no completion for %lld ms with %lld of %lld "
                            "requests outstanding; giving up\n", name, (long long)stall_ms,
                            (long long)(submitted.load() - received.load()), (long long)n);
                    fflush(stderr);
                    poll_error.store(BF_ERR_TIMEOUT);
                    stop.store(true);
                    return;
                }
                continue;
            }
            if (k < 0) {
                poll_error.store(k);
                stop.store(true);
                return;
            }
            last_seen = now;
            for (int32_t j = 0; j < k; ++j) {
                const uint64_t i = buf[j].tag;
                if (i < (uint64_t)n)
                    done[i] = buf[j];
            }
            const int64_t got = received.fetch_add(k) + k;
            if (got >= next_report) {
                fprintf(stderr, "[loadgen %s] %lld of %lld completed, %.3f s\n", name,
                        (long long)got, (long long)n, (double)(now - t_begin) * 1e-9);
                fflush(stderr);
                while (next_report <= got)
                    next_report += progress_every;
            }
        }
    });
    const int64_t t0 = bf_now_ns() + 1000000;   // start 1 ms from now
    int64_t busy = 0;
    int64_t in_submit = 0;
    int rc = BF_OK;
    // Requests due at the same time go to the server in one bf_submit_batch
    // call (up to 4096 at a time), others one by one.
    constexpr int64_t kChunk = 4096;
    for (int64_t i = 0; i < n && rc == BF_OK && !stop.load();) {
        const int64_t when = t0 + t_offset_ns[i];
        int64_t j = i + 1;
        while (j < n && j - i < kChunk && t_offset_ns[j] == t_offset_ns[i])
            ++j;
        while (bf_now_ns() < when) {
        }
        for (int64_t k = i; k < j; ++k) {
            reqs[k].tag = (uint64_t)k;
            reqs[k].t_arrival_ns = when;
        }
        while (i < j && rc == BF_OK && !stop.load()) {
            const int64_t ts = bf_now_ns();
            int32_t got;
            if (j - i == 1) {
                const bf_status st = bf_submit(s, &reqs[i], nullptr);
                got = st == BF_OK ? 1 : (st == BF_ERR_BUSY ? 0 : st);
            } else {
                got = bf_submit_batch(s, &reqs[i], (int32_t)(j - i), nullptr);
            }
            in_submit += bf_now_ns() - ts;
            if (got < 0) {
                rc = got;
                break;
            }
            if (got == 0)
                ++busy;
            i += got;
            submitted.fetch_add(got);
        }
    }
    if (rc != BF_OK) {
        // Stop waiting for requests that were never submitted.
        stop.store(true);
    }
    poller.join();
    if (submit_ns)
        *submit_ns = in_submit;
    if (rc != BF_OK)
        return rc;
    if (poll_error.load() != 0)
        return poll_error.load();
    return busy;
}

}  // extern "C"
