// Load generator for the serving loop of libbf (benchmark helper, not part
// of the beamforming path): replays a schedule of requests against a
// bf_server from one native thread while another drains completions.
#include <stdint.h>

#include <atomic>
#include <thread>

#include "bf.h"

extern "C" {

/* Submits reqs[i] at t_start + t_offset_ns[i] (t_offset_ns non-decreasing;
 * busy-waits for each), retrying while the submission queue is full, and
 * collects every completion.  reqs[i].t_arrival_ns is set to the scheduled
 * time, so latency is measured from the schedule, not from the submit.
 * done[i] receives the completion of reqs[i] (matched by tag = i).
 * Returns the number of BF_ERR_BUSY retries (>= 0), or a bf_status. */
int64_t bf_loadgen_replay(bf_server s, bf_request *reqs, const int64_t *t_offset_ns, int64_t n,
                          bf_completion *done)
{
    if (!s || (n > 0 && (!reqs || !t_offset_ns || !done)) || n < 0)
        return BF_ERR_INVALID;
    std::atomic<int64_t> received{0};
    std::atomic<int> poll_error{0};
    std::thread poller([&] {
        bf_completion buf[256];
        while (received.load() < n) {
            const int32_t k = bf_poll(s, buf, 256, 1000);
            if (k == BF_ERR_TIMEOUT)
                continue;
            if (k < 0) {
                poll_error.store(k);
                return;
            }
            for (int32_t j = 0; j < k; ++j) {
                const uint64_t i = buf[j].tag;
                if (i < (uint64_t)n)
                    done[i] = buf[j];
            }
            received.fetch_add(k);
        }
    });
    const int64_t t0 = bf_now_ns() + 1000000;   // start 1 ms from now
    int64_t busy = 0;
    int rc = BF_OK;
    for (int64_t i = 0; i < n && rc == BF_OK; ++i) {
        const int64_t when = t0 + t_offset_ns[i];
        while (bf_now_ns() < when) {
        }
        reqs[i].tag = (uint64_t)i;
        reqs[i].t_arrival_ns = when;
        for (;;) {
            const bf_status st = bf_submit(s, &reqs[i], nullptr);
            if (st == BF_OK)
                break;
            if (st != BF_ERR_BUSY) {
                rc = st;
                break;
            }
            ++busy;
        }
    }
    if (rc != BF_OK) {
        // Stop waiting for requests that were never submitted.
        received.store(n);
    }
    poller.join();
    if (rc != BF_OK)
        return rc;
    if (poll_error.load() != 0)
        return poll_error.load();
    return busy;
}

}  // extern "C"
