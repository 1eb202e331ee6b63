// Device-independent core of the serving loop (no HIP): submission ring,
// admission by an HBM budget, continuous batching onto device streams,
// completion reporting.  The device side is reached only through `Device`,
// which libbf implements with HIP streams and events (bf_server.cpp) and
// the host executor implements with a null device and a settable clock
// (hostexec/), so the same loop runs, and is tested, with and without a GPU.
#pragma once

#include <stdint.h>

#include <vector>

#include "bf.h"

namespace bfs {

// A request as the loop keeps it.
struct Req {
    bf_request r;
    uint64_t ticket;
    int64_t t_arrival;
    int64_t t_submit;
    uint64_t bytes;
};

// S + R bytes of a request (what it holds of the HBM budget).
uint64_t request_bytes(const bf_request &r);

// CLOCK_MONOTONIC in nanoseconds.
int64_t monotonic_ns();

// Calls fn(S, R, w_id, f) once per S block of reqs, in order: block k of a
// request reads S + k f 60 and writes R + k 64 60 complex elements (S is
// null when f = 0).
template <class Fn>
void for_each_block(const std::vector<Req> &reqs, Fn &&fn)
{
    for (const Req &q : reqs) {
        const char *S = static_cast<const char *>(q.r.S);
        char *R = static_cast<char *>(q.r.R);
        for (int k = 0; k < q.r.n_s; ++k)
            fn(q.r.f > 0 ? S + (size_t)k * q.r.f * BF_B * 8 : nullptr,
               R + (size_t)k * BF_M * BF_B * 8, q.r.w_id, q.r.f);
    }
}

// What the loop needs of a device.  launch() is called from the batcher
// thread only; done() and release() from the completion thread only;
// now_ns() from any thread.
class Device {
public:
    virtual ~Device() = default;
    virtual int64_t now_ns() = 0;
    // Enqueues one launch covering every S block of reqs (n_items blocks in
    // all) on stream `stream` (0 .. n_streams - 1; launches on one stream
    // run in order).  On BF_OK, *token names the launch for done() and
    // release(); on an error nothing reached the device.
    virtual bf_status launch(int stream, const std::vector<Req> &reqs, int n_items, void **token) = 0;
    // 1: the launch has finished, 0: not yet, < 0: the bf_status of a failure.
    virtual int done(void *token) = 0;
    // The token is not used again.
    virtual void release(void *token) = 0;
};

struct Server;

// Checks cfg (budget > 0, 1..8 streams, max_batch_items >= 1,
// queue_capacity a power of two >= 2) and starts the batcher and completion
// threads.  n_w and f_max bound the requests' w_id and f.  The device must
// outlive the server.
bf_status server_create(Server **out, Device *dev, const bf_server_cfg &cfg, int n_w, int f_max);
bf_status server_submit(Server *s, const bf_request *req, uint64_t *ticket);
// Checks all n requests (nothing is queued if one fails), then queues as
// many as the ring has room for, in order, with consecutive tickets from
// *first_ticket; returns that count (0 .. n) or a bf_status.
int32_t server_submit_batch(Server *s, const bf_request *reqs, int32_t n, uint64_t *first_ticket);
int32_t server_poll(Server *s, bf_completion *out, int32_t max, int64_t timeout_us);
bf_status server_stats(Server *s, bf_server_stats *out);
// Drains every submitted request, joins the threads and frees the server
// (not the device).  BF_ERR_DEVICE if any launch failed.
bf_status server_destroy(Server *s);

}  // namespace bfs
