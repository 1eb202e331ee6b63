// Device-independent core of the serving loop: submission ring -> batcher
// thread (admission by HBM budget, continuous batching over a few streams)
// -> completion thread -> poll.  The device is reached through bfs::Device.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "bf_serve_core.h"
#include "bf_status.h"

namespace bfs {

uint64_t request_bytes(const bf_request &r)
{
    return (uint64_t)r.n_s * ((uint64_t)r.f * BF_B * 8 + (uint64_t)BF_M * BF_B * 8);
}

int64_t monotonic_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

namespace {

constexpr int kMaxStreams = 8;
constexpr uint64_t kRateMinBytes = 8ull << 20;

struct Launch {
    void *token = nullptr;
    int64_t t_launch = 0;
    uint64_t bytes = 0;
    int status = BF_OK;
    std::vector<Req> reqs;
};

}  // namespace

struct Server {
    Device *dev = nullptr;
    bf_server_cfg cfg{};
    int n_w = 0;
    int f_max = 0;

    // Submission ring: one producer (submit), one consumer (batcher).
    std::vector<Req> ring;
    uint64_t mask = 0;
    std::atomic<uint64_t> head{0};   // next slot the producer writes
    std::atomic<uint64_t> tail{0};   // next slot the consumer reads
    uint64_t next_ticket = 1;        // producer only

    // Batcher state (batcher thread only).
    std::deque<Req> pending;         // popped from the ring, not yet admitted
    std::deque<Req> admitted;        // admitted, not yet launched
    int64_t admitted_items = 0;      // S blocks of `admitted`
    int rr = 0;

    // Launches in flight, one FIFO per stream.
    std::mutex fl_mu;
    std::deque<Launch *> inflight[kMaxStreams];
    std::atomic<int> n_inflight{0};
    std::atomic<uint64_t> inflight_bytes{0};
    std::vector<Launch *> spare;     // guarded by fl_mu

    // Completions waiting for poll.
    std::mutex cq_mu;
    std::condition_variable cq_cv;
    std::deque<bf_completion> cq;

    // Wakeups of the batcher.
    std::mutex wake_mu;
    std::condition_variable wake_cv;
    std::atomic<bool> batcher_sleeping{false};

    std::atomic<bool> stopping{false};
    std::atomic<bool> batcher_done{false};
    std::atomic<bool> completer_done{false};
    std::atomic<int> failed{0};

    // Throughput estimate for closing launches early (bytes per ns).
    std::atomic<double> rate{0.0};

    // Statistics.
    // (submitted requests are counted by head)
    std::atomic<uint64_t> n_admitted{0}, completed{0}, refused{0}, launches{0}, misses{0},
        peak_bytes{0}, launch_host_ns{0};

    std::thread batcher, completer;
};

namespace {

void wake_batcher(Server *s)
{
    if (s->batcher_sleeping.load()) {
        std::lock_guard<std::mutex> lk(s->wake_mu);
        s->wake_cv.notify_one();
    }
}

void post_completions(Server *s, const Launch &L, int64_t t_done)
{
    uint64_t n_miss = 0;
    {
        std::lock_guard<std::mutex> lk(s->cq_mu);
        for (const Req &q : L.reqs) {
            bf_completion c{};
            c.ticket = q.ticket;
            c.tag = q.r.tag;
            c.status = L.status;
            c.t_arrival_ns = q.t_arrival;
            c.t_submit_ns = q.t_submit;
            c.t_launch_ns = L.t_launch;
            c.t_done_ns = t_done;
            c.deadline_missed =
                s->cfg.deadline_us > 0 && t_done > q.t_arrival + s->cfg.deadline_us * 1000 ? 1 : 0;
            n_miss += (uint64_t)c.deadline_missed;
            s->cq.push_back(c);
        }
    }
    s->cq_cv.notify_all();
    s->completed.fetch_add(L.reqs.size());
    s->misses.fetch_add(n_miss);
}

// Packs the leading `count` requests of `admitted` into one launch.
void launch_front(Server *s, size_t count, int stream_idx)
{
    Launch *L = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->fl_mu);
        if (!s->spare.empty()) {
            L = s->spare.back();
            s->spare.pop_back();
        }
    }
    if (!L)
        L = new Launch();
    L->reqs.clear();
    L->bytes = 0;
    L->status = BF_OK;
    L->token = nullptr;
    int items = 0;
    for (size_t k = 0; k < count; ++k) {
        const Req &q = s->admitted.front();
        L->bytes += q.bytes;
        items += q.r.n_s;
        L->reqs.push_back(q);
        s->admitted.pop_front();
    }
    s->admitted_items -= items;
    L->t_launch = s->dev->now_ns();
    const bf_status rc = s->dev->launch(stream_idx, L->reqs, items, &L->token);
    s->launches.fetch_add(1);
    s->launch_host_ns.fetch_add((uint64_t)std::max<int64_t>(0, s->dev->now_ns() - L->t_launch));
    if (rc != BF_OK) {
        // Nothing reached the device: report the requests as failed now.
        L->status = rc;
        s->failed.store(1);
        s->inflight_bytes.fetch_sub(L->bytes);
        post_completions(s, *L, s->dev->now_ns());
        std::lock_guard<std::mutex> lk(s->fl_mu);
        s->spare.push_back(L);
        return;
    }
    std::lock_guard<std::mutex> lk(s->fl_mu);
    s->inflight[stream_idx].push_back(L);
    s->n_inflight.fetch_add(1);
}

// A stream with no launch in flight, else (with `deep`) one with a single
// launch in flight; -1 if none.  Under load (deep: the admitted work fills
// at least half a launch) the next launch is then packed and queued behind
// the running one, so the device does not wait for the host between the
// two; otherwise work waits for a free stream and gathers into larger
// launches.
int free_stream(Server *s, bool deep)
{
    std::lock_guard<std::mutex> lk(s->fl_mu);
    for (size_t depth = 1; depth <= (deep ? 2u : 1u); ++depth) {
        for (int k = 0; k < s->cfg.n_streams; ++k) {
            const int i = (s->rr + k) % s->cfg.n_streams;
            if (s->inflight[i].size() < depth) {
                s->rr = (i + 1) % s->cfg.n_streams;
                return i;
            }
        }
    }
    return -1;
}

void batcher_loop(Server *s)
{
    for (;;) {
        bool progress = false;
        // 1. Drain the submission ring.
        uint64_t t = s->tail.load(std::memory_order_relaxed);
        const uint64_t h = s->head.load(std::memory_order_acquire);
        for (; t != h; ++t) {
            s->pending.push_back(s->ring[t & s->mask]);
            progress = true;
        }
        s->tail.store(t, std::memory_order_release);

        // 2. Admit in arrival order while the budget allows.  (The bytes in
        // flight only fall behind the batcher's back, so one reading of
        // them bounds the whole pass; the counters move once per pass.)
        if (!s->pending.empty()) {
            const uint64_t in_use = s->inflight_bytes.load();
            uint64_t add = 0, n_add = 0;
            while (!s->pending.empty()) {
                const Req &q = s->pending.front();
                if (in_use + add + q.bytes > s->cfg.hbm_budget_bytes)
                    break;
                add += q.bytes;
                ++n_add;
                s->admitted_items += q.r.n_s;
                s->admitted.push_back(q);
                s->pending.pop_front();
            }
            if (n_add > 0) {
                const uint64_t now_b = s->inflight_bytes.fetch_add(add) + add;
                s->n_admitted.fetch_add(n_add);
                uint64_t peak = s->peak_bytes.load();
                while (now_b > peak && !s->peak_bytes.compare_exchange_weak(peak, now_b)) {
                }
                progress = true;
            }
        }

        // 3. Launch admitted work on free streams.
        while (!s->admitted.empty()) {
            const int si = free_stream(s, 2 * s->admitted_items >= s->cfg.max_batch_items);
            if (si < 0)
                break;
            size_t count = 0;
            int items = 0;
            uint64_t bytes = 0;
            // Close the launch early only while the oldest member can still
            // make its deadline: a launch of `allow` bytes is predicted to end
            // in time.  Once that deadline is lost, throughput matters more
            // and the launch takes everything admitted.
            uint64_t allow = ~0ull;
            const double rate = s->rate.load();
            if (s->cfg.deadline_us > 0 && rate > 0.0) {
                const int64_t left = s->admitted.front().t_arrival + s->cfg.deadline_us * 1000 -
                                     s->dev->now_ns();
                if (left > 0)
                    allow = (uint64_t)(rate * (double)left);
            }
            for (const Req &q : s->admitted) {
                if (count > 0 && (items + q.r.n_s > s->cfg.max_batch_items || bytes + q.bytes > allow))
                    break;
                ++count;
                items += q.r.n_s;
                bytes += q.bytes;
            }
            launch_front(s, count, si);
            progress = true;
        }

        if (progress)
            continue;
        if (s->stopping.load() && s->head.load() == s->tail.load() && s->pending.empty() &&
            s->admitted.empty())
            break;
        // 4. Nothing to do now.  While requests wait for launches in flight
        // (for a stream or for budget), the next event is a completion:
        // poll for it, so the stream or budget it frees is used at once (a
        // sleeping thread is woken tens to hundreds of microseconds after
        // the notification).  Otherwise sleep until a submission, a
        // completion or 50 us.
        if ((!s->admitted.empty() || !s->pending.empty()) && s->n_inflight.load() > 0) {
            std::this_thread::yield();
            continue;
        }
        std::unique_lock<std::mutex> lk(s->wake_mu);
        // (sequentially consistent flag and head accesses on both sides, so a
        // submission either sees the flag or is seen here)
        s->batcher_sleeping.store(true);
        if (s->head.load() == s->tail.load())
            s->wake_cv.wait_for(lk, std::chrono::microseconds(50));
        s->batcher_sleeping.store(false);
    }
    s->batcher_done.store(true);
}

void completer_loop(Server *s)
{
    int idle_polls = 0;
    for (;;) {
        bool any = false;
        for (int i = 0; i < s->cfg.n_streams; ++i) {
            Launch *L = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->fl_mu);
                if (!s->inflight[i].empty())
                    L = s->inflight[i].front();
            }
            if (!L)
                continue;
            const int d = s->dev->done(L->token);
            if (d == 0)
                continue;
            const int64_t t_done = s->dev->now_ns();
            if (d < 0) {
                L->status = d;
                s->failed.store(1);
            } else if (t_done > L->t_launch && L->bytes >= kRateMinBytes) {
                // (small launches measure launch overhead, not throughput)
                const double r = (double)L->bytes / (double)(t_done - L->t_launch);
                const double old = s->rate.load();
                s->rate.store(old > 0.0 ? 0.8 * old + 0.2 * r : r);
            }
            s->dev->release(L->token);
            L->token = nullptr;
            // The bytes go back to the budget before the completions are
            // posted, so a poller that has seen them never finds them still
            // counted in flight.
            s->inflight_bytes.fetch_sub(L->bytes);
            post_completions(s, *L, t_done);
            {
                std::lock_guard<std::mutex> lk(s->fl_mu);
                s->inflight[i].pop_front();
                s->spare.push_back(L);
            }
            s->n_inflight.fetch_sub(1);
            wake_batcher(s);
            any = true;
        }
        if (any) {
            idle_polls = 0;
            continue;
        }
        if (s->batcher_done.load() && s->n_inflight.load() == 0)
            break;
        // Poll back-to-back while launches are in flight (lowest latency);
        // nap between polls when idle so an idle server does not hold a core.
        if (s->n_inflight.load() > 0)
            std::this_thread::yield();
        else if (++idle_polls > 2000)
            std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    s->completer_done.store(true);
    {
        // (taken so that a poller between its check and its wait cannot
        // miss the notification)
        std::lock_guard<std::mutex> lk(s->cq_mu);
    }
    s->cq_cv.notify_all();
}

}  // namespace

bf_status server_create(Server **out, Device *dev, const bf_server_cfg &cfg, int n_w, int f_max)
{
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!dev)
        return bf_fail(BF_ERR_INVALID, "device is null");
    if (cfg.hbm_budget_bytes == 0 || cfg.n_streams < 1 || cfg.n_streams > kMaxStreams ||
        cfg.max_batch_items < 1 || cfg.queue_capacity < 2 ||
        (cfg.queue_capacity & (cfg.queue_capacity - 1)) != 0)
        return bf_fail(BF_ERR_INVALID,
                       "bad server config (budget > 0, 1..8 streams, max_batch_items >= 1, "
                       "queue_capacity a power of two >= 2)");
    Server *s = new (std::nothrow) Server();
    if (!s)
        return bf_fail(BF_ERR_OOM, "server allocation");
    s->dev = dev;
    s->cfg = cfg;
    s->n_w = n_w;
    s->f_max = f_max;
    try {
        s->ring.resize((size_t)cfg.queue_capacity);
    } catch (...) {
        delete s;
        return bf_fail(BF_ERR_OOM, "submission ring of %d slots", cfg.queue_capacity);
    }
    s->mask = (uint64_t)cfg.queue_capacity - 1;
    s->batcher = std::thread(batcher_loop, s);
    s->completer = std::thread(completer_loop, s);
    *out = s;
    return BF_OK;
}

namespace {

// The checks of one request (index names it in the message of a batch).
bf_status check_request(const Server *s, const bf_request &r, int index)
{
    if (r.w_id < 0 || r.w_id >= s->n_w)
        return bf_fail(BF_ERR_INVALID, "request %d: w_id %d outside [0, %d)", index, r.w_id, s->n_w);
    if (r.f < 0 || r.f > s->f_max)
        return bf_fail(BF_ERR_INVALID, "request %d: f %d outside [0, %d]", index, r.f, s->f_max);
    if (r.n_s < 1 || r.n_s > s->cfg.max_batch_items)
        return bf_fail(BF_ERR_INVALID, "request %d: n_s %d outside [1, %d]", index, r.n_s,
                       s->cfg.max_batch_items);
    if (!r.R || (reinterpret_cast<uintptr_t>(r.R) & 15u))
        return bf_fail(BF_ERR_INVALID, "request %d: R null or not 16-byte aligned", index);
    if (r.f > 0 && (!r.S || (reinterpret_cast<uintptr_t>(r.S) & 7u)))
        return bf_fail(BF_ERR_INVALID, "request %d: S null or not 8-byte aligned", index);
    if (request_bytes(r) > s->cfg.hbm_budget_bytes)
        return bf_fail(BF_ERR_INVALID, "request %d of %llu bytes exceeds the whole budget", index,
                       (unsigned long long)request_bytes(r));
    return BF_OK;
}

// Writes reqs[0 .. n) into the ring from head h on and publishes them.
void publish(Server *s, const bf_request *reqs, int n, uint64_t h, uint64_t *first_ticket)
{
    const int64_t now = s->dev->now_ns();
    if (first_ticket)
        *first_ticket = s->next_ticket;
    for (int i = 0; i < n; ++i) {
        Req &slot = s->ring[(h + (uint64_t)i) & s->mask];
        slot.r = reqs[i];
        slot.ticket = s->next_ticket++;
        slot.t_submit = now;
        slot.t_arrival = reqs[i].t_arrival_ns > 0 ? reqs[i].t_arrival_ns : now;
        slot.bytes = request_bytes(reqs[i]);
    }
    // (sequentially consistent, against the batcher's sleeping flag)
    s->head.store(h + (uint64_t)n);
    wake_batcher(s);
}

}  // namespace

bf_status server_submit(Server *s, const bf_request *req, uint64_t *ticket)
{
    if (!s || !req)
        return bf_fail(BF_ERR_INVALID, "null argument");
    if (s->stopping.load(std::memory_order_relaxed))
        return bf_fail(BF_ERR_INVALID, "server is shutting down");
    const bf_status rc = check_request(s, *req, 0);
    if (rc != BF_OK)
        return rc;
    const uint64_t h = s->head.load(std::memory_order_relaxed);
    if (h - s->tail.load(std::memory_order_acquire) >= s->ring.size()) {
        s->refused.fetch_add(1);
        return bf_fail(BF_ERR_BUSY, "submission queue full");
    }
    publish(s, req, 1, h, ticket);
    return BF_OK;
}

int32_t server_submit_batch(Server *s, const bf_request *reqs, int32_t n, uint64_t *first_ticket)
{
    if (!s || n < 0 || (n > 0 && !reqs))
        return bf_fail(BF_ERR_INVALID, "bad bf_submit_batch arguments");
    if (s->stopping.load(std::memory_order_relaxed))
        return bf_fail(BF_ERR_INVALID, "server is shutting down");
    for (int32_t i = 0; i < n; ++i) {
        const bf_status rc = check_request(s, reqs[i], i);
        if (rc != BF_OK)
            return rc;
    }
    const uint64_t h = s->head.load(std::memory_order_relaxed);
    const uint64_t room = s->ring.size() - (h - s->tail.load(std::memory_order_acquire));
    const int32_t take = (int32_t)std::min<uint64_t>(room, (uint64_t)n);
    if (take < n)
        s->refused.fetch_add(1);
    if (take > 0)
        publish(s, reqs, take, h, first_ticket);
    return take;
}

int32_t server_poll(Server *s, bf_completion *out, int32_t max, int64_t timeout_us)
{
    if (!s || (!out && max > 0) || max < 0)
        return bf_fail(BF_ERR_INVALID, "bad bf_poll arguments");
    std::unique_lock<std::mutex> lk(s->cq_mu);
    auto ready = [&] { return !s->cq.empty() || s->completer_done.load(); };
    if (!ready()) {
        if (timeout_us == 0)
            return 0;
        if (timeout_us < 0)
            s->cq_cv.wait(lk, ready);
        else if (!s->cq_cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
            return bf_fail(BF_ERR_TIMEOUT, "no completion within %lld us", (long long)timeout_us);
    }
    int32_t n = 0;
    while (n < max && !s->cq.empty()) {
        out[n++] = s->cq.front();
        s->cq.pop_front();
    }
    return n;
}

bf_status server_stats(Server *s, bf_server_stats *o)
{
    if (!s || !o)
        return bf_fail(BF_ERR_INVALID, "null argument");
    o->submitted = s->head.load();
    o->admitted = s->n_admitted.load();
    o->completed = s->completed.load();
    o->refused = s->refused.load();
    o->launches = s->launches.load();
    o->deadline_misses = s->misses.load();
    o->inflight_bytes = s->inflight_bytes.load();
    o->peak_inflight_bytes = s->peak_bytes.load();
    o->queued = s->head.load() - s->tail.load();
    o->launch_host_ns = s->launch_host_ns.load();
    return BF_OK;
}

bf_status server_destroy(Server *s)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "server is null");
    s->stopping.store(true);
    {
        std::lock_guard<std::mutex> lk(s->wake_mu);
        s->wake_cv.notify_all();
    }
    s->batcher.join();
    s->completer.join();
    for (Launch *L : s->spare)
        delete L;
    const int failed = s->failed.load();
    delete s;
    return failed ? bf_fail(BF_ERR_DEVICE, "a launch of this server failed") : BF_OK;
}

}  // namespace bfs
