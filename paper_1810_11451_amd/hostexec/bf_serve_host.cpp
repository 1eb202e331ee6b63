// Host-only executor of the serving loop: the device-independent core of
// csrc/bf_serve_core.cpp driven by a null device (no HIP).  See
// include/bf_serve_host.h.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "bf_serve_core.h"
#include "bf_serve_host.h"
#include "bf_status.h"

namespace {

struct Rec {
    bfh_launch_rec pub{};
    std::vector<uint64_t> tickets;
    bool finished = false;   // manual completion: set by bfh_device_complete
    int fin_status = BF_OK;
    bool released = false;
};

}  // namespace

struct bfh_device_s final : public bfs::Device {
    bfh_device_cfg cfg{};
    std::atomic<int64_t> clock{1000000000LL};

    std::mutex mu;                     // guards everything below
    std::deque<Rec> recs;              // one per launch, stable addresses
    std::vector<std::pair<int64_t, int>> fail_at;   // (launch index, status)
    int64_t stream_end[8] = {};
    int32_t peak_unfinished = 0;
    std::atomic<int> users{0};

    int64_t now_ns() override
    {
        return cfg.manual_clock ? clock.load() : bfs::monotonic_ns();
    }

    // Caller holds mu.
    bool finished_locked(const Rec &r, int64_t now) const
    {
        if (r.finished || r.pub.status != BF_OK)
            return true;
        return !cfg.manual_complete && now >= r.pub.t_end_ns;
    }

    int32_t unfinished_locked(int stream, int64_t now) const
    {
        int32_t n = 0;
        for (const Rec &r : recs)
            if ((stream < 0 || r.pub.stream == stream) && !finished_locked(r, now))
                ++n;
        return n;
    }

    void write_marks(const std::vector<bfs::Req> &reqs)
    {
        bfs::for_each_block(reqs, [](const void *S, void *R, int32_t w_id, int32_t f) {
            float *r = static_cast<float *>(R);
            const float *s = static_cast<const float *>(S);
            const float id[2] = {(float)w_id, (float)f};
            std::memcpy(r, id, sizeof id);
            float first[2] = {0.f, 0.f}, last[2] = {0.f, 0.f};
            if (f > 0) {
                std::memcpy(first, s, sizeof first);
                std::memcpy(last, s + 2 * ((size_t)f * BF_B - 1), sizeof last);
            }
            std::memcpy(r + 2, first, sizeof first);
            std::memcpy(r + 4, last, sizeof last);
            std::memcpy(r + 2 * ((size_t)BF_M * BF_B - 1), id, sizeof id);
        });
    }

    bf_status launch(int stream, const std::vector<bfs::Req> &reqs, int n_items, void **token) override
    {
        const int64_t now = now_ns();
        std::lock_guard<std::mutex> lk(mu);
        const int64_t index = (int64_t)recs.size();
        recs.emplace_back();
        Rec &r = recs.back();
        r.pub.stream = stream;
        r.pub.n_reqs = (int32_t)reqs.size();
        r.pub.n_items = n_items;
        r.pub.t_launch_ns = now;
        r.pub.first_ticket = reqs.empty() ? 0 : reqs.front().ticket;
        for (const bfs::Req &q : reqs) {
            r.pub.bytes += q.bytes;
            r.tickets.push_back(q.ticket);
        }
        for (const auto &fa : fail_at) {
            if (fa.first == index) {
                r.pub.status = fa.second;
                r.released = true;
                return bf_fail((bf_status)fa.second, "null device: launch %lld made to fail",
                               (long long)index);
            }
        }
        if (cfg.write_marks)
            write_marks(reqs);
        if (!cfg.manual_complete) {
            const int64_t cost = cfg.launch_ns + (cfg.bytes_per_ns > 0.0
                                                      ? (int64_t)((double)r.pub.bytes / cfg.bytes_per_ns)
                                                      : 0);
            r.pub.t_end_ns = std::max(now, stream_end[stream]) + cost;
            stream_end[stream] = r.pub.t_end_ns;
        }
        peak_unfinished = std::max(peak_unfinished, unfinished_locked(-1, now));
        *token = &r;
        return BF_OK;
    }

    int done(void *token) override
    {
        const int64_t now = now_ns();
        std::lock_guard<std::mutex> lk(mu);
        const Rec &r = *static_cast<const Rec *>(token);
        if (!finished_locked(r, now))
            return 0;
        if (cfg.manual_complete && r.fin_status != BF_OK)
            return r.fin_status;
        return 1;
    }

    void release(void *token) override
    {
        std::lock_guard<std::mutex> lk(mu);
        static_cast<Rec *>(token)->released = true;
    }
};

struct bfh_server_s {
    bfs::Server *core = nullptr;
    bfh_device dev = nullptr;
};

extern "C" bf_status bfh_device_create(bfh_device *out, const bfh_device_cfg *cfg)
{
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    bfh_device d = new (std::nothrow) bfh_device_s();
    if (!d)
        return bf_fail(BF_ERR_OOM, "device allocation");
    if (cfg) {
        d->cfg = *cfg;
    } else {
        d->cfg.launch_ns = 5000;
        d->cfg.bytes_per_ns = 5000.0;
    }
    if (d->cfg.launch_ns < 0) {
        delete d;
        return bf_fail(BF_ERR_INVALID, "launch_ns < 0");
    }
    *out = d;
    return BF_OK;
}

extern "C" bf_status bfh_device_destroy(bfh_device d)
{
    if (!d)
        return bf_fail(BF_ERR_INVALID, "device is null");
    if (d->users.load() != 0)
        return bf_fail(BF_ERR_INVALID, "device still used by a server");
    delete d;
    return BF_OK;
}

extern "C" void bfh_clock_set(bfh_device d, int64_t t_ns)
{
    if (d && d->cfg.manual_clock)
        d->clock.store(t_ns);
}

extern "C" int64_t bfh_clock_now(bfh_device d) { return d ? d->now_ns() : 0; }

extern "C" int32_t bfh_device_complete(bfh_device d, int32_t stream, int32_t count, int32_t status)
{
    if (!d || count < 0 || status > 0)
        return bf_fail(BF_ERR_INVALID, "bad bfh_device_complete arguments");
    const int64_t now = d->now_ns();
    std::lock_guard<std::mutex> lk(d->mu);
    int32_t n = 0;
    for (Rec &r : d->recs) {
        if (n >= count)
            break;
        // (launches that failed when enqueued never reached the device)
        if (r.pub.stream != stream || r.pub.status != BF_OK || r.finished)
            continue;
        r.finished = true;
        r.fin_status = status;
        r.pub.t_end_ns = now;
        r.pub.status = status;
        ++n;
    }
    return n;
}

extern "C" bf_status bfh_device_fail_launch(bfh_device d, int64_t index, int32_t status)
{
    if (!d || index < 0 || status >= 0)
        return bf_fail(BF_ERR_INVALID, "bad bfh_device_fail_launch arguments");
    std::lock_guard<std::mutex> lk(d->mu);
    d->fail_at.emplace_back(index, status);
    return BF_OK;
}

extern "C" int64_t bfh_device_launches(bfh_device d, bfh_launch_rec *out, int64_t max)
{
    if (!d || (max > 0 && !out))
        return bf_fail(BF_ERR_INVALID, "bad bfh_device_launches arguments");
    std::lock_guard<std::mutex> lk(d->mu);
    const int64_t n = (int64_t)d->recs.size();
    for (int64_t k = 0; k < std::min(n, max); ++k)
        out[k] = d->recs[(size_t)k].pub;
    return n;
}

extern "C" int64_t bfh_device_launch_tickets(bfh_device d, int64_t k, uint64_t *out, int64_t max)
{
    if (!d || (max > 0 && !out))
        return bf_fail(BF_ERR_INVALID, "bad bfh_device_launch_tickets arguments");
    std::lock_guard<std::mutex> lk(d->mu);
    if (k < 0 || k >= (int64_t)d->recs.size())
        return bf_fail(BF_ERR_INVALID, "launch %lld unknown", (long long)k);
    const std::vector<uint64_t> &t = d->recs[(size_t)k].tickets;
    for (int64_t i = 0; i < std::min((int64_t)t.size(), max); ++i)
        out[i] = t[(size_t)i];
    return (int64_t)t.size();
}

extern "C" int32_t bfh_device_unfinished(bfh_device d, int32_t stream)
{
    if (!d)
        return bf_fail(BF_ERR_INVALID, "device is null");
    const int64_t now = d->now_ns();
    std::lock_guard<std::mutex> lk(d->mu);
    return d->unfinished_locked(stream, now);
}

extern "C" int32_t bfh_device_peak_unfinished(bfh_device d)
{
    if (!d)
        return bf_fail(BF_ERR_INVALID, "device is null");
    std::lock_guard<std::mutex> lk(d->mu);
    return d->peak_unfinished;
}

extern "C" bf_status bfh_server_create(bfh_server *out, bfh_device dev, const bf_server_cfg *cfg_in,
                                       int32_t n_w, int32_t f_max)
{
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!dev)
        return bf_fail(BF_ERR_INVALID, "device is null");
    if (n_w < 1 || f_max < 0 || f_max > BF_FMAX)
        return bf_fail(BF_ERR_INVALID, "n_w %d or f_max %d out of range", n_w, f_max);
    bf_server_cfg cfg{};
    cfg.hbm_budget_bytes = 16ull << 30;
    cfg.deadline_us = 0;
    cfg.n_streams = 2;
    cfg.max_batch_items = 16384;
    cfg.queue_capacity = 65536;
    cfg.prec = BF_FP32;
    if (cfg_in)
        cfg = *cfg_in;
    if (cfg.prec < 0 || cfg.prec > BF_BF16X2)
        return bf_fail(BF_ERR_INVALID, "unknown precision %d", cfg.prec);
    bfh_server s = new (std::nothrow) bfh_server_s();
    if (!s)
        return bf_fail(BF_ERR_OOM, "server allocation");
    s->dev = dev;
    const bf_status rc = bfs::server_create(&s->core, dev, cfg, n_w, f_max);
    if (rc != BF_OK) {
        delete s;
        return rc;
    }
    dev->users.fetch_add(1);
    *out = s;
    return BF_OK;
}

extern "C" bf_status bfh_submit(bfh_server s, const bf_request *req, uint64_t *ticket)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "null argument");
    return bfs::server_submit(s->core, req, ticket);
}

extern "C" int32_t bfh_submit_batch(bfh_server s, const bf_request *reqs, int32_t n, uint64_t *first_ticket)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "null argument");
    return bfs::server_submit_batch(s->core, reqs, n, first_ticket);
}

extern "C" int32_t bfh_poll(bfh_server s, bf_completion *out, int32_t max, int64_t timeout_us)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "bad bf_poll arguments");
    return bfs::server_poll(s->core, out, max, timeout_us);
}

extern "C" bf_status bfh_server_stats_get(bfh_server s, bf_server_stats *o)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "null argument");
    return bfs::server_stats(s->core, o);
}

extern "C" bf_status bfh_server_destroy(bfh_server s)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "server is null");
    const bf_status rc = bfs::server_destroy(s->core);
    s->dev->users.fetch_sub(1);
    delete s;
    return rc;
}
