// Serving loop of libbf (the C ABI of the serving section of include/bf.h):
// the device-independent loop of bf_serve_core.cpp driven by HIP streams,
// with each launch's completion marked by an event.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <vector>

#include "bf_host.h"
#include "bf_serve_core.h"

extern "C" int64_t bf_now_ns(void) { return bfs::monotonic_ns(); }

namespace {

constexpr int kMaxStreams = 8;

class HipDevice final : public bfs::Device {
public:
    HipDevice(bf_plan plan, bf_prec prec) : plan_(plan), prec_(prec) {}
    ~HipDevice() override
    {
        for (hipEvent_t e : spare_)
            (void)hipEventDestroy(e);
        for (int i = 0; i < n_streams_; ++i)
            (void)hipStreamDestroy(streams_[i]);
    }

    bf_status open(int n_streams, int max_items)
    {
        const bf_status rs = reserve_staging(plan_, max_items);
        if (rs != BF_OK)
            return rs;
        for (int i = 0; i < n_streams; ++i) {
            const hipError_t e = hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking);
            if (e != hipSuccess)
                return bf_fail(BF_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
            n_streams_ = i + 1;
        }
        return BF_OK;
    }

    int64_t now_ns() override { return bfs::monotonic_ns(); }

    bf_status launch(int stream, const std::vector<bfs::Req> &reqs, int n_items, void **token) override
    {
        hipEvent_t ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (!spare_.empty()) {
                ev = spare_.back();
                spare_.pop_back();
            }
        }
        if (!ev) {
            const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess)
                return bf_fail(BF_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
        // One record per request; the device expands them into items.
        recs_.clear();
        for (const bfs::Req &q : reqs)
            recs_.push_back(BfReqRec{static_cast<const float2 *>(q.r.f > 0 ? q.r.S : nullptr),
                                     static_cast<float2 *>(q.r.R), q.r.w_id, q.r.f, q.r.n_s, 0});
        const hipStream_t st = streams_[stream];
        bf_status rc = enqueue_requests(plan_, prec_, recs_, n_items, st);
        if (rc == BF_OK) {
            const hipError_t e = hipEventRecord(ev, st);
            if (e != hipSuccess)
                rc = bf_fail(BF_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
        }
        if (rc != BF_OK) {
            release(ev);
            return rc;
        }
        *token = ev;
        return BF_OK;
    }

    int done(void *token) override
    {
        const hipError_t e = hipEventQuery(static_cast<hipEvent_t>(token));
        if (e == hipErrorNotReady)
            return 0;
        return e == hipSuccess ? 1 : BF_ERR_DEVICE;
    }

    void release(void *token) override
    {
        std::lock_guard<std::mutex> lk(mu_);
        spare_.push_back(static_cast<hipEvent_t>(token));
    }

private:
    bf_plan plan_;
    bf_prec prec_;
    hipStream_t streams_[kMaxStreams] = {};
    int n_streams_ = 0;
    std::mutex mu_;                   // guards spare_ (launch and release run on different threads)
    std::vector<hipEvent_t> spare_;
    std::vector<BfReqRec> recs_;      // batcher thread only
};

}  // namespace

struct bf_server_s {
    HipDevice dev;
    bfs::Server *core = nullptr;
    bf_server_s(bf_plan plan, bf_prec prec) : dev(plan, prec) {}
};

extern "C" bf_status bf_server_create(bf_server *out, bf_plan plan, const bf_server_cfg *cfg_in)
{
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!plan)
        return bf_fail(BF_ERR_INVALID, "plan is null");
    bf_server_cfg cfg{};
    cfg.hbm_budget_bytes = 16ull << 30;
    cfg.deadline_us = 0;
    cfg.n_streams = 2;
    cfg.max_batch_items = 16384;
    cfg.queue_capacity = 65536;
    cfg.prec = BF_FP32;
    if (cfg_in)
        cfg = *cfg_in;
    if (cfg.n_streams < 1 || cfg.n_streams > kMaxStreams || cfg.max_batch_items < 1)
        return bf_fail(BF_ERR_INVALID,
                       "bad server config (budget > 0, 1..8 streams, max_batch_items >= 1, "
                       "queue_capacity a power of two >= 2)");
    if (cfg.prec < 0 || cfg.prec >= kPrecCount)
        return bf_fail(BF_ERR_INVALID, "unknown precision %d", cfg.prec);
    if (!(plan->mask & BF_PREC_BIT(cfg.prec)))
        return bf_fail(BF_ERR_UNSUPPORTED, "precision %d not prepared by the plan", cfg.prec);

    bf_server s = new (std::nothrow) bf_server_s(plan, (bf_prec)cfg.prec);
    if (!s)
        return bf_fail(BF_ERR_OOM, "server allocation");
    bf_status rc = s->dev.open(cfg.n_streams, cfg.max_batch_items);
    if (rc == BF_OK)
        rc = bfs::server_create(&s->core, &s->dev, cfg, plan->n_w, plan->f_max);
    if (rc != BF_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return BF_OK;
}

extern "C" bf_status bf_submit(bf_server s, const bf_request *req, uint64_t *ticket)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "null argument");
    return bfs::server_submit(s->core, req, ticket);
}

extern "C" int32_t bf_submit_batch(bf_server s, const bf_request *reqs, int32_t n, uint64_t *first_ticket)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "null argument");
    return bfs::server_submit_batch(s->core, reqs, n, first_ticket);
}

extern "C" int32_t bf_poll(bf_server s, bf_completion *out, int32_t max, int64_t timeout_us)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "bad bf_poll arguments");
    return bfs::server_poll(s->core, out, max, timeout_us);
}

extern "C" bf_status bf_server_stats_get(bf_server s, bf_server_stats *o)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "null argument");
    return bfs::server_stats(s->core, o);
}

extern "C" bf_status bf_server_destroy(bf_server s)
{
    if (!s)
        return bf_fail(BF_ERR_INVALID, "server is null");
    // (the loop drains and stops before the streams and events go)
    const bf_status rc = bfs::server_destroy(s->core);
    delete s;
    return rc;
}
