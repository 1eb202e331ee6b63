// Concurrency stress of the serving loop on the host executor (null device),
// built with ThreadSanitizer by tests/test_serve_stress.py.  The loop's own
// threads (batcher, completion) run against a submitter, a poller and a
// thread reading statistics; every scenario checks that each request
// completes exactly once, with the expected status, and that the budget
// held.  Exit status 0 on success, 1 on a failed check, 2 on a stall.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "bf_serve_host.h"

namespace {

uint64_t g_state = 0x9e3779b97f4a7c15ull;
uint64_t next_u64()
{
    // splitmix64
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
int uniform(int lo, int hi) { return lo + (int)(next_u64() % (uint64_t)(hi - lo + 1)); }

#define CHECK(cond, ...)                                                                   \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            fprintf(stderr, "check failed at line %d: %s: ", __LINE__, #cond);             \
            fprintf(stderr, __VA_ARGS__);                                                  \
            fprintf(stderr, "\n");                                                         \
            exit(1);                                                                       \
        }                                                                                  \
    } while (0)

constexpr int kM = BF_M, kB = BF_B;
constexpr size_t kBlockR = (size_t)kM * kB * 2;   // floats per R block

struct Scenario {
    const char *name;
    int n_req;
    int ns_max;
    int n_streams;
    int max_items;
    int queue;
    uint64_t budget;
    int64_t deadline_us;
    bool marks;               // distinct R per request, marks checked by the poller
    std::vector<int64_t> fail_at;
    int batch = 1;            // requests per submit call (> 1: bfh_submit_batch)
};

int run(const Scenario &sc)
{
    fprintf(stderr, "[stress] %s: %d requests\n", sc.name, sc.n_req);
    bfh_device_cfg dc{};
    dc.launch_ns = 3000;
    dc.bytes_per_ns = 4000.0;
    dc.write_marks = sc.marks ? 1 : 0;
    bfh_device dev = nullptr;
    CHECK(bfh_device_create(&dev, &dc) == BF_OK, "%s", bf_last_error());
    for (int64_t k : sc.fail_at)
        CHECK(bfh_device_fail_launch(dev, k, BF_ERR_DEVICE) == BF_OK, "%s", bf_last_error());

    // requests: S from a shared read-only arena; R distinct per request
    // (marks) or from a ring twice the budget (admitted requests never share)
    std::vector<bf_request> reqs((size_t)sc.n_req);
    size_t r_blocks = 0, s_need = 0;
    for (int i = 0; i < sc.n_req; ++i) {
        bf_request &r = reqs[(size_t)i];
        memset(&r, 0, sizeof r);
        r.w_id = uniform(0, 63);
        r.f = uniform(0, 36);
        r.n_s = uniform(1, sc.ns_max);
        r.tag = (uint64_t)i;
        r_blocks += (size_t)r.n_s;
        s_need = std::max(s_need, (size_t)r.f * r.n_s * kB * 2);
    }
    const size_t ring_blocks = sc.marks ? r_blocks : std::max<size_t>(2 * sc.budget / (kBlockR * 4) + 64, 64);
    std::vector<float> S(s_need + 2 * kB * 36 * 2 + 16, 1.0f);
    for (size_t k = 0; k < S.size(); ++k)
        S[k] = (float)(k % 1021);
    std::vector<float> R(ring_blocks * kBlockR + 4);
    float *R16 = reinterpret_cast<float *>((reinterpret_cast<uintptr_t>(R.data()) + 15) & ~uintptr_t(15));
    size_t pos = 0;
    std::vector<size_t> r_at((size_t)sc.n_req), s_at((size_t)sc.n_req);
    for (int i = 0; i < sc.n_req; ++i) {
        bf_request &r = reqs[(size_t)i];
        if (!sc.marks && pos + (size_t)r.n_s > ring_blocks)
            pos = 0;
        r_at[(size_t)i] = pos;
        r.R = R16 + pos * kBlockR;
        pos += (size_t)r.n_s;
        s_at[(size_t)i] = (size_t)uniform(0, 36 * kB) * 2;
        r.S = r.f > 0 ? S.data() + s_at[(size_t)i] : nullptr;
    }

    bf_server_cfg cfg{};
    cfg.hbm_budget_bytes = sc.budget;
    cfg.deadline_us = sc.deadline_us;
    cfg.n_streams = sc.n_streams;
    cfg.max_batch_items = sc.max_items;
    cfg.queue_capacity = sc.queue;
    cfg.prec = BF_FP32;
    bfh_server srv = nullptr;
    CHECK(bfh_server_create(&srv, dev, &cfg, 64, 36) == BF_OK, "%s", bf_last_error());

    std::vector<int> seen((size_t)sc.n_req, 0);
    std::vector<int> status((size_t)sc.n_req, 1);
    std::atomic<int> got{0};
    std::atomic<bool> stop{false};
    std::atomic<int> bad{0};
    std::thread poller([&] {
        bf_completion buf[128];
        auto last = std::chrono::steady_clock::now();
        while (got.load() < sc.n_req) {
            const int32_t k = bfh_poll(srv, buf, 128, 2000);
            if (k == BF_ERR_TIMEOUT) {
                if (std::chrono::steady_clock::now() - last > std::chrono::seconds(10)) {
                    fprintf(stderr, "[stress] %s: no completion for 10 s (%d of %d)\n", sc.name,
                            got.load(), sc.n_req);
                    bf_server_stats st{};
                    bfh_server_stats_get(srv, &st);
                    fprintf(stderr, "  submitted %llu admitted %llu completed %llu launches %llu "
                            "inflight %llu queued %llu unfinished %d\n",
                            (unsigned long long)st.submitted, (unsigned long long)st.admitted,
                            (unsigned long long)st.completed, (unsigned long long)st.launches,
                            (unsigned long long)st.inflight_bytes, (unsigned long long)st.queued,
                            bfh_device_unfinished(dev, -1));
                    fflush(stderr);
                    _Exit(2);
                }
                continue;
            }
            if (k < 0) {
                bad.store(1);
                return;
            }
            last = std::chrono::steady_clock::now();
            for (int j = 0; j < k; ++j) {
                const size_t i = (size_t)buf[j].tag;
                if (i >= (size_t)sc.n_req) {
                    bad.store(2);
                    continue;
                }
                seen[i] += 1;
                status[i] = buf[j].status;
                if (sc.marks && buf[j].status == BF_OK) {
                    const bf_request &r = reqs[i];
                    for (int b = 0; b < r.n_s; ++b) {
                        const float *blk = R16 + (r_at[i] + (size_t)b) * kBlockR;
                        const float *s0 = S.data() + s_at[i] + (size_t)b * r.f * kB * 2;
                        bool ok = blk[0] == (float)r.w_id && blk[1] == (float)r.f &&
                                  blk[kBlockR - 2] == (float)r.w_id && blk[kBlockR - 1] == (float)r.f;
                        if (r.f > 0)
                            ok = ok && blk[2] == s0[0] && blk[5] == s0[(size_t)r.f * kB * 2 - 1];
                        if (!ok)
                            bad.store(3);
                    }
                }
            }
            got.fetch_add(k);
        }
    });
    std::thread watcher([&] {
        while (!stop.load()) {
            bf_server_stats st{};
            if (bfh_server_stats_get(srv, &st) != BF_OK || st.inflight_bytes > sc.budget)
                bad.store(4);
            (void)bfh_device_unfinished(dev, -1);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });

    int busy = 0;
    uint64_t next_ticket = 1;
    for (int i = 0; i < sc.n_req;) {
        if (sc.batch > 1) {
            const int want = std::min(uniform(1, sc.batch), sc.n_req - i);
            uint64_t first = 0;
            const int32_t got = bfh_submit_batch(srv, &reqs[(size_t)i], want, &first);
            CHECK(got >= 0 && got <= want, "batch at %d: %d (%s)", i, got, bf_last_error());
            if (got == 0) {
                ++busy;
                std::this_thread::yield();
                continue;
            }
            CHECK(first == next_ticket, "tickets not consecutive at %d", i);
            next_ticket += (uint64_t)got;
            i += got;
        } else {
            for (;;) {
                const bf_status rc = bfh_submit(srv, &reqs[(size_t)i], nullptr);
                if (rc == BF_OK)
                    break;
                CHECK(rc == BF_ERR_BUSY, "submit %d: %s", i, bf_last_error());
                ++busy;
                std::this_thread::yield();
            }
            ++i;
        }
        if ((i & 255) == 0)
            std::this_thread::sleep_for(std::chrono::microseconds(uniform(0, 300)));
    }
    poller.join();
    bf_server_stats st{};
    CHECK(bfh_server_stats_get(srv, &st) == BF_OK, "%s", bf_last_error());
    stop.store(true);
    watcher.join();
    const bf_status drc = bfh_server_destroy(srv);
    CHECK(bad.load() == 0, "poller/watcher found problem %d", bad.load());
    CHECK(st.completed == (uint64_t)sc.n_req && st.submitted == (uint64_t)sc.n_req, "counts");
    CHECK(st.inflight_bytes == 0, "inflight %llu after all completions", (unsigned long long)st.inflight_bytes);
    CHECK(st.peak_inflight_bytes <= sc.budget, "peak over budget");
    int n_failed = 0;
    for (int i = 0; i < sc.n_req; ++i) {
        CHECK(seen[(size_t)i] == 1, "request %d completed %d times", i, seen[(size_t)i]);
        n_failed += status[(size_t)i] != BF_OK;
    }
    // the failed requests are exactly those of the launches made to fail
    std::vector<bfh_launch_rec> L((size_t)st.launches);
    const int64_t nl = bfh_device_launches(dev, L.data(), (int64_t)L.size());
    int expect_failed = 0;
    for (int64_t k : sc.fail_at)
        if (k < nl)
            expect_failed += L[(size_t)k].n_reqs;
    CHECK(n_failed == expect_failed, "%d failed, %d expected", n_failed, expect_failed);
    CHECK(drc == (expect_failed ? BF_ERR_DEVICE : BF_OK), "destroy returned %d", drc);
    for (int64_t k = 0; k < nl; ++k)
        CHECK(L[(size_t)k].n_items <= sc.max_items, "launch %lld has %d items", (long long)k,
              L[(size_t)k].n_items);
    CHECK(bfh_device_destroy(dev) == BF_OK, "%s", bf_last_error());
    fprintf(stderr, "[stress] %s ok: %lld launches, %d busy retries, %d failed\n", sc.name,
            (long long)nl, busy, n_failed);
    return 0;
}

}  // namespace

int main(int argc, char **argv)
{
    const int scale = argc > 1 ? atoi(argv[1]) : 1;
    const uint64_t MB = 1ull << 20;
    Scenario a{"mixed, 2 streams", 6000 * scale, 16, 2, 512, 1024, 256 * MB, 500, false, {}};
    Scenario b{"marks, 3 streams", 1500 * scale, 8, 3, 64, 256, 64 * MB, 0, true, {}};
    Scenario c{"small budget, small queue", 3000 * scale, 4, 2, 32, 8, 2 * MB, 500, false, {}};
    Scenario d{"failures", 2000 * scale, 8, 2, 64, 512, 32 * MB, 0, false, {3, 10, 11, 40}};
    Scenario e{"one stream, one item", 1000 * scale, 1, 1, 1, 64, 8 * MB, 200, true, {}};
    Scenario f{"batched submits, small queue", 4000 * scale, 16, 2, 256, 64, 64 * MB, 500, true, {}, 48};
    Scenario g{"batched submits, failures", 2000 * scale, 8, 3, 128, 256, 16 * MB, 0, false, {2, 7}, 200};
    for (const Scenario *s : {&a, &b, &c, &d, &e, &f, &g})
        if (run(*s) != 0)
            return 1;
    fprintf(stderr, "[stress] all scenarios ok\n");
    return 0;
}
