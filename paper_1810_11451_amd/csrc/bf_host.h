// Host-side internals of libbf (plan object, staging ring, helpers).
#pragma once

#include <hip/hip_runtime.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <functional>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "bf_internal.h"
#include "bf_status.h"

#define BF_STRINGIFY2(x) #x
#define BF_STRINGIFY(x) BF_STRINGIFY2(x)

constexpr int kPrecCount = 6;
constexpr int kBucketCount = 5;
constexpr int kRingSlots = 8;
// Items per descriptor block that every staging slot holds from plan creation.
constexpr int kReserveItems = 16384;
static_assert(kReserveItems >= BF_NOALLOC_MAX_ITEMS, "staging reserve covers bf_apply_noalloc");
constexpr uint32_t kSupportedMask = BF_PREC_ALL;

// One slot of the descriptor staging ring: a pinned host block, its device
// copy, an event recorded on the plan's copy stream after the upload, and
// an event recorded on the caller's stream after the launch that reads it.
struct StagingSlot {
    void *host = nullptr;
    void *host_dev = nullptr;   // host's device-side address (kernels read records there)
    void *dev = nullptr;
    size_t cap = 0;
    void *sorted = nullptr;     // pinned block the ordered items are written to and uploaded from
    size_t sorted_cap = 0;
    hipEvent_t copied = nullptr;
    hipEvent_t ev = nullptr;
    bool launched = false;   // ev has been recorded after a launch
};

// ws_deal as a table on the host: pos[i] = ws_deal(i, n, G) for every i,
// walking the parts and workgroup blocks with running offsets instead of
// ws_deal's divisions per item.
inline void ws_deal_table(int *pos, int n, int G)
{
    const int X = G < 8 ? G : 8;
    if (X <= 0) {
        for (int i = 0; i < n; ++i)
            pos[i] = i;
        return;
    }
    const int q = n / X, r = n % X;
    int i = 0;
    for (int x = 0; x < X; ++x) {
        const int lo = x * q + (x < r ? x : r);
        const int cnt = q + (x < r ? 1 : 0);
        const int nb = G / X + (x < G % X ? 1 : 0);
        const int a = cnt / nb, b = cnt % nb;
        for (int j = 0; j < nb; ++j) {
            const int nj = a + (j < b ? 1 : 0);
            for (int k = 0; k < nj; ++k)
                pos[i++] = lo + j + k * nb;
        }
    }
}

// Balanced dealing (product order 4) as a table on the host: for the
// items of each of the wave-specialised schedule's parts (one per XCD,
// positions lo .. lo + cnt - 1, nb workgroups), ranked r = 0 .. cnt - 1
// longest f first, pos[lo + r] is the position rank r goes to.  Ranks are
// dealt in rounds of nb, alternately forwards and backwards over the
// workgroups (so each workgroup's summed f comes out close to the mean; a
// short last round goes to the workgroups that take one product more),
// and each workgroup j takes its round-ordered products starting at round
// (j n_j) / nb, so that at any moment the workgroups of an XCD are at
// different f.  The layout of each workgroup's share is ws_share's (lo + j
// + k nb).  Depends only on n and G.
inline void ws_balance_table(int *pos, int n, int G)
{
    const int X = G < 8 ? G : 8;
    if (X <= 0) {
        for (int i = 0; i < n; ++i)
            pos[i] = i;
        return;
    }
    const int q = n / X, r = n % X;
    for (int x = 0; x < X; ++x) {
        const int lo = x * q + (x < r ? x : r);
        const int cnt = q + (x < r ? 1 : 0);
        const int nb = G / X + (x < G % X ? 1 : 0);
        const int a = cnt / nb, b = cnt % nb;
        for (int s = 0; s < cnt; ++s) {
            const int rnd = s / nb, u = s % nb;
            const int j = rnd < a ? ((rnd & 1) ? nb - 1 - u : u) : u;
            const int nj = a + (j < b ? 1 : 0);
            const int k = (rnd + (int)((long)j * nj / nb)) % nj;
            pos[lo + s] = lo + j + k * nb;
        }
    }
}

// Part (XCD share) of each position of the wave-specialised schedule's item
// list: part[p] = x for lo_x <= p < lo_x + cnt_x.
inline void ws_part_table(int *part, int n, int G)
{
    const int X = G < 8 ? G : 8;
    if (X <= 0) {
        for (int i = 0; i < n; ++i)
            part[i] = 0;
        return;
    }
    const int q = n / X, r = n % X;
    int p = 0;
    for (int x = 0; x < X; ++x) {
        const int cnt = q + (x < r ? 1 : 0);
        for (int c = 0; c < cnt; ++c)
            part[p++] = x;
    }
}

// Dealt positions of order 3 (ws_deal) for n items on a grid of g; for
// order 4 the balanced positions by rank (ws_balance_table) and the part of
// each position (ws_part_table).
struct DealTable {
    int n = -1, g = -1;
    std::vector<int> pos;
};
struct BalanceTable {
    int n = -1, g = -1;
    std::vector<int> pos, part;
};

struct bf_plan_s {
    int device = 0;
    int n_cu = 1;
    int n_w = 0;
    int f_max = 0;
    int pairs = 0;
    uint32_t mask = 0;

    float2 *a_fp32 = nullptr;   // FP32 operand layout, a_fp32_stride float2 per W
    size_t a_fp32_stride = 0;
    float *a_3m = nullptr;      // FP32 three-product layout, a_3m_stride floats per W
    size_t a_3m_stride = 0;
    // 16-bit operand layouts, index 0 = FP16, 1 = BF16 (lo only for split forms)
    void *lp_hi[2] = {nullptr, nullptr};
    bool lp_split[2] = {false, false};   // compact layout holds the lo part
    int *lp_exp[2] = {nullptr, nullptr};
    uint32_t *lp_wc[2] = {nullptr, nullptr};   // compact 16-bit W (wave-specialised schedule)
    size_t lp_wc_stride[2] = {0, 0};           // dwords per W
    size_t lp_stride = 0;       // 16-byte units per W

    // Pool updates.  Every entry has two device slots, w and w + n_w, in each
    // operand layout; half[w] says which one is current.  Launches read the
    // slot that was current when they were enqueued (descriptors carry slot
    // numbers).  An update writes the other slot on update_stream, which
    // first waits for guard[w]: an event on marker_stream that completes
    // when every launch issued before the entry's previous update has.
    std::vector<uint8_t> half;
    std::vector<hipEvent_t> guard;
    hipStream_t update_stream = nullptr;
    hipStream_t marker_stream = nullptr;
    hipEvent_t updated = nullptr;        // after the latest update's transforms
    hipEvent_t stage_free = nullptr;     // after the latest update's upload of its W
    void *w_pinned = nullptr;            // one W, pinned host memory
    float2 *w_stage = nullptr;           // one W, device memory
    bool any_update = false;

    hipStream_t copy_stream = nullptr;   // descriptor uploads (overlap the previous launch)
    std::mutex mu;              // guards the ring, the tables, the sort buffers, kev_* and logged
    hipEvent_t kev_start = nullptr;   // kernel timing events (bf_plan_set_kernel_events)
    hipEvent_t kev_stop = nullptr;

    // Environment at creation (include/bf.h, "Environment").
    bool env_force_set = false;  // BF_FORCE_VARIANT
    bf_variant env_force{};
    std::string tune_cache;      // BF_AUTOTUNE_CACHE
    int log = 0;                 // BF_LOG
    bool tuning = false;         // bf_autotune is running (its launches are not logged)
    std::set<std::string> logged;   // launch configurations already logged
    std::vector<StagingSlot> ring;
    size_t ring_next = 0;
    bf_variant table[kPrecCount][kBucketCount];
    float tuned_us[kPrecCount][kBucketCount] = {};   // measured by autotune or loaded; 0: default
    std::vector<BfReqRec> rec_tmp;
    std::vector<int> sort_scratch;
    DealTable deal;
    BalanceTable balance;
};

struct FillStats {
    int max_f;
    bool vec16;
    int64_t sum_f;
    int min_f = BF_FMAX + 1;   // smallest f (above BF_FMAX for an empty batch)
};
// Tuning-table bucket of a batch: bf_f_bucket of its mean f, rounded.
int batch_bucket(int64_t sum_f, int n);
// The variant a launch of the plan takes: the caller's, else BF_FORCE_VARIANT,
// else the plan's table.  Caller holds p->mu.
bf_variant pick_variant(bf_plan p, bf_prec prec, int bucket, const bf_variant *force);
// With BF_LOG set, one stderr line for each launch configuration the first
// time the plan launches it.  Caller holds p->mu.
void log_launch(bf_plan p, bf_prec prec, int n, const bfk::LaunchCfg &cfg, const bf_variant &v,
                const char *path);

// A roctx range over a host-side phase (shown by rocprofv3 --marker-trace).
class HostRange {
public:
    explicit HostRange(const char *name) { roctxRangePushA(name); }
    ~HostRange() { roctxRangePop(); }
    HostRange(const HostRange &) = delete;
    HostRange &operator=(const HostRange &) = delete;
};
using FillFn = std::function<FillStats(BfItem *)>;

void order_items(const BfItem *in, BfItem *out, int n, int n_w, std::vector<int> &scratch, int mode,
                 const int *deal = nullptr, const BalanceTable *balance = nullptr);
bfk::LaunchCfg choose_launch(bf_plan p, bf_prec prec, int n, int max_f, bool vec16,
                             bool uniform_f, const bf_variant *force);
bf_status reserve_staging(bf_plan p, int n);
// Serving launches: one record per request (S, R, w_id, f, n_s; item0 is
// set here), n_items the sum of their n_s.  The records are put in the
// product order of the plan's variant for the batch (in place), written to
// pinned staging and expanded into items on the device ahead of the apply
// kernel, so the host's work grows with the requests, not with their S
// blocks.
bf_status enqueue_requests(bf_plan p, bf_prec prec, std::vector<BfReqRec> &recs, int n_items,
                           hipStream_t st);
bf_status enqueue_items(bf_plan p, bf_prec prec, int n, const FillFn &fill, hipStream_t st,
                        const bf_variant *force, int *grid_out);
hipError_t launch_for_plan(bf_plan p, const bfk::LaunchCfg &cfg, BfHeader *blk, int n,
                           hipStream_t st);
