// Host side of libbf: the C ABI declared in include/bf.h.
//
// plan   : W pool upload and plan-time operand layouts (W is constant).
// apply  : all-or-nothing argument check, descriptor packing into a pinned
//          staging ring, one H2D copy and one kernel launch per batch.
// graph  : descriptors uploaded once, persistent kernel captured in a
//          hipGraph for replay.
// tuning : variant table per (precision, f bucket), autotuner, text cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bf_internal.h"
#include "bf_host.h"

// ---------------------------------------------------------------------------
// Argument checks (host only).

static inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
static inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

extern "C" bf_status bf_check_batch(int32_t n_w, int32_t f_max, int32_t batch,
                                    const int32_t *w_ids, const int32_t *f, const void *const *S,
                                    void *const *R)
{
    if (batch < 0)
        return bf_fail(BF_ERR_INVALID, "batch %d < 0", batch);
    if (batch == 0)
        return BF_OK;
    if (!w_ids || !f || !S || !R)
        return bf_fail(BF_ERR_INVALID, "null array argument");
    for (int32_t t = 0; t < batch; ++t) {
        if (w_ids[t] < 0 || w_ids[t] >= n_w)
            return bf_fail(BF_ERR_INVALID, "item %d: w_id %d outside [0, %d)", t, w_ids[t], n_w);
        if (f[t] < 0 || f[t] > f_max)
            return bf_fail(BF_ERR_INVALID, "item %d: f %d outside [0, %d]", t, f[t], f_max);
        if (!R[t] || !aligned16(R[t]))
            return bf_fail(BF_ERR_INVALID, "item %d: R pointer null or not 16-byte aligned", t);
        if (f[t] > 0 && (!S[t] || !aligned8(S[t])))
            return bf_fail(BF_ERR_INVALID, "item %d: S pointer null or not 8-byte aligned", t);
    }
    return BF_OK;
}

// ---------------------------------------------------------------------------
// Plan.

static void release_slot(StagingSlot &s)
{
    if (s.ev)
        (void)hipEventSynchronize(s.ev);
    if (s.host)
        (void)hipHostFree(s.host);
    if (s.sorted)
        (void)hipHostFree(s.sorted);
    if (s.dev)
        (void)hipFree(s.dev);
    if (s.ev)
        (void)hipEventDestroy(s.ev);
    if (s.copied)
        (void)hipEventDestroy(s.copied);
    s = StagingSlot{};
}

// Defaults measured on MI355X at steady state, with S not left in the
// memory-side cache by earlier launches.  Full-width batches (mean f 36) run
// the wave-specialised schedule: both FP32 forms on 16 x 16 tiles with the
// matrix-core waves copying W into LDS, the items sorted by W id (order 1;
// at one f it sorts by W only), so that a workgroup's consecutive products
// mostly share W and copy it once (three-product kernel 163.8-166.9 against
// 167.4-171.4 us in the caller's order; whole-job throughput the same or
// better, where order 3 lost 4% to per-step costs of the apply path; the
// four-product form, with S copied to LDS too, 187.3-189.7 us, against 222
// us for 32 x 32 tiles and 12 producers); the split 16-bit forms with 12
// producers (168 against 178 us for the streaming schedule on the gain
// workload).  Batches of mixed or smaller f: the FP32 forms run the same
// 16 x 16 kernels with W and S copied; the three-product form with the items
// grouped by W id modulo 8, so that each XCD's L2 holds an eighth of the
// pool (uneven batch, 8192 products, f ~ U{1..36}, 256 W: 69.0 against 77.4
// us for one product per workgroup, and serving capacity 3.54-3.57 M
// against 3.14-3.22 M requests/s; order 3 gains under 1% there), the
// four-product form dealt in W blocks (order 3: 81.0 against 85.1 us for
// order 2); the 16-bit forms, whose wave-specialised kernel takes one f per
// batch, run one product per workgroup, grouped by W id modulo 8, with
// staged R stores (FP16x2 74.4 us on the uneven batch).
static bf_status default_variants(bf_plan p)
{
    for (int pr = 0; pr < kPrecCount; ++pr)
        for (int b = 0; b < kBucketCount; ++b) {
            bf_variant v{};
            const bool full = b == kBucketCount - 1;
            const bool fp32 = pr == BF_FP32 || pr == BF_FP32_3M;
            if (!full && pr == BF_FP32_3M)
                v = bf_variant{3, 0, 2, 9};   // wave-specialised, 16 x 16 tiles, W and S copied
                                              // to LDS, grouped by W id mod 8
            else if (!full && fp32)
                v = bf_variant{3, 0, 3, 9};   // the same, dealt to the workgroups in W blocks
            else if (!full)
                v = bf_variant{0, 0, 2, 1};   // one per workgroup, grouped by W id mod 8, staged
            else if (pr == BF_FP32_3M)
                v = bf_variant{3, 0, 1, 8};   // wave-specialised, 16 x 16 tiles, W copied by the
                                              // matrix-core waves, depth 2, sorted by W id
            else if (fp32)
                v = bf_variant{3, 0, 1, 9};   // wave-specialised, 16 x 16 tiles, W copied by the
                                              // matrix-core waves and S by the producers, by W id
            else if (pr == BF_FP16 || pr == BF_BF16)
                v = bf_variant{3, 0, 0, 4};   // plain 16-bit: wave-specialised, 12 producers
            else
                v = bf_variant{3, 0, 0, 5};   // split 16-bit: wave-specialised, 12 producers, depth 2
            p->table[pr][b] = v;
        }
    return BF_OK;
}

static void read_env(bf_plan p);

extern "C" bf_status bf_plan_create(bf_plan *out, const void *w_pool, int32_t n_w, int32_t f_max,
                                    uint32_t prec_mask, void *hip_stream)
{
    HostRange range("bf_plan_create");
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!w_pool)
        return bf_fail(BF_ERR_INVALID, "w_pool is null");
    if (n_w < 1)
        return bf_fail(BF_ERR_INVALID, "n_w %d < 1", n_w);
    if (f_max < 0 || f_max > BF_FMAX)
        return bf_fail(BF_ERR_INVALID, "f_max %d outside [0, %d]", f_max, BF_FMAX);
    if (prec_mask == 0)
        prec_mask = BF_PREC_BIT(BF_FP32);
    if (prec_mask & ~BF_PREC_ALL)
        return bf_fail(BF_ERR_INVALID, "unknown precision bits 0x%x", prec_mask);
    if (prec_mask & ~kSupportedMask)
        return bf_fail(BF_ERR_UNSUPPORTED, "precision form not built in this library (mask 0x%x)",
                       prec_mask);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);

    bf_plan p = new (std::nothrow) bf_plan_s();
    if (!p)
        return bf_fail(BF_ERR_OOM, "plan allocation");
    p->n_w = n_w;
    p->f_max = f_max;
    p->mask = prec_mask;
    p->pairs = (f_max + 1) / 2;
    p->half.assign((size_t)n_w, 0);
    p->guard.assign((size_t)n_w, nullptr);
    default_variants(p);
    read_env(p);

    auto fail_dev = [&](const char *what, hipError_t e) {
        bf_status s = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? BF_ERR_OOM
                                                                                   : BF_ERR_DEVICE;
        bf_plan_destroy(p);
        return bf_fail(s, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess)
        return fail_dev("hipGetDevice", e);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess)
        return fail_dev("hipDeviceGetAttribute", e);
    p->n_cu = cus > 0 ? cus : 1;
    e = hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess)
        return fail_dev("hipStreamCreate(copy)", e);

    const size_t w_bytes = (size_t)n_w * BF_M * f_max * sizeof(float2);
    float2 *w_dev = nullptr;
    if (w_bytes) {
        e = hipMalloc(&w_dev, w_bytes);
        if (e != hipSuccess)
            return fail_dev("hipMalloc(W staging)", e);
        e = hipMemcpyAsync(w_dev, w_pool, w_bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            (void)hipFree(w_dev);
            return fail_dev("hipMemcpyAsync(W)", e);
        }
    }
    if (prec_mask & BF_PREC_BIT(BF_FP32)) {
        p->a_fp32_stride = bfk::fp32_w_stride(p->pairs);
        const size_t bytes = std::max<size_t>(1, 2 * (size_t)n_w * p->a_fp32_stride * sizeof(float2));
        e = hipMalloc(&p->a_fp32, bytes);
        if (e == hipSuccess && p->pairs > 0)
            e = bfk::launch_w_transform_fp32(w_dev, n_w, f_max, p->a_fp32, p->pairs, st);
        if (e != hipSuccess) {
            if (w_dev)
                (void)hipFree(w_dev);
            return fail_dev("FP32 W layout", e);
        }
    }
    // The three-product layout serves both FP32 forms: the 16 x 16 kernels
    // of the four-product form read its Wr and Wi as well.
    if (prec_mask & (BF_PREC_BIT(BF_FP32_3M) | BF_PREC_BIT(BF_FP32))) {
        p->a_3m_stride = bfk::fp32_3m_w_stride(p->pairs);
        const size_t bytes = std::max<size_t>(16, 2 * (size_t)n_w * p->a_3m_stride * sizeof(float));
        e = hipMalloc(&p->a_3m, bytes);
        if (e == hipSuccess && p->pairs > 0)
            e = bfk::launch_w_transform_3m(w_dev, n_w, f_max, p->a_3m, p->pairs, st);
        if (e != hipSuccess) {
            if (w_dev)
                (void)hipFree(w_dev);
            return fail_dev("three-product W layout", e);
        }
    }
    p->lp_stride = bfk::lp_w_units(f_max);
    for (int ty = 0; ty < 2; ++ty) {
        const bf_prec plain = ty == 0 ? BF_FP16 : BF_BF16;
        const bf_prec split = ty == 0 ? BF_FP16X2 : BF_BF16X2;
        const bool want = prec_mask & (BF_PREC_BIT(plain) | BF_PREC_BIT(split));
        if (!want)
            continue;
        const bool want_lo = prec_mask & BF_PREC_BIT(split);
        p->lp_split[ty] = want_lo;
        // the per-lane operand layout serves the plain form only
        if (prec_mask & BF_PREC_BIT(plain)) {
            const size_t bytes = std::max<size_t>(16, 2 * (size_t)n_w * p->lp_stride * 16);
            e = hipMalloc(&p->lp_hi[ty], bytes);
        }
        if (e == hipSuccess)
            e = hipMalloc(&p->lp_exp[ty], sizeof(int) * 2 * (size_t)n_w);
        p->lp_wc_stride[ty] = bfk::lp_wc_stride(want_lo);
        if (e == hipSuccess)
            e = hipMalloc(&p->lp_wc[ty], sizeof(uint32_t) * 2 * (size_t)n_w * p->lp_wc_stride[ty]);
        if (e == hipSuccess && w_dev)
            e = bfk::launch_w_transform_lp(w_dev, n_w, f_max, ty == 1, p->lp_hi[ty], p->lp_split[ty],
                                           p->lp_exp[ty], p->lp_wc[ty], st);
        if (e != hipSuccess) {
            if (w_dev)
                (void)hipFree(w_dev);
            return fail_dev("16-bit W layout", e);
        }
    }
    e = hipStreamSynchronize(st);
    if (w_dev)
        (void)hipFree(w_dev);
    if (e != hipSuccess)
        return fail_dev("hipStreamSynchronize(plan)", e);
    // Every staging slot gets its pinned and device blocks now: allocating
    // them on first use cost each of a fresh plan's first eight launches
    // about 0.2 ms.
    const bf_status rs = reserve_staging(p, kReserveItems);
    if (rs != BF_OK) {
        bf_plan_destroy(p);
        return rs;
    }
    // One upload per slot now: a slot's first upload took about 0.1 ms more
    // than later ones, which the first launches of a fresh plan paid.
    for (StagingSlot &slot : p->ring) {
        std::memset(slot.host, 0, slot.cap);
        std::memset(slot.sorted, 0, slot.sorted_cap);
        e = hipMemcpyAsync(slot.dev, slot.host, slot.cap, hipMemcpyHostToDevice, p->copy_stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot.dev, slot.sorted, slot.sorted_cap, hipMemcpyHostToDevice, p->copy_stream);
        if (e != hipSuccess)
            return fail_dev("hipMemcpyAsync(staging)", e);
    }
    e = hipStreamSynchronize(p->copy_stream);
    if (e != hipSuccess)
        return fail_dev("hipStreamSynchronize(staging)", e);
    if (!p->tune_cache.empty()) {
        if (FILE *fp = fopen(p->tune_cache.c_str(), "r")) {
            fclose(fp);
            if (bf_tune_load(p, p->tune_cache.c_str()) != BF_OK)
                fprintf(stderr, "[bf] BF_AUTOTUNE_CACHE %s not loaded: %s\n", p->tune_cache.c_str(),
                        bf_last_error());
        }
    }
    if (p->log)
        fprintf(stderr, "[bf] plan: %d W of 64 x %d, forms 0x%x, device %d (%d CUs)%s%s%s\n", n_w, f_max,
                prec_mask, p->device, p->n_cu, p->env_force_set ? ", BF_FORCE_VARIANT set" : "",
                p->tune_cache.empty() ? "" : ", tune cache ", p->tune_cache.c_str());
    *out = p;
    return BF_OK;
}

extern "C" bf_status bf_plan_destroy(bf_plan p)
{
    if (!p)
        return bf_fail(BF_ERR_INVALID, "plan is null");
    {
        std::lock_guard<std::mutex> lk(p->mu);
        for (auto &s : p->ring)
            release_slot(s);
    }
    if (p->a_fp32)
        (void)hipFree(p->a_fp32);
    if (p->a_3m)
        (void)hipFree(p->a_3m);
    for (int ty = 0; ty < 2; ++ty) {
        if (p->lp_hi[ty])
            (void)hipFree(p->lp_hi[ty]);
        if (p->lp_exp[ty])
            (void)hipFree(p->lp_exp[ty]);
        if (p->lp_wc[ty])
            (void)hipFree(p->lp_wc[ty]);
    }
    if (p->update_stream) {
        (void)hipStreamSynchronize(p->update_stream);
        (void)hipStreamDestroy(p->update_stream);
    }
    if (p->marker_stream) {
        (void)hipStreamSynchronize(p->marker_stream);
        (void)hipStreamDestroy(p->marker_stream);
    }
    for (hipEvent_t g : p->guard)
        if (g)
            (void)hipEventDestroy(g);
    if (p->updated)
        (void)hipEventDestroy(p->updated);
    if (p->stage_free)
        (void)hipEventDestroy(p->stage_free);
    if (p->w_stage)
        (void)hipFree(p->w_stage);
    if (p->w_pinned)
        (void)hipHostFree(p->w_pinned);
    if (p->copy_stream)
        (void)hipStreamDestroy(p->copy_stream);
    delete p;
    return BF_OK;
}

extern "C" bf_status bf_plan_info(bf_plan p, int32_t *n_w, int32_t *f_max, uint32_t *mask)
{
    if (!p)
        return bf_fail(BF_ERR_INVALID, "plan is null");
    if (n_w)
        *n_w = p->n_w;
    if (f_max)
        *f_max = p->f_max;
    if (mask)
        *mask = p->mask;
    return BF_OK;
}

extern "C" bf_status bf_plan_set_kernel_events(bf_plan p, void *start, void *stop)
{
    if (!p)
        return bf_fail(BF_ERR_INVALID, "plan is null");
    if ((start == nullptr) != (stop == nullptr))
        return bf_fail(BF_ERR_INVALID, "kernel events: give both or neither");
    std::lock_guard<std::mutex> lk(p->mu);
    p->kev_start = static_cast<hipEvent_t>(start);
    p->kev_stop = static_cast<hipEvent_t>(stop);
    return BF_OK;
}

extern "C" bf_status bf_plan_update(bf_plan p, int32_t w_id, const void *w, void *hip_stream)
{
    HostRange range("bf_plan_update");
    if (!p)
        return bf_fail(BF_ERR_INVALID, "plan is null");
    if (!w)
        return bf_fail(BF_ERR_INVALID, "w is null");
    if (w_id < 0 || w_id >= p->n_w)
        return bf_fail(BF_ERR_INVALID, "w_id %d outside [0, %d)", w_id, p->n_w);
    if (p->f_max == 0)
        return BF_OK;   // no flows: every product is the empty sum, W is never read
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lk(p->mu);
    const size_t w_bytes = (size_t)BF_M * p->f_max * sizeof(float2);
    auto dev_fail = [&](const char *what, hipError_t e) {
        return bf_fail(e == hipErrorOutOfMemory ? BF_ERR_OOM : BF_ERR_DEVICE, "%s: %s", what,
                       hipGetErrorString(e));
    };
    hipError_t e = hipSuccess;
    if (!p->update_stream) {
        e = hipStreamCreateWithFlags(&p->update_stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&p->marker_stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&p->updated, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&p->stage_free, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc(&p->w_pinned, w_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc(&p->w_stage, w_bytes);
        if (e == hipSuccess)
            e = hipEventRecord(p->stage_free, p->update_stream);
        if (e != hipSuccess)
            return dev_fail("update resources", e);
    }
    // The pinned buffer is free once the previous update's upload is done.
    e = hipEventSynchronize(p->stage_free);
    if (e != hipSuccess)
        return dev_fail("hipEventSynchronize(update staging)", e);
    std::memcpy(p->w_pinned, w, w_bytes);

    const int next = 1 - (int)p->half[(size_t)w_id];
    const size_t slot = (size_t)w_id + (size_t)p->n_w * next;
    // The slot being written was current before this entry's previous update:
    // launches issued before that update may still read it.
    if (p->guard[(size_t)w_id])
        e = hipStreamWaitEvent(p->update_stream, p->guard[(size_t)w_id], 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->w_stage, p->w_pinned, w_bytes, hipMemcpyHostToDevice, p->update_stream);
    if (e == hipSuccess)
        e = hipEventRecord(p->stage_free, p->update_stream);
    if (e == hipSuccess && p->a_fp32)
        e = bfk::launch_w_transform_fp32(p->w_stage, 1, p->f_max, p->a_fp32 + slot * p->a_fp32_stride,
                                         p->pairs, p->update_stream);
    if (e == hipSuccess && p->a_3m)
        e = bfk::launch_w_transform_3m(p->w_stage, 1, p->f_max, p->a_3m + slot * p->a_3m_stride,
                                       p->pairs, p->update_stream);
    for (int ty = 0; ty < 2 && e == hipSuccess; ++ty) {
        if (!p->lp_wc[ty])
            continue;
        const size_t off = slot * p->lp_stride * 16;
        e = bfk::launch_w_transform_lp(p->w_stage, 1, p->f_max, ty == 1,
                                       p->lp_hi[ty] ? static_cast<char *>(p->lp_hi[ty]) + off : nullptr,
                                       p->lp_split[ty],
                                       p->lp_exp[ty] + slot, p->lp_wc[ty] + slot * p->lp_wc_stride[ty],
                                       p->update_stream);
    }
    if (e == hipSuccess)
        e = hipEventRecord(p->updated, p->update_stream);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(st, p->updated, 0);
    if (e != hipSuccess)
        return dev_fail("pool update", e);

    // Guard for this entry's next update: every launch issued so far.  A
    // staging slot is reused only after its previous launch finished, so the
    // launches not yet known to be done are the latest one of each slot.
    if (!p->guard[(size_t)w_id]) {
        e = hipEventCreateWithFlags(&p->guard[(size_t)w_id], hipEventDisableTiming);
        if (e != hipSuccess)
            return dev_fail("hipEventCreate(guard)", e);
    }
    for (const StagingSlot &s : p->ring)
        if (s.launched && e == hipSuccess)
            e = hipStreamWaitEvent(p->marker_stream, s.ev, 0);
    if (e == hipSuccess)
        e = hipEventRecord(p->guard[(size_t)w_id], p->marker_stream);
    if (e != hipSuccess)
        return dev_fail("update guard", e);
    p->half[(size_t)w_id] = (uint8_t)next;
    p->any_update = true;
    return BF_OK;
}

// ---------------------------------------------------------------------------
// Descriptor packing.

extern "C" int32_t bf_f_bucket(int32_t f)
{
    if (f <= 0)
        return 0;
    const int32_t b = f / 9;
    return b < kBucketCount ? b : kBucketCount - 1;
}

// Batches are keyed by their mean f (rounded): uniform full-width batches
// and uneven batches with the same largest f want different schedules.
int batch_bucket(int64_t sum_f, int n)
{
    if (n <= 0)
        return 0;
    return bf_f_bucket((int32_t)((sum_f + n / 2) / n));
}

bf_variant pick_variant(bf_plan p, bf_prec prec, int bucket, const bf_variant *force)
{
    if (force)
        return *force;
    if (p->env_force_set)
        return p->env_force;
    return p->table[prec][bucket];
}

static const char *const kPrecNames[kPrecCount] = {"fp32", "fp16", "bf16", "fp16x2", "bf16x2", "fp32_3m"};

void log_launch(bf_plan p, bf_prec prec, int n, const bfk::LaunchCfg &cfg, const bf_variant &v,
                const char *path)
{
    if (!p->log || p->tuning)
        return;
    char key[160];
    snprintf(key, sizeof key, "%s %s variant %d:%d:%d:%d -> schedule %d grid %d%s%s%s", path,
             kPrecNames[prec], v.schedule, v.wg_per_cu, v.order, v.store, cfg.schedule, cfg.grid,
             cfg.vec16 ? " vec16" : "", cfg.stage ? " staged" : "", cfg.tile16 ? " 16x16" : "");
    if (p->logged.insert(key).second)
        fprintf(stderr, "[bf] launch %s (first: %d items)\n", key, n);
}

// BF_FORCE_VARIANT, BF_AUTOTUNE_CACHE and BF_LOG, read when a plan is made.
static void read_env(bf_plan p)
{
    const char *lg = getenv("BF_LOG");
    p->log = lg && *lg && strcmp(lg, "0") != 0 ? 1 : 0;
    const char *fv = getenv("BF_FORCE_VARIANT");
    if (fv && *fv) {
        bf_variant v{};
        char tail = 0;
        const int got = sscanf(fv, "%d:%d:%d:%d%c", &v.schedule, &v.wg_per_cu, &v.order, &v.store, &tail);
        const bool ok = got == 4 && v.schedule >= 0 && v.schedule <= 3 && v.wg_per_cu >= 0 &&
                        v.wg_per_cu <= 64 && v.order >= 0 && v.order <= 4 && v.store >= 0 &&
                        v.store <= (v.schedule == 3 ? 9 : 1);
        if (ok) {
            p->env_force_set = true;
            p->env_force = v;
        } else {
            // (a bad setting must not go unnoticed, logging or not)
            fprintf(stderr, "[bf] BF_FORCE_VARIANT=\"%s\" ignored: expected schedule:wg_per_cu:order:store "
                    "within the ranges of bf_variant\n", fv);
        }
    }
    const char *tc = getenv("BF_AUTOTUNE_CACHE");
    if (tc && *tc)
        p->tune_cache = tc;
}

// Product orders of the variants (items carry pool W ids at this point):
//   1: longest f first, then by W id (counting sorts; stable);
//   2: grouped by W id modulo 8, caller order within each group.  The
//      kernels give each of the 8 XCDs one contiguous eighth of the item
//      list, so this lets each XCD's L2 hold the operands of an eighth of
//      the pool only;
//   3: grouped by W id modulo 8 and by W id within each group (one stable
//      counting sort), and given `deal` (ws_deal's table for the
//      wave-specialised schedule's grid) dealt to its workgroups in
//      contiguous blocks in the same pass, so that consecutive products of
//      a workgroup mostly share their W and copy it into LDS once;
//   4: grouped by W id modulo 8 and, given `balance` (the wave-specialised
//      schedule's tables), each XCD part's items ranked longest f first and
//      dealt by ws_balance_table, so that the workgroups' summed f match and
//      an XCD's workgroups are at different f at any moment.  One pass
//      counts, one places every item: p = its grouped position, x = the part
//      of p, r = its f rank within x (caller order among equal f).
// The sort key of order 3: W ids of one residue modulo 8 together, in
// increasing order within it.
static inline int order3_key(int w, int g8) { return (w % 8) * g8 + w / 8; }

// Order 4's tables for n items on a grid of G, rebuilt only when n or G
// change.
static const BalanceTable *balance_table(BalanceTable &t, int n, int G)
{
    if (t.n != n || t.g != G) {
        t.pos.resize((size_t)n);
        t.part.resize((size_t)n);
        ws_balance_table(t.pos.data(), n, G);
        ws_part_table(t.part.data(), n, G);
        t.n = n;
        t.g = G;
    }
    return &t;
}

// ws_deal's table for n items on a grid of G, rebuilt only when n or G
// change (a caller that launches batches of one size builds it once).
static const int *deal_table(DealTable &t, int n, int G)
{
    if (t.n != n || t.g != G) {
        t.pos.resize((size_t)n);
        ws_deal_table(t.pos.data(), n, G);
        t.n = n;
        t.g = G;
    }
    return t.pos.data();
}

void order_items(const BfItem *in, BfItem *out, int n, int n_w, std::vector<int> &scratch, int mode,
                 const int *deal, const BalanceTable *balance)
{
    if (mode == 4 && balance) {
        constexpr int kGroups = 8, kF = BF_FMAX + 1;
        const int X = balance->g < 8 ? std::max(balance->g, 1) : 8;   // parts of the schedule
        // scratch: [group cursors 8][rank cursors X x kF][part of each item n]
        scratch.assign((size_t)kGroups + (size_t)X * kF + (size_t)n, 0);
        int *gcur = scratch.data();
        int *rcur = gcur + kGroups;
        int *xs = rcur + (size_t)X * kF;
        for (int t = 0; t < n; ++t)
            gcur[in[t].w_id % kGroups]++;
        for (int g = 0, run = 0; g < kGroups; ++g) {
            const int c = gcur[g];
            gcur[g] = run;
            run += c;
        }
        for (int t = 0; t < n; ++t) {
            const int x = balance->part[(size_t)gcur[in[t].w_id % kGroups]++];
            xs[t] = x;
            rcur[(size_t)x * kF + (BF_FMAX - in[t].f)]++;
        }
        for (int x = 0, run = 0; x < X; ++x)
            for (int k = 0; k < kF; ++k) {
                const int c = rcur[(size_t)x * kF + k];
                rcur[(size_t)x * kF + k] = run;
                run += c;
            }
        for (int t = 0; t < n; ++t)
            out[balance->pos[(size_t)rcur[(size_t)xs[t] * kF + (BF_FMAX - in[t].f)]++]] = in[t];
        return;
    }
    if (mode == 4)
        mode = 2;   // (not wave-specialised: grouped only)
    if (mode == 3) {
        const int g8 = (n_w + 7) / 8;
        scratch.assign((size_t)8 * g8 + 1, 0);
        for (int t = 0; t < n; ++t)
            scratch[(size_t)order3_key(in[t].w_id, g8) + 1]++;
        for (int k = 0; k < 8 * g8; ++k)
            scratch[(size_t)k + 1] += scratch[(size_t)k];
        for (int t = 0; t < n; ++t) {
            const int s = scratch[(size_t)order3_key(in[t].w_id, g8)]++;
            out[deal ? deal[s] : s] = in[t];
        }
        return;
    }
    if (mode == 2) {
        constexpr int kGroups = 8;
        int cnt[kGroups + 1] = {0};
        for (int t = 0; t < n; ++t)
            cnt[in[t].w_id % kGroups + 1]++;
        for (int g = 0; g < kGroups; ++g)
            cnt[g + 1] += cnt[g];
        for (int t = 0; t < n; ++t)
            out[cnt[in[t].w_id % kGroups]++] = in[t];
        return;
    }
    // Mode 1: stable counting sort by W id, then by f descending.  With one
    // f in the batch the second pass is the identity, so the first writes
    // straight to out.  (in and out never overlap; the intermediate buffer
    // is kept across calls, so a hot loop does not allocate.)
    scratch.assign((size_t)n_w + 1, 0);
    bool one_f = true;
    for (int t = 0; t < n; ++t) {
        scratch[(size_t)in[t].w_id + 1]++;
        one_f = one_f && in[t].f == in[0].f;
    }
    for (int k = 0; k < n_w; ++k)
        scratch[(size_t)k + 1] += scratch[(size_t)k];
    if (one_f) {
        for (int t = 0; t < n; ++t)
            out[scratch[(size_t)in[t].w_id]++] = in[t];
        return;
    }
    static thread_local std::vector<BfItem> by_w;
    by_w.resize((size_t)n);
    for (int t = 0; t < n; ++t)
        by_w[(size_t)scratch[(size_t)in[t].w_id]++] = in[t];
    int cnt[BF_FMAX + 2] = {0};
    for (int t = 0; t < n; ++t)
        cnt[BF_FMAX - by_w[(size_t)t].f + 1]++;
    for (int k = 0; k <= BF_FMAX; ++k)
        cnt[k + 1] += cnt[k];
    for (int t = 0; t < n; ++t)
        out[cnt[BF_FMAX - by_w[(size_t)t].f]++] = by_w[(size_t)t];
}

bfk::LaunchCfg choose_launch(bf_plan p, bf_prec prec, int n, int max_f, bool vec16,
                             bool uniform_f, const bf_variant *force)
{
    const bf_variant v = force ? *force : p->table[prec][bf_f_bucket(max_f)];
    (void)max_f;
    bfk::LaunchCfg cfg{};
    cfg.prec = prec;
    cfg.schedule = v.schedule;
    const bool lp = prec != BF_FP32 && prec != BF_FP32_3M;
    if (prec == BF_FP32_3M && cfg.schedule != 0)
        cfg.schedule = 3;   // the three-product form runs one-per-workgroup or wave-specialised
    else if (lp && cfg.schedule == 1)
        cfg.schedule = 2;   // the 16-bit forms have no claim schedule
    cfg.vec16 = vec16;
    if (cfg.schedule == 3 && !vec16)   // its producers move S in 16-byte chunks only
        cfg.schedule = prec == BF_FP32_3M ? 0 : 2;
    // A pool without columns has no W operands: every product is the empty
    // sum.  The wave-specialised kernels load W unconditionally, so such
    // batches run the schedules whose W loads are guarded.
    if (cfg.schedule == 3 && p->f_max < 1)
        cfg.schedule = lp ? 2 : 0;
    // The 16-bit wave-specialised kernel runs only batches whose products
    // all have the same f.  A serving benchmark that launched it on batches
    // of mixed f (two streams, many small launches) was stopped after three
    // silent minutes and the record did not show whether the device had
    // hung; until that is settled such batches take the streaming schedule.
    if (cfg.schedule == 3 && lp && !uniform_f)
        cfg.schedule = 2;
    cfg.stage = cfg.schedule == 3 || prec == BF_FP32_3M || (v.store >= 1 && cfg.schedule != 1);
    // For schedule 3 the store field selects producer waves and prefetch
    // depth: 0 -> (4, 1), 1 -> (8, 1), 2 -> (8, 2), 3 -> (8, 3), 4 -> (12, 1),
    // 5 -> (12, 2).
    static const int kProducers[6] = {4, 8, 8, 8, 12, 12};
    static const int kDepths[6] = {1, 1, 2, 3, 1, 2};
    const int ws = (cfg.schedule == 3 && v.store >= 0 && v.store <= 5) ? v.store : 0;
    cfg.producers = kProducers[ws];
    cfg.depth = kDepths[ws];
    if (prec == BF_FP32_3M && cfg.producers > 8)
        cfg.producers = 8;   // its two accumulator sets leave registers for 12 waves only
    // Store fields 6 to 9 (both FP32 forms): 8 matrix-core waves on 16 x 16
    // tiles and 8 producers at prefetch depth 1 (6) or 2 (7); 8 adds the
    // matrix-core waves copying W into LDS themselves, 9 the producers
    // copying S the same way.  The 16-bit forms read them as 0.
    cfg.tile16 = (prec == BF_FP32_3M || prec == BF_FP32) && cfg.schedule == 3 && v.store >= 6;
    if (cfg.tile16) {
        cfg.producers = 8;
        cfg.depth = v.store >= 7 ? 2 : 1;
        cfg.w_dma = v.store >= 8;
        cfg.s_dma = v.store == 9;
    }
    if (v.schedule == 0) {
        cfg.grid = n;
    } else {
        const int occ = bfk::apply_occupancy(prec, cfg.schedule, vec16, cfg.stage);
        const int per_cu = v.wg_per_cu > 0 ? v.wg_per_cu : occ;
        const long g = (long)per_cu * p->n_cu;
        cfg.grid = (int)std::min<long>(g, n);
    }
    return cfg;
}

// Makes a staging slot ready for a block of `bytes`: waits for the launch
// that last read it, then grows it if needed.
static bf_status ensure_slot(StagingSlot &s, size_t bytes)
{
    if (s.ev) {
        hipError_t e = hipEventSynchronize(s.ev);
        if (e != hipSuccess)
            return bf_fail(BF_ERR_DEVICE, "hipEventSynchronize(staging): %s", hipGetErrorString(e));
    } else {
        // Both events only order work on this device (the upload before the
        // launch) and tell the host that the slot is free again; neither
        // publishes device memory to the host, so they skip the system-scope
        // fence (2.5 us less per launch).
        const unsigned flags = hipEventDisableTiming | hipEventDisableSystemFence;
        hipError_t e = hipEventCreateWithFlags(&s.ev, flags);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&s.copied, flags);
        if (e != hipSuccess)
            return bf_fail(BF_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    if (s.cap >= bytes)
        return BF_OK;
    size_t cap = std::max<size_t>(bytes, 64 * 1024);
    cap = std::max(cap, s.cap * 2);
    if (s.host)
        (void)hipHostFree(s.host);
    if (s.dev)
        (void)hipFree(s.dev);
    s.host = nullptr;
    s.dev = nullptr;
    s.cap = 0;
    if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess)
        return bf_fail(BF_ERR_OOM, "pinned staging of %zu bytes", cap);
    if (hipHostGetDevicePointer(&s.host_dev, s.host, 0) != hipSuccess) {
        (void)hipHostFree(s.host);
        s.host = nullptr;
        return bf_fail(BF_ERR_DEVICE, "device address of pinned staging");
    }
    if (hipMalloc(&s.dev, cap) != hipSuccess) {
        (void)hipHostFree(s.host);
        s.host = nullptr;
        return bf_fail(BF_ERR_OOM, "device staging of %zu bytes", cap);
    }
    s.cap = cap;
    return BF_OK;
}

// Gives every staging slot room for a block of n items up front, so that a
// hot loop never reallocates (a device free waits for the whole device).
bf_status reserve_staging(bf_plan p, int n)
{
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->ring.empty())
        p->ring.resize(kRingSlots);
    for (StagingSlot &slot : p->ring) {
        // (a serving launch of n items has at most n request records)
        bf_status s = ensure_slot(slot, block_bytes(n) + (size_t)n * sizeof(BfReqRec));
        if (s != BF_OK)
            return s;
        if (slot.sorted_cap < slot.cap) {   // where ordered blocks are written
            if (slot.sorted)
                (void)hipHostFree(slot.sorted);
            slot.sorted = nullptr;
            slot.sorted_cap = 0;
            if (hipHostMalloc(&slot.sorted, slot.cap, hipHostMallocDefault) != hipSuccess)
                return bf_fail(BF_ERR_OOM, "pinned staging of %zu bytes", slot.cap);
            slot.sorted_cap = slot.cap;
        }
    }
    return BF_OK;
}

// Descriptors name pool entries by W id until they are ordered; the kernels
// read the entry's current slot.  Caller holds p->mu.
static void map_slots(bf_plan p, BfItem *items, int n)
{
    if (!p->any_update)
        return;
    for (int t = 0; t < n; ++t)
        items[t].w_id += p->n_w * (int)p->half[(size_t)items[t].w_id];
}

// Uploads the descriptor block that `slot.host` holds (header, sink, n
// items filled in, with statistics fs) to the device block `dev_blk` and
// launches the apply kernel on st.  The upload runs on `copy_st`, which the
// launch waits for.  With `may_order` the variant's product order is
// applied (on host buffers of the plan).  Caller holds p->mu, and the
// slot's previous launch has finished.
static bf_status upload_and_launch(bf_plan p, bf_prec prec, int n, const FillStats &fs, StagingSlot &slot,
                                   void *dev_blk, hipStream_t copy_st, hipStream_t st, bool may_order,
                                   const bf_variant *force, int *grid_out)
{
    const size_t bytes = block_bytes(n);
    BfItem *items = reinterpret_cast<BfItem *>(static_cast<char *>(slot.host) + sizeof(BfHeader) +
                                               kSinkBytes);
    const bool uniform_f = fs.min_f == fs.max_f;
    bf_variant chosen = pick_variant(p, prec, batch_bucket(fs.sum_f, n), force);
    bfk::LaunchCfg cfg = choose_launch(p, prec, n, fs.max_f, fs.vec16, uniform_f, &chosen);
    // The ordered block goes to the slot's second pinned buffer (header
    // copied, items written in order there) and is uploaded from it: no copy
    // back into the first one.
    const void *upload = slot.host;
    if (chosen.order >= 1 && n > 1 && may_order) {
        if (slot.sorted_cap < bytes) {
            if (slot.sorted)
                (void)hipHostFree(slot.sorted);
            slot.sorted = nullptr;
            slot.sorted_cap = 0;
            if (hipHostMalloc(&slot.sorted, slot.cap, hipHostMallocDefault) != hipSuccess)
                return bf_fail(BF_ERR_OOM, "pinned staging of %zu bytes", slot.cap);
            slot.sorted_cap = slot.cap;
        }
        std::memcpy(slot.sorted, slot.host, sizeof(BfHeader));
        BfItem *dst = reinterpret_cast<BfItem *>(static_cast<char *>(slot.sorted) + sizeof(BfHeader) + kSinkBytes);
        const bool deal = chosen.order == 3 && cfg.schedule == 3;
        const bool bal = chosen.order == 4 && cfg.schedule == 3;
        order_items(items, dst, n, p->n_w, p->sort_scratch, chosen.order,
                    deal ? deal_table(p->deal, n, cfg.grid) : nullptr,
                    bal ? balance_table(p->balance, n, cfg.grid) : nullptr);
        items = dst;
        upload = slot.sorted;
    }
    cfg.ev_start = p->kev_start;
    cfg.ev_stop = p->kev_stop;
    log_launch(p, prec, n, cfg, chosen, "apply");
    if (grid_out)
        *grid_out = cfg.grid;
    map_slots(p, items, n);

    hipError_t e = hipMemcpyAsync(dev_blk, upload, bytes, hipMemcpyHostToDevice, copy_st);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "hipMemcpyAsync(descriptors): %s", hipGetErrorString(e));
    if (copy_st != st) {
        e = hipEventRecord(slot.copied, copy_st);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(st, slot.copied, 0);
        if (e != hipSuccess)
            return bf_fail(BF_ERR_DEVICE, "descriptor upload ordering: %s", hipGetErrorString(e));
    }
    if (p->any_update) {   // the W of updated entries must be in place
        e = hipStreamWaitEvent(st, p->updated, 0);
        if (e != hipSuccess)
            return bf_fail(BF_ERR_DEVICE, "update ordering: %s", hipGetErrorString(e));
    }
    e = launch_for_plan(p, cfg, static_cast<BfHeader *>(dev_blk), n, st);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    e = hipEventRecord(slot.ev, st);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    slot.launched = true;
    return BF_OK;
}

// Record-level form of order_items (mode 1: by W id, then f descending;
// mode 2: grouped by W id modulo 8; mode 3: grouped by W id modulo 8, by W
// id within a group, the dealing to workgroups left to the expansion
// kernel).  Every item of a record shares its W id and f, so the items come
// out in the order order_items gives them.
static void order_records(std::vector<BfReqRec> &recs, std::vector<BfReqRec> &tmp, int mode, int n_w)
{
    if (mode == 4)
        mode = 2;   // (a record's items stay together: grouped only)
    const size_t n = recs.size();
    tmp.resize(n);
    if (mode == 2) {
        constexpr int kGroups = 8;
        size_t cnt[kGroups + 1] = {0};
        for (const BfReqRec &q : recs)
            cnt[q.w_id % kGroups + 1]++;
        for (int g = 0; g < kGroups; ++g)
            cnt[g + 1] += cnt[g];
        for (const BfReqRec &q : recs)
            tmp[cnt[q.w_id % kGroups]++] = q;
        recs.swap(tmp);
        return;
    }
    if (mode == 3) {
        const int g8 = (n_w + 7) / 8;
        std::stable_sort(recs.begin(), recs.end(), [g8](const BfReqRec &a, const BfReqRec &b) {
            return order3_key(a.w_id, g8) < order3_key(b.w_id, g8);
        });
        return;
    }
    std::stable_sort(recs.begin(), recs.end(), [](const BfReqRec &a, const BfReqRec &b) {
        return a.f != b.f ? a.f > b.f : a.w_id < b.w_id;
    });
}

bf_status enqueue_requests(bf_plan p, bf_prec prec, std::vector<BfReqRec> &recs, int n_items,
                           hipStream_t st)
{
    HostRange range("bf_serve_launch");
    const int n_recs = (int)recs.size();
    if (n_items == 0)
        return BF_OK;
    FillStats fs{0, true, 0};
    for (const BfReqRec &q : recs) {
        fs.max_f = std::max(fs.max_f, (int)q.f);
        fs.min_f = std::min(fs.min_f, (int)q.f);
        fs.sum_f += (int64_t)q.f * q.n_s;
        // (block k starts k f 480 bytes after S, a multiple of 16)
        if (q.f > 0 && !aligned16(q.S))
            fs.vec16 = false;
    }
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->ring.empty())
        p->ring.resize(kRingSlots);
    StagingSlot &slot = p->ring[p->ring_next];
    p->ring_next = (p->ring_next + 1) % p->ring.size();
    const size_t rec_off = block_bytes(n_items);
    bf_status s = ensure_slot(slot, rec_off + (size_t)n_recs * sizeof(BfReqRec));
    if (s != BF_OK)
        return s;
    bf_variant chosen = pick_variant(p, prec, batch_bucket(fs.sum_f, n_items), nullptr);
    if (chosen.order >= 1 && n_recs > 1)
        order_records(recs, p->rec_tmp, chosen.order, p->n_w);
    bfk::LaunchCfg cfg = choose_launch(p, prec, n_items, fs.max_f, fs.vec16, fs.min_f == fs.max_f, &chosen);
    const int deal_grid = chosen.order == 3 && cfg.schedule == 3 ? cfg.grid : 0;
    cfg.ev_start = p->kev_start;
    cfg.ev_stop = p->kev_stop;
    log_launch(p, prec, n_items, cfg, chosen, "serve");
    BfReqRec *dst = reinterpret_cast<BfReqRec *>(static_cast<char *>(slot.host) + rec_off);
    int item0 = 0;
    for (int k = 0; k < n_recs; ++k) {
        dst[k] = recs[(size_t)k];
        dst[k].item0 = item0;
        item0 += recs[(size_t)k].n_s;
        if (p->any_update)   // the slot of the entry current now (see map_slots)
            dst[k].w_id += p->n_w * (int)p->half[(size_t)dst[k].w_id];
    }
    if (item0 != n_items)
        return bf_fail(BF_ERR_INVALID, "request records hold %d items, not %d", item0, n_items);
    // The expansion kernel reads the records straight from pinned host
    // memory (a few kilobytes: one request is 32 bytes however many S blocks
    // it has), so nothing is uploaded and the launch waits on no other
    // queue; the slot is not written again before slot.ev (after the apply
    // kernel) has completed.
    char *dev_blk = static_cast<char *>(slot.dev);
    hipError_t e = hipSuccess;
    if (p->any_update)
        e = hipStreamWaitEvent(st, p->updated, 0);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "update ordering: %s", hipGetErrorString(e));
    e = bfk::launch_expand(reinterpret_cast<const BfReqRec *>(static_cast<char *>(slot.host_dev) + rec_off),
                           n_recs, reinterpret_cast<BfHeader *>(dev_blk), n_items, deal_grid, st);
    if (e == hipSuccess)
        e = launch_for_plan(p, cfg, reinterpret_cast<BfHeader *>(dev_blk), n_items, st);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    e = hipEventRecord(slot.ev, st);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    slot.launched = true;
    return BF_OK;
}

// Common tail of bf_apply / bf_apply_packed / the serving batcher: items
// are already validated and written by `fill` into host memory.
bf_status enqueue_items(bf_plan p, bf_prec prec, int n, const FillFn &fill, hipStream_t st,
                        const bf_variant *force, int *grid_out)
{
    if (n == 0)
        return BF_OK;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->ring.empty())
        p->ring.resize(kRingSlots);
    StagingSlot &slot = p->ring[p->ring_next];
    p->ring_next = (p->ring_next + 1) % p->ring.size();
    bf_status s = ensure_slot(slot, block_bytes(n));
    if (s != BF_OK)
        return s;
    BfHeader *hdr = static_cast<BfHeader *>(slot.host);
    std::memset(hdr, 0, sizeof *hdr);
    hdr->n_items = (uint32_t)n;
    const FillStats fs = fill(reinterpret_cast<BfItem *>(static_cast<char *>(slot.host) + sizeof(BfHeader) +
                                                         kSinkBytes));
    // The slot's previous launch has finished (ensure_slot waited for it), so
    // the upload may run on the copy stream while the caller's stream is
    // still busy with earlier work; the launch waits only for the upload.
    return upload_and_launch(p, prec, n, fs, slot, slot.dev, p->copy_stream, st, true, force, grid_out);
}

hipError_t launch_for_plan(bf_plan p, const bfk::LaunchCfg &cfg, BfHeader *blk, int n,
                           hipStream_t st)
{
    bfk::PlanDev pd{};
    pd.a_fp32 = p->a_fp32;
    pd.a_fp32_stride = (int)p->a_fp32_stride;
    pd.pairs = p->pairs;
    pd.a_3m = p->a_3m;
    pd.a_3m_stride = (int)p->a_3m_stride;
    const int ty = (cfg.prec == BF_BF16 || cfg.prec == BF_BF16X2) ? 1 : 0;
    pd.lp_hi = p->lp_hi[ty];
    pd.lp_exp = p->lp_exp[ty];
    pd.lp_stride = (int)p->lp_stride;
    pd.lp_chunks = bfk::lp_chunks(p->f_max);
    pd.lp_wc = p->lp_wc[ty];
    pd.lp_wc_stride = (int)p->lp_wc_stride[ty];
    return bfk::launch_apply(cfg, blk, n, pd, st);
}

static bf_status check_plan_prec(bf_plan p, bf_prec prec)
{
    if (!p)
        return bf_fail(BF_ERR_INVALID, "plan is null");
    if ((int)prec < 0 || (int)prec >= kPrecCount)
        return bf_fail(BF_ERR_INVALID, "unknown precision %d", (int)prec);
    if (!(p->mask & BF_PREC_BIT(prec)))
        return bf_fail(BF_ERR_UNSUPPORTED, "precision %d not prepared by this plan", (int)prec);
    return BF_OK;
}

extern "C" bf_status bf_apply(bf_plan p, int32_t batch, const int32_t *w_ids, const int32_t *f,
                              const void *const *S, void *const *R, bf_prec prec, void *hip_stream)
{
    HostRange range("bf_apply");
    bf_status s = check_plan_prec(p, prec);
    if (s != BF_OK)
        return s;
    s = bf_check_batch(p->n_w, p->f_max, batch, w_ids, f, S, R);
    if (s != BF_OK || batch == 0)
        return s;
    FillFn fill = [&](BfItem *items) {
        FillStats fs{0, true, 0};
        for (int32_t t = 0; t < batch; ++t) {
            BfItem &it = items[t];
            it.S = static_cast<const float2 *>(S[t]);
            it.R = static_cast<float2 *>(R[t]);
            it.w_id = w_ids[t];
            it.f = f[t];
            it.pad0 = it.pad1 = 0;
            fs.max_f = std::max(fs.max_f, (int)f[t]);
            fs.min_f = std::min(fs.min_f, (int)f[t]);
            fs.sum_f += f[t];
            if (f[t] > 0 && !aligned16(S[t]))
                fs.vec16 = false;
        }
        return fs;
    };
    return enqueue_items(p, prec, batch, fill, static_cast<hipStream_t>(hip_stream), nullptr,
                         nullptr);
}

// ---------------------------------------------------------------------------
// bf_apply_noalloc: bf_apply with its descriptor block (header with the
// persistent kernels' counters, sink, items) in `scratch`, a fixed array of
// the library that each device holds until the process ends, instead of a
// staging slot's device block.  Host code reaches the array only through the
// device address looked up once per device (g_scratch_ptr): the array's own
// name is a host-side stand-in, not a device address.

constexpr size_t kScratchBytes = sizeof(BfHeader) + kSinkBytes + (size_t)BF_NOALLOC_MAX_ITEMS * sizeof(BfItem);
// (Referenced from host code, the array is emitted as a global symbol of
// the device code object, which the runtime resolves by name.  An explicit
// `used` attribute would keep it as a local symbol instead, which the
// runtime cannot find.)
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on device dev, which must be current.
static bf_status scratch_on(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return bf_fail(BF_ERR_UNSUPPORTED, "device %d beyond the %d this library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return bf_fail(BF_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BF_OK;
}

extern "C" bf_status bf_apply_noalloc(bf_plan p, int32_t batch, const int32_t *w_ids, const int32_t *f,
                                      const void *const *S, void *const *R, bf_prec prec, void *hip_stream)
{
    HostRange range("bf_apply_noalloc");
    bf_status s = check_plan_prec(p, prec);
    if (s != BF_OK)
        return s;
    if (batch > BF_NOALLOC_MAX_ITEMS)
        return bf_fail(BF_ERR_INVALID, "batch %d above the %d products bf_apply_noalloc holds", batch,
                       BF_NOALLOC_MAX_ITEMS);
    s = bf_check_batch(p->n_w, p->f_max, batch, w_ids, f, S, R);
    if (s != BF_OK || batch == 0)
        return s;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != p->device)
        return bf_fail(BF_ERR_INVALID, "current device %d is not the plan's device %d", dev, p->device);
    void *blk = nullptr;
    s = scratch_on(dev, &blk);
    if (s != BF_OK)
        return s;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);

    std::lock_guard<std::mutex> lk(p->mu);
    const size_t bytes = block_bytes(batch);
    if (p->ring.empty())
        return bf_fail(BF_ERR_DEVICE, "plan has no staging ring");
    StagingSlot &slot = p->ring[p->ring_next];
    // (every slot holds kReserveItems >= BF_NOALLOC_MAX_ITEMS items from plan creation on)
    if (slot.cap < bytes || !slot.ev || !slot.host)
        return bf_fail(BF_ERR_DEVICE, "staging slot below its reserve");
    p->ring_next = (p->ring_next + 1) % p->ring.size();
    e = hipEventSynchronize(slot.ev);   // the slot's previous launch is done with its host block
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "hipEventSynchronize(staging): %s", hipGetErrorString(e));
    BfHeader *hdr = static_cast<BfHeader *>(slot.host);
    std::memset(hdr, 0, sizeof *hdr);   // the kernels' counters start at zero
    hdr->n_items = (uint32_t)batch;
    BfItem *items = reinterpret_cast<BfItem *>(static_cast<char *>(slot.host) + sizeof(BfHeader) + kSinkBytes);
    FillStats fs{0, true, 0};
    for (int32_t t = 0; t < batch; ++t) {
        BfItem &it = items[t];
        it.S = static_cast<const float2 *>(S[t]);
        it.R = static_cast<float2 *>(R[t]);
        it.w_id = w_ids[t];
        it.f = f[t];
        it.pad0 = it.pad1 = 0;
        fs.max_f = std::max(fs.max_f, (int)f[t]);
        fs.min_f = std::min(fs.min_f, (int)f[t]);
        fs.sum_f += f[t];
        if (f[t] > 0 && !aligned16(S[t]))
            fs.vec16 = false;
    }
    // The upload is ordered on the caller's stream: the array is shared by
    // every call on this device, so it must not be overwritten while an
    // earlier call's kernel on that stream still reads it.
    return upload_and_launch(p, prec, batch, fs, slot, blk, st, st, false, nullptr, nullptr);
}

extern "C" bf_status bf_apply_packed(bf_plan p, int32_t batch, const int32_t *w_ids,
                                     const int32_t *f, const void *S_base, const int64_t *s_off,
                                     void *R_base, bf_prec prec, void *hip_stream)
{
    HostRange range("bf_apply_packed");
    bf_status s = check_plan_prec(p, prec);
    if (s != BF_OK)
        return s;
    if (batch < 0)
        return bf_fail(BF_ERR_INVALID, "batch %d < 0", batch);
    if (batch == 0)
        return BF_OK;
    if (!w_ids || !f || !s_off || !R_base)
        return bf_fail(BF_ERR_INVALID, "null argument");
    if (!aligned16(R_base) || (S_base && !aligned8(S_base)))
        return bf_fail(BF_ERR_INVALID, "R_base not 16-byte aligned or S_base not 8-byte aligned");
    for (int32_t t = 0; t < batch; ++t) {
        if (w_ids[t] < 0 || w_ids[t] >= p->n_w)
            return bf_fail(BF_ERR_INVALID, "item %d: w_id %d outside [0, %d)", t, w_ids[t], p->n_w);
        if (f[t] < 0 || f[t] > p->f_max)
            return bf_fail(BF_ERR_INVALID, "item %d: f %d outside [0, %d]", t, f[t], p->f_max);
        if (f[t] > 0 && (!S_base || s_off[t] < 0))
            return bf_fail(BF_ERR_INVALID, "item %d: S_base null or negative offset", t);
    }
    const float2 *sb = static_cast<const float2 *>(S_base);
    float2 *rb = static_cast<float2 *>(R_base);
    FillFn fill = [&](BfItem *items) {
        FillStats fs{0, aligned16(S_base) || !S_base, 0};
        for (int32_t t = 0; t < batch; ++t) {
            BfItem &it = items[t];
            it.S = f[t] > 0 ? sb + s_off[t] : nullptr;
            it.R = rb + (size_t)t * BF_M * BF_B;
            it.w_id = w_ids[t];
            it.f = f[t];
            it.pad0 = it.pad1 = 0;
            fs.max_f = std::max(fs.max_f, (int)f[t]);
            fs.min_f = std::min(fs.min_f, (int)f[t]);
            fs.sum_f += f[t];
            if (f[t] > 0 && (s_off[t] & 1))
                fs.vec16 = false;
        }
        return fs;
    };
    return enqueue_items(p, prec, batch, fill, static_cast<hipStream_t>(hip_stream), nullptr,
                         nullptr);
}

// ---------------------------------------------------------------------------
// Graphs.

// A fixed batch: its descriptor block, ordered and uploaded once, and the
// launch configuration chosen for it.  A replay is one kernel launch: no
// upload, no event, no hipGraphLaunch (whose extra queue packets cost about
// 5 us per launch against 0.4 us between two plain launches).
struct bf_graph_s {
    bf_plan plan = nullptr;
    void *blk = nullptr;
    bfk::LaunchCfg cfg{};
    int n = 0;
};

extern "C" bf_status bf_graph_create(bf_graph *out, bf_plan p, int32_t batch, const int32_t *w_ids,
                                     const int32_t *f, const void *const *S, void *const *R,
                                     bf_prec prec, void *hip_stream)
{
    HostRange range("bf_graph_create");
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    bf_status s = check_plan_prec(p, prec);
    if (s != BF_OK)
        return s;
    s = bf_check_batch(p->n_w, p->f_max, batch, w_ids, f, S, R);
    if (s != BF_OK)
        return s;
    if (batch == 0)
        return bf_fail(BF_ERR_INVALID, "a graph needs at least one item");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);

    std::vector<BfItem> raw((size_t)batch), items((size_t)batch);
    int max_f = 0, min_f = BF_FMAX + 1;
    int64_t sum_f = 0;
    bool vec16 = true;
    for (int32_t t = 0; t < batch; ++t) {
        raw[(size_t)t] = BfItem{static_cast<const float2 *>(S[t]), static_cast<float2 *>(R[t]),
                                w_ids[t], f[t], 0, 0};
        max_f = std::max(max_f, (int)f[t]);
        min_f = std::min(min_f, (int)f[t]);
        sum_f += f[t];
        if (f[t] > 0 && !aligned16(S[t]))
            vec16 = false;
    }
    std::vector<int> scratch;
    bf_variant v;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        v = pick_variant(p, prec, batch_bucket(sum_f, batch), nullptr);
    }
    bfk::LaunchCfg cfg = choose_launch(p, prec, batch, max_f, vec16, min_f == max_f, &v);
    DealTable dt;
    BalanceTable bt;
    if (v.order >= 1)
        order_items(raw.data(), items.data(), batch, p->n_w, scratch, v.order,
                    v.order == 3 && cfg.schedule == 3 ? deal_table(dt, batch, cfg.grid) : nullptr,
                    v.order == 4 && cfg.schedule == 3 ? balance_table(bt, batch, cfg.grid) : nullptr);
    else
        items = raw;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        log_launch(p, prec, batch, cfg, v, "graph");
    }

    bool after_update = false;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        map_slots(p, items.data(), batch);
        after_update = p->any_update;
    }
    if (after_update && hipStreamWaitEvent(st, p->updated, 0) != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "update ordering");

    bf_graph g = new (std::nothrow) bf_graph_s();
    if (!g)
        return bf_fail(BF_ERR_OOM, "graph allocation");
    g->plan = p;
    g->n = batch;
    const size_t bytes = block_bytes(batch);
    std::vector<unsigned char> host(bytes, 0);
    reinterpret_cast<BfHeader *>(host.data())->n_items = (uint32_t)batch;
    std::memcpy(host.data() + sizeof(BfHeader) + kSinkBytes, items.data(),
                (size_t)batch * sizeof(BfItem));
    g->cfg = cfg;
    hipError_t e = hipMalloc(&g->blk, bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->blk, host.data(), bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        bf_graph_destroy(g);
        return bf_fail(BF_ERR_DEVICE, "graph descriptors: %s", hipGetErrorString(e));
    }
    *out = g;
    return BF_OK;
}

extern "C" bf_status bf_graph_launch(bf_graph g, void *hip_stream)
{
    if (!g || !g->blk)
        return bf_fail(BF_ERR_INVALID, "graph is null");
    bfk::LaunchCfg cfg = g->cfg;
    {
        std::lock_guard<std::mutex> lk(g->plan->mu);
        cfg.ev_start = g->plan->kev_start;
        cfg.ev_stop = g->plan->kev_stop;
    }
    hipError_t e = launch_for_plan(g->plan, cfg, static_cast<BfHeader *>(g->blk), g->n,
                                   static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
    return BF_OK;
}

extern "C" bf_status bf_graph_destroy(bf_graph g)
{
    if (!g)
        return bf_fail(BF_ERR_INVALID, "graph is null");
    (void)hipDeviceSynchronize();
    if (g->blk)
        (void)hipFree(g->blk);
    delete g;
    return BF_OK;
}

// ---------------------------------------------------------------------------
// Variants and tuning.

static bool valid_variant(const bf_variant &v)
{
    return v.schedule >= 0 && v.schedule <= 3 && v.wg_per_cu >= 0 && v.wg_per_cu <= 64 &&
           v.order >= 0 && v.order <= 4 && v.store >= 0 && v.store <= (v.schedule == 3 ? 9 : 1);
}

extern "C" bf_status bf_set_variant(bf_plan p, bf_prec prec, int32_t bucket, const bf_variant *v)
{
    if (!p || !v)
        return bf_fail(BF_ERR_INVALID, "null argument");
    if ((int)prec < 0 || (int)prec >= kPrecCount || bucket < 0 || bucket >= kBucketCount)
        return bf_fail(BF_ERR_INVALID, "precision %d or bucket %d out of range", (int)prec, bucket);
    if (!valid_variant(*v))
        return bf_fail(BF_ERR_INVALID, "invalid variant");
    std::lock_guard<std::mutex> lk(p->mu);
    p->table[prec][bucket] = *v;
    return BF_OK;
}

extern "C" bf_status bf_get_variant(bf_plan p, bf_prec prec, int32_t bucket, bf_variant *v)
{
    if (!p || !v)
        return bf_fail(BF_ERR_INVALID, "null argument");
    if ((int)prec < 0 || (int)prec >= kPrecCount || bucket < 0 || bucket >= kBucketCount)
        return bf_fail(BF_ERR_INVALID, "precision %d or bucket %d out of range", (int)prec, bucket);
    std::lock_guard<std::mutex> lk(p->mu);
    *v = p->table[prec][bucket];
    return BF_OK;
}

extern "C" bf_status bf_autotune(bf_plan p, int32_t batch, const int32_t *w_ids, const int32_t *f,
                                 const void *const *S, void *const *R, bf_prec prec, int32_t reps,
                                 void *hip_stream, bf_variant *best, float *best_us)
{
    bf_status s = check_plan_prec(p, prec);
    if (s != BF_OK)
        return s;
    s = bf_check_batch(p->n_w, p->f_max, batch, w_ids, f, S, R);
    if (s != BF_OK)
        return s;
    if (batch == 0)
        return bf_fail(BF_ERR_INVALID, "cannot tune an empty batch");
    if (reps < 1)
        reps = 1;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int64_t sum_f = 0;
    int min_f = BF_FMAX + 1, max_f = 0;
    for (int32_t t = 0; t < batch; ++t) {
        sum_f += f[t];
        min_f = std::min(min_f, (int)f[t]);
        max_f = std::max(max_f, (int)f[t]);
    }
    const bool lp = prec != BF_FP32 && prec != BF_FP32_3M;

    std::vector<bf_variant> cands;
    for (int st = 0; st < 2; ++st)
        for (int o = 0; o < 4; ++o)
            cands.push_back(bf_variant{0, 0, o, st});
    const int per_cu[] = {1, 2, 3, 4, 6};
    for (int w : per_cu)
        cands.push_back(bf_variant{1, w, 1, 0});
    for (int st = 0; st < 2; ++st)
        for (int w : per_cu)
            for (int o = 0; o < 2; ++o)
                cands.push_back(bf_variant{2, w, o, st});
    // (the 16-bit wave-specialised kernel takes batches of one f only; store
    // fields 6 to 9 exist for the FP32 forms only)
    if (!lp || min_f == max_f)
        for (int o = 0; o < 5; ++o)
            for (int st = 0; st < (lp ? 6 : 10); ++st)
                cands.push_back(bf_variant{3, 0, o, st});

    // Each timed launch records its kernel's own start and end (the plan's
    // kernel events, set per launch), so the host's packing and upload and
    // the queue's gaps stay out of the comparison.  The caller's events are
    // put back afterwards.
    HostRange range("bf_autotune");
    std::vector<hipEvent_t> kev((size_t)2 * reps, nullptr);
    for (hipEvent_t &e : kev)
        if (hipEventCreate(&e) != hipSuccess) {
            s = bf_fail(BF_ERR_DEVICE, "hipEventCreate(autotune)");
            break;
        }
    hipEvent_t saved[2];
    {
        std::lock_guard<std::mutex> lk(p->mu);
        saved[0] = p->kev_start;
        saved[1] = p->kev_stop;
        p->kev_start = p->kev_stop = nullptr;
        p->tuning = true;
    }
    float best_t = 1e30f;
    bf_variant best_v = cands[0];
    for (size_t c = 0; c < cands.size() && s == BF_OK; ++c) {
        const bf_variant &v = cands[c];
        FillFn fill = [&](BfItem *items) {
            FillStats fs{0, true, 0};
            for (int32_t t = 0; t < batch; ++t) {
                items[t] = BfItem{static_cast<const float2 *>(S[t]), static_cast<float2 *>(R[t]),
                                  w_ids[t], f[t], 0, 0};
                fs.max_f = std::max(fs.max_f, (int)f[t]);
                fs.min_f = std::min(fs.min_f, (int)f[t]);
                fs.sum_f += f[t];
                if (f[t] > 0 && !aligned16(S[t]))
                    fs.vec16 = false;
            }
            return fs;
        };
        for (int w = 0; w < 2 && s == BF_OK; ++w)
            s = enqueue_items(p, prec, batch, fill, st, &v, nullptr);
        for (int r = 0; r < reps && s == BF_OK; ++r) {
            {
                std::lock_guard<std::mutex> lk(p->mu);
                p->kev_start = kev[(size_t)2 * r];
                p->kev_stop = kev[(size_t)2 * r + 1];
            }
            s = enqueue_items(p, prec, batch, fill, st, &v, nullptr);
        }
        {
            std::lock_guard<std::mutex> lk(p->mu);
            p->kev_start = p->kev_stop = nullptr;
        }
        if (s != BF_OK)
            break;
        if (hipStreamSynchronize(st) != hipSuccess) {
            s = bf_fail(BF_ERR_DEVICE, "hipStreamSynchronize(autotune)");
            break;
        }
        float total_ms = 0.f;
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, kev[(size_t)2 * r], kev[(size_t)2 * r + 1]);
            total_ms += ms;
        }
        const float us = total_ms * 1000.f / (float)reps;
        if (us < best_t) {
            best_t = us;
            best_v = v;
        }
    }
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->kev_start = saved[0];
        p->kev_stop = saved[1];
        p->tuning = false;
    }
    for (hipEvent_t e : kev)
        if (e)
            (void)hipEventDestroy(e);
    if (s != BF_OK)
        return s;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->table[prec][batch_bucket(sum_f, batch)] = best_v;
        p->tuned_us[prec][batch_bucket(sum_f, batch)] = best_t;
    }
    if (p->log)
        fprintf(stderr, "[bf] autotune %s bucket %d: %d:%d:%d:%d, %.2f us (%zu candidates)\n",
                kPrecNames[prec], batch_bucket(sum_f, batch), best_v.schedule, best_v.wg_per_cu,
                best_v.order, best_v.store, best_t, cands.size());
    if (!p->tune_cache.empty() && bf_tune_save(p, p->tune_cache.c_str()) != BF_OK)
        fprintf(stderr, "[bf] BF_AUTOTUNE_CACHE %s not written: %s\n", p->tune_cache.c_str(), bf_last_error());
    if (best)
        *best = best_v;
    if (best_us)
        *best_us = best_t;
    return BF_OK;
}

// Architecture key of the tuning database: the device's gfx name without
// feature suffixes (e.g. "gfx950").
static std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

namespace {
// One database entry: the best variant of a (precision form, f bucket) on
// one architecture and CU count, with its measured time (0: not measured).
struct TuneRow {
    std::string arch;
    int cus, prec, bucket;
    bf_variant v;
    float us;
};

// Parses a tuning file: v2 lines "arch cus prec bucket schedule wg_per_cu
// order store us", or v1 lines "prec bucket schedule wg_per_cu order store"
// (no architecture: they apply anywhere).  Returns false on a malformed line.
bool read_tune_file(const char *path, std::vector<TuneRow> &rows)
{
    FILE *fp = fopen(path, "r");
    if (!fp)
        return false;
    char line[256];
    bool ok = true;
    while (fgets(line, sizeof line, fp)) {
        if (line[0] == '#' || line[0] == '\n')
            continue;
        TuneRow r{};
        char arch[64] = {0};
        int sc = 0, w = 0, o = 0, st = 0;
        float us = 0.f;
        if (std::isalpha((unsigned char)line[0])) {
            if (sscanf(line, "%63s %d %d %d %d %d %d %d %f", arch, &r.cus, &r.prec, &r.bucket, &sc, &w, &o,
                       &st, &us) != 9) {
                ok = false;
                break;
            }
            r.arch = arch;
        } else {
            const int got = sscanf(line, "%d %d %d %d %d %d", &r.prec, &r.bucket, &sc, &w, &o, &st);
            if (got < 5) {
                ok = false;
                break;
            }
            r.cus = -1;   // v1: any device
        }
        r.v = bf_variant{sc, w, o, st};
        r.us = us;
        if (r.prec < 0 || r.prec >= kPrecCount || r.bucket < 0 || r.bucket >= kBucketCount ||
            !valid_variant(r.v)) {
            ok = false;
            break;
        }
        rows.push_back(r);
    }
    fclose(fp);
    return ok;
}
}  // namespace

extern "C" bf_status bf_tune_save(bf_plan p, const char *path)
{
    if (!p || !path)
        return bf_fail(BF_ERR_INVALID, "null argument");
    const std::string arch = arch_name();
    // Entries of other architectures or CU counts already in the file stay.
    std::vector<TuneRow> keep, old;
    if (read_tune_file(path, old))
        for (const TuneRow &r : old)
            if (r.cus >= 0 && !(r.arch == arch && r.cus == p->n_cu))
                keep.push_back(r);
    FILE *fp = fopen(path, "w");
    if (!fp)
        return bf_fail(BF_ERR_INVALID, "cannot open %s for writing", path);
    std::lock_guard<std::mutex> lk(p->mu);
    fprintf(fp, "# bf tune v2: the best variant per (architecture, CUs, precision form, f bucket)\n");
    fprintf(fp, "# arch cus prec bucket schedule wg_per_cu order store us\n");
    for (const TuneRow &r : keep)
        fprintf(fp, "%s %d %d %d %d %d %d %d %.2f\n", r.arch.c_str(), r.cus, r.prec, r.bucket,
                r.v.schedule, r.v.wg_per_cu, r.v.order, r.v.store, r.us);
    for (int pr = 0; pr < kPrecCount; ++pr)
        for (int b = 0; b < kBucketCount; ++b) {
            const bf_variant &v = p->table[pr][b];
            fprintf(fp, "%s %d %d %d %d %d %d %d %.2f\n", arch.c_str(), p->n_cu, pr, b, v.schedule,
                    v.wg_per_cu, v.order, v.store, p->tuned_us[pr][b]);
        }
    fclose(fp);
    return BF_OK;
}

extern "C" bf_status bf_tune_load(bf_plan p, const char *path)
{
    if (!p || !path)
        return bf_fail(BF_ERR_INVALID, "null argument");
    std::vector<TuneRow> rows;
    if (!read_tune_file(path, rows))
        return bf_fail(BF_ERR_INVALID, "cannot read or malformed tune file %s", path);
    const std::string arch = arch_name();
    std::lock_guard<std::mutex> lk(p->mu);
    for (const TuneRow &r : rows)
        if (r.cus < 0 || (r.arch == arch && r.cus == p->n_cu)) {
            p->table[r.prec][r.bucket] = r.v;
            p->tuned_us[r.prec][r.bucket] = r.us;
        }
    return BF_OK;
}

extern "C" bf_status bf_tune_query(bf_plan p, bf_prec prec, int32_t f, bf_variant *v, float *tuned_us)
{
    if (!p || !v)
        return bf_fail(BF_ERR_INVALID, "null argument");
    if ((int)prec < 0 || (int)prec >= kPrecCount || f < 0 || f > BF_FMAX)
        return bf_fail(BF_ERR_INVALID, "precision %d or f %d out of range", (int)prec, f);
    std::lock_guard<std::mutex> lk(p->mu);
    const int b = bf_f_bucket(f);
    *v = p->table[prec][b];
    if (tuned_us)
        *tuned_us = p->tuned_us[prec][b];
    return BF_OK;
}

// ---------------------------------------------------------------------------
// Diagnostics.

extern "C" const char *bf_build_info(void)
{
    return "libbf gfx950 hip-" BF_STRINGIFY(HIP_VERSION_MAJOR) "." BF_STRINGIFY(HIP_VERSION_MINOR)
           " fp32-mfma fp32-3m fp16/bf16-mfma split";
}

extern "C" int32_t bf_device_cu_count(void)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "device query: %s", hipGetErrorString(e));
    return cus;
}
