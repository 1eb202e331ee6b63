#!/usr/bin/env python3
"""Benchmark: batched beamforming R = W x S on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload full-width] [--prec fp32_3m]

A step is one bf_apply over the whole batch (descriptor packing and upload,
one kernel launch), with S already resident in HBM.  Before the --warmup
steps the path runs for --settle-ms of wall time, so that the device has
raised its clock as it does under continuous load.  The default workload
is the full-width batch: 16384 products of 64x36 by 36x60 complex64, W from
a pool of 64 unit-norm precoders, S normalised 256-QAM.  Three disjoint
S/R buffer sets (2.4 GB) rotate so that the 256 MB last-level cache cannot
serve repeated reads.

Prints one JSON line: whole-job complex GFLOP/s (8 real flops per complex
multiply-add, 8*64*60*f per product), the roofline of the apply kernel
(kernel time from HIP events on the launch stream, algorithmic flops or
bytes per launch), and the FP64 oracle timed on the host on a bounded
sample of the same workload.  The default line also carries the uneven
batch, the gain workload in the four 16-bit forms, and the serving
workload (closed-loop capacity, p50/p99 at half of it); --no-compare
leaves all of these out, --no-serving only the serving workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

from paper_1810_11451_amd import bf  # noqa: E402
from paper_1810_11451_amd import workloads as wl  # noqa: E402

METRIC = "complex GFLOP/s + %roofline for batched 64×f·f×60 beamforming; p50/p99 latency"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_LP_TFLOPS = 2500.0
PRECS = {"fp32": bf.BF_FP32, "fp32_3m": bf.BF_FP32_3M, "fp16": bf.BF_FP16, "bf16": bf.BF_BF16,
         "fp16x2": bf.BF_FP16X2, "bf16x2": bf.BF_BF16X2}
# Workloads: batches of products (generator), the serving replay and the
# filter stage (None: handled apart).
WORKLOADS = {"single-w": wl.single_w_batch, "full-width": wl.full_width_batch,
             "uneven": wl.uneven_batch, "gain": wl.gain_batch, "serving": None, "filter": None}
FILTER_METRIC = "blocks/s + %roofline for the batched 2048-point FFT -> MULT -> IFFT filter stage"
from paper_1810_11451_amd.probe.traffic import kernel_sha  # noqa: E402


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(batch, target_s: float) -> dict:
    """The FP64 oracle (as it stands) on a bounded sample of the workload:
    seeded products of the same batch, repeated until about target_s."""
    from oracle import oracle as orc
    threads = host_threads()
    rng = np.random.default_rng(12345)
    probe = rng.choice(batch.n, size=min(batch.n, 8 * threads), replace=False)
    t0 = time.perf_counter()
    orc.apply(batch, items=probe, threads=threads)
    dt = max(time.perf_counter() - t0, 1e-6)
    n = int(min(batch.n, max(len(probe), len(probe) * target_s / dt)))
    items = rng.choice(batch.n, size=n, replace=False)
    reps, t0 = 0, time.perf_counter()
    while True:
        orc.apply(batch, items=items, threads=threads)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= target_s:
            break
    flops = reps * 8 * wl.M * wl.B * int(np.sum(batch.f[items].astype(np.int64)))
    return {"value": round(flops / dt / 1e9, 3), "unit": "complex GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} of the {batch.n} products of the same workload (seeded choice), "
                      f"x{reps} passes, C FP64 triple loop, {dt:.1f} s"}


def cpu_extra(batch, target_s: float) -> dict:
    """Second CPU data points on bounded samples: the C oracle on one core
    and the oracle's numpy rendering (complex128), each about target_s."""
    from oracle import oracle as orc
    rng = np.random.default_rng(54321)
    out = {}
    for name, fn in (("c_oracle_one_core", lambda it: orc.apply(batch, items=it, threads=1)),
                     ("numpy_oracle_one_core", lambda it: [orc.apply_numpy(batch.w_block(int(t)),
                                                                           batch.s_block(int(t)))
                                                          for t in it])):
        items = rng.choice(batch.n, size=min(batch.n, 64), replace=False)
        reps, t0 = 0, time.perf_counter()
        while True:
            fn(items)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= target_s:
                break
        flops = reps * 8 * wl.M * wl.B * int(np.sum(batch.f[items].astype(np.int64)))
        out[name] = {"value": round(flops / dt / 1e9, 3), "unit": "complex GFLOP/s", "cores": 1,
                     "sample": f"{len(items)} seeded products, x{reps} passes, {dt:.1f} s"}
    return out


def probe_mfma() -> dict | None:
    """Measured sustained FP32 matrix-core rate on this device (the probe's
    register-only MFMA loop), as a second denominator for MFMA-bound
    rooflines."""
    try:
        from paper_1810_11451_amd.probe import hbm
        return hbm.measure_mfma()
    except (RuntimeError, OSError) as e:   # probe library not built
        print(f"[bench] matrix-core probe unavailable: {e}", file=sys.stderr, flush=True)
        return None


def probe_copy(mib: int = 1024) -> dict | None:
    """Measured HBM copy bandwidth on this device (the probe's streaming
    copy), as a second denominator for HBM-bound rooflines."""
    try:
        from paper_1810_11451_amd.probe import hbm
        return hbm.measure(mib=mib, iters=10)
    except (RuntimeError, OSError) as e:   # probe library not built
        print(f"[bench] copy probe unavailable: {e}", file=sys.stderr, flush=True)
        return None


GROUP = 10   # launches per event pair in the kernel timing
MALL_BYTES = 256 << 20   # the device's memory-side cache (Infinity Cache)


def buffer_sets(batch, requested: int) -> int:
    """Disjoint S/R buffer sets to rotate: at least `requested`, and enough
    that the S of all sets is twice the memory-side cache, so that no launch
    reads S an earlier launch left there.  (With three sets the uneven
    batch's 219 MB of S was largely served from that cache: 64 against 78 us
    per launch with eight sets.)  At most 16: a batch too small for that is
    launch-bound anyway."""
    s_bytes = int(batch.f.astype(np.int64).sum()) * wl.B * 8
    if s_bytes == 0:
        return requested
    return max(requested, min(16, -(-2 * MALL_BYTES // s_bytes)))


def settle(step, ms: float, torch) -> int:
    """Runs step(i) back to back for `ms` milliseconds of wall time and
    returns how many ran.  The device raises its engine clock over the
    first tens of milliseconds of sustained load (about 2.2 to 2.45 GHz,
    GRBM_GUI_ACTIVE per dispatch) and lowers it again after a pause of a
    few hundred milliseconds, so a fixed number of warm-up steps alone
    would time part of that ramp instead of the continuous operation the
    stage is built for."""
    if ms <= 0:
        return 0
    t0 = time.perf_counter()
    i = 0
    while (time.perf_counter() - t0) * 1e3 < ms:
        step(i)
        i += 1
        if i % 32 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return i


def time_launches(launch, steps, torch, stream, group=GROUP):
    """Average duration per launch, in ms, of `steps` calls of launch(i),
    timed with HIP events on `stream` around groups of `group` back-to-back
    launches; one entry per group.  Back-to-back launches keep the
    dispatch of each kernel off the timed interval of a single event pair."""
    n_groups = max(1, steps // group)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_groups)]
    torch.cuda.synchronize()
    i = 0
    for g in range(n_groups):
        ev[g][0].record(stream)
        for _ in range(group):
            launch(i)
            i += 1
        ev[g][1].record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) / group for a, b in ev])


def own_kernel_times(plan, prec, apply, launches, torch, stream):
    """Durations, in ms, of the apply kernels of `launches` calls of
    apply(i) (each a bf_apply* call on `plan` for precision `prec`), from
    the event pair each kernel records at its own start and end
    (bf_plan_set_kernel_events): the kernel alone, without the descriptor
    upload or the queue's gap between two launches."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for a, b in ev:   # creates the events
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    try:
        for i in range(launches):
            bf.bf_plan_set_kernel_events(plan, ev[i][0], ev[i][1])
            apply(i)
    finally:
        bf.bf_plan_set_kernel_events(plan, None, None)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def kernel_time(plan, db, batch, prec, steps, copies, torch, stream, settle_ms: float = 200.0):
    """Duration of the apply kernel at steady state: the batch fixed on the
    device once per buffer set (bf_graph_create; same kernel, grid and
    product order as bf_apply), replays launched back to back over the sets
    in turn for settle_ms (what ran before may have left the device idle
    long enough for its clock to drop), then at least 200 replays timed
    with HIP events on the launch stream around groups of GROUP of them.
    A replay is one plain kernel launch, so the queue leaves about 0.4 us
    between two kernels: the per-launch mean is the kernel's duration to
    within that.  Then as many replays again, each timed by the start and
    end events the kernel records itself (hipExtLaunchKernel), which read
    a few microseconds longer.  Returns (per-launch ms of each group,
    per-kernel ms from the kernels' own events)."""
    graphs = [bf.bf_graph_create(plan, batch.w_ids, batch.f, db.s_ptrs[c], db.r_ptrs[c], prec)
              for c in range(copies)]
    launch = lambda i: bf.bf_graph_launch(graphs[i % copies], stream)  # noqa: E731
    try:
        settle(launch, settle_ms, torch)
        n = max(steps, 200)
        grouped = time_launches(launch, n, torch, stream)
        own = own_kernel_times(plan, prec, launch, n, torch, stream)
        return grouped, own
    finally:
        torch.cuda.synchronize()
        for g in graphs:
            g.close()


def workload_kernel(batch, prec: int, torch, stream, copies: int, settle_ms: float, launches: int,
                    sample: int = 256) -> dict:
    """Kernel time of one precision form on one workload at steady state
    (kernel_time: the plan's default variant over `copies` disjoint buffer
    sets, settle_ms, then `launches` kernels each timed by its own start
    and end events).  Also returns (under "_sample") host copies of a
    seeded sample of the products of the last launch, for the CPU leg's
    error check."""
    from paper_1810_11451_amd.device import DeviceBatch
    plan = bf.bf_plan_create(batch.W, bf.BF_PREC_BIT(prec))
    db = DeviceBatch(batch, copies=copies, fill_r=None)
    ms, own = kernel_time(plan, db, batch, prec, launches, copies, torch, stream, settle_ms)
    last = (len(own) - 1) % copies
    items = np.sort(np.random.default_rng(777).choice(batch.n, size=min(sample, batch.n), replace=False))
    got = db.R[last].index_select(0, torch.as_tensor(items, device=db.R[last].device)).cpu().numpy()
    variant = bf.bf_get_variant(plan, prec, bf.batch_bucket(batch.f))
    plan.close()
    del db
    torch.cuda.empty_cache()
    us = float(np.mean(ms)) * 1e3
    nbytes = batch.bytes_moved()
    sched = launched_schedule(prec, variant[0])
    return {"prec": bf.PREC_NAMES[prec], "kernel": kernel_symbol(prec, sched, variant[3]),
            "variant": list(variant), "buffer_sets": copies, "kernel_us_mean": round(us, 2),
            "kernel_us_p50": round(float(np.median(ms)) * 1e3, 2),
            "kernel_us_own_events": round(float(np.mean(own)) * 1e3, 2),
            "hbm_gbs": round(nbytes / (us * 1e-6) / 1e9, 1),
            "hbm_frac": round(nbytes / (us * 1e-6) / (PEAK_HBM_GBS * 1e9), 4),
            "complex_gflops": round(batch.flops() / (us * 1e-6) / 1e9, 1),
            "_sample": (items, got)}


def side_workloads(args, torch, stream) -> dict:
    """The two further workloads in the same run, kernel time only: the
    uneven batch (8192 products, f ~ U{1..36}, pool of 256 W) in the
    three-product FP32 form, and the gain workload (the full-width batch
    with per-product gains 10^U(-3, 3)) in the four 16-bit forms."""
    out = {}
    ub = wl.uneven_batch()
    e = workload_kernel(ub, bf.BF_FP32_3M, torch, stream, buffer_sets(ub, args.copies), 200.0, 200)
    e["traffic"] = load_traffic("uneven-fp32_3m", e["kernel"], e["variant"])
    e["workload"] = ub.name
    e["_batch"] = ub
    out["uneven_batch"] = e
    gb = wl.gain_batch()
    forms = {}
    for name in ("fp16x2", "bf16x2", "fp16", "bf16"):
        r = workload_kernel(gb, PRECS[name], torch, stream, buffer_sets(gb, args.copies), 200.0, 200)
        r["traffic"] = load_traffic(f"gain-{name}", r["kernel"], r["variant"])
        forms[name] = r
        print(f"[bench] gain workload {name}: {r['kernel_us_mean']} us", file=sys.stderr, flush=True)
    out["gain_workload"] = {"workload": gb.name, "forms": forms, "_batch": gb}
    return out


def side_errors(side: dict) -> None:
    """CPU leg: relative Frobenius error of the sampled products of each side
    workload against the FP64 oracle (FP32 bar 2e-6, split forms 2e-5,
    plain 16-bit forms reported only)."""
    from oracle import oracle as orc

    def err_of(batch, entry):
        items, got = entry.pop("_sample")
        nz = batch.f[items] > 0
        err = orc.rel_frobenius(got, orc.apply(batch, items=items))
        entry["max_rel_err_sample"] = float(f"{np.max(err[nz]):.3g}") if np.any(nz) else 0.0
        entry["sample"] = f"{len(items)} seeded products of the last launch"

    ue = side["uneven_batch"]
    err_of(ue.pop("_batch"), ue)
    g = side["gain_workload"]
    gb = g.pop("_batch")
    for entry in g["forms"].values():
        err_of(gb, entry)


def issued_flops(batch, prec: int) -> int:
    """Real flops the matrix cores execute for a batch in a given form
    (padding included): the FP32 forms run a real GEMM per product with
    N = 60 padded to 64, four real products per complex one (64 x 64 x f
    each) or three (Gauss); the 16-bit forms run M = 128 real rows (antenna,
    re/im) by N = 64 by K = 2f padded to 16 per step, once (plain) or three
    times (split: hi*hi, hi*lo, lo*hi)."""
    f = batch.f.astype(np.int64)
    if prec == bf.BF_FP32:
        return int(np.sum(4 * 2 * 64 * 64 * f))
    if prec == bf.BF_FP32_3M:
        return int(np.sum(3 * 2 * 64 * 64 * f))
    steps = (f + 7) // 8
    terms = 3 if prec in (bf.BF_FP16X2, bf.BF_BF16X2) else 1
    return int(np.sum(terms * 2 * 128 * 64 * 16 * steps))


def roof_floors_us(batch, prec: int) -> dict:
    """Time of one launch at the spec-sheet peaks: the issued matrix-core
    work at the form's peak, and the algorithmic bytes at the HBM peak.  The
    larger one names the roof the kernel is measured against."""
    lp = prec not in (bf.BF_FP32, bf.BF_FP32_3M)
    peak = (PEAK_LP_TFLOPS if lp else PEAK_FP32_TFLOPS) * 1e12
    return {"compute_us": round(issued_flops(batch, prec) / peak * 1e6, 2),
            "hbm_us": round(batch.bytes_moved() / (PEAK_HBM_GBS * 1e9) * 1e6, 2),
            "issued_flops": issued_flops(batch, prec)}


def launched_schedule(prec: int, schedule: int) -> int:
    """The schedule the library runs for a variant's schedule field (S
    16-byte aligned): the three-product form has schedules 0 and 3 only,
    the 16-bit forms no claim schedule."""
    if prec == bf.BF_FP32_3M:
        return 0 if schedule == 0 else 3
    if prec != bf.BF_FP32 and schedule == 1:
        return 2
    return schedule


def kernel_symbol(prec: int, schedule: int, store: int = 0) -> str:
    """Name (as rocprofv3 lists it, without template arguments) of the apply
    kernel that a precision form, launched schedule and variant store field
    run (store 6 to 9: the FP32 forms on 16 x 16 tiles)."""
    if prec in (bf.BF_FP32, bf.BF_FP32_3M):
        if schedule == 3:
            if store >= 6:
                return "apply_fp32_3m16_ws" if prec == bf.BF_FP32_3M else "apply_fp32_4m16_ws"
            return "apply_fp32_ws"
        if prec == bf.BF_FP32_3M:
            return "apply_fp32_3m_single"
        return {0: "apply_fp32_single", 1: "apply_fp32_claim", 2: "apply_fp32_stream"}[schedule]
    return {0: "apply_lp_single", 2: "apply_lp_stream", 3: "apply_lp_ws"}[schedule]


def load_traffic(workload_key: str, symbol: str | None = None, variant=None):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source (and, given `symbol` and
    `variant`, on that kernel in that launch variant); else None."""
    path = ROOT / "profiles" / "traffic.json"
    if not path.exists():
        return None
    try:
        data = json.loads(path.read_text())
    except ValueError:
        return None
    entry = data.get(workload_key)
    if not entry or entry.get("kernel_sha") != kernel_sha(workload_key):
        return None
    if symbol is not None and entry.get("kernel") != symbol:
        return None
    if variant is not None and entry.get("variant") != ":".join(str(int(x)) for x in variant):
        return None
    return entry.get("traffic_bytes_per_launch")


def _qam_on_device(torch, n, seed):
    """n normalised 256-QAM symbols generated on the device (seeded)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    lv = torch.randint(0, 16, (2, n), generator=g, device="cuda", dtype=torch.int32)
    x = ((2 * lv - 15).to(torch.float32) / float(np.sqrt(170.0)))
    return torch.complex(x[0], x[1])


def serve_bench(args, torch) -> dict:
    """Serving workload: Poisson arrivals of requests (W id from a pool of
    1024, f ~ U{1..36}, 1..64 S blocks of normalised 256-QAM), admission by
    an HBM budget, 0.5 ms per-request deadline.  The FP32 form is the
    three-product one.  Offered load = half its closed-loop capacity
    (40000 requests submitted at once after settle_ms of such loops, submit
    path included); the split form's capacity is measured the same way."""
    rng = np.random.default_rng(5)
    n_w, n_req = 1024, args.requests
    W = wl.unit_norm_pool(rng, n_w, wl.F_MAX)
    split = PRECS[args.serve_split]
    fp32 = bf.BF_FP32_3M
    plan = bf.bf_plan_create(W, bf.BF_PREC_BIT(fp32) | bf.BF_PREC_BIT(split))
    w_ids = rng.integers(0, n_w, n_req).astype(np.int32)
    f = rng.integers(1, wl.F_MAX + 1, n_req).astype(np.int32)
    ns = rng.integers(1, 65, n_req).astype(np.int32)
    s_elems = 1 << 27                                   # 1 GiB S arena
    S = _qam_on_device(torch, s_elems, 5)
    need = f.astype(np.int64) * ns * wl.B
    s_off = (rng.integers(0, s_elems - need.max(), n_req) // 2 * 2).astype(np.int64)
    budget = args.budget_gib << 30
    r_blocks = (2 * budget) // (wl.M * wl.B * 8)        # R ring twice the budget
    R = torch.empty((int(r_blocks), wl.M, wl.B), dtype=torch.complex64, device="cuda")
    r_off = np.zeros(n_req, np.int64)
    pos = 0
    for i in range(n_req):
        if pos + ns[i] > r_blocks:
            pos = 0
        r_off[i] = pos
        pos += ns[i]
    reqs = np.zeros(n_req, bf.REQUEST_DTYPE)
    reqs["w_id"], reqs["f"], reqs["n_s"] = w_ids, f, ns
    reqs["S"] = S.data_ptr() + s_off * 8
    reqs["R"] = R.data_ptr() + r_off * (wl.M * wl.B * 8)
    flops_req = 8 * wl.M * wl.B * f.astype(np.int64) * ns
    bytes_req = ns.astype(np.int64) * (f.astype(np.int64) * wl.B * 8 + wl.M * wl.B * 8)

    def run(prec, t_off, n, budget_bytes, streams, label):
        print(f"[bench] serving run {label}: {n} requests", file=sys.stderr, flush=True)
        srv = bf.bf_server_create(plan, hbm_budget_bytes=budget_bytes, deadline_us=500,
                                  n_streams=streams, max_batch_items=16384, prec=prec)
        try:
            done, busy, submit_ns = bf.loadgen_replay(srv, reqs[:n].copy(), t_off[:n],
                                                      progress_every=20000, stall_ms=20000,
                                                      label=label, with_submit_ns=True)
        except bf.BfError as e:
            # A stalled run is reported and the process ends at once: the
            # server's drain would wait for the stalled work.
            print(f"[bench] serving run {label} failed: {e}", file=sys.stderr, flush=True)
            os._exit(3)
        st = bf.bf_server_stats_get(srv)
        srv.close()
        assert np.all(done["status"] == bf.BF_OK), "serving run reported errors"
        st["submit_ns_per_request"] = submit_ns / max(n, 1)
        print(f"[bench] serving run {label} done", file=sys.stderr, flush=True)
        return done, busy, st

    def summary(done, busy, st, n):
        k0 = n // 100                                    # first 1% is warm-up
        d = done[k0:n]
        lat = (d["t_done_ns"] - d["t_arrival_ns"]) / 1e3
        queue = (d["t_launch_ns"] - d["t_arrival_ns"]) / 1e3
        span = (done["t_done_ns"].max() - done["t_arrival_ns"].min()) / 1e9
        return {"requests": int(n), "p50_us": round(float(np.percentile(lat, 50)), 1),
                "p99_us": round(float(np.percentile(lat, 99)), 1),
                "queue_p50_us": round(float(np.percentile(queue, 50)), 1),
                "deadline_miss_rate": round(float(np.mean(d["deadline_missed"])), 5),
                "complex_gflops": round(float(flops_req[:n].sum()) / span / 1e9, 1),
                "gbs": round(float(bytes_req[:n].sum()) / span / 1e9, 1),
                "req_per_s": round(n / span, 1), "launches": st["launches"],
                "peak_inflight_mb": round(st["peak_inflight_bytes"] / 2 ** 20, 1),
                "queue_full_retries": busy,
                "submit_ns_per_request": round(st["submit_ns_per_request"], 1),
                "batcher_us_per_launch": round(st["launch_host_ns"] / max(st["launches"], 1) / 1e3, 2),
                "requests_per_launch": round(n / max(st["launches"], 1), 1)}

    streams = args.streams
    n_cap = min(n_req, 40000)
    # Warm-up: closed loops of up to 20000 requests for settle_ms (at least
    # one), so the capacity is measured at the device's sustained clock.
    t_warm = time.perf_counter()
    k = 0
    while k == 0 or (time.perf_counter() - t_warm) * 1e3 < args.settle_ms:
        run(fp32, np.zeros(n_cap, np.int64), min(n_cap, 20000), budget, streams, f"warm-up {k}")
        k += 1
    done, busy, st = run(fp32, np.zeros(n_cap, np.int64), n_cap, budget, streams,
                         "fp32_3m closed loop")
    span = (done["t_done_ns"].max() - done["t_arrival_ns"].min()) / 1e9
    capacity = n_cap / span
    lam = 0.5 * capacity
    gaps = rng.exponential(1e9 / lam, n_req)
    t_off = np.cumsum(gaps).astype(np.int64)
    out = {"capacity_req_per_s": round(capacity, 1),
           "capacity_gbs": round(float(bytes_req[:n_cap].sum()) / span / 1e9, 1),
           "closed_loop": summary(done, busy, st, n_cap),
           "offered_req_per_s": round(lam, 1),
           "offered_gbs": round(lam * float(bytes_req.mean()) / 1e9, 1)}
    d2, b2, s2 = run(split, np.zeros(n_cap, np.int64), n_cap, budget, streams,
                     f"{args.serve_split} closed loop")
    out[f"closed_loop_{args.serve_split}"] = summary(d2, b2, s2, n_cap)
    for name, prec in (("fp32_3m", fp32), (args.serve_split, split)):
        print(f"[bench] serving {name} at {lam:.0f} req/s", file=sys.stderr, flush=True)
        out[name] = summary(*run(prec, t_off, n_req, budget, streams, name), n_req)
    n_small = min(n_req, 20000)
    out["fp32_3m_budget_16mib"] = summary(*run(fp32, t_off, n_small, 16 << 20, streams,
                                               "fp32_3m 16 MiB budget"), n_small)
    plan.close()
    return out


def filter_cpu_baseline(s, h, target_s: float) -> dict:
    """The filter oracle (numpy complex128 FFTs, as it stands) on seeded
    blocks of the same workload, repeated until about target_s."""
    from oracle import filter_oracle as fo
    rng = np.random.default_rng(54321)
    pick = rng.choice(s.shape[0], size=min(s.shape[0], 256), replace=False)
    sample = s[pick]
    reps, t0 = 0, time.perf_counter()
    while True:
        fo.filter_apply(sample, h)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= target_s:
            break
    return {"value": round(reps * len(pick) / dt, 1), "unit": "blocks/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{len(pick)} of the {s.shape[0]} blocks of the same workload (seeded choice), "
                      f"x{reps} passes, numpy complex128 FFTs on one thread, {dt:.1f} s"}


def filter_bench(args, torch) -> dict:
    """Filter stage: 16384 blocks of 2048 CN(0,1) samples through a 127-tap
    windowed-sinc lowpass (cutoff 0.1); three disjoint x/y buffer sets
    rotate.  A step is one bf_filter_apply over all blocks."""
    n, n_taps = 16384, 127
    rng = np.random.default_rng(6)
    s = wl.filter_signals(rng, n)
    h = wl.lowpass_taps(n_taps, 0.1)
    flt = bf.bf_filter_create(h)
    xs = [torch.from_numpy(s).cuda() for _ in range(args.copies)]
    ys = [torch.empty_like(xs[0]) for _ in range(args.copies)]
    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup
    settle(lambda i: bf.bf_filter_apply(flt, n, xs[i % args.copies], ys[i % args.copies]),
           args.settle_ms, torch)
    for i in range(W):
        bf.bf_filter_apply(flt, n, xs[i % args.copies], ys[i % args.copies])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        bf.bf_filter_apply(flt, n, xs[i % args.copies], ys[i % args.copies])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = time_launches(lambda i: bf.bf_filter_apply(flt, n, xs[i % args.copies], ys[i % args.copies]),
                            K, torch, stream)
    kern_s = float(np.mean(kern_ms)) / 1e3
    nbytes = n * wl.N_FILTER * 8 * 2                    # each block read once, written once
    flops_conv = n * (2 * 5 * wl.N_FILTER * 11 + 6 * wl.N_FILTER)   # 5 N log2 N per FFT + complex mult
    ach = nbytes / kern_s / 1e9
    out = {"metric": FILTER_METRIC, "value": round(n * K / wall, 1), "unit": "blocks/s",
           "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(wall / K * 1e3, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"filter: {n} blocks of 2048 CN(0,1) samples, {n_taps}-tap "
                                  "windowed-sinc lowpass", "n_blocks": n, "n_taps": n_taps,
                      "buffer_sets": args.copies},
           "latency_us": {"p50": round(float(np.percentile(kern_ms, 50)) * 1e3, 2),
                          "p99": round(float(np.percentile(kern_ms, 99)) * 1e3, 2)},
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": load_traffic("filter"),
                        "kernel": "filter_kernel", "kernel_us_mean": round(kern_s * 1e6, 2),
                        "kernel_timing": "HIP events on the launch stream around groups of 10 back-to-back launches",
                        "algorithmic": {"bytes_per_launch": nbytes, "flops_conventional": flops_conv,
                                        "ai_flop_per_byte": round(flops_conv / nbytes, 2)},
                        "gflops_conventional": round(flops_conv / kern_s / 1e9, 1)}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = filter_cpu_baseline(s, h, min(args.cpu_seconds, 10.0))
    flt.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    # Warm-up: --settle-ms of continuous running (the device's clock ramp),
    # then --warmup steps.
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--settle-ms", type=float, default=400.0,
                    help="run the path this long before the warm-up steps (device clock ramp)")
    ap.add_argument("--workload", default="full-width", choices=list(WORKLOADS))
    ap.add_argument("--prec", default="fp32_3m", choices=sorted(PRECS),
                    help="arithmetic form (default: FP32, three real products per complex one)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the four-product FP32 kernel alongside")
    ap.add_argument("--copies", type=int, default=3,
                    help="disjoint S/R buffer sets rotated (at least; more where that many would hold "
                         "less S than twice the memory-side cache)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="tune the variant before timing")
    ap.add_argument("--requests", type=int, default=200000, help="serving: requests replayed")
    ap.add_argument("--no-serving", action="store_true",
                    help="full-width line: leave out the serving workload")
    ap.add_argument("--budget-gib", type=int, default=16, help="serving: HBM budget")
    ap.add_argument("--streams", type=int, default=2, help="serving: device streams")
    ap.add_argument("--serve-split", default="fp16x2", choices=["fp16x2", "bf16x2", "fp16", "bf16"],
                    help="serving: the 16-bit form compared with FP32")
    ap.add_argument("--variant", default=None,
                    help="force schedule:wg_per_cu:order (e.g. 2:3:1) instead of the plan table")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the products are "
              "independent and this library has no multi-GPU path (a multi-GPU version would "
              "shard the items, with no exchange between GPUs).", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    from paper_1810_11451_amd.device import DeviceBatch

    torch.cuda.set_device(0)
    if args.workload == "filter":
        print(json.dumps(filter_bench(args, torch)), flush=True)
        return 0
    if args.workload == "serving":
        res = serve_bench(args, torch)
        fp = res["fp32_3m"]
        out = {"metric": METRIC, "value": fp["complex_gflops"], "unit": "complex GFLOP/s",
               "n_gpus": 1, "steps": fp["requests"], "warmup": 0,
               "ms_per_step": round(1e3 / fp["req_per_s"], 6), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": "serving: Poisson requests, pool 1024 W 64x36, f~U{1..36}, "
                                      "1..64 S of 256-QAM, 0.5 ms deadline",
                          "budget_gib": args.budget_gib, "streams": args.streams},
               "latency_us": {"p50": fp["p50_us"], "p99": fp["p99_us"]},
               "serving": res}
        print(json.dumps(out), flush=True)
        return 0
    prec = PRECS[args.prec]
    batch = WORKLOADS[args.workload]()
    print(f"[bench] {args.workload}: {batch.name}, prec {args.prec}", file=sys.stderr, flush=True)
    plan = bf.bf_plan_create(batch.W, bf.BF_PREC_BIT(prec))
    copies = buffer_sets(batch, args.copies)
    db = DeviceBatch(batch, copies=copies, fill_r=None)
    stream = torch.cuda.current_stream()
    tuned = None
    if args.variant:
        v = [int(x) for x in args.variant.split(":")]
        for bk in range(5):
            bf.bf_set_variant(plan, prec, bk, *v)
    if args.autotune:
        tuned = bf.bf_autotune(plan, batch.w_ids, batch.f, db.s_ptrs[0], db.r_ptrs[0], prec, reps=5)
    variant = bf.bf_get_variant(plan, prec, bf.batch_bucket(batch.f))

    settle_steps = settle(lambda i: db.apply(plan, prec, copy=i % copies), args.settle_ms, torch)
    for i in range(args.warmup):
        db.apply(plan, prec, copy=i % copies)
    torch.cuda.synchronize()

    K = args.steps
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        db.apply(plan, prec, copy=i % copies)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    wall = t1 - t0
    # Per-step latency in a second pass of K steps: event pairs around every
    # step cost the stream a few microseconds each, so they stay out of the
    # throughput pass above.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for i in range(K):
        ev[i][0].record(stream)
        db.apply(plan, prec, copy=i % copies)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    kern_ms, kern_own = kernel_time(plan, db, batch, prec, K, copies, torch, stream)
    kern_s = float(np.mean(kern_ms)) / 1e3

    compare = None
    if prec == bf.BF_FP32_3M and not args.no_compare:
        # The four-product FP32 form on the same workload, kernel time only.
        plan4 = bf.bf_plan_create(batch.W, bf.BF_PREC_BIT(bf.BF_FP32))
        k4, _ = kernel_time(plan4, db, batch, bf.BF_FP32, K, copies, torch, stream)
        v4 = bf.bf_get_variant(plan4, bf.BF_FP32, bf.batch_bucket(batch.f))
        plan4.close()
        t4 = float(np.mean(k4)) / 1e3
        sym4 = kernel_symbol(bf.BF_FP32, launched_schedule(bf.BF_FP32, v4[0]), v4[3])
        compare = {"prec": "fp32", "kernel": sym4, "kernel_us_mean": round(t4 * 1e6, 2),
                   "tflops": round(batch.flops() / t4 / 1e12, 2),
                   "frac": round(batch.flops() / t4 / 1e12 / PEAK_FP32_TFLOPS, 4),
                   "variant": list(v4), "traffic": load_traffic("full-width-fp32", sym4, v4)}
    split = None
    if prec == bf.BF_FP32_3M and not args.no_compare:
        # The 2-term split FP16 form (FP32-class accuracy from 16-bit matrix
        # cores) on the same workload, kernel time only, against this form.
        plans = bf.bf_plan_create(batch.W, bf.BF_PREC_BIT(bf.BF_FP16X2))
        ks, _ = kernel_time(plans, db, batch, bf.BF_FP16X2, K, copies, torch, stream)
        vs = bf.bf_get_variant(plans, bf.BF_FP16X2, bf.batch_bucket(batch.f))
        plans.close()
        split = {"prec": "fp16x2", "kernel_us_mean": round(float(np.mean(ks)) * 1e3, 2),
                 "hbm_gbs_equiv": round(batch.bytes_moved() / (float(np.mean(ks)) / 1e3) / 1e9, 1),
                 "variant": list(vs)}

    side = None
    serving = None
    if args.workload == "full-width" and prec == bf.BF_FP32_3M and not args.no_compare:
        side = side_workloads(args, torch, stream)
        if not args.no_serving:
            # The serving workload (Poisson requests against a pool of 1024 W)
            # in the same run: closed-loop capacity, then p50/p99 of the
            # three-product FP32 and split forms at half of it.
            serving = serve_bench(args, torch)
            torch.cuda.empty_cache()

    flops = batch.flops()
    nbytes = batch.bytes_moved()
    value = flops * K / wall / 1e9
    ai = flops / nbytes
    lp = prec not in (bf.BF_FP32, bf.BF_FP32_3M)
    peak_flops = (PEAK_LP_TFLOPS if lp else PEAK_FP32_TFLOPS) * 1e12
    key = f"{args.workload}-{args.prec}"
    sched = launched_schedule(prec, variant[0])
    traffic = load_traffic(key, kernel_symbol(prec, sched, variant[3]), variant)
    floors = roof_floors_us(batch, prec)
    if floors["compute_us"] > floors["hbm_us"]:
        ach = flops / kern_s / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 2), "peak": peak_flops / 1e12,
                "unit": "TFLOP/s", "frac": round(ach / (peak_flops / 1e12), 4)}
    else:
        ach = nbytes / kern_s / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4)}
    roof["traffic"] = traffic
    roof["kernel"] = kernel_symbol(prec, sched, variant[3])
    roof["kernel_us_mean"] = round(kern_s * 1e6, 2)
    roof["kernel_us_p50"] = round(float(np.median(kern_ms)) * 1e3, 2)
    roof["kernel_us_min"] = round(float(np.min(kern_ms)) * 1e3, 2)
    roof["kernel_timing"] = (f"HIP events on the launch stream around groups of {GROUP} back-to-back launches "
                             "of the batch fixed on the device (bf_graph_launch: one plain kernel launch each, "
                             "same kernel and grid as bf_apply), after 200 ms of them")
    roof["kernel_us_own_events"] = round(float(np.mean(kern_own)) * 1e3, 2)
    roof["step_us_mean"] = round(float(np.mean(step_ms)) * 1e3, 2)
    roof["launch_period_us"] = round(wall / K * 1e6, 2)
    roof["algorithmic"] = {"flops_per_launch": flops, "bytes_per_launch": nbytes,
                           "ai_flop_per_byte": round(ai, 2)}
    roof["floors_us"] = floors
    roof["hbm_gbs_equiv"] = round(nbytes / kern_s / 1e9, 1)
    if roof["bound"] == "hbm":
        pc = probe_copy()
        if pc is not None:
            roof["measured_probe"] = {"kind": "streaming copy, 1 GiB read + 1 GiB written",
                                      "GBps": pc["GBps"],
                                      "frac": round(roof["hbm_gbs_equiv"] / pc["GBps"], 4)}
    elif not lp:
        pm = probe_mfma()
        if pm is not None:
            roof["measured_probe"] = {"kind": "FP32 matrix-core loop from registers "
                                              "(v_mfma_f32_32x32x2_f32)",
                                      "TFLOPs": pm["TFLOPs"],
                                      "frac": round(roof["achieved"] / pm["TFLOPs"], 4)}
        # The kernel also moves its bytes; on this device the measured copy
        # rate, not the spec-sheet one, sets the memory floor.
        pc = probe_copy()
        if pm is not None and pc is not None:
            t_mfma = flops / (pm["TFLOPs"] * 1e12) * 1e6
            t_hbm = nbytes / (pc["GBps"] * 1e9) * 1e6
            roof["measured_floors_us"] = {
                "mfma_probe": round(t_mfma, 1), "hbm_copy_probe": round(t_hbm, 1),
                "copy_probe_GBps": pc["GBps"],
                "slower_floor_over_kernel": round(max(t_mfma, t_hbm) / (kern_s * 1e6), 4)}

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "complex GFLOP/s",
        "complex_gmac_per_s": round(value / 8, 2),
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_3m": "f32", "fp16": "f16", "bf16": "bf16",
                  "fp16x2": "f16x2", "bf16x2": "bf16x2"}[args.prec],
        "data": "synthetic",
        "config": {"workload": batch.name, "n_products": batch.n, "n_w": batch.n_w,
                   "f": int(batch.f.max()) if batch.f.min() == batch.f.max() else "U{1..36}",
                   "prec": args.prec, "variant": {"schedule": variant[0], "wg_per_cu": variant[1],
                                                  "order": variant[2], "store": variant[3]},
                   "buffer_sets": copies,
                   "settle": {"ms": args.settle_ms, "steps": settle_steps}},
        "latency_us": {"p50": round(float(np.percentile(step_ms, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(step_ms, 99)) * 1e3, 2)},
        "roofline": roof,
    }
    if tuned is not None:
        out["config"]["autotuned_us"] = round(tuned[1], 2)
    if prec == bf.BF_FP32_3M:
        out["config"]["product"] = ("FP32, three real products per complex product (Gauss); "
                                    "flops counted as 8 per complex multiply-add")
    if compare is not None:
        out["compare_fp32_four_product"] = compare
    if split is not None:
        split["speedup_over_this_form"] = round(kern_s * 1e6 / split["kernel_us_mean"], 3)
        out["compare_split_fp16x2"] = split
    if side is not None:
        g = side["gain_workload"]
        for entry in g["forms"].values():
            entry["speedup_over_fp32_3m_full_width"] = round(kern_s * 1e6 / entry["kernel_us_mean"], 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(batch, args.cpu_seconds)
        out["cpu_other"] = cpu_extra(batch, min(3.0, args.cpu_seconds))
        if side is not None:
            side_errors(side)
    if side is not None:
        for entry in [side["uneven_batch"]] + list(side["gain_workload"]["forms"].values()):
            entry.pop("_sample", None)
        side["uneven_batch"].pop("_batch", None)
        side["gain_workload"].pop("_batch", None)
        out["uneven_batch"] = side["uneven_batch"]
        out["gain_workload"] = side["gain_workload"]
    if serving is not None:
        serving["workload"] = ("serving: Poisson requests, pool 1024 W 64x36, f~U{1..36}, 1..64 S of "
                               f"256-QAM, 0.5 ms deadline, {args.budget_gib} GiB budget, "
                               f"{args.streams} streams")
        out["serving_workload"] = serving
    plan.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
