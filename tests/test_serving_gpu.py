"""GPU tests of the serving loop (bf_server_*): results, admission, deadlines.

Each request's results are compared with the FP64 oracle (2e-6, FP32) and,
for "alone == in the mix", bitwise with the same request served alone:
every product is computed by the same kernel code whatever else shares
its launch.
"""
import time

import numpy as np
import pytest

from gpu_util import FP32_TOL, announce, require_gpu
from oracle import oracle as orc
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl

pytestmark = pytest.mark.gpu

RB = wl.M * wl.B * 8   # bytes of one R block


class Arena:
    """Device S and R arenas for a list of requests (w, f, n_s)."""

    def __init__(self, torch, rng, shapes, n_w):
        self.torch = torch
        self.shapes = shapes
        s_sizes = [f * n * wl.B for (_, f, n) in shapes]
        self.s_off = np.concatenate([[0], np.cumsum(s_sizes)[:-1]]).astype(np.int64)
        self.S_host = wl.qam256(rng, (max(1, int(sum(s_sizes))),)).astype(np.complex64)
        self.S = torch.from_numpy(self.S_host).cuda()
        n_r = sum(n for (_, _, n) in shapes)
        self.r_off = np.concatenate([[0], np.cumsum([n for (_, _, n) in shapes])[:-1]]).astype(np.int64)
        self.R = torch.full((n_r, wl.M, wl.B), float("nan"), dtype=torch.complex64, device="cuda")

    def request(self, i, tag=None):
        w, f, n = self.shapes[i]
        S = self.S.data_ptr() + int(self.s_off[i]) * 8 if f > 0 else 0
        R = self.R.data_ptr() + int(self.r_off[i]) * RB
        return bf.make_request(w, f, n, S, R, tag=i if tag is None else tag)

    def result(self, i):
        w, f, n = self.shapes[i]
        self.torch.cuda.synchronize()
        return self.R[int(self.r_off[i]): int(self.r_off[i]) + n].cpu().numpy()

    def reference(self, W, i):
        w, f, n = self.shapes[i]
        blocks = self.S_host[int(self.s_off[i]): int(self.s_off[i]) + f * n * wl.B]
        s_off = np.arange(n, dtype=np.int64) * f * wl.B
        return orc.apply_arrays(W, np.full(n, w, np.int32), np.full(n, f, np.int32),
                                blocks if blocks.size else np.zeros(1, np.complex64), s_off)


def _shapes(rng, n_req, n_w, max_ns=6):
    return [(int(rng.integers(0, n_w)), int(rng.integers(0, 37)), int(rng.integers(1, max_ns + 1)))
            for _ in range(n_req)]


def _drain(server, n, timeout_s=30.0):
    got = []
    t_end = time.time() + timeout_s
    while len(got) < n and time.time() < t_end:
        got.extend(bf.bf_poll(server, 256, 100000).tolist())
    assert len(got) == n, f"only {len(got)} of {n} completions"
    return np.array(got, dtype=bf.COMPLETION_DTYPE)


def test_serve_matches_oracle():
    torch = require_gpu()
    rng = np.random.default_rng(701)
    W = wl.unit_norm_pool(rng, 16, 36)
    shapes = _shapes(rng, 30, 16)
    ar = Arena(torch, rng, shapes, 16)
    plan = bf.bf_plan_create(W)
    announce("serve 30 requests")
    with bf.bf_server_create(plan, n_streams=2) as srv:
        tickets = [bf.bf_submit(srv, ar.request(i)) for i in range(len(shapes))]
        assert tickets == sorted(tickets) and len(set(tickets)) == len(tickets)
        done = _drain(srv, len(shapes))
        assert np.all(done["status"] == bf.BF_OK)
        assert np.all(done["t_done_ns"] >= done["t_launch_ns"])
        assert np.all(done["t_launch_ns"] >= done["t_arrival_ns"])
        st = bf.bf_server_stats_get(srv)
        assert st["completed"] == len(shapes) and st["inflight_bytes"] == 0
    for i, (w, f, n) in enumerate(shapes):
        got = ar.result(i)
        ref = ar.reference(W, i)
        if f == 0:
            assert np.all(got == 0)
        else:
            assert np.max(orc.rel_frobenius(got, ref)) <= FP32_TOL, f"request {i}"
    plan.close()


@pytest.mark.parametrize("prec,variant", [(bf.BF_FP32, (0, 0, 1, 1)), (bf.BF_FP32, (2, 0, 0)),
                                          (bf.BF_FP32, (1, 0, 2)), (bf.BF_FP32_3M, (0, 0, 2, 1)),
                                          (bf.BF_FP32_3M, (3, 0, 1, 7)), (bf.BF_FP32_3M, (3, 0, 3, 9)),
                                          (bf.BF_FP32, (3, 0, 3, 8)), (bf.BF_FP32_3M, (0, 0, 3, 1)),
                                          (bf.BF_FP32_3M, (3, 0, 4, 9))],
                         ids=["fp32-single-byw", "fp32-stream-asgiven", "fp32-claim-xcd",
                              "fp32_3m-single-xcd", "fp32_3m-ws16-byw", "fp32_3m-ws16-w-blocked",
                              "fp32-ws16-w-blocked", "fp32_3m-single-w-sorted", "fp32_3m-ws16-f-balanced"])
def test_serve_under_each_product_order(prec, variant):
    """Requests expand into items on the device in the order the variant
    asks for (as given, by W id then f, grouped by W id modulo 8, grouped
    and sorted by W id and, on the wave-specialised schedule, dealt to the
    workgroups in blocks); n_s up to 70 takes a record past one wave's 64
    lanes.  Every request against the oracle."""
    torch = require_gpu()
    rng = np.random.default_rng(703)
    W = wl.unit_norm_pool(rng, 24, 36)
    shapes = _shapes(rng, 40, 24, max_ns=70)
    ar = Arena(torch, rng, shapes, 24)
    plan = bf.bf_plan_create(W, bf.BF_PREC_BIT(prec))
    for bk in range(5):
        bf.bf_set_variant(plan, prec, bk, *variant)
    announce(f"serve 40 requests prec={bf.PREC_NAMES[prec]} variant={variant}")
    with bf.bf_server_create(plan, n_streams=2, prec=prec) as srv:
        for i in range(len(shapes)):
            bf.bf_submit(srv, ar.request(i))
        done = _drain(srv, len(shapes))
        assert np.all(done["status"] == bf.BF_OK)
    for i, (w, f, n) in enumerate(shapes):
        got = ar.result(i)
        if f == 0:
            assert np.all(got == 0)
        else:
            assert np.max(orc.rel_frobenius(got, ar.reference(W, i))) <= FP32_TOL, f"request {i}"
    plan.close()


@pytest.mark.parametrize("prec", [bf.BF_FP32, bf.BF_FP16X2])
def test_alone_equals_in_mix(prec):
    torch = require_gpu()
    rng = np.random.default_rng(702)
    W = wl.unit_norm_pool(rng, 8, 36)
    shapes = _shapes(rng, 40, 8)
    plan = bf.bf_plan_create(W, bf.BF_PREC_BIT(prec))
    alone = Arena(torch, np.random.default_rng(9), shapes, 8)
    mix = Arena(torch, np.random.default_rng(9), shapes, 8)
    announce(f"alone vs mix prec={prec}")
    with bf.bf_server_create(plan, n_streams=3, prec=prec) as srv:
        for i in range(len(shapes)):
            bf.bf_submit(srv, alone.request(i))
            _drain(srv, 1)
        for i in range(len(shapes)):
            bf.bf_submit(srv, mix.request(i))
        _drain(srv, len(shapes))
        assert bf.bf_server_stats_get(srv)["launches"] < 2 * len(shapes)
    for i in range(len(shapes)):
        a, m = alone.result(i), mix.result(i)
        assert np.array_equal(a.view(np.uint32), m.view(np.uint32)), f"request {i} differs"
    plan.close()


def test_admission_respects_budget():
    torch = require_gpu()
    rng = np.random.default_rng(703)
    W = wl.unit_norm_pool(rng, 4, 36)
    shapes = [(int(rng.integers(0, 4)), 36, 8) for _ in range(25)]
    per_req = 8 * (36 * wl.B * 8 + RB)
    budget = 3 * per_req
    ar = Arena(torch, rng, shapes, 4)
    plan = bf.bf_plan_create(W)
    announce("budget of three requests")
    with bf.bf_server_create(plan, hbm_budget_bytes=budget, n_streams=4) as srv:
        for i in range(len(shapes)):
            bf.bf_submit(srv, ar.request(i))
        done = _drain(srv, len(shapes))
        st = bf.bf_server_stats_get(srv)
        assert st["peak_inflight_bytes"] <= budget
        assert st["peak_inflight_bytes"] >= per_req
        assert np.all(done["status"] == bf.BF_OK)
        with pytest.raises(bf.BfError) as ei:
            bf.bf_submit(srv, bf.make_request(0, 36, 100, ar.S, ar.R))   # larger than the budget
        assert ei.value.status == bf.BF_ERR_INVALID
        with pytest.raises(bf.BfError) as ei:
            bf.bf_submit(srv, bf.make_request(9, 3, 1, ar.S, ar.R))    # no such W
        assert ei.value.status == bf.BF_ERR_INVALID
    for i in range(len(shapes)):
        ref = ar.reference(W, i)
        assert np.max(orc.rel_frobenius(ar.result(i), ref)) <= FP32_TOL
    plan.close()


def test_deadline_misses_are_reported_not_dropped():
    torch = require_gpu()
    rng = np.random.default_rng(704)
    W = wl.unit_norm_pool(rng, 4, 36)
    shapes = _shapes(rng, 20, 4, max_ns=4)
    ar = Arena(torch, rng, shapes, 4)
    plan = bf.bf_plan_create(W)
    announce("1 us deadline")
    with bf.bf_server_create(plan, deadline_us=1) as srv:
        past = bf.bf_now_ns() - 10_000_000
        for i in range(len(shapes)):
            r = ar.request(i)
            r["t_arrival_ns"] = past
            bf.bf_submit(srv, r)
        done = _drain(srv, len(shapes))
        assert np.all(done["deadline_missed"] == 1)
        assert bf.bf_server_stats_get(srv)["deadline_misses"] == len(shapes)
    for i in range(len(shapes)):
        w, f, n = shapes[i]
        if f:
            assert np.max(orc.rel_frobenius(ar.result(i), ar.reference(W, i))) <= FP32_TOL
    plan.close()


def test_destroy_drains():
    torch = require_gpu()
    rng = np.random.default_rng(705)
    W = wl.unit_norm_pool(rng, 4, 36)
    shapes = _shapes(rng, 60, 4)
    ar = Arena(torch, rng, shapes, 4)
    plan = bf.bf_plan_create(W)
    announce("destroy right after submitting")
    srv = bf.bf_server_create(plan, n_streams=2)
    for i in range(len(shapes)):
        bf.bf_submit(srv, ar.request(i))
    srv.close()
    torch.cuda.synchronize()
    for i in range(len(shapes)):
        w, f, n = shapes[i]
        got = ar.result(i)
        assert not np.any(np.isnan(got.view(np.float32))), f"request {i} not written"
    plan.close()


def test_loadgen_poisson_replay():
    torch = require_gpu()
    rng = np.random.default_rng(706)
    W = wl.unit_norm_pool(rng, 32, 36)
    shapes = _shapes(rng, 3000, 32, max_ns=8)
    ar = Arena(torch, rng, shapes, 32)
    plan = bf.bf_plan_create(W)
    reqs = np.concatenate([ar.request(i) for i in range(len(shapes))])
    gaps = rng.exponential(2000.0, size=len(shapes))       # ~500k requests/s offered
    t_off = np.cumsum(gaps).astype(np.int64)
    announce(f"loadgen replay n={len(shapes)}")
    with bf.bf_server_create(plan, n_streams=2, deadline_us=500) as srv:
        done, busy = bf.loadgen_replay(srv, reqs, t_off)
    assert np.all(done["status"] == bf.BF_OK)
    assert np.array_equal(done["tag"], np.arange(len(shapes)))
    lat = (done["t_done_ns"] - done["t_arrival_ns"]) / 1e3
    print(f"latency us p50 {np.percentile(lat, 50):.1f} p99 {np.percentile(lat, 99):.1f}", flush=True)
    assert np.all(lat > 0)
    for i in rng.choice(len(shapes), size=60, replace=False):
        w, f, n = shapes[i]
        if f:
            assert np.max(orc.rel_frobenius(ar.result(i), ar.reference(W, i))) <= FP32_TOL
    plan.close()
