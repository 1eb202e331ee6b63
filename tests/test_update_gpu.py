"""GPU tests of bf_plan_update: one pool entry replaced while the plan is in use.

Every result is compared with the FP64 oracle run on the pool that the
launch should have seen: the old W for launches issued before an update,
the new W for launches issued after it, whatever streams they run on.
Bars as in the parity tests: FP32 forms 2e-6, split forms 2e-5, plain
16-bit forms 4u*sqrt(2).
"""
import dataclasses
import math

import numpy as np
import pytest

from gpu_util import FP32_TOL, announce, require_gpu
from oracle import oracle as orc
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl
from paper_1810_11451_amd.device import DeviceBatch

pytestmark = pytest.mark.gpu

FORMS = {"fp32": bf.BF_FP32, "fp32_3m": bf.BF_FP32_3M, "fp16": bf.BF_FP16, "bf16": bf.BF_BF16,
         "fp16x2": bf.BF_FP16X2, "bf16x2": bf.BF_BF16X2}
BAR = {"fp32": FP32_TOL, "fp32_3m": FP32_TOL, "fp16x2": 2e-5, "bf16x2": 2e-5,
       "fp16": 4 * 2.0 ** -11 * math.sqrt(2), "bf16": 4 * 2.0 ** -8 * math.sqrt(2)}


def with_pool(batch, W):
    return dataclasses.replace(batch, W=np.ascontiguousarray(W, dtype=np.complex64))


def check(batch, W, R, bar, what):
    ref = orc.apply(with_pool(batch, W))
    err = orc.rel_frobenius(R, ref)
    nz = batch.f > 0
    assert np.all(R[~nz] == 0), what
    assert np.max(err[nz], initial=0.0) <= bar, f"{what}: max rel err {np.max(err[nz]):.3g}"


def big_batch(rng, n, n_w, w_id):
    """n full-width products, all on pool entry w_id (long enough to still run
    while the host issues an update)."""
    S3 = wl.qam256(rng, (n, wl.F_MAX, wl.B)).astype(np.complex64)
    return wl._uniform_f_batch("one entry", np.zeros((n_w, wl.M, wl.F_MAX), np.complex64),
                               np.full(n, w_id), wl.F_MAX, S3)


@pytest.mark.parametrize("form", sorted(FORMS))
def test_update_then_apply(form):
    """After an update, every entry reads right: the updated one its new W,
    the others their old W."""
    require_gpu()
    rng = np.random.default_rng(901)
    b = wl.random_batch(rng, 120, 5, f_values=np.arange(0, 37), dist="qam")
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(FORMS[form]))
    W2 = b.W.copy()
    W2[3] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    announce(f"update then apply form={form}")
    bf.bf_plan_update(plan, 3, W2[3])
    db = DeviceBatch(b)
    db.apply(plan, FORMS[form])
    check(b, W2, db.result(), BAR[form], form)
    # a second update of the same entry, and one of another entry
    W2[3] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    W2[0] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    bf.bf_plan_update(plan, 3, W2[3])
    bf.bf_plan_update(plan, 0, W2[0])
    db.apply(plan, FORMS[form])
    check(b, W2, db.result(), BAR[form], form + " after two more updates")
    plan.close()


@pytest.mark.parametrize("form", sorted(FORMS))
def test_update_then_apply_wave_specialised(form):
    """The same through the wave-specialised schedule, which reads the
    16-bit forms' compact W layout (rewritten by the update too)."""
    require_gpu()
    rng = np.random.default_rng(907)
    b = wl.random_batch(rng, 700, 5, f_values=np.arange(0, 37), dist="qam")
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(FORMS[form]))
    for bk in range(5):
        bf.bf_set_variant(plan, FORMS[form], bk, 3, 0, 0, 1)
    W2 = b.W.copy()
    W2[2] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0] * 3.0   # a new scale exponent as well
    announce(f"update then apply, wave-specialised, form={form}")
    bf.bf_plan_update(plan, 2, W2[2])
    db = DeviceBatch(b)
    db.apply(plan, FORMS[form])
    check(b, W2, db.result(), BAR[form], form)
    plan.close()


def test_before_and_after_on_one_stream():
    """apply(old) ; update ; apply(new) issued back to back on one stream."""
    torch = require_gpu()
    rng = np.random.default_rng(902)
    W0 = wl.unit_norm_pool(rng, 4, wl.F_MAX)
    W1 = W0.copy()
    W1[2] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    b = with_pool(big_batch(rng, 4096, 4, 2), W0)
    plan = bf.bf_plan_create(W0, bf.BF_PREC_BIT(bf.BF_FP32_3M))
    st = torch.cuda.Stream()
    a, c = DeviceBatch(b), DeviceBatch(b)
    torch.cuda.synchronize()   # the R fills run on the default stream
    announce("before/after on one stream")
    with torch.cuda.stream(st):
        a.apply(plan, bf.BF_FP32_3M, stream=st.cuda_stream)
        bf.bf_plan_update(plan, 2, W1[2], stream=st.cuda_stream)
        c.apply(plan, bf.BF_FP32_3M, stream=st.cuda_stream)
    torch.cuda.synchronize()
    items = np.random.default_rng(1).choice(b.n, 64, replace=False)
    for db, W, what in ((a, W0, "before"), (c, W1, "after")):
        R = db.result()
        ref = orc.apply(with_pool(b, W), items=items)
        assert np.max(orc.rel_frobenius(R[items], ref)) <= FP32_TOL, what
    plan.close()


def test_updates_across_streams():
    """Launches on one stream, updates on another: each launch sees the pool
    as it was when it was issued, and the second update of the entry waits
    for the launch issued before the first."""
    torch = require_gpu()
    rng = np.random.default_rng(903)
    W0 = wl.unit_norm_pool(rng, 3, wl.F_MAX)
    W1, W2 = W0.copy(), W0.copy()
    W1[1] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    W2[1] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    b = with_pool(big_batch(rng, 4096, 3, 1), W0)
    plan = bf.bf_plan_create(W0, bf.BF_PREC_BIT(bf.BF_FP32) | bf.BF_PREC_BIT(bf.BF_FP32_3M))
    s_apply, s_update = torch.cuda.Stream(), torch.cuda.Stream()
    dbs = [DeviceBatch(b) for _ in range(3)]
    torch.cuda.synchronize()   # the R fills run on the default stream
    announce("updates on a second stream")
    dbs[0].apply(plan, bf.BF_FP32_3M, stream=s_apply.cuda_stream)
    bf.bf_plan_update(plan, 1, W1[1], stream=s_update.cuda_stream)
    dbs[1].apply(plan, bf.BF_FP32, stream=s_apply.cuda_stream)
    bf.bf_plan_update(plan, 1, W2[1], stream=s_update.cuda_stream)
    dbs[2].apply(plan, bf.BF_FP32_3M, stream=s_apply.cuda_stream)
    torch.cuda.synchronize()
    items = np.random.default_rng(2).choice(b.n, 64, replace=False)
    for db, W, what in zip(dbs, (W0, W1, W2), ("first", "second", "third")):
        ref = orc.apply(with_pool(b, W), items=items)
        assert np.max(orc.rel_frobenius(db.result()[items], ref)) <= FP32_TOL, what
    plan.close()


def test_graph_created_after_update():
    torch = require_gpu()
    rng = np.random.default_rng(904)
    b = wl.random_batch(rng, 200, 4, dist="qam")
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(bf.BF_FP32_3M))
    W1 = b.W.copy()
    W1[0] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    bf.bf_plan_update(plan, 0, W1[0])
    db = DeviceBatch(b)
    announce("graph after update")
    g = bf.bf_graph_create(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0], bf.BF_FP32_3M)
    st = torch.cuda.current_stream()
    for _ in range(2):
        bf.bf_graph_launch(g, st)
    check(b, W1, db.result(), FP32_TOL, "graph")
    g.close()
    plan.close()


def test_server_launches_after_update():
    torch = require_gpu()
    rng = np.random.default_rng(905)
    W0 = wl.unit_norm_pool(rng, 2, wl.F_MAX)
    W1 = W0.copy()
    W1[1] = wl.unit_norm_pool(rng, 1, wl.F_MAX)[0]
    plan = bf.bf_plan_create(W0)
    S = torch.from_numpy(wl.qam256(rng, (4 * wl.F_MAX * wl.B,)).astype(np.complex64)).cuda()
    R = torch.full((8, wl.M, wl.B), float("nan"), dtype=torch.complex64, device="cuda")
    rb = wl.M * wl.B * 8
    announce("server across an update")
    with bf.bf_server_create(plan, n_streams=2) as srv:
        bf.bf_submit(srv, bf.make_request(1, wl.F_MAX, 4, S.data_ptr(), R.data_ptr(), tag=0))
        got = []
        while len(got) < 1:
            got.extend(bf.bf_poll(srv, 8, 100000).tolist())
        bf.bf_plan_update(plan, 1, W1[1])
        bf.bf_submit(srv, bf.make_request(1, wl.F_MAX, 4, S.data_ptr(), R.data_ptr() + 4 * rb, tag=1))
        while len(got) < 2:
            got.extend(bf.bf_poll(srv, 8, 100000).tolist())
    torch.cuda.synchronize()
    blocks = S.cpu().numpy()
    s_off = np.arange(4, dtype=np.int64) * wl.F_MAX * wl.B
    res = R.cpu().numpy()
    for half, W in ((0, W0), (1, W1)):
        ref = orc.apply_arrays(W, np.full(4, 1, np.int32), np.full(4, wl.F_MAX, np.int32), blocks, s_off)
        assert np.max(orc.rel_frobenius(res[4 * half: 4 * half + 4], ref)) <= FP32_TOL, f"request {half}"
    plan.close()


def test_update_rejects_bad_arguments():
    require_gpu()
    rng = np.random.default_rng(906)
    plan = bf.bf_plan_create(wl.unit_norm_pool(rng, 2, 8))
    for w_id in (-1, 2):
        with pytest.raises(bf.BfError) as ei:
            bf.bf_plan_update(plan, w_id, np.zeros((64, 8), np.complex64))
        assert ei.value.status == bf.BF_ERR_INVALID
    with pytest.raises(ValueError):
        bf.bf_plan_update(plan, 0, np.zeros((64, 9), np.complex64))
    plan.close()
