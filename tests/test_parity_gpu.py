"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (FP32 path): relative Frobenius error <= 2e-6 per product; exact
(bitwise) where the arithmetic is exact (identity W, f = 0, Gaussian
integers).  Sizes span several workgroups and ragged f; the full-size
workloads are checked on every item, in the launch configuration the
benchmark uses.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, all_errors, announce, rel_errors, require_gpu, run_batch
from oracle import oracle as orc
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl
from paper_1810_11451_amd.device import DeviceBatch

pytestmark = pytest.mark.gpu

VARIANTS = {
    "one-per-wg": (0, 0, 0),
    "claim-occ-sorted": (1, 0, 1),
    "claim-1-asgiven": (1, 1, 0),
    "claim-3-sorted": (1, 3, 1),
    "stream-occ-sorted": (2, 0, 1),
    "stream-1-asgiven": (2, 1, 0),
    "stream-2-sorted": (2, 2, 1),
    "single-staged": (0, 0, 0, 1),
    "stream-staged": (2, 0, 1, 1),
    "stream-1-staged-asgiven": (2, 1, 0, 1),
    "ws-sorted": (3, 0, 1),
    "ws-asgiven": (3, 0, 0),
    "ws-2-per-cu": (3, 2, 1),
    "ws-8-producers": (3, 0, 1, 1),
    "ws-8-producers-depth-2": (3, 0, 1, 2),
    "ws-8-producers-depth-3": (3, 0, 1, 3),
    "ws-12-producers-asgiven": (3, 0, 0, 4),
    "ws-12-producers-depth-2": (3, 0, 1, 5),
    "ws-xcd-grouped": (3, 0, 2, 1),
    "stream-xcd-grouped": (2, 2, 2),
    "one-per-wg-xcd-grouped": (0, 0, 2),
    "ws16": (3, 0, 0, 6),
    "ws16-sorted-depth-2": (3, 0, 1, 7),
    "ws16-w-copied": (3, 0, 0, 8),
    "ws16-w-copied-xcd-grouped": (3, 0, 2, 8),
    "ws16-w-and-s-copied": (3, 0, 0, 9),
    "ws16-w-blocked": (3, 0, 3, 8),
    "ws16-w-and-s-copied-w-blocked": (3, 0, 3, 9),
    "one-per-wg-w-sorted": (0, 0, 3, 1),
    "ws16-f-balanced": (3, 0, 4, 9),
    "one-per-wg-f-balanced": (0, 0, 4, 1),
}
# 16 x 16 tiles, four products per step (store fields 6 to 9)
WS16 = ["ws16", "ws16-sorted-depth-2", "ws16-w-copied", "ws16-w-and-s-copied"]
WS_VARIANTS = ["ws-sorted", "ws-8-producers", "ws-8-producers-depth-2", "ws-8-producers-depth-3",
               "ws-12-producers-asgiven", "ws-12-producers-depth-2", "ws16", "ws16-w-copied",
               "ws16-w-and-s-copied", "ws16-w-and-s-copied-w-blocked", "ws16-f-balanced"]


@pytest.mark.parametrize("vname", sorted(VARIANTS))
def test_single_w_fp32(vname):
    b = wl.single_w_batch()
    announce(f"single-W fp32 variant={vname} n={b.n}")
    R = run_batch(b, variant=VARIANTS[vname])
    err, _ = rel_errors(b, R)
    assert np.max(err) <= FP32_TOL, f"max rel err {np.max(err):.3g}"


@pytest.mark.parametrize("vname", sorted(VARIANTS))
@pytest.mark.parametrize("seed", [101, 102])
def test_ragged_all_f(vname, seed):
    """Every f in 0..36, several pool entries, items in random order."""
    rng = np.random.default_rng(seed)
    f_values = np.repeat(np.arange(0, 37), 3)
    b = wl.random_batch(rng, len(f_values), 7, f_values=f_values)
    announce(f"ragged seed={seed} variant={vname} n={b.n}")
    R = run_batch(b, variant=VARIANTS[vname])
    err, ref = rel_errors(b, R)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL, f"max rel err {np.max(err[nz]):.3g}"
    assert np.all(R[~nz] == 0), "f = 0 items must be all zeros"


@pytest.mark.parametrize("vname", [None] + WS16)
@pytest.mark.parametrize("f_max", [1, 2, 7, 36])
def test_small_pools(f_max, vname):
    """Pools narrower than 36 (odd and even f_max); the 16 x 16 kernels
    read the three-product W layout, whose offsets follow from f_max."""
    rng = np.random.default_rng(200 + f_max)
    b = wl.random_batch(rng, 50, 3, f_max=f_max)
    announce(f"pool f_max={f_max} n={b.n} variant={vname}")
    R = run_batch(b, variant=VARIANTS[vname] if vname else None)
    err, _ = rel_errors(b, R)
    nz = b.f > 0
    assert np.max(err[nz], initial=0) <= FP32_TOL
    assert np.all(R[~nz] == 0)


def test_packed_entry_point_and_unaligned_s():
    """bf_apply_packed, and S blocks that are only 8-byte aligned."""
    rng = np.random.default_rng(301)
    f = np.array([3, 1, 36, 5, 0, 2, 35], np.int32)
    b = wl.random_batch(rng, len(f), 2, f_values=[0])
    blocks = [wl.cn01(rng, (int(x), wl.B)) for x in f]
    b = wl._pack("unaligned", b.W, b.w_ids, f, blocks)
    # shift every block by one complex element: S offsets become odd
    S2 = np.zeros(b.S.size + len(f), np.complex64)
    off2 = b.s_off + np.arange(len(f)) + 1
    for t in range(len(f)):
        S2[off2[t]: off2[t] + f[t] * wl.B] = b.s_block(t).reshape(-1)
    b2 = wl.Batch("unaligned", b.W, b.w_ids, f, S2, off2)
    announce("packed + 8-byte aligned S")
    for packed in (False, True):
        R = run_batch(b2, packed=packed)
        err, _ = rel_errors(b2, R)
        nz = f > 0
        assert np.max(err[nz]) <= FP32_TOL
        assert np.all(R[~nz] == 0)


def test_identity_is_exact():
    rng = np.random.default_rng(401)
    W = np.stack([wl.identity_w(f, 36) for f in (1, 2, 17, 36)])
    f = np.array([1, 2, 17, 36, 36, 17], np.int32)
    w_ids = np.array([0, 1, 2, 3, 3, 2], np.int32)
    blocks = [wl.cn01(rng, (int(x), wl.B)) for x in f]
    b = wl._pack("identity", W, w_ids, f, blocks)
    announce("identity W")
    R = run_batch(b)
    for t in range(b.n):
        S = b.s_block(t)
        assert np.array_equal(R[t, : f[t]], S), f"item {t}: identity rows differ"
        assert np.all(R[t, f[t]:] == 0)


@pytest.mark.parametrize("vname", [None] + WS16)
def test_exact_integers_bitwise(vname):
    rng = np.random.default_rng(402)
    b = wl.exact_integer_batch(rng, 200, 5)
    announce(f"exact integers n={b.n} variant={vname}")
    R = run_batch(b, variant=VARIANTS[vname] if vname else None)
    ref = orc.apply(b)
    assert np.array_equal(R.astype(np.complex128), ref)


def test_16x16_variants_agree_bitwise():
    """The four-product 16 x 16 kernels (store fields 6 to 9, every
    product order) run the same chain, so they agree bit for bit; the
    32 x 32 kernels group the flows differently and agree within the bar
    only."""
    require_gpu()
    n = bf.bf_device_cu_count() * 3 + 5
    rng = np.random.default_rng(433)
    b = wl.random_batch(rng, n, 9, f_values=np.arange(0, 37))
    announce(f"fp32 16x16 variants bitwise n={n}")
    ref = run_batch(b, variant=VARIANTS["ws16"])
    for v in [(3, 0, 0, 7), (3, 0, 0, 8), (3, 0, 2, 8), (3, 0, 0, 9), (3, 0, 2, 9), (3, 0, 3, 8), (3, 0, 3, 9),
              (3, 0, 4, 8), (3, 0, 4, 9)]:
        R = run_batch(b, variant=v)
        assert np.array_equal(R.view(np.uint32), ref.view(np.uint32)), v
    err, _ = rel_errors(b, ref)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL and np.all(ref[~nz] == 0)


def test_dft_closed_form():
    rng = np.random.default_rng(403)
    W = wl.dft_w(36)[None]
    f = np.array([1, 8, 36], np.int32)
    blocks = [wl.qam256(rng, (int(x), wl.B)) for x in f]
    b = wl._pack("dft", W, np.zeros(3, np.int32), f, blocks)
    announce("DFT W")
    R = run_batch(b)
    for t in range(3):
        pad = np.zeros((wl.M, wl.B), np.complex128)
        pad[: f[t]] = b.s_block(t)
        ref = np.fft.fft(pad, axis=0) / 8.0
        e = np.linalg.norm(R[t] - ref) / np.linalg.norm(ref)
        assert e <= FP32_TOL, f"f={f[t]}: {e:.3g}"


def test_nothing_written_on_invalid_batch():
    torch = require_gpu()
    b = wl.single_w_batch(n=10)
    plan = bf.bf_plan_create(b.W)
    db = DeviceBatch(b)
    w_ids = b.w_ids.copy()
    w_ids[7] = 1   # pool has one entry
    announce("invalid batch leaves R untouched")
    with pytest.raises(bf.BfError) as ei:
        bf.bf_apply(plan, w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0])
    assert ei.value.status == bf.BF_ERR_INVALID and "item 7" in ei.value.detail
    torch.cuda.synchronize()
    assert np.all(np.isnan(db.result().view(np.float32)))
    with pytest.raises(bf.BfError) as ei:
        bf.bf_apply(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0], prec=bf.BF_BF16X2)
    assert ei.value.status == bf.BF_ERR_UNSUPPORTED
    bf.bf_apply(plan, b.w_ids[:0], b.f[:0], db.s_ptrs[0][:0], db.r_ptrs[0][:0])   # no-op
    plan.close()


def test_r_must_be_16_byte_aligned():
    """R is written with 16-byte stores: an R offset by one complex element
    (8-byte aligned only) is refused before anything is launched, in the
    pointer-array, packed and serving entry points."""
    torch = require_gpu()
    b = wl.single_w_batch(n=6)
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(bf.BF_FP32) | bf.BF_PREC_BIT(bf.BF_FP32_3M))
    db = DeviceBatch(b)
    r_ptrs = db.r_ptrs[0].copy()
    r_ptrs[3] += 8
    announce("R offset by one complex element is refused")
    for prec in (bf.BF_FP32, bf.BF_FP32_3M):
        with pytest.raises(bf.BfError) as ei:
            bf.bf_apply(plan, b.w_ids, b.f, db.s_ptrs[0], r_ptrs, prec)
        assert ei.value.status == bf.BF_ERR_INVALID and "item 3" in ei.value.detail
    R = torch.empty((b.n * 64 * 60 + 1,), dtype=torch.complex64, device="cuda")
    R.view(torch.float32).fill_(float("nan"))
    with pytest.raises(bf.BfError) as ei:
        bf.bf_apply_packed(plan, b.w_ids, b.f, db.S[0], db.s_off, R[1:], bf.BF_FP32_3M)
    assert ei.value.status == bf.BF_ERR_INVALID and "16-byte" in ei.value.detail
    torch.cuda.synchronize()
    assert np.all(np.isnan(db.result().view(np.float32)))
    assert torch.isnan(R.view(torch.float32)).all().item()
    with bf.bf_server_create(plan, prec=bf.BF_FP32_3M) as srv:
        req = np.zeros(1, bf.REQUEST_DTYPE)
        req["w_id"], req["f"], req["n_s"] = 0, int(b.f[0]), 1
        req["S"] = int(db.s_ptrs[0][0])
        req["R"] = int(db.r_ptrs[0][0]) + 8
        with pytest.raises(bf.BfError) as ei:
            bf.bf_submit(srv, req[0])
        assert ei.value.status == bf.BF_ERR_INVALID and "16-byte" in ei.value.detail
    plan.close()


def test_two_streams_and_plan_reuse():
    torch = require_gpu()
    rng = np.random.default_rng(501)
    b = wl.random_batch(rng, 300, 4, dist="qam")
    plan = bf.bf_plan_create(b.W)
    db = DeviceBatch(b, copies=2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    announce("two streams")
    for _ in range(3):
        db.apply(plan, copy=0, stream=s1)
        db.apply(plan, copy=1, stream=s2)
    torch.cuda.synchronize()
    ref = orc.apply(b)
    for c in range(2):
        err = orc.rel_frobenius(db.result(c), ref)
        nz = b.f > 0
        assert np.max(err[nz]) <= FP32_TOL
    plan.close()


def test_graph_replay_matches_direct():
    torch = require_gpu()
    b = wl.uneven_batch(n=700)
    plan = bf.bf_plan_create(b.W)
    direct = DeviceBatch(b)
    direct.apply(plan)
    Rd = direct.result()
    db = DeviceBatch(b)
    announce("graph replay x4")
    g = bf.bf_graph_create(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0])
    for rep in range(4):
        db.R[0].view(torch.float32).fill_(float("nan"))
        bf.bf_graph_launch(g)
        torch.cuda.synchronize()
        Rg = db.result()
        assert np.array_equal(Rg.view(np.uint32), Rd.view(np.uint32)), f"replay {rep} differs"
        direct.apply(plan)          # eager work between replays
        torch.cuda.synchronize()
    g.close()
    err, _ = rel_errors(b, Rd)
    assert np.max(err) <= FP32_TOL


@pytest.mark.parametrize("prec,variant", [(bf.BF_FP32, (1, 0, 1)), (bf.BF_FP32, (3, 0, 0, 8)),
                                          (bf.BF_FP32_3M, (3, 0, 0, 7)), (bf.BF_FP32_3M, (3, 0, 0, 8)),
                                          (bf.BF_FP32_3M, (3, 0, 0, 9))],
                         ids=["fp32-claim", "fp32-ws16-w-copied", "fp32_3m-ws16", "fp32_3m-ws16-w-copied",
                              "fp32_3m-ws16-w-and-s-copied"])
def test_graph_launch_inside_a_captured_hip_graph(prec, variant):
    """bf_graph_launch captured into the caller's own hipGraph (torch's
    CUDAGraph): every replay, with eager work between replays, gives the
    direct launch's products bit for bit (the persistent schedules re-arm
    their counters at the end of each launch)."""
    torch = require_gpu()
    b = wl.uneven_batch(n=900)
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(prec))
    for bk in range(5):
        bf.bf_set_variant(plan, prec, bk, *variant)
    direct = DeviceBatch(b)
    direct.apply(plan, prec)
    Rd = direct.result()
    db = DeviceBatch(b)
    g = bf.bf_graph_create(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0], prec)
    announce(f"bf_graph_launch captured, prec={bf.PREC_NAMES[prec]} variant={variant}")
    outer = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(outer):
        bf.bf_graph_launch(g, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        db.R[0].view(torch.float32).fill_(float("nan"))
        outer.replay()
        torch.cuda.synchronize()
        assert np.array_equal(db.result().view(np.uint32), Rd.view(np.uint32)), f"replay {rep} differs"
        direct.apply(plan, prec)    # eager work between replays
        torch.cuda.synchronize()
    del outer
    g.close()
    plan.close()
    plan.close()


def test_autotune_and_cache(tmp_path):
    """The autotuner stores its pick (timed by the kernels' own events) and
    puts back the caller's kernel events; the pick survives save and load."""
    torch = require_gpu()
    b = wl.uneven_batch(n=2000)
    plan = bf.bf_plan_create(b.W)
    db = DeviceBatch(b)
    st = torch.cuda.current_stream()
    mine = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for e in mine:
        e.record(st)
    torch.cuda.synchronize()
    bf.bf_plan_set_kernel_events(plan, mine[0], mine[1])
    announce("autotune")
    best, us = bf.bf_autotune(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0], reps=2)
    assert us > 0
    torch.cuda.synchronize()
    before = mine[0].elapsed_time(mine[1])
    db.apply(plan)                  # records the caller's pair again
    torch.cuda.synchronize()
    after = mine[0].elapsed_time(mine[1])
    assert after > 0 and after != before
    bf.bf_plan_set_kernel_events(plan, None, None)
    bucket = bf.batch_bucket(b.f)
    assert bf.bf_get_variant(plan, bf.BF_FP32, bucket) == best
    f_mean = int(round(float(np.mean(b.f))))
    q_v, q_us = bf.bf_tune_query(plan, bf.BF_FP32, f_mean)
    assert q_v == best and abs(q_us - us) < 1e-3
    path = tmp_path / "tune.txt"
    bf.bf_tune_save(plan, path)
    plan2 = bf.bf_plan_create(b.W)
    bf.bf_tune_load(plan2, path)
    assert bf.bf_get_variant(plan2, bf.BF_FP32, bucket) == best
    db.R[0].fill_(float("nan"))
    db.apply(plan2)
    err, _ = rel_errors(b, db.result())
    assert np.max(err) <= FP32_TOL
    plan.close()
    plan2.close()


def test_full_width_workload_all_items():
    """16384 products, f = 36, pool of 64: the benchmark's workload and
    launch; every product checked against the oracle."""
    b = wl.full_width_batch()
    announce(f"full-width n={b.n}")
    R = run_batch(b)
    assert not np.any(np.isnan(R.view(np.float32))), "some R not written"
    err = all_errors(b, R)
    assert np.max(err) <= FP32_TOL, f"max rel err {np.max(err):.3g}"


def test_uneven_workload_all_items():
    """8192 products with f ~ U{1..36} from a pool of 256: every item checked."""
    b = wl.uneven_batch()
    announce(f"uneven n={b.n}")
    R = run_batch(b)
    err, _ = rel_errors(b, R)
    assert np.max(err) <= FP32_TOL, f"max rel err {np.max(err):.3g}"


@pytest.mark.parametrize("vname", WS_VARIANTS)
@pytest.mark.parametrize("per_wg", [5, 6, 7])
def test_ws_long_shares(vname, per_wg):
    """Persistent wave-specialised schedule with 5-8 products per workgroup
    (one workgroup per CU), so that the producers' prefetch ring wraps and
    every remainder of its unrolled loop occurs; ragged f in random order."""
    torch = require_gpu()
    n_cu = bf.bf_device_cu_count()
    n = n_cu * per_wg + (37 * per_wg) % n_cu
    rng = np.random.default_rng(120 + per_wg)
    b = wl.random_batch(rng, n, 9, f_values=np.arange(0, 37))
    announce(f"ws long shares variant={vname} n={n}")
    R = run_batch(b, variant=VARIANTS[vname])
    err, _ = rel_errors(b, R)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL, f"max rel err {np.max(err[nz]):.3g}"
    assert np.all(R[~nz] == 0)


def test_tune_database(tmp_path):
    """The tuning table as a database keyed by (architecture, CUs, form, f
    bucket): loads only this device's entries (and architecture-free ones),
    keeps other devices' entries when saving, rejects malformed files."""
    torch = require_gpu()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cus = bf.bf_device_cu_count()
    rng = np.random.default_rng(131)
    b = wl.random_batch(rng, 80, 3, dist="qam")
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_ALL)
    default4 = bf.bf_tune_query(plan, bf.BF_FP32, 36)
    path = tmp_path / "db.txt"
    path.write_text("# hand-written entries\n"
                    f"gfx942 304 {bf.BF_FP32} 2 1 2 1 0 99.00\n"
                    f"{arch} {cus} {bf.BF_FP32} 2 2 1 0 1 12.50\n"
                    f"{arch} {cus + 1} {bf.BF_FP32} 3 1 1 1 0 7.00\n"
                    f"{bf.BF_BF16} 1 2 3 0 0\n")
    announce("tune database")
    bf.bf_tune_load(plan, path)
    assert bf.bf_tune_query(plan, bf.BF_FP32, 20) == ((2, 1, 0, 1), 12.5)
    assert bf.bf_tune_query(plan, bf.BF_BF16, 10) == ((2, 3, 0, 0), 0.0)
    assert bf.bf_tune_query(plan, bf.BF_FP32, 27)[0] != (1, 1, 1, 0)   # other CU count: ignored
    assert bf.bf_tune_query(plan, bf.BF_FP32, 36) == default4
    bf.bf_tune_save(plan, path)
    text = path.read_text()
    assert "gfx942 304" in text and f"{arch} {cus + 1}" in text
    plan2 = bf.bf_plan_create(b.W, bf.BF_PREC_ALL)
    bf.bf_tune_load(plan2, path)
    assert bf.bf_tune_query(plan2, bf.BF_FP32, 20) == ((2, 1, 0, 1), 12.5)
    db = DeviceBatch(b)
    db.apply(plan2, bf.BF_FP32)
    err, _ = rel_errors(b, db.result())
    assert np.max(err) <= FP32_TOL
    bad = tmp_path / "bad.txt"
    bad.write_text(f"{arch} {cus} 0 2 9 0 0 0 1.0\n")   # schedule 9 does not exist
    with pytest.raises(bf.BfError) as ei:
        bf.bf_tune_load(plan2, bad)
    assert ei.value.status == bf.BF_ERR_INVALID
    assert bf.bf_tune_query(plan2, bf.BF_FP32, 20) == ((2, 1, 0, 1), 12.5)
    plan.close()
    plan2.close()
