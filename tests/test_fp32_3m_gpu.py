"""GPU parity of the three-product (Gauss) FP32 form against the FP64 oracle.

Bar: relative Frobenius error <= 2e-6 per product, as for the four-product
form.  Exact-integer inputs stay exact (every partial sum, including
(Wr + Wi)(Sr + Si), is an integer far below 2^24), so there the comparison
is bitwise.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, all_errors, announce, rel_errors, require_gpu, run_batch
from oracle import oracle as orc
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl

pytestmark = pytest.mark.gpu
P = bf.BF_FP32_3M
VARIANTS = {"one-per-wg": (0, 0, 0), "ws-sorted": (3, 0, 1), "ws-asgiven": (3, 0, 0),
            "mapped-from-stream": (2, 2, 1), "ws-8-producers": (3, 0, 1, 1),
            "ws-8-producers-depth-2": (3, 0, 1, 2), "ws-8-producers-depth-3": (3, 0, 1, 3),
            "ws-12-producers-asgiven": (3, 0, 0, 4), "ws-12-producers-depth-2": (3, 0, 1, 5),
            "ws16": (3, 0, 0, 6), "ws16-sorted-depth-2": (3, 0, 1, 7),
            "ws16-xcd-grouped-depth-2": (3, 0, 2, 7), "one-per-wg-xcd-grouped": (0, 0, 2),
            "ws16-w-copied-by-matrix-waves": (3, 0, 0, 8), "ws16-w-copied-xcd-grouped": (3, 0, 2, 8),
            "ws16-w-and-s-copied": (3, 0, 0, 9), "ws16-w-and-s-copied-sorted": (3, 0, 1, 9),
            "ws16-w-blocked": (3, 0, 3, 8), "ws16-w-and-s-copied-w-blocked": (3, 0, 3, 9),
            "one-per-wg-w-sorted": (0, 0, 3, 1), "ws16-f-balanced": (3, 0, 4, 9),
            "ws16-f-balanced-w-staged": (3, 0, 4, 7)}
WS16 = ["ws16", "ws16-sorted-depth-2", "ws16-w-copied-by-matrix-waves", "ws16-w-and-s-copied"]


@pytest.mark.parametrize("vname", sorted(VARIANTS))
@pytest.mark.parametrize("seed", [801, 802])
def test_ragged_all_f(vname, seed):
    rng = np.random.default_rng(seed)
    f_values = np.repeat(np.arange(0, 37), 3)
    b = wl.random_batch(rng, len(f_values), 6, f_values=f_values)
    announce(f"3m ragged seed={seed} variant={vname}")
    R = run_batch(b, prec=P, variant=VARIANTS[vname])
    err, _ = rel_errors(b, R)
    nz = b.f > 0
    assert np.all(R[~nz] == 0)
    assert np.max(err[nz]) <= FP32_TOL, f"max rel err {np.max(err[nz]):.3g}"


@pytest.mark.parametrize("vname", ["one-per-wg", "ws-sorted"] + WS16)
def test_exact_integers_bitwise(vname):
    rng = np.random.default_rng(803)
    b = wl.exact_integer_batch(rng, 200, 5)
    announce(f"3m exact integers variant={vname}")
    R = run_batch(b, prec=P, variant=VARIANTS[vname])
    assert np.array_equal(R.astype(np.complex128), orc.apply(b))


@pytest.mark.parametrize("vname", [None] + WS16)
@pytest.mark.parametrize("f_max", [1, 2, 3, 5, 7, 36])
def test_small_pools(f_max, vname):
    """Pools narrower than 36 flows: both W layouts of an entry, and their
    offsets, follow from f_max."""
    rng = np.random.default_rng(810 + f_max)
    b = wl.random_batch(rng, 60, 3, f_max=f_max)
    announce(f"3m pool f_max={f_max} variant={vname}")
    R = run_batch(b, prec=P, variant=VARIANTS[vname] if vname else None)
    err, _ = rel_errors(b, R)
    nz = b.f > 0
    assert np.max(err[nz], initial=0) <= FP32_TOL
    assert np.all(R[~nz] == 0)


def test_dft_and_identity_within_bar():
    rng = np.random.default_rng(804)
    W = np.stack([wl.dft_w(36), wl.identity_w(36, 36)])
    f = np.array([36, 36, 17, 36], np.int32)
    w_ids = np.array([0, 1, 1, 0], np.int32)
    blocks = [wl.qam256(rng, (int(x), wl.B)) for x in f]
    b = wl._pack("dft+identity", W, w_ids, f, blocks)
    announce("3m dft + identity")
    R = run_batch(b, prec=P)
    err, _ = rel_errors(b, R)
    assert np.max(err) <= FP32_TOL


@pytest.mark.parametrize("vname", [None] + WS16)
def test_full_width_workload_all_items(vname):
    b = wl.full_width_batch()
    announce(f"3m full-width n={b.n} variant={vname}")
    R = run_batch(b, prec=P, variant=VARIANTS[vname] if vname else None)
    assert not np.any(np.isnan(R.view(np.float32)))
    err = all_errors(b, R)
    print(f"[fp32_3m] rel err p50 {np.median(err):.3g} max {err.max():.3g}", flush=True)
    assert np.max(err) <= FP32_TOL


@pytest.mark.parametrize("vname", [None] + WS16)
def test_uneven_workload_all_items(vname):
    b = wl.uneven_batch()
    announce(f"3m uneven n={b.n} variant={vname}")
    R = run_batch(b, prec=P, variant=VARIANTS[vname] if vname else None)
    err = all_errors(b, R)
    assert np.max(err) <= FP32_TOL


@pytest.mark.parametrize("vname", ["ws-sorted", "ws-8-producers", "ws-8-producers-depth-2",
                                   "ws-8-producers-depth-3", "ws-12-producers-asgiven",
                                   "ws-12-producers-depth-2"] + WS16)
@pytest.mark.parametrize("per_wg", [1, 2, 5, 6, 7])
def test_ws_long_shares(vname, per_wg):
    """5-8 products per persistent workgroup: the producers' prefetch ring
    wraps and every remainder of its unrolled loop occurs."""
    require_gpu()
    n_cu = bf.bf_device_cu_count()
    n = n_cu * per_wg + (37 * per_wg) % n_cu
    rng = np.random.default_rng(820 + per_wg)
    b = wl.random_batch(rng, n, 9, f_values=np.arange(0, 37))
    announce(f"3m ws long shares variant={vname} n={n}")
    R = run_batch(b, prec=P, variant=VARIANTS[vname])
    err, _ = rel_errors(b, R)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL, f"max rel err {np.max(err[nz]):.3g}"
    assert np.all(R[~nz] == 0)


def test_variants_agree_bitwise():
    """The one-product-per-workgroup and wave-specialised kernels issue the
    same matrix-core steps in the same order on the same operands (Wr + Wi
    formed by one FP32 add in both), so their results agree bit for bit on
    random data, every f included."""
    require_gpu()
    n = bf.bf_device_cu_count() * 3 + 5
    rng = np.random.default_rng(832)
    b = wl.random_batch(rng, n, 9, f_values=np.arange(0, 37))
    announce(f"3m variants bitwise n={n}")
    ref = run_batch(b, prec=P, variant=VARIANTS["one-per-wg"])
    for vname in ["ws-8-producers", "ws-8-producers-depth-2", "ws-asgiven"]:
        R = run_batch(b, prec=P, variant=VARIANTS[vname])
        assert np.array_equal(R.view(np.uint32), ref.view(np.uint32)), vname


def test_16x16_variants_agree_bitwise():
    """The prefetch depths of the 16 x 16 kernel, and its variants whose
    matrix-core waves copy W themselves (and whose producers copy S straight
    to LDS), issue the same matrix-core steps on the same operands, so they
    agree bit for bit; the
    32 x 32 kernels sum the flows in another grouping and agree within the
    bar only."""
    require_gpu()
    n = bf.bf_device_cu_count() * 3 + 5
    rng = np.random.default_rng(833)
    b = wl.random_batch(rng, n, 9, f_values=np.arange(0, 37))
    announce(f"3m 16x16 variants bitwise n={n}")
    ref = run_batch(b, prec=P, variant=VARIANTS["ws16"])
    for v in [(3, 0, 0, 7), (3, 0, 0, 8), (3, 0, 2, 8), (3, 0, 0, 9), (3, 0, 2, 9), (3, 0, 3, 8), (3, 0, 3, 9),
              (3, 0, 4, 8), (3, 0, 4, 9)]:
        R = run_batch(b, prec=P, variant=v)
        assert np.array_equal(R.view(np.uint32), ref.view(np.uint32)), v
    err, _ = rel_errors(b, ref)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL and np.all(ref[~nz] == 0)
