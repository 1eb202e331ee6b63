"""W reuse in the 16 x 16 kernels whose matrix-core waves copy W into LDS
(store fields 8 and 9): a product whose predecessor in the workgroup's
share read the same pool entry, with at least as many 4-flow steps, reads
that copy instead of copying W again.

The batches below are laid out (product order as given, one workgroup per
CU, so workgroup j takes items j, j + nb, j + 2 nb, ... of its XCD's
eighth) so that consecutive products of a workgroup share W while f rises,
falls and stays, and so that the pool entry changes and changes back.
Every product must agree bit for bit with the 16 x 16 kernel whose
producers stage W for every product (store 7, same chain), and with the
FP64 oracle within the FP32 bar.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, announce, rel_errors, require_gpu, run_batch
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl

pytestmark = pytest.mark.gpu

FORMS = {"fp32_3m": bf.BF_FP32_3M, "fp32": bf.BF_FP32}


def _batch(pattern: str, n_cu: int, seed: int) -> wl.Batch:
    rng = np.random.default_rng(seed)
    n = n_cu * 6 + 7
    nb = max(n_cu // 8, 1)        # workgroups per XCD
    t = np.arange(n)
    W = wl.cn01_pool(rng, 3, wl.F_MAX)
    if pattern == "one-w-random-f":
        w_ids = np.zeros(n, np.int32)
        f = rng.integers(0, wl.F_MAX + 1, n)
    elif pattern == "one-w-rising-f":
        # each workgroup's products: f = 1, 7, 13, ... (a new step count each time)
        w_ids = np.ones(n, np.int32)
        f = np.minimum(1 + 6 * (t // nb), wl.F_MAX)
    elif pattern == "runs-of-two":
        # pool entries change every second product of a workgroup, and come back
        w_ids = ((t // (2 * nb)) % 3).astype(np.int32)
        f = rng.integers(1, wl.F_MAX + 1, n)
    else:   # "falling-then-rising": f high first, then low, then high again, one W
        w_ids = np.full(n, 2, np.int32)
        k = t // nb
        f = np.where(k % 3 == 0, 36, np.where(k % 3 == 1, 3, 20))
    f = np.asarray(f, np.int32)
    blocks = [wl.cn01(rng, (int(x), wl.B)) for x in f]
    return wl._pack(pattern, W, w_ids.astype(np.int32), f, blocks)


@pytest.mark.parametrize("pattern", ["one-w-random-f", "one-w-rising-f", "runs-of-two",
                                     "falling-then-rising"])
@pytest.mark.parametrize("form", sorted(FORMS))
def test_w_reuse_matches_per_product_staging(form, pattern):
    require_gpu()
    prec = FORMS[form]
    b = _batch(pattern, bf.bf_device_cu_count(), 950 + len(pattern))
    announce(f"w reuse form={form} pattern={pattern} n={b.n}")
    ref = run_batch(b, prec=prec, variant=(3, 0, 0, 7))
    for v in [(3, 0, 0, 8), (3, 0, 0, 9)]:
        R = run_batch(b, prec=prec, variant=v)
        assert np.array_equal(R.view(np.uint32), ref.view(np.uint32)), (form, pattern, v)
    err, _ = rel_errors(b, ref)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL, f"max rel err {np.max(err[nz]):.3g}"
    assert np.all(ref[~nz] == 0)


@pytest.mark.parametrize("n_w", [1, 5, 64])
@pytest.mark.parametrize("form", sorted(FORMS))
def test_w_blocked_order_matches_per_product_staging(form, n_w):
    """Order 3 (grouped and sorted by W id, dealt to the workgroups in
    blocks) on a random batch of mixed f: the same products, bit for bit,
    as the 16 x 16 kernel with per-product staging in the caller's order."""
    require_gpu()
    prec = FORMS[form]
    rng = np.random.default_rng(970 + n_w)
    n = bf.bf_device_cu_count() * 5 + 11
    b = wl.random_batch(rng, n, n_w, f_values=np.arange(0, 37))
    announce(f"w blocked order form={form} n_w={n_w} n={n}")
    ref = run_batch(b, prec=prec, variant=(3, 0, 0, 7))
    for v in [(3, 0, 3, 8), (3, 0, 3, 9), (3, 0, 4, 9)]:
        R = run_batch(b, prec=prec, variant=v)
        assert np.array_equal(R.view(np.uint32), ref.view(np.uint32)), (form, n_w, v)
    err, _ = rel_errors(b, ref)
    nz = b.f > 0
    assert np.max(err[nz]) <= FP32_TOL and np.all(ref[~nz] == 0)
