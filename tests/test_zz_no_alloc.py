"""bf_apply_noalloc (descriptor block in the library's fixed device array)
against bf_apply on the same inputs, through the C ABI.

Two calls in a row on one plan and stream, the second with a smaller batch
(ragged f, f = 0 included) than the first (the largest the call holds), so
the array keeps the first call's contents when the second runs.  Each
result must equal bf_apply's bit for bit (the same kernels run on the same
descriptors) and meet the FP32 bar against the FP64 oracle on every
product.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, all_errors, announce, require_gpu
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl
from paper_1810_11451_amd.device import DeviceBatch

pytestmark = pytest.mark.gpu

TOL = {bf.BF_FP32: FP32_TOL, bf.BF_FP32_3M: FP32_TOL, bf.BF_FP16X2: 2e-5}


def _batches():
    big = wl.full_width_batch(n=bf_max())
    rng = np.random.default_rng(77)
    f_values = np.concatenate([np.arange(0, 37), rng.integers(0, 37, 1963)])
    small = wl.random_batch(rng, len(f_values), 64, f_values=f_values, dist="unit")
    return big, small


def bf_max():
    return 16384


@pytest.mark.parametrize("prec", [bf.BF_FP32_3M, bf.BF_FP32, bf.BF_FP16X2],
                         ids=["fp32_3m", "fp32", "fp16x2"])
def test_noalloc_matches_apply_on_two_calls(prec):
    torch = require_gpu()
    big, small = _batches()
    stream = torch.cuda.current_stream()
    for k, b in enumerate((big, small)):
        announce(f"noalloc prec={bf.PREC_NAMES[prec]} call={k} n={b.n}")
        plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(prec))
        ref = DeviceBatch(b)
        got = DeviceBatch(b)
        bf.bf_apply(plan, b.w_ids, b.f, ref.s_ptrs[0], ref.r_ptrs[0], prec, stream)
        bf.bf_apply_noalloc(plan, b.w_ids, b.f, got.s_ptrs[0], got.r_ptrs[0], prec, stream)
        R_ref = ref.result()
        R_got = got.result()
        plan.close()
        assert np.array_equal(R_got.view(np.uint32), R_ref.view(np.uint32)), \
            f"call {k}: bf_apply_noalloc differs from bf_apply"
        nz = b.f > 0
        assert np.all(R_got[~nz] == 0)
        err = all_errors(b, R_got)
        assert np.max(err[nz]) <= TOL[prec], f"call {k}: max rel err {np.max(err[nz]):.3g}"


def test_noalloc_rejects_batches_above_its_array():
    torch = require_gpu()
    b = wl.full_width_batch(n=bf_max() + 1)
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(bf.BF_FP32_3M))
    db = DeviceBatch(b)
    with pytest.raises(bf.BfError) as e:
        bf.bf_apply_noalloc(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0], bf.BF_FP32_3M,
                            torch.cuda.current_stream())
    assert e.value.status == bf.BF_ERR_INVALID and "16384" in e.value.detail
    torch.cuda.synchronize()
    assert np.all(np.isnan(db.result().view(np.float32))), "nothing may be launched"
    plan.close()
