"""Edge cases of the batch entry points on the GPU, for every precision form:
empty batches, batches made only of empty products (f = 0: R must be all
zeros, S may be null), and one batch four times the full-width workload,
checked against the oracle on every product."""
import math

import numpy as np
import pytest

from gpu_util import FP32_TOL, all_errors, announce, rel_errors, require_gpu
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl
from paper_1810_11451_amd.device import DeviceBatch

pytestmark = pytest.mark.gpu
FORMS = {"fp32": bf.BF_FP32, "fp32_3m": bf.BF_FP32_3M, "fp16": bf.BF_FP16, "bf16": bf.BF_BF16,
         "fp16x2": bf.BF_FP16X2, "bf16x2": bf.BF_BF16X2}
# the parity bars of each form (plain 16-bit: 4 u sqrt(2), u the unit roundoff)
BAR = {"fp32": FP32_TOL, "fp32_3m": FP32_TOL, "fp16x2": 2e-5, "bf16x2": 2e-5,
       "fp16": 4 * 2.0 ** -11 * math.sqrt(2), "bf16": 4 * 2.0 ** -8 * math.sqrt(2)}


def test_empty_batches_are_no_ops():
    """batch = 0 returns at once, launches nothing and leaves the plan usable."""
    torch = require_gpu()
    rng = np.random.default_rng(901)
    b = wl.random_batch(rng, 5, 2, f_values=[3, 36])
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_ALL)
    R_empty = torch.empty((0,), dtype=torch.complex64, device="cuda")
    announce("empty batches, every form")
    for name, prec in FORMS.items():
        bf.bf_apply(plan, [], [], [], [], prec)
        bf.bf_apply_packed(plan, [], [], None, [], R_empty, prec)
        db = DeviceBatch(b)
        db.apply(plan, prec)
        err, _ = rel_errors(b, db.result())
        assert np.max(err) <= BAR[name], name
    plan.close()


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("n", [1, 300])
def test_only_empty_products_write_zeros(form, n):
    """Every product has f = 0 and a null S: R is overwritten with zeros
    (the empty sum), whatever it held before."""
    torch = require_gpu()
    rng = np.random.default_rng(902 + n)
    W = wl.unit_norm_pool(rng, 3, 36)
    w_ids = rng.integers(0, 3, size=n).astype(np.int32)
    R = torch.empty((n, bf.BF_M, bf.BF_B), dtype=torch.complex64, device="cuda")
    R.view(torch.float32).fill_(float("nan"))
    r_ptrs = (R.data_ptr() + np.arange(n, dtype=np.uint64) * (bf.BF_M * bf.BF_B * 8)).astype(np.uint64)
    plan = bf.bf_plan_create(W, bf.BF_PREC_BIT(FORMS[form]))
    announce(f"only f = 0 form={form} n={n}")
    bf.bf_apply(plan, w_ids, np.zeros(n, np.int32), np.zeros(n, np.uint64), r_ptrs, FORMS[form])
    torch.cuda.synchronize()
    assert torch.count_nonzero(R.view(torch.float32)).item() == 0
    plan.close()


@pytest.mark.parametrize("form", ["fp32_3m", "fp16x2"])
def test_four_times_full_width_all_items(form):
    """65536 products in one launch (four times the full-width workload):
    every product against the oracle, chunk by chunk."""
    torch = require_gpu()
    n = 4 * 16384
    b = wl.full_width_batch(seed=903, n=n)
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(FORMS[form]))
    db = DeviceBatch(b, fill_r=float("nan"))
    announce(f"four times full width form={form} n={n}")
    db.apply(plan, FORMS[form])
    torch.cuda.synchronize()
    err = all_errors(b, db.R[0])
    assert np.max(err) <= BAR[form], f"max rel err {np.max(err):.3g}"
    plan.close()


@pytest.mark.parametrize("variant", [None, (3, 0, 0, 2), (3, 0, 0, 5), (3, 0, 0, 8), (3, 0, 0, 9), (2, 2, 0, 0),
                                     (1, 2, 1, 0)])
@pytest.mark.parametrize("form", sorted(FORMS))
def test_pool_without_columns(form, variant):
    """A pool with f_max = 0 (every product is the empty sum): the plan is
    valid in every form, and R comes back all zeros under the default and
    under forced variants (the wave-specialised ones, which load W
    unconditionally, are routed to schedules that do not)."""
    torch = require_gpu()
    n = 70
    W = np.zeros((2, bf.BF_M, 0), np.complex64)
    R = torch.empty((n, bf.BF_M, bf.BF_B), dtype=torch.complex64, device="cuda")
    R.view(torch.float32).fill_(float("nan"))
    r_ptrs = (R.data_ptr() + np.arange(n, dtype=np.uint64) * (bf.BF_M * bf.BF_B * 8)).astype(np.uint64)
    plan = bf.bf_plan_create(W, bf.BF_PREC_BIT(FORMS[form]))
    assert bf.bf_plan_info(plan)[1] == 0
    if variant is not None:
        for bk in range(5):
            bf.bf_set_variant(plan, FORMS[form], bk, *variant)
    announce(f"pool with f_max = 0 form={form} variant={variant}")
    bf.bf_apply(plan, np.arange(n, dtype=np.int32) % 2, np.zeros(n, np.int32), np.zeros(n, np.uint64),
                r_ptrs, FORMS[form])
    torch.cuda.synchronize()
    assert torch.count_nonzero(R.view(torch.float32)).item() == 0
    plan.close()
