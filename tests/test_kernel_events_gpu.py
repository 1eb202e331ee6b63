"""Kernel timing events (bf_plan_set_kernel_events) through the C ABI.

With a pair set, each apply kernel records it at its own start and end.
For every launch path (each schedule of the FP32, three-product and 16-bit
forms) the products must be bit for bit those of a launch without events,
the recorded interval must be positive and lie inside an event pair that
the test records around the whole call, and after the pair is cleared a
later launch must leave it untouched.
"""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl
from paper_1810_11451_amd.device import DeviceBatch

pytestmark = pytest.mark.gpu

CASES = [
    (bf.BF_FP32, (0, 0, 0)), (bf.BF_FP32, (1, 0, 1)), (bf.BF_FP32, (2, 0, 1, 1)),
    (bf.BF_FP32, (3, 0, 1, 5)), (bf.BF_FP32, (3, 0, 0, 8)), (bf.BF_FP32, (3, 0, 0, 9)),
    (bf.BF_FP32_3M, (0, 0, 2, 1)), (bf.BF_FP32_3M, (3, 0, 0, 1)), (bf.BF_FP32_3M, (3, 0, 0, 7)),
    (bf.BF_FP32_3M, (3, 0, 0, 8)), (bf.BF_FP32_3M, (3, 0, 0, 9)),
    (bf.BF_FP16, (0, 0, 0)), (bf.BF_FP16X2, (2, 0, 1)), (bf.BF_BF16X2, (3, 0, 0, 5)),
    (bf.BF_FP16, (3, 0, 0, 4)),
]


@pytest.mark.parametrize("prec,variant", CASES,
                         ids=[f"{bf.PREC_NAMES[p]}-{':'.join(map(str, v))}" for p, v in CASES])
def test_kernel_events_time_the_kernel_and_change_nothing(prec, variant):
    torch = require_gpu()
    rng = np.random.default_rng(31)
    f_values = np.concatenate([np.arange(0, 37), rng.integers(0, 37, 1500)])
    b = wl.random_batch(rng, len(f_values), 32, f_values=f_values, dist="unit")
    announce(f"kernel events prec={bf.PREC_NAMES[prec]} variant={variant} n={b.n}")
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(prec))
    for bk in range(5):
        bf.bf_set_variant(plan, prec, bk, *variant)
    st = torch.cuda.current_stream()
    ref = DeviceBatch(b)
    got = DeviceBatch(b)
    ref.apply(plan, prec)
    outer = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    inner = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for e in inner:
        e.record(st)   # creates the events
    torch.cuda.synchronize()
    outer[0].record(st)
    bf.bf_plan_set_kernel_events(plan, inner[0], inner[1])
    got.apply(plan, prec)
    bf.bf_plan_set_kernel_events(plan, None, None)
    outer[1].record(st)
    torch.cuda.synchronize()
    k_ms = inner[0].elapsed_time(inner[1])
    o_ms = outer[0].elapsed_time(outer[1])
    # Launched again without events: the pair keeps the first interval.
    got.apply(plan, prec)
    torch.cuda.synchronize()
    assert inner[0].elapsed_time(inner[1]) == k_ms
    assert 0.0 < k_ms <= o_ms, f"kernel {k_ms} ms, whole call {o_ms} ms"
    assert 0.0 <= outer[0].elapsed_time(inner[0])
    assert 0.0 <= inner[1].elapsed_time(outer[1])
    assert np.array_equal(got.result().view(np.uint32), ref.result().view(np.uint32))
    plan.close()


def test_kernel_events_need_both_or_neither():
    torch = require_gpu()
    b = wl.full_width_batch(n=64)
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(bf.BF_FP32))
    e = torch.cuda.Event(enable_timing=True)
    e.record(torch.cuda.current_stream())
    with pytest.raises(bf.BfError):
        bf.bf_plan_set_kernel_events(plan, e, None)
    bf.bf_plan_set_kernel_events(plan, None, None)
    plan.close()
