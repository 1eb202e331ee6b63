"""Helpers shared by the GPU tests (not collected by pytest)."""
import sys

import numpy as np

from oracle import oracle as orc
from paper_1810_11451_amd import bf
from paper_1810_11451_amd.device import DeviceBatch

FP32_TOL = 2e-6     # relative Frobenius error per product, FP32 path


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm GPU (run with -m 'not gpu' on CPU)")
    if not bf.LIB_PATH.exists():
        raise RuntimeError("libbf.so is not built")
    return torch


def run_batch(batch, prec=bf.BF_FP32, mask=None, packed=False, variant=None, plan=None):
    """Plan + apply through the C ABI; returns (R as complex64 [n,64,60], plan)."""
    require_gpu()
    own = plan is None
    if own:
        plan = bf.bf_plan_create(batch.W, mask if mask is not None else bf.BF_PREC_BIT(prec))
    if variant is not None:
        for b in range(5):
            bf.bf_set_variant(plan, prec, b, *variant)
    db = DeviceBatch(batch)
    db.apply(plan, prec, packed=packed)
    R = db.result()
    if own:
        plan.close()
    return R


def rel_errors(batch, R, items=None):
    ref = orc.apply(batch, items=items)
    got = R if items is None else R[np.asarray(items)]
    return orc.rel_frobenius(got, ref), ref


def all_errors(batch, R, chunk: int = 2048) -> np.ndarray:
    """Relative Frobenius error of every product against the oracle, in
    chunks of products so that the complex128 reference of a full-size
    batch is never held at once.  R is a complex64 numpy array [n, 64, 60]
    or a device tensor of that shape (copied to the host chunk by chunk)."""
    n = batch.n
    err = np.empty(n, np.float64)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        items = np.arange(lo, hi)
        got = R[lo:hi]
        if not isinstance(got, np.ndarray):
            got = got.cpu().numpy()
        err[lo:hi] = orc.rel_frobenius(got, orc.apply(batch, items=items))
    return err
