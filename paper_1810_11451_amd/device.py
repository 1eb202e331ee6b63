"""Device buffers for a workloads.Batch (torch is used for memory only).

Uploads a batch's S buffer, allocates R, and builds the per-item device
pointer arrays that bf_apply takes.  No product arithmetic happens here.
"""
from __future__ import annotations

import numpy as np

from . import bf
from .workloads import B, M, Batch

R_ELEMS = M * B            # complex elements per R
R_BYTES = R_ELEMS * 8


class DeviceBatch:
    def __init__(self, batch: Batch, device: str = "cuda", fill_r: float | None = float("nan"),
                 copies: int = 1):
        import torch
        self.batch = batch
        self.torch = torch
        self.n = batch.n
        self.copies = copies
        S = batch.S if batch.S.size else np.zeros(1, np.complex64)
        self.S = [torch.from_numpy(S).to(device) for _ in range(copies)]
        self.R = [torch.empty((max(self.n, 1), M, B), dtype=torch.complex64, device=device)
                  for _ in range(copies)]
        if fill_r is not None:
            for r in self.R:
                r.view(torch.float32).fill_(fill_r)
        self.s_off = batch.s_off.astype(np.int64)
        self.s_ptrs = [np.where(batch.f > 0, s.data_ptr() + self.s_off * 8, 0).astype(np.uint64)
                       for s in self.S]
        self.r_ptrs = [(r.data_ptr() + np.arange(self.n, dtype=np.uint64) * R_BYTES).astype(np.uint64)
                       for r in self.R]

    def apply(self, plan, prec=bf.BF_FP32, copy: int = 0, stream=None, packed: bool = False):
        b = self.batch
        if packed:
            bf.bf_apply_packed(plan, b.w_ids, b.f, self.S[copy], self.s_off, self.R[copy], prec, stream)
        else:
            bf.bf_apply(plan, b.w_ids, b.f, self.s_ptrs[copy], self.r_ptrs[copy], prec, stream)

    def result(self, copy: int = 0) -> np.ndarray:
        self.torch.cuda.synchronize()
        return self.R[copy][: self.n].cpu().numpy()
