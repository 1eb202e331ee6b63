"""Per-step time of bf_apply over a fresh process's first steps.

    python -m paper_1810_11451_amd.probe.startup [--steps 600] [--pre none|mfma|copy|apply|touch]
        [--pre-ms 800] [--gap-ms 0] [--graph] [--variant S:W:O:T]

Runs the three-product FP32 form on the full-width batch (16384 products of
64x36 by 36x60, three rotating buffer sets) for --steps steps, each bracketed
by an event pair, and prints one JSON line: the first ten step times and the
means of consecutive groups of 25 steps (microseconds).  Before that the
process may load the GPU for --pre-ms with the matrix-core probe, the copy
probe, or the apply path itself, then stay idle for --gap-ms; --pre touch
fills the R buffers first.  --graph launches captured graphs instead of
bf_apply.  Under `rocprofv3 --kernel-trace` or `--pmc GRBM_GUI_ACTIVE` the
same command gives each dispatch's duration and engine clock.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--pre", default="none", choices=["none", "mfma", "copy", "apply", "touch"])
    ap.add_argument("--pre-ms", type=float, default=800.0)
    ap.add_argument("--gap-ms", type=float, default=0.0)
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--variant", default=None, help="schedule:wg_per_cu:order:store for every f bucket")
    a = ap.parse_args(argv)

    import torch

    from paper_1810_11451_amd import bf
    from paper_1810_11451_amd import workloads as wl
    from paper_1810_11451_amd.device import DeviceBatch

    prec = bf.BF_FP32_3M
    torch.cuda.set_device(0)
    batch = wl.full_width_batch()
    plan = bf.bf_plan_create(batch.W, bf.BF_PREC_BIT(prec))
    if a.variant:
        v = [int(x) for x in a.variant.split(":")]
        for bk in range(5):
            bf.bf_set_variant(plan, prec, bk, *v)
    db = DeviceBatch(batch, copies=3, fill_r=None)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    print(f"[startup] setup done, pre {a.pre}", file=sys.stderr, flush=True)
    if a.pre == "touch":
        for r in db.R:
            r.view(torch.float32).fill_(0.0)
        torch.cuda.synchronize()
    elif a.pre in ("mfma", "copy"):
        from paper_1810_11451_amd.probe import hbm
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < a.pre_ms:
            if a.pre == "mfma":
                hbm.measure_mfma(iters=20000, reps=1)
            else:
                hbm.measure(mib=1024, iters=10)
        torch.cuda.synchronize()
    elif a.pre == "apply":
        t0 = time.perf_counter()
        i = 0
        while (time.perf_counter() - t0) * 1e3 < a.pre_ms:
            db.apply(plan, prec, copy=i % 3)
            i += 1
            if i % 50 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
    if a.gap_ms > 0:
        time.sleep(a.gap_ms / 1e3)
    if a.graph:
        graphs = [bf.bf_graph_create(plan, batch.w_ids, batch.f, db.s_ptrs[c], db.r_ptrs[c], prec)
                  for c in range(3)]
        step = lambda i: bf.bf_graph_launch(graphs[i % 3], st)  # noqa: E731
    else:
        step = lambda i: db.apply(plan, prec, copy=i % 3)  # noqa: E731
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    for i in range(a.steps):
        ev[i][0].record(st)
        step(i)
        ev[i][1].record(st)
    torch.cuda.synchronize()
    us = np.array([x.elapsed_time(y) for x, y in ev]) * 1e3
    groups = [round(float(us[i:i + 25].mean()), 1) for i in range(0, a.steps, 25)]
    print(json.dumps({"pre": a.pre, "pre_ms": a.pre_ms, "gap_ms": a.gap_ms, "graph": a.graph,
                      "variant": a.variant, "first10": [round(float(x), 1) for x in us[:10]],
                      "bucket25_us": groups}), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
