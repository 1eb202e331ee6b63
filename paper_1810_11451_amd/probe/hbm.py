"""Achievable HBM bandwidth: time a plain streaming copy of known size
(and, with --mode mfma, the sustained FP32 matrix-core rate).

    python -m paper_1810_11451_amd.probe.hbm [--mib 1024] [--iters 20] [--grid G] [--mode M]

Prints one JSON line with the copy's read+write GB/s.  Under a counter run
(rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE) the same command gives the bytes
the counters report for a known traffic of `mib` MiB read and written per
dispatch, which scales the counters of the beamforming kernel.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
LIB = HERE / "libbfprobe.so"


def build() -> Path:
    from paper_1810_11451_amd.build import ARCH, COMMON, hipcc
    cmd = [hipcc(), *COMMON, "-x", "hip", "-shared", "-fPIC", str(HERE / "hbm_probe.hip"),
           "-o", str(LIB)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"probe build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return LIB


def measure(mib: int = 1024, iters: int = 20, mode: str = "copy", grid: int = 0,
            variant: int = 1) -> dict:
    """Times the streaming kernel on `mib` MiB (read, written or both) with
    HIP events; returns its figures as a dict (GBps counts read + written)."""
    import torch
    if not LIB.exists():
        raise RuntimeError(f"{LIB} not built")
    L = ctypes.CDLL(str(LIB))
    L.bfprobe_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    m = {"copy": 0, "read": 1, "write": 2}[mode]
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    grid = grid or 256 * 8
    st = torch.cuda.current_stream()
    for _ in range(3):
        if L.bfprobe_stream(src.data_ptr(), dst.data_ptr(), nbytes, grid, variant, m,
                            st.cuda_stream) != 0:
            raise RuntimeError("probe launch failed")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(iters):
        L.bfprobe_stream(src.data_ptr(), dst.data_ptr(), nbytes, grid, variant, m, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    rd = nbytes if m != 2 else 0
    wr = nbytes if m != 1 else 0
    if m == 0 and not bool(torch.equal(src[:1024], dst[:1024])):
        raise RuntimeError("probe copy is wrong")
    del src, dst
    return {"probe": "hbm_" + mode, "bytes_read": rd, "bytes_written": wr,
            "us": round(ms * 1e3, 2), "GBps": round((rd + wr) / ms / 1e6, 1), "grid": grid,
            "variant": variant}


def measure_mfma(iters: int = 20000, grid: int = 0, reps: int = 3) -> dict:
    """Times the FP32 matrix-core loop (v_mfma_f32_32x32x2_f32, four
    independent chains per wave, two waves per SIMD) with HIP events;
    returns its sustained TFLOP/s."""
    import torch
    if not LIB.exists():
        raise RuntimeError(f"{LIB} not built")
    L = ctypes.CDLL(str(LIB))
    L.bfprobe_mfma.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    grid = grid or 256 * 2
    out = torch.empty(grid * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    if L.bfprobe_mfma(out.data_ptr(), grid, 100, st.cuda_stream) != 0:
        raise RuntimeError("mfma probe launch failed")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        L.bfprobe_mfma(out.data_ptr(), grid, iters, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = grid * 4 * iters * 4 * 4096
    del out
    return {"probe": "mfma_fp32_32x32x2", "us": round(ms * 1e3, 2),
            "TFLOPs": round(flops / ms / 1e9, 2), "grid": grid, "iters": iters}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--grid", type=int, default=0, help="workgroups (0: 256 CUs x 8)")
    ap.add_argument("--variant", type=int, default=1,
                    help="bit 0 non-temporal, bits 1-2 log2 unroll (default 1: plain nt copy)")
    ap.add_argument("--mode", default="copy", choices=["copy", "read", "write", "mfma"])
    a = ap.parse_args(argv)
    if a.mode == "mfma":
        print(json.dumps(measure_mfma(grid=a.grid)), flush=True)
    else:
        print(json.dumps(measure(a.mib, a.iters, a.mode, a.grid, a.variant)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
