"""Build libbf.so in-tree for gfx950 with hipcc.

    python -m paper_1810_11451_amd.build          # build (always recompiles)

Objects go to paper_1810_11451_amd/_build/, the library to
paper_1810_11451_amd/libbf.so.  Every HIP source is compiled with packed
FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
BUILD = PKG / "_build"
LIB = PKG / "libbf.so"
LOADGEN_SRC = PKG / "loadgen" / "bf_loadgen.cpp"
LOADGEN = PKG / "loadgen" / "libbf_loadgen.so"
HOSTEXEC = PKG / "hostexec" / "libbf_serve_host.so"
# The serving loop's device-independent core, shared by libbf.so and the
# host executor (no HIP in these sources).
SERVE_CORE = [CSRC / "bf_serve_core.cpp", CSRC / "bf_status.cpp"]
HOSTEXEC_SRC = PKG / "hostexec" / "bf_serve_host.cpp"

ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Wno-unused-command-line-argument",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", str(INCLUDE), "-I", str(CSRC),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libbf)")


def sources() -> list[Path]:
    return sorted(CSRC.glob("*.hip")) + sorted(CSRC.glob("*.cpp"))


def _compile(src: Path) -> Path:
    obj = BUILD / (src.name + ".o")
    cmd = [hipcc(), *COMMON, "-x", "hip", "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                     and "not a recognized feature" not in l and l.strip())
    if warn:
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-soname,libbf.so",
           "-o", str(tmp), *map(str, objs), "-lpthread", "-L", "/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # benchmark helper: the serving load generator, linked against libbf.so
    tmp = LOADGEN.with_suffix(".so.tmp")
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-I", str(INCLUDE),
           str(LOADGEN_SRC), "-o", str(tmp), "-L", str(PKG), "-lbf",
           "-Wl,-rpath,$ORIGIN/.."]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LOADGEN)
    build_hostexec()
    if verbose:
        print(f"built {LIB}, {LOADGEN} and {HOSTEXEC}", file=sys.stderr)
    return LIB


def hostexec_cmd(out: Path, extra=()) -> list[str]:
    """g++ line of the host executor (the serving core on a null device)."""
    return ["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra",
            "-I", str(INCLUDE), "-I", str(CSRC), *extra,
            str(HOSTEXEC_SRC), *map(str, SERVE_CORE), "-o", str(out)]


def build_hostexec() -> Path:
    """Builds hostexec/libbf_serve_host.so with g++ (no ROCm needed)."""
    tmp = HOSTEXEC.with_suffix(".so.tmp")
    cmd = hostexec_cmd(tmp, ["-shared"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host executor build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, HOSTEXEC)
    return HOSTEXEC


if __name__ == "__main__":
    build(verbose=True)
