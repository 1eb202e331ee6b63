"""Host check of the block dealing used by product order 3 (ws_deal in
csrc/bf_internal.h, shared by the host ordering and the serving expansion
kernel): tests/native/deal_check.cpp, built with hipcc for the host, checks
that it is a bijection and that each wave-specialised workgroup's share is a
run of consecutive items, for item counts and grids of every size class."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def test_ws_deal_is_a_bijection_onto_workgroup_runs(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if Path("/opt/rocm/bin/hipcc").exists() else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("no hipcc")
    exe = tmp_path / "deal_check"
    cmd = [hipcc, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", str(ROOT / "include"),
           "-I", str(ROOT / "paper_1810_11451_amd" / "csrc"), "-x", "hip",
           str(ROOT / "tests" / "native" / "deal_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ws_deal ok" in r.stderr
