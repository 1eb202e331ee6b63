"""Host check of the library's product orders 1 to 4 (order_items in
libbf.so, called from tests/native/order_check.cpp built with hipcc for the
host): all are permutations; orders 1 and 2 sort as documented, stably, on
batches of mixed and of one f; order 3 gives each wave-specialised
workgroup runs of one W; order 4 balances the workgroups' summed f within
each XCD part."""
import shutil
import subprocess
from pathlib import Path

import pytest

from paper_1810_11451_amd import bf

ROOT = Path(__file__).resolve().parents[1]


def test_product_orders(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if Path("/opt/rocm/bin/hipcc").exists() else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("no hipcc")
    if not bf.LIB_PATH.exists():
        from paper_1810_11451_amd import build
        build.build()
    exe = tmp_path / "order_check"
    lib_dir = bf.LIB_PATH.parent
    cmd = [hipcc, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", str(ROOT / "include"),
           "-I", str(ROOT / "paper_1810_11451_amd" / "csrc"), "-x", "hip",
           str(ROOT / "tests" / "native" / "order_check.cpp"), "-o", str(exe),
           "-L", str(lib_dir), "-lbf", f"-Wl,-rpath,{lib_dir}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "orders ok" in r.stderr
