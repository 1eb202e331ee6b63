"""The serving loop under ThreadSanitizer, on the host executor (no GPU).

tests/native/serve_stress.cpp drives the loop's batcher and completion
threads against a submitter, a poller and a statistics reader through five
scenarios (two and three streams, a budget and queue small enough to refuse
and stall admission, launches made to fail, one item per launch).  It is
built twice: with -fsanitize=thread, where any data race or lock-order
problem ends the run with TSan's exit code, and plainly at a larger scale.

The sanitizer build uses ROCm's clang: the ThreadSanitizer runtime of the
system GCC (11) does not intercept pthread_cond_clockwait, which
std::condition_variable::wait_for uses, and so reports a false double lock
on every timed wait.
"""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
PKG = ROOT / "paper_1810_11451_amd"
SOURCES = [ROOT / "tests" / "native" / "serve_stress.cpp", PKG / "hostexec" / "bf_serve_host.cpp",
           PKG / "csrc" / "bf_serve_core.cpp", PKG / "csrc" / "bf_status.cpp"]
INCLUDES = ["-I", str(ROOT / "include"), "-I", str(PKG / "csrc")]


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and Path(c).exists():
            return c
    return None


def _build(tmp_path, compiler, flags, name):
    out = tmp_path / name
    cmd = [compiler, "-std=c++17", "-pthread", "-g", *flags, *INCLUDES, *map(str, SOURCES), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stderr}"
    return out


def test_serving_loop_has_no_data_races(tmp_path):
    cxx = _clang()
    if cxx is None:
        pytest.skip("no clang++ with a ThreadSanitizer runtime")
    exe = _build(tmp_path, cxx, ["-O1", "-fsanitize=thread"], "serve_stress_tsan")
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 second_deadlock_stack=1")
    r = subprocess.run([str(exe), "1"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stderr[-6000:]}"
    assert "all scenarios ok" in r.stderr


def test_serving_loop_stress_at_scale(tmp_path):
    exe = _build(tmp_path, "g++", ["-O2", "-Wall", "-Wextra"], "serve_stress")
    r = subprocess.run([str(exe), "8"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stderr[-6000:]}"
    assert "all scenarios ok" in r.stderr
