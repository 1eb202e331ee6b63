"""CPU tests of the C ABI: exports, status strings and host-side argument checks.

None of these touch a GPU: the library loads without one, and every check
exercised here rejects its arguments before any HIP call.
"""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_1810_11451_amd import bf

ROOT = Path(__file__).resolve().parents[1]


def declared_functions(header="bf.h", prefix="bf_"):
    text = (ROOT / "include" / header).read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(" + prefix + r"[a-z_0-9]+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not bf.LIB_PATH.exists():
        from paper_1810_11451_amd import build
        build.build()
    return bf.lib()


@pytest.mark.parametrize("header", ["bf.h", "bf_serve_host.h"])
@pytest.mark.parametrize("lang,std,compiler", [("c", "-std=c99", "gcc"), ("c++", "-std=c++17", "g++")])
def test_headers_compile_on_their_own(header, lang, std, compiler):
    """Each public header is valid C and C++ by itself (a stray comment end
    or a missing include shows up here, not only in the library build)."""
    import shutil
    import subprocess
    if shutil.which(compiler) is None:
        pytest.skip(f"no {compiler}")
    r = subprocess.run([compiler, std, "-fsyntax-only", "-Wall", "-Werror", "-x", lang,
                        str(ROOT / "include" / header)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("bf_plan_create", "bf_plan_destroy", "bf_apply", "bf_status_str", "bf_last_error",
                 "bf_graph_create", "bf_autotune"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_names_match_header():
    import paper_1810_11451_amd.bf as mod
    for n in declared_functions():
        assert hasattr(mod, n) and n in mod._SIGS, n


def test_status_strings(L):
    for code, name in [(0, "BF_OK"), (-1, "BF_ERR_INVALID"), (-2, "BF_ERR_OOM"),
                       (-3, "BF_ERR_DEVICE"), (-4, "BF_ERR_BUSY"), (-5, "BF_ERR_TIMEOUT"),
                       (-6, "BF_ERR_UNSUPPORTED")]:
        assert bf.bf_status_str(code) == name
    assert "gfx950" in bf.bf_build_info()


def _good(n=4):
    w = np.array([0, 1, 2, 1], np.int32)[:n]
    f = np.array([36, 0, 5, 1], np.int32)[:n]
    S = np.array([0x1000, 0, 0x2008, 0x3010], np.uint64)[:n]
    R = np.array([0x10000, 0x20000, 0x30010, 0x40000], np.uint64)[:n]
    return w, f, S, R


def test_check_batch_accepts_valid(L):
    w, f, S, R = _good()
    assert bf.bf_check_batch(3, 36, w, f, S, R) == bf.BF_OK
    assert bf.bf_check_batch(3, 36, w[:0], f[:0], S[:0], R[:0]) == bf.BF_OK


@pytest.mark.parametrize("mutate,needle", [
    (lambda w, f, S, R: w.__setitem__(2, 3), "w_id 3"),
    (lambda w, f, S, R: w.__setitem__(0, -1), "w_id -1"),
    (lambda w, f, S, R: f.__setitem__(3, 37), "f 37"),
    (lambda w, f, S, R: f.__setitem__(1, -2), "f -2"),
    (lambda w, f, S, R: S.__setitem__(0, 0), "S pointer"),
    (lambda w, f, S, R: S.__setitem__(2, 0x2004), "S pointer"),
    (lambda w, f, S, R: R.__setitem__(1, 0), "R pointer"),
    (lambda w, f, S, R: R.__setitem__(3, 0x40001), "R pointer"),
    (lambda w, f, S, R: R.__setitem__(2, 0x30008), "16-byte"),
])
def test_check_batch_rejects(L, mutate, needle):
    w, f, S, R = _good()
    mutate(w, f, S, R)
    assert bf.bf_check_batch(3, 36, w, f, S, R) == bf.BF_ERR_INVALID
    assert needle in bf.bf_last_error()


def test_check_batch_f_limited_by_pool(L):
    w, f, S, R = _good()
    assert bf.bf_check_batch(3, 8, w, f, S, R) == bf.BF_ERR_INVALID
    assert "item 0" in bf.bf_last_error()


def test_null_s_allowed_for_f_zero(L):
    w, f, S, R = _good()
    assert S[1] == 0 and f[1] == 0
    assert bf.bf_check_batch(3, 36, w, f, S, R) == bf.BF_OK


def test_plan_create_rejects_bad_arguments_before_device(L):
    h = ctypes.c_void_p()
    w = np.zeros((1, 64, 4), np.complex64)
    assert L.bf_plan_create(ctypes.byref(h), None, 1, 4, 0, None) == bf.BF_ERR_INVALID
    assert L.bf_plan_create(ctypes.byref(h), w.ctypes.data, 0, 4, 0, None) == bf.BF_ERR_INVALID
    assert L.bf_plan_create(ctypes.byref(h), w.ctypes.data, 1, 37, 0, None) == bf.BF_ERR_INVALID
    assert L.bf_plan_create(ctypes.byref(h), w.ctypes.data, 1, 4, 1 << 7, None) == bf.BF_ERR_INVALID
    assert L.bf_plan_create(None, w.ctypes.data, 1, 4, 0, None) == bf.BF_ERR_INVALID
    assert h.value is None


def test_calls_on_null_handles(L):
    assert L.bf_apply(None, 0, None, None, None, None, 0, None) == bf.BF_ERR_INVALID
    assert L.bf_plan_destroy(None) == bf.BF_ERR_INVALID
    assert L.bf_graph_launch(None, None) == bf.BF_ERR_INVALID
    assert L.bf_graph_destroy(None) == bf.BF_ERR_INVALID
    assert L.bf_tune_save(None, b"/tmp/x") == bf.BF_ERR_INVALID
    assert L.bf_tune_load(None, b"/tmp/x") == bf.BF_ERR_INVALID
    assert L.bf_tune_query(None, 0, 36, None, None) == bf.BF_ERR_INVALID


def test_plan_update_rejects_null_arguments(L):
    w = np.zeros((64, 4), np.complex64)
    assert L.bf_plan_update(None, 0, w.ctypes.data, None) == bf.BF_ERR_INVALID
    assert "plan is null" in bf.bf_last_error()


def test_filter_rejects_bad_arguments_before_device(L):
    h = ctypes.c_void_p()
    taps = np.ones(4, np.complex64)
    assert L.bf_filter_create(None, taps.ctypes.data, 4, None) == bf.BF_ERR_INVALID
    assert L.bf_filter_create(ctypes.byref(h), None, 4, None) == bf.BF_ERR_INVALID
    assert L.bf_filter_create(ctypes.byref(h), taps.ctypes.data, 0, None) == bf.BF_ERR_INVALID
    assert L.bf_filter_create(ctypes.byref(h), taps.ctypes.data, 2049, None) == bf.BF_ERR_INVALID
    assert "n_taps" in bf.bf_last_error()
    assert L.bf_filter_apply(None, 1, None, None, None) == bf.BF_ERR_INVALID
    assert L.bf_filter_destroy(None) == bf.BF_ERR_INVALID
    assert h.value is None


def test_server_create_rejects_null_plan(L):
    h = ctypes.c_void_p()
    assert L.bf_server_create(ctypes.byref(h), None, None) == bf.BF_ERR_INVALID
    assert L.bf_submit(None, None, None) == bf.BF_ERR_INVALID
    assert L.bf_poll(None, None, 0, 0) == bf.BF_ERR_INVALID
    assert L.bf_server_destroy(None) == bf.BF_ERR_INVALID


def test_record_layouts_match_header():
    assert ctypes.sizeof(bf.bf_server_cfg) == 32
    assert ctypes.sizeof(bf.bf_server_stats) == 80
    assert bf.REQUEST_DTYPE.itemsize == 48 and bf.COMPLETION_DTYPE.itemsize == 56


def test_monotonic_clock(L):
    import time
    a = bf.bf_now_ns()
    b = time.monotonic_ns()
    assert abs(a - b) < 10_000_000_000


def test_f_bucket(L):
    assert [bf.bf_f_bucket(f) for f in (0, 1, 8, 9, 17, 18, 27, 35, 36)] == [0, 0, 0, 1, 1, 2, 3, 3, 4]


def test_python_wrapper_raises_with_detail(L):
    with pytest.raises(bf.BfError) as ei:
        bf.bf_plan_create(np.zeros((1, 64, 40), np.complex64))
    assert ei.value.status == bf.BF_ERR_INVALID and "f_max" in ei.value.detail


def test_filter_binding_checks_tensor_sizes():
    """The binding refuses tensors that cannot hold the batch (CPU tensors
    stand in: the check happens before anything reaches the library)."""
    import torch
    small = torch.zeros((2, bf.N_FILTER), dtype=torch.complex64)
    ok = torch.zeros((3, bf.N_FILTER), dtype=torch.complex64)
    with pytest.raises(ValueError, match="bytes"):
        bf._filter_buffer(small, 3, "x")
    assert bf._filter_buffer(ok, 3, "x") == ok.data_ptr()
    with pytest.raises(ValueError, match="contiguous"):
        bf._filter_buffer(ok.t(), 1, "x")
    with pytest.raises(ValueError, match="complex64"):
        bf._filter_buffer(torch.zeros((3, bf.N_FILTER), dtype=torch.float64), 1, "x")
    assert bf._filter_buffer(12345, 7, "x") == 12345


def test_packed_binding_checks_tensor_sizes():
    """bf_apply_packed refuses S or R tensors too small for the batch before
    the library is called (plan handle unused: the check comes first)."""
    import torch

    class NoPlan:
        handle = None

    f = np.array([2, 0, 3], np.int32)
    s_off = np.array([0, 0, 120], np.int64)      # last item ends at 120 + 180 = 300
    w = np.zeros(3, np.int32)
    S_small = torch.zeros(299, dtype=torch.complex64)
    R_ok = torch.zeros((3, bf.BF_M, bf.BF_B), dtype=torch.complex64)
    with pytest.raises(ValueError, match="S_base"):
        bf.bf_apply_packed(NoPlan(), w, f, S_small, s_off, R_ok)
    S_ok = torch.zeros(300, dtype=torch.complex64)
    with pytest.raises(ValueError, match="R_base"):
        bf.bf_apply_packed(NoPlan(), w, f, S_ok, s_off, R_ok[:2])


def test_host_executor_exports_its_header():
    """include/bf_serve_host.h: the host-only executor of the serving loop
    exports every declared call, and its binding names them all."""
    from paper_1810_11451_amd import hostexec
    names = declared_functions("bf_serve_host.h", "bfh_")
    assert "bfh_submit" in names and "bfh_device_complete" in names
    H = hostexec.lib()
    missing = [n for n in names if not hasattr(H, n)]
    assert not missing, f"not exported: {missing}"
    assert set(names) <= set(hostexec._SIGS), set(names) - set(hostexec._SIGS)
