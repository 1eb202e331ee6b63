"""Python binding of the host-only executor of the serving loop
(include/bf_serve_host.h): libbf's request loop on a null device with a
settable clock, for running and checking the loop without a GPU.

Argument marshalling only; names match the C entry points.  Requests and
completions use the numpy layouts of the main binding (bf.REQUEST_DTYPE,
bf.COMPLETION_DTYPE); S and R are host memory here.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

from .. import bf

LIB_PATH = Path(__file__).resolve().with_name("libbf_serve_host.so")


class bfh_device_cfg(ctypes.Structure):
    _fields_ = [("manual_clock", ctypes.c_int32), ("manual_complete", ctypes.c_int32),
                ("launch_ns", ctypes.c_int64), ("bytes_per_ns", ctypes.c_double),
                ("write_marks", ctypes.c_int32), ("reserved", ctypes.c_int32)]


LAUNCH_DTYPE = np.dtype([("stream", "<i4"), ("n_reqs", "<i4"), ("n_items", "<i4"), ("status", "<i4"),
                         ("bytes", "<u8"), ("t_launch_ns", "<i8"), ("t_end_ns", "<i8"),
                         ("first_ticket", "<u8")])
assert LAUNCH_DTYPE.itemsize == 48

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_SIGS = {
    "bfh_device_create": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(bfh_device_cfg)]),
    "bfh_device_destroy": (_i32, [_vp]),
    "bfh_clock_set": (None, [_vp, _i64]),
    "bfh_clock_now": (_i64, [_vp]),
    "bfh_device_complete": (_i32, [_vp, _i32, _i32, _i32]),
    "bfh_device_fail_launch": (_i32, [_vp, _i64, _i32]),
    "bfh_device_launches": (_i64, [_vp, _vp, _i64]),
    "bfh_device_launch_tickets": (_i64, [_vp, _i64, _vp, _i64]),
    "bfh_device_unfinished": (_i32, [_vp, _i32]),
    "bfh_device_peak_unfinished": (_i32, [_vp]),
    "bfh_server_create": (_i32, [ctypes.POINTER(_vp), _vp, ctypes.POINTER(bf.bf_server_cfg), _i32, _i32]),
    "bfh_submit": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "bfh_submit_batch": (_i32, [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_uint64)]),
    "bfh_poll": (_i32, [_vp, _vp, _i32, _i64]),
    "bfh_server_stats_get": (_i32, [_vp, ctypes.POINTER(bf.bf_server_stats)]),
    "bfh_server_destroy": (_i32, [_vp]),
    "bf_status_str": (ctypes.c_char_p, [_i32]),
    "bf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libbf_serve_host.so (once), building it with g++ if missing."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            from .. import build
            build.build_hostexec()
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise bf.BfError(rc, where, lib().bf_last_error().decode())
    return rc


class Device:
    """A null device; destroyed on close()."""

    def __init__(self, manual_clock=False, manual_complete=False, launch_ns=5000,
                 bytes_per_ns=5000.0, write_marks=False):
        cfg = bfh_device_cfg(int(manual_clock), int(manual_complete), int(launch_ns),
                             float(bytes_per_ns), int(write_marks), 0)
        h = _vp()
        _check(lib().bfh_device_create(ctypes.byref(h), ctypes.byref(cfg)), "bfh_device_create")
        self.handle = h.value

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(lib().bfh_device_destroy(h), "bfh_device_destroy")

    def clock_set(self, t_ns: int) -> None:
        lib().bfh_clock_set(self.handle, int(t_ns))

    def clock_now(self) -> int:
        return int(lib().bfh_clock_now(self.handle))

    def complete(self, stream: int, count: int = 1, status: int = bf.BF_OK) -> int:
        return _check(lib().bfh_device_complete(self.handle, int(stream), int(count), int(status)),
                      "bfh_device_complete")

    def fail_launch(self, index: int, status: int = bf.BF_ERR_DEVICE) -> None:
        _check(lib().bfh_device_fail_launch(self.handle, int(index), int(status)),
               "bfh_device_fail_launch")

    def launches(self) -> np.ndarray:
        n = _check(lib().bfh_device_launches(self.handle, None, 0), "bfh_device_launches")
        out = np.zeros(n, LAUNCH_DTYPE)
        m = _check(lib().bfh_device_launches(self.handle, out.ctypes.data, n), "bfh_device_launches")
        return out[:min(n, m)]

    def launch_tickets(self, k: int) -> np.ndarray:
        n = _check(lib().bfh_device_launch_tickets(self.handle, int(k), None, 0),
                   "bfh_device_launch_tickets")
        out = np.zeros(n, np.uint64)
        _check(lib().bfh_device_launch_tickets(self.handle, int(k), out.ctypes.data, n),
               "bfh_device_launch_tickets")
        return out

    def unfinished(self, stream: int = -1) -> int:
        return _check(lib().bfh_device_unfinished(self.handle, int(stream)), "bfh_device_unfinished")

    def peak_unfinished(self) -> int:
        return _check(lib().bfh_device_peak_unfinished(self.handle), "bfh_device_peak_unfinished")


class Server:
    """The serving loop on a null device; drained and destroyed on close()."""

    def __init__(self, dev: Device, n_w: int, f_max: int = bf.BF_FMAX, hbm_budget_bytes: int = 16 << 30,
                 deadline_us: int = 0, n_streams: int = 2, max_batch_items: int = 16384,
                 queue_capacity: int = 65536, prec: int = bf.BF_FP32):
        cfg = bf.bf_server_cfg(int(hbm_budget_bytes), int(deadline_us), int(n_streams),
                               int(max_batch_items), int(queue_capacity), int(prec))
        h = _vp()
        _check(lib().bfh_server_create(ctypes.byref(h), dev.handle, ctypes.byref(cfg), int(n_w),
                                       int(f_max)), "bfh_server_create")
        self.handle = h.value
        self.dev = dev

    def close(self) -> None:
        if self.handle:
            h, self.handle = self.handle, None
            _check(lib().bfh_server_destroy(h), "bfh_server_destroy")

    def submit(self, req) -> int:
        req = np.ascontiguousarray(req, dtype=bf.REQUEST_DTYPE)
        t = ctypes.c_uint64()
        _check(lib().bfh_submit(self.handle, req.ctypes.data, ctypes.byref(t)), "bfh_submit")
        return int(t.value)

    def submit_batch(self, reqs) -> tuple:
        """Returns (requests queued, first ticket)."""
        reqs = np.ascontiguousarray(reqs, dtype=bf.REQUEST_DTYPE)
        t = ctypes.c_uint64()
        rc = lib().bfh_submit_batch(self.handle, reqs.ctypes.data, int(reqs.shape[0]), ctypes.byref(t))
        _check(rc, "bfh_submit_batch")
        return int(rc), int(t.value)

    def poll(self, max_n: int = 1024, timeout_us: int = 0) -> np.ndarray:
        out = np.zeros(max_n, bf.COMPLETION_DTYPE)
        rc = lib().bfh_poll(self.handle, out.ctypes.data, int(max_n), int(timeout_us))
        if rc == bf.BF_ERR_TIMEOUT:
            return out[:0]
        _check(rc, "bfh_poll")
        return out[:rc]

    def stats(self) -> dict:
        st = bf.bf_server_stats()
        _check(lib().bfh_server_stats_get(self.handle, ctypes.byref(st)), "bfh_server_stats_get")
        return st.as_dict()
