"""Python binding of libbf (the C ABI in include/bf.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libbf.so.  Function names match the C entry points.  Device
buffers may be given as torch tensors (anything with ``data_ptr()``) or as
integer addresses; streams as ``torch.cuda.Stream``, a raw ``hipStream_t``
integer, or None (torch's current stream when torch has a GPU, else the
default stream).

There is no fallback: if libbf.so is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().with_name("libbf.so")

BF_M, BF_B, BF_FMAX = 64, 60, 36
BF_OK, BF_ERR_INVALID, BF_ERR_OOM, BF_ERR_DEVICE = 0, -1, -2, -3
BF_ERR_BUSY, BF_ERR_TIMEOUT, BF_ERR_UNSUPPORTED = -4, -5, -6
BF_FP32, BF_FP16, BF_BF16, BF_FP16X2, BF_BF16X2, BF_FP32_3M = 0, 1, 2, 3, 4, 5
PREC_NAMES = {BF_FP32: "fp32", BF_FP16: "fp16", BF_BF16: "bf16",
              BF_FP16X2: "fp16x2", BF_BF16X2: "bf16x2", BF_FP32_3M: "fp32_3m"}
PREC_ALL = BF_PREC_ALL = 0x3F


def BF_PREC_BIT(p: int) -> int:
    return 1 << int(p)


class BfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status_name(status)} ({detail})")
        self.status = status
        self.detail = detail


class bf_variant(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32), ("store", ctypes.c_int32)]

    def as_tuple(self):
        return (self.schedule, self.wg_per_cu, self.order, self.store)


class bf_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("deadline_us", ctypes.c_int64),
                ("n_streams", ctypes.c_int32), ("max_batch_items", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("prec", ctypes.c_int32)]


class bf_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("submitted", "admitted", "completed", "refused", "launches", "deadline_misses",
                 "inflight_bytes", "peak_inflight_bytes", "queued", "launch_host_ns")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


# numpy layouts of bf_request (48 bytes) and bf_completion (56 bytes)
REQUEST_DTYPE = np.dtype([("w_id", "<i4"), ("f", "<i4"), ("n_s", "<i4"), ("reserved", "<i4"),
                          ("S", "<u8"), ("R", "<u8"), ("tag", "<u8"), ("t_arrival_ns", "<i8")])
COMPLETION_DTYPE = np.dtype([("ticket", "<u8"), ("tag", "<u8"), ("status", "<i4"),
                             ("deadline_missed", "<i4"), ("t_arrival_ns", "<i8"),
                             ("t_submit_ns", "<i8"), ("t_launch_ns", "<i8"), ("t_done_ns", "<i8")])
assert REQUEST_DTYPE.itemsize == 48 and COMPLETION_DTYPE.itemsize == 56

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_SIGS = {
    "bf_plan_create": (_i32, [ctypes.POINTER(_vp), _vp, _i32, _i32, _u32, _vp]),
    "bf_plan_destroy": (_i32, [_vp]),
    "bf_plan_info": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_u32)]),
    "bf_plan_update": (_i32, [_vp, _i32, _vp, _vp]),
    "bf_filter_create": (_i32, [ctypes.POINTER(_vp), _vp, _i32, _vp]),
    "bf_filter_apply": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "bf_filter_spectrum": (_i32, [_vp, _vp]),
    "bf_filter_destroy": (_i32, [_vp]),
    "bf_apply": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp]),
    "bf_apply_packed": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "bf_apply_noalloc": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp]),
    "bf_plan_set_kernel_events": (_i32, [_vp, _vp, _vp]),
    "bf_check_batch": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "bf_graph_create": (_i32, [ctypes.POINTER(_vp), _vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp]),
    "bf_graph_launch": (_i32, [_vp, _vp]),
    "bf_graph_destroy": (_i32, [_vp]),
    "bf_set_variant": (_i32, [_vp, _i32, _i32, ctypes.POINTER(bf_variant)]),
    "bf_get_variant": (_i32, [_vp, _i32, _i32, ctypes.POINTER(bf_variant)]),
    "bf_f_bucket": (_i32, [_i32]),
    "bf_autotune": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _i32, _vp,
                           ctypes.POINTER(bf_variant), ctypes.POINTER(ctypes.c_float)]),
    "bf_tune_save": (_i32, [_vp, ctypes.c_char_p]),
    "bf_tune_load": (_i32, [_vp, ctypes.c_char_p]),
    "bf_tune_query": (_i32, [_vp, _i32, _i32, ctypes.POINTER(bf_variant), ctypes.POINTER(ctypes.c_float)]),
    "bf_status_str": (ctypes.c_char_p, [_i32]),
    "bf_last_error": (ctypes.c_char_p, []),
    "bf_build_info": (ctypes.c_char_p, []),
    "bf_device_cu_count": (_i32, []),
    "bf_server_create": (_i32, [ctypes.POINTER(_vp), _vp, ctypes.POINTER(bf_server_cfg)]),
    "bf_submit": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "bf_submit_batch": (_i32, [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_uint64)]),
    "bf_poll": (_i32, [_vp, _vp, _i32, _i64]),
    "bf_server_stats_get": (_i32, [_vp, ctypes.POINTER(bf_server_stats)]),
    "bf_server_destroy": (_i32, [_vp]),
    "bf_now_ns": (_i64, []),
}

_lib = None


def lib():
    """Load libbf.so (once).  Raises if it is not built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1810_11451_amd.build`. "
                               "The beamforming path has no CPU fallback.")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_name(s: int) -> str:
    try:
        return lib().bf_status_str(int(s)).decode()
    except Exception:  # pragma: no cover - library not loadable
        return str(s)


def bf_last_error() -> str:
    return lib().bf_last_error().decode()


def bf_status_str(s: int) -> str:
    return lib().bf_status_str(int(s)).decode()


def bf_build_info() -> str:
    return lib().bf_build_info().decode()


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise BfError(rc, where, bf_last_error())
    return rc


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, (int, np.integer)):
        return int(x)
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError(f"cannot take a device address of {type(x)}")


def _stream(s) -> int:
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream)
        except Exception:  # pragma: no cover
            pass
        return 0
    if isinstance(s, (int, np.integer)):
        return int(s)
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    raise TypeError(f"not a stream: {type(s)}")


def _i32_array(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a), dtype=np.int32)
    if n is not None and a.shape != (n,):
        raise ValueError(f"expected {n} entries, got shape {a.shape}")
    return a


def _ptr_array(ptrs, n) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray([_ptr(p) for p in ptrs] if not isinstance(ptrs, np.ndarray)
                                        else ptrs, dtype=np.uint64))
    if a.shape != (n,):
        raise ValueError(f"expected {n} pointers, got shape {a.shape}")
    return a


class Plan:
    """Owns a bf_plan handle; destroyed with bf_plan_destroy on close()."""

    def __init__(self, handle: int, n_w: int, f_max: int, mask: int):
        self.handle = handle
        self.n_w = n_w
        self.f_max = f_max
        self.mask = mask

    def close(self):
        if self.handle:
            _check(lib().bf_plan_destroy(self.handle), "bf_plan_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover - best effort
        try:
            if self.handle:
                lib().bf_plan_destroy(self.handle)
        except Exception:
            pass


def bf_plan_create(w_pool: np.ndarray, prec_mask: int = 0, stream=None) -> Plan:
    w = np.ascontiguousarray(w_pool, dtype=np.complex64)
    if w.ndim != 3 or w.shape[1] != BF_M:
        raise ValueError(f"w_pool must be [n_w, 64, f_max], got {w.shape}")
    h = _vp()
    _check(lib().bf_plan_create(ctypes.byref(h), w.ctypes.data, w.shape[0], w.shape[2],
                                int(prec_mask), _stream(stream)), "bf_plan_create")
    return Plan(h.value, w.shape[0], w.shape[2], int(prec_mask) or 1)


def bf_plan_destroy(plan: Plan) -> None:
    plan.close()


def bf_plan_info(plan: Plan):
    n_w, f_max, mask = _i32(), _i32(), _u32()
    _check(lib().bf_plan_info(plan.handle, ctypes.byref(n_w), ctypes.byref(f_max),
                              ctypes.byref(mask)), "bf_plan_info")
    return n_w.value, f_max.value, mask.value


def bf_plan_update(plan: Plan, w_id: int, w: np.ndarray, stream=None) -> None:
    """Replace pool entry w_id with w (complex64 [64, f_max]); see bf.h."""
    w = np.ascontiguousarray(w, dtype=np.complex64)
    if w.shape != (BF_M, plan.f_max):
        raise ValueError(f"w must be [64, {plan.f_max}], got {w.shape}")
    _check(lib().bf_plan_update(plan.handle, int(w_id), w.ctypes.data, _stream(stream)),
           "bf_plan_update")


def bf_apply(plan: Plan, w_ids, f, S_ptrs, R_ptrs, prec: int = BF_FP32, stream=None) -> None:
    w_ids = _i32_array(w_ids)
    n = w_ids.shape[0]
    f = _i32_array(f, n)
    S = _ptr_array(S_ptrs, n)
    R = _ptr_array(R_ptrs, n)
    _check(lib().bf_apply(plan.handle, n, w_ids.ctypes.data, f.ctypes.data, S.ctypes.data,
                          R.ctypes.data, int(prec), _stream(stream)), "bf_apply")


def bf_apply_noalloc(plan: Plan, w_ids, f, S_ptrs, R_ptrs, prec: int = BF_FP32, stream=None) -> None:
    w_ids = _i32_array(w_ids)
    n = w_ids.shape[0]
    f = _i32_array(f, n)
    S = _ptr_array(S_ptrs, n)
    R = _ptr_array(R_ptrs, n)
    _check(lib().bf_apply_noalloc(plan.handle, n, w_ids.ctypes.data, f.ctypes.data, S.ctypes.data,
                                  R.ctypes.data, int(prec), _stream(stream)), "bf_apply_noalloc")


def bf_plan_set_kernel_events(plan: Plan, start=None, stop=None) -> None:
    """Events (torch.cuda.Event(enable_timing=True), or raw hipEvent_t
    handles) that the apply kernel of each later bf_apply* call on the plan
    records at its own start and end; None, None switches it off."""
    def handle(e):
        if e is None:
            return None
        return int(e.cuda_event) if hasattr(e, "cuda_event") else int(e)
    _check(lib().bf_plan_set_kernel_events(plan.handle, handle(start), handle(stop)),
           "bf_plan_set_kernel_events")


def bf_apply_packed(plan: Plan, w_ids, f, S_base, s_off, R_base, prec: int = BF_FP32,
                    stream=None) -> None:
    w_ids = _i32_array(w_ids)
    n = w_ids.shape[0]
    f = _i32_array(f, n)
    s_off = np.ascontiguousarray(np.asarray(s_off), dtype=np.int64)
    if s_off.shape != (n,):
        raise ValueError("s_off must have one entry per item")
    # Tensors are checked for size: the library sees only addresses.
    if hasattr(S_base, "numel"):
        live = f > 0
        need = int(np.max(s_off[live] + f[live].astype(np.int64) * BF_B)) if np.any(live) else 0
        if not S_base.is_contiguous() or S_base.numel() * S_base.element_size() < need * 8:
            raise ValueError(f"S_base must be contiguous and hold {need} complex64 values")
    if hasattr(R_base, "numel"):
        need = n * BF_M * BF_B
        if not R_base.is_contiguous() or R_base.numel() * R_base.element_size() < need * 8:
            raise ValueError(f"R_base must be contiguous and hold {need} complex64 values")
    _check(lib().bf_apply_packed(plan.handle, n, w_ids.ctypes.data, f.ctypes.data, _ptr(S_base),
                                 s_off.ctypes.data, _ptr(R_base), int(prec), _stream(stream)),
           "bf_apply_packed")


def bf_check_batch(n_w: int, f_max: int, w_ids, f, S_ptrs, R_ptrs) -> int:
    """Host-only check; returns the bf_status (does not raise)."""
    w_ids = _i32_array(w_ids)
    n = w_ids.shape[0]
    f = _i32_array(f, n)
    S = _ptr_array(S_ptrs, n)
    R = _ptr_array(R_ptrs, n)
    return int(lib().bf_check_batch(n_w, f_max, n, w_ids.ctypes.data, f.ctypes.data,
                                    S.ctypes.data, R.ctypes.data))


class Graph:
    def __init__(self, handle: int):
        self.handle = handle

    def close(self):
        if self.handle:
            _check(lib().bf_graph_destroy(self.handle), "bf_graph_destroy")
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            if self.handle:
                lib().bf_graph_destroy(self.handle)
        except Exception:
            pass


def bf_graph_create(plan: Plan, w_ids, f, S_ptrs, R_ptrs, prec: int = BF_FP32,
                    stream=None) -> Graph:
    w_ids = _i32_array(w_ids)
    n = w_ids.shape[0]
    f = _i32_array(f, n)
    S = _ptr_array(S_ptrs, n)
    R = _ptr_array(R_ptrs, n)
    h = _vp()
    _check(lib().bf_graph_create(ctypes.byref(h), plan.handle, n, w_ids.ctypes.data, f.ctypes.data,
                                 S.ctypes.data, R.ctypes.data, int(prec), _stream(stream)),
           "bf_graph_create")
    return Graph(h.value)


def bf_graph_launch(graph: Graph, stream=None) -> None:
    _check(lib().bf_graph_launch(graph.handle, _stream(stream)), "bf_graph_launch")


def bf_graph_destroy(graph: Graph) -> None:
    graph.close()


def bf_f_bucket(f: int) -> int:
    return int(lib().bf_f_bucket(int(f)))


def batch_bucket(f) -> int:
    """Tuning-table bucket the library uses for a batch: that of its mean f."""
    f = np.asarray(f, dtype=np.int64)
    if f.size == 0:
        return 0
    return bf_f_bucket(int((int(f.sum()) + f.size // 2) // f.size))


def bf_set_variant(plan: Plan, prec: int, bucket: int, schedule: int, wg_per_cu: int = 0,
                   order: int = 1, store: int = 0) -> None:
    v = bf_variant(schedule, wg_per_cu, order, store)
    _check(lib().bf_set_variant(plan.handle, int(prec), int(bucket), ctypes.byref(v)),
           "bf_set_variant")


def bf_get_variant(plan: Plan, prec: int, bucket: int):
    v = bf_variant()
    _check(lib().bf_get_variant(plan.handle, int(prec), int(bucket), ctypes.byref(v)),
           "bf_get_variant")
    return v.as_tuple()


def bf_autotune(plan: Plan, w_ids, f, S_ptrs, R_ptrs, prec: int = BF_FP32, reps: int = 5,
                stream=None):
    w_ids = _i32_array(w_ids)
    n = w_ids.shape[0]
    f = _i32_array(f, n)
    S = _ptr_array(S_ptrs, n)
    R = _ptr_array(R_ptrs, n)
    best = bf_variant()
    us = ctypes.c_float()
    _check(lib().bf_autotune(plan.handle, n, w_ids.ctypes.data, f.ctypes.data, S.ctypes.data,
                             R.ctypes.data, int(prec), int(reps), _stream(stream),
                             ctypes.byref(best), ctypes.byref(us)), "bf_autotune")
    return best.as_tuple(), float(us.value)


def bf_tune_save(plan: Plan, path: str) -> None:
    _check(lib().bf_tune_save(plan.handle, str(path).encode()), "bf_tune_save")


def bf_tune_load(plan: Plan, path: str) -> None:
    _check(lib().bf_tune_load(plan.handle, str(path).encode()), "bf_tune_load")


def bf_device_cu_count() -> int:
    return _check(lib().bf_device_cu_count(), "bf_device_cu_count")


# ---- serving ---------------------------------------------------------------

class Server:
    def __init__(self, handle: int, plan: Plan):
        self.handle = handle
        self.plan = plan   # keeps the plan alive while the server runs

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(lib().bf_server_destroy(h), "bf_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def bf_server_create(plan: Plan, hbm_budget_bytes: int = 16 << 30, deadline_us: int = 0,
                     n_streams: int = 2, max_batch_items: int = 16384,
                     queue_capacity: int = 65536, prec: int = BF_FP32) -> Server:
    cfg = bf_server_cfg(int(hbm_budget_bytes), int(deadline_us), int(n_streams),
                        int(max_batch_items), int(queue_capacity), int(prec))
    h = _vp()
    _check(lib().bf_server_create(ctypes.byref(h), plan.handle, ctypes.byref(cfg)),
           "bf_server_create")
    return Server(h.value, plan)


def make_request(w_id: int, f: int, n_s: int, S, R, tag: int = 0, t_arrival_ns: int = 0):
    r = np.zeros(1, REQUEST_DTYPE)
    r["w_id"], r["f"], r["n_s"] = w_id, f, n_s
    r["S"], r["R"], r["tag"], r["t_arrival_ns"] = _ptr(S), _ptr(R), tag, t_arrival_ns
    return r


def bf_submit_batch(server: Server, reqs) -> tuple:
    """Submit REQUEST_DTYPE records in one call; returns (requests queued,
    first ticket).  Fewer than given means the queue filled."""
    reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
    t = ctypes.c_uint64()
    n = _check(lib().bf_submit_batch(server.handle, reqs.ctypes.data, int(reqs.shape[0]),
                                     ctypes.byref(t)), "bf_submit_batch")
    return int(n), int(t.value)


def bf_submit(server: Server, req) -> int:
    """Submit one request (a REQUEST_DTYPE record); returns its ticket."""
    req = np.ascontiguousarray(req, dtype=REQUEST_DTYPE)
    t = ctypes.c_uint64()
    _check(lib().bf_submit(server.handle, req.ctypes.data, ctypes.byref(t)), "bf_submit")
    return int(t.value)


def bf_poll(server: Server, max_n: int = 1024, timeout_us: int = 0) -> np.ndarray:
    """Up to max_n completions (COMPLETION_DTYPE); empty on timeout."""
    out = np.zeros(max_n, COMPLETION_DTYPE)
    rc = lib().bf_poll(server.handle, out.ctypes.data, int(max_n), int(timeout_us))
    if rc == BF_ERR_TIMEOUT:
        return out[:0]
    _check(rc, "bf_poll")
    return out[:rc]


def bf_server_stats_get(server: Server) -> dict:
    st = bf_server_stats()
    _check(lib().bf_server_stats_get(server.handle, ctypes.byref(st)), "bf_server_stats_get")
    return st.as_dict()


def bf_server_destroy(server: Server) -> None:
    server.close()


def bf_now_ns() -> int:
    return int(lib().bf_now_ns())


LOADGEN_PATH = LIB_PATH.parent / "loadgen" / "libbf_loadgen.so"
_loadgen = None


def loadgen_replay(server: Server, reqs: np.ndarray, t_offset_ns: np.ndarray,
                   progress_every: int = 0, stall_ms: int = 0, label: str = "replay",
                   with_submit_ns: bool = False) -> tuple:
    """Replays reqs (REQUEST_DTYPE) at the given offsets from a native thread
    (benchmark helper); returns (completions in request order, busy retries),
    and with with_submit_ns the nanoseconds spent inside bf_submit calls.
    progress_every > 0 prints a stderr line per that many completions;
    stall_ms > 0 gives up (BfError, BF_ERR_TIMEOUT) when requests are
    outstanding and none completes for that long."""
    global _loadgen
    lib()
    if _loadgen is None:
        if not LOADGEN_PATH.exists():
            raise RuntimeError(f"{LOADGEN_PATH} is not built")
        L = ctypes.CDLL(str(LOADGEN_PATH))
        L.bf_loadgen_replay.restype = _i64
        L.bf_loadgen_replay.argtypes = [_vp, _vp, _vp, _i64, _vp, _i64, _i64, ctypes.c_char_p,
                                        ctypes.POINTER(_i64)]
        _loadgen = L
    reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
    t_off = np.ascontiguousarray(t_offset_ns, dtype=np.int64)
    if t_off.shape != (reqs.shape[0],):
        raise ValueError("one offset per request")
    done = np.zeros(reqs.shape[0], COMPLETION_DTYPE)
    submit_ns = _i64(0)
    rc = _loadgen.bf_loadgen_replay(server.handle, reqs.ctypes.data, t_off.ctypes.data,
                                   reqs.shape[0], done.ctypes.data, int(progress_every),
                                   int(stall_ms), label.encode(), ctypes.byref(submit_ns))
    _check(rc, "bf_loadgen_replay")
    if with_submit_ns:
        return done, int(rc), int(submit_ns.value)
    return done, int(rc)


# ---- filter stage ----------------------------------------------------------

N_FILTER = 2048


class Filter:
    """Owns a bf_filter handle; destroyed with bf_filter_destroy on close()."""

    def __init__(self, handle: int, n_taps: int):
        self.handle = handle
        self.n_taps = n_taps

    def close(self):
        if self.handle:
            _check(lib().bf_filter_destroy(self.handle), "bf_filter_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover
        try:
            if self.handle:
                lib().bf_filter_destroy(self.handle)
        except Exception:
            pass


def bf_filter_create(h, stream=None) -> Filter:
    h = np.ascontiguousarray(np.asarray(h).reshape(-1), dtype=np.complex64)
    out = _vp()
    _check(lib().bf_filter_create(ctypes.byref(out), h.ctypes.data, int(h.shape[0]), _stream(stream)),
           "bf_filter_create")
    return Filter(out.value, int(h.shape[0]))


def _filter_buffer(a, batch: int, name: str) -> int:
    """Device address of a filter buffer: an int, or a tensor, which must be
    contiguous and hold at least batch x 2048 complex64 values."""
    if not hasattr(a, "data_ptr"):
        return int(a)
    need = int(batch) * N_FILTER * 8
    if not a.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if str(a.dtype) not in ("torch.complex64", "torch.float32"):
        raise ValueError(f"{name} must be complex64 (or float32 pairs), got {a.dtype}")
    have = a.numel() * a.element_size()
    if have < need:
        raise ValueError(f"{name} holds {have} bytes, {need} needed for {batch} blocks")
    return a.data_ptr()


def bf_filter_apply(flt: Filter, batch: int, x, y, stream=None) -> None:
    """x, y: device pointers (int) or contiguous torch tensors of complex64
    [batch, 2048] (checked for size)."""
    xp = _filter_buffer(x, batch, "x")
    yp = _filter_buffer(y, batch, "y")
    _check(lib().bf_filter_apply(flt.handle, int(batch), xp, yp, _stream(stream)), "bf_filter_apply")


def bf_filter_spectrum(flt: Filter) -> np.ndarray:
    H = np.zeros(N_FILTER, np.complex64)
    _check(lib().bf_filter_spectrum(flt.handle, H.ctypes.data), "bf_filter_spectrum")
    return H


def bf_filter_destroy(flt: Filter) -> None:
    flt.close()


def bf_tune_query(plan: Plan, prec: int, f: int):
    """(variant tuple, recorded kernel us or 0) the plan uses for mean f."""
    v = bf_variant()
    us = ctypes.c_float()
    _check(lib().bf_tune_query(plan.handle, int(prec), int(f), ctypes.byref(v), ctypes.byref(us)),
           "bf_tune_query")
    return v.as_tuple(), float(us.value)
