"""FP64 oracle for the beamforming product R = W x S.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.
Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  It shares no code with the GPU library.

What it computes (Section III of the paper, beamforming paragraph and its
equation): for every item t of a batch,

    R_t[i][j] = sum_{k < f_t} W_{w_t}[i][k] * S_t[k][j],   i < 64, j < 60,

where W_{w_t} is one precoder of a pool (one row per antenna) whose leading
f_t columns are used, and S_t is the f_t x 60 symbol matrix.  The method is
exactly this matrix product, so the oracle is that definition written out.

Two independent renderings are provided:

* ``apply``: the plain C triple loop in ``bf_oracle.c`` (complex64 inputs
  widened exactly to double, k summed in order 0..f-1, no contraction into
  FMA), threaded over items.  This is the oracle the parity tests and the
  CPU baseline use.
* ``apply_numpy``: the same definition as a numpy sum of rank-one terms in
  complex128, used as a second opinion on small cases.

``rel_frobenius`` is the error metric of the parity bar:
||R_gpu - R_ref||_F / ||R_ref||_F per product, evaluated in FP64.

Parity status: pinned.  The paper prints no worked beamforming values, so
the pins are mathematical (exact rational brute force, a hand-worked
example, identity and DFT closed forms, Parseval, linearity, exact
Gaussian-integer products) plus planted-mistake builds of the C oracle
that those pins must reject.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "bf_oracle.c"
LIB = HERE / "liboracle.so"
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC", "-pthread"]

_lib = None


def build(out: Path = LIB, mutant: int = 0, force: bool = True) -> Path:
    """Compile bf_oracle.c with gcc (mutant > 0 plants a mistake; tests only)."""
    out = Path(out)
    if not force and out.exists() and out.stat().st_mtime >= SRC.stat().st_mtime:
        return out
    cmd = ["gcc", *CFLAGS, f"-DORACLE_MUTANT={int(mutant)}", str(SRC), "-o", str(out) + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(str(out) + ".tmp", out)
    return out


def _bind(path: Path):
    lib = ctypes.CDLL(str(path))
    fn = lib.oracle_bf_apply
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    return lib


def load(path: Path | None = None):
    """Load the oracle library, building it when missing or older than its source."""
    global _lib
    if path is not None:
        return _bind(Path(path))
    if _lib is None:
        build(force=False)
        _lib = _bind(LIB)
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def apply_arrays(W, w_ids, f, S, s_off, m: int | None = None, b: int = 60,
                 threads: int | None = None, lib=None) -> np.ndarray:
    """Run the C oracle on raw arrays.

    W      complex64 [n_w, m, ldw]
    w_ids  int32 [n];  f int32 [n]
    S      complex64 flat buffer, item t's f[t] x b block at complex offset s_off[t]
    Returns complex128 [n, m, b].
    """
    W = np.ascontiguousarray(W, dtype=np.complex64)
    n_w, mm, ldw = W.shape
    m = mm if m is None else m
    w_ids = np.ascontiguousarray(w_ids, dtype=np.int32)
    f = np.ascontiguousarray(f, dtype=np.int32)
    S = np.ascontiguousarray(S, dtype=np.complex64).reshape(-1)
    s_off = np.ascontiguousarray(s_off, dtype=np.int64)
    n = int(w_ids.shape[0])
    if n and int(np.max(s_off + f.astype(np.int64) * b)) > S.shape[0]:
        raise ValueError("S buffer too small for the given offsets")
    R = np.zeros((n, m, b), dtype=np.complex128)
    lib = load() if lib is None else lib
    rc = lib.oracle_bf_apply(n, m, b, ldw, n_w, W.ctypes.data, w_ids.ctypes.data, f.ctypes.data,
                             S.ctypes.data if S.size else None, s_off.ctypes.data, R.ctypes.data,
                             int(threads or default_threads()))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return R


def apply(batch, items=None, threads: int | None = None, lib=None) -> np.ndarray:
    """Oracle results for a workloads.Batch (all items, or the listed ones)."""
    if items is None:
        return apply_arrays(batch.W, batch.w_ids, batch.f, batch.S, batch.s_off,
                            threads=threads, lib=lib)
    items = np.asarray(items, dtype=np.int64)
    return apply_arrays(batch.W, batch.w_ids[items], batch.f[items], batch.S,
                        batch.s_off[items], threads=threads, lib=lib)


def apply_numpy(W, S) -> np.ndarray:
    """One product in complex128 as a sum of rank-one terms, k = 0..f-1.

    W is m x f (or wider; the leading S.shape[0] columns are used), S is f x b.
    """
    W = np.asarray(W, dtype=np.complex128)
    S = np.asarray(S, dtype=np.complex128)
    f = S.shape[0]
    R = np.zeros((W.shape[0], S.shape[1]), dtype=np.complex128)
    for k in range(f):
        R += W[:, k][:, None] * S[k, :][None, :]
    return R


def rel_frobenius(got, ref) -> np.ndarray:
    """Per-product ||got - ref||_F / ||ref||_F in FP64 (leading axis = product).

    A product whose reference is exactly zero (f = 0) scores 0 if the result
    is exactly zero (either sign) and +inf otherwise.
    """
    got = np.asarray(got).astype(np.complex128)
    ref = np.asarray(ref).astype(np.complex128)
    if got.shape != ref.shape:
        raise ValueError(f"shape mismatch {got.shape} vs {ref.shape}")
    axes = tuple(range(1, ref.ndim))
    num = np.sqrt(np.sum(np.abs(got - ref) ** 2, axis=axes))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=axes))
    out = np.empty(num.shape, dtype=np.float64)
    zero = den == 0
    out[~zero] = num[~zero] / den[~zero]
    out[zero] = np.where(num[zero] == 0, 0.0, np.inf)
    return out


if __name__ == "__main__":  # pragma: no cover
    print(build(), file=sys.stderr)
