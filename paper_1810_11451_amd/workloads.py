"""Seeded synthetic inputs for the beamforming product R = W x S.

This module only draws and lays out inputs; it contains none of the
product's arithmetic, so both the GPU path and the FP64 oracle can take
their inputs from it without sharing any computation.

Shapes follow the beamforming paragraph of Section III of the paper: W is
64 x f (one row per antenna of the 4 x 8 x 2 array of Section II), S is
f x 60 (one row per flow, one column per resource element), and f ranges
from 0 to 36.  The paper gives no value distributions; these are used:

* CN(0,1): real and imaginary parts independently N(0, 1/2).
* normalised 256-QAM: I and Q independently uniform over the odd levels
  {+-1, +-3, ..., +-15}, divided by sqrt(170) so that E|s|^2 = 1.
* unit-norm-column W: CN(0,1) drawn in FP64, each column divided by its
  2-norm in FP64, then rounded to complex64.
* per-request gains: g = 10**u with u ~ U(-3, 3), applied to S in FP64
  before rounding to complex64.

Every generator takes a ``numpy.random.Generator`` and draws in a fixed
order (W, then W ids, then f, then S, then gains), so a seed fixes the
whole workload.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

M = 64          # antennas (rows of W and R)
B = 60          # resource elements (columns of S and R)
F_MAX = 36      # largest number of flows

QAM_LEVELS = np.arange(-15, 16, 2, dtype=np.int64)   # 16 odd levels
QAM_NORM = math.sqrt(170.0)


def cn01(rng: np.random.Generator, shape) -> np.ndarray:
    """CN(0,1) samples in complex128 (re, im each N(0, 1/2))."""
    s = math.sqrt(0.5)
    re = rng.standard_normal(shape) * s
    im = rng.standard_normal(shape) * s
    return re + 1j * im


def qam256_levels(rng: np.random.Generator, shape) -> np.ndarray:
    """Unnormalised 256-QAM symbols: odd integers in [-15, 15] on each axis."""
    i = QAM_LEVELS[rng.integers(0, 16, size=shape)]
    q = QAM_LEVELS[rng.integers(0, 16, size=shape)]
    return i.astype(np.float64) + 1j * q.astype(np.float64)


def qam256(rng: np.random.Generator, shape) -> np.ndarray:
    """Normalised 256-QAM symbols (unit average power), complex128."""
    return qam256_levels(rng, shape) / QAM_NORM


def unit_norm_pool(rng: np.random.Generator, n_w: int, f_max: int = F_MAX) -> np.ndarray:
    """Pool of n_w precoders 64 x f_max with unit-norm columns, complex64."""
    w = cn01(rng, (n_w, M, f_max))
    norms = np.sqrt(np.sum(np.abs(w) ** 2, axis=1, keepdims=True))
    return (w / norms).astype(np.complex64)


def cn01_pool(rng: np.random.Generator, n_w: int, f_max: int) -> np.ndarray:
    return cn01(rng, (n_w, M, f_max)).astype(np.complex64)


def identity_w(f: int, f_max: int | None = None) -> np.ndarray:
    """W = [I_f ; 0] (64 x f), padded with zero columns up to f_max."""
    f_max = f if f_max is None else f_max
    w = np.zeros((M, f_max), dtype=np.complex64)
    for k in range(f):
        w[k, k] = 1.0
    return w


def dft_w(f: int, f_max: int | None = None) -> np.ndarray:
    """Leading f columns of the unitary 64-point DFT matrix, complex64.

    W[i, k] = exp(-2 pi i * i k / 64) / 8, built in FP64 with the angle
    reduced modulo 64 before the trig call, then rounded.
    """
    f_max = f if f_max is None else f_max
    w = np.zeros((M, f_max), dtype=np.complex128)
    i = np.arange(M)[:, None]
    k = np.arange(f)[None, :]
    ang = -2.0 * np.pi * ((i * k) % M) / M
    w[:, :f] = (np.cos(ang) + 1j * np.sin(ang)) / 8.0
    return w.astype(np.complex64)


def gaussian_int_w(rng: np.random.Generator, n_w: int, f_max: int, bound: int = 8) -> np.ndarray:
    """Precoders with Gaussian-integer entries, |re|, |im| <= bound."""
    re = rng.integers(-bound, bound + 1, size=(n_w, M, f_max))
    im = rng.integers(-bound, bound + 1, size=(n_w, M, f_max))
    return (re + 1j * im).astype(np.complex64)


@dataclasses.dataclass
class Batch:
    """A batch of products R_t = W[w_ids[t]][:, :f[t]] . S_t.

    W      complex64 [n_w, 64, f_max], row-major; entry t uses the leading
           f[t] columns (row stride f_max).
    w_ids  int32 [n]
    f      int32 [n]
    S      complex64 flat buffer; S_t is the f[t] x 60 row-major block that
           starts at complex element s_off[t].
    s_off  int64 [n], offsets in complex elements (multiples of 60).
    gains  float64 [n] or None: the gains already folded into S (reporting).
    """
    name: str
    W: np.ndarray
    w_ids: np.ndarray
    f: np.ndarray
    S: np.ndarray
    s_off: np.ndarray
    gains: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.w_ids.shape[0])

    @property
    def n_w(self) -> int:
        return int(self.W.shape[0])

    @property
    def f_max(self) -> int:
        return int(self.W.shape[2])

    def s_block(self, t: int) -> np.ndarray:
        ft = int(self.f[t])
        o = int(self.s_off[t])
        return self.S[o:o + ft * B].reshape(ft, B)

    def w_block(self, t: int) -> np.ndarray:
        return self.W[int(self.w_ids[t]), :, : int(self.f[t])]

    def flops(self) -> int:
        """Algorithmic flop count: 8 real flops per complex multiply-add."""
        return int(8 * M * B * np.sum(self.f.astype(np.int64)))

    def bytes_moved(self) -> int:
        """Algorithmic HBM bytes per pass: every S read once, every R written once."""
        return int(np.sum(self.f.astype(np.int64)) * B * 8 + self.n * M * B * 8)


def _pack(name, W, w_ids, f, blocks, gains=None) -> Batch:
    f = np.asarray(f, dtype=np.int32)
    sizes = f.astype(np.int64) * B
    s_off = np.zeros(len(f), dtype=np.int64)
    if len(f) > 1:
        s_off[1:] = np.cumsum(sizes)[:-1]
    total = int(np.sum(sizes))
    S = np.zeros(total, dtype=np.complex64)
    for t, blk in enumerate(blocks):
        S[s_off[t]: s_off[t] + sizes[t]] = np.asarray(blk).reshape(-1)
    return Batch(name, np.ascontiguousarray(W, dtype=np.complex64),
                 np.asarray(w_ids, dtype=np.int32), f, S, s_off, gains)


def _uniform_f_batch(name, W, w_ids, f_val, S3) -> Batch:
    """Batch whose items all have the same f, S given as [n, f, 60]."""
    n = S3.shape[0]
    f = np.full(n, f_val, dtype=np.int32)
    s_off = np.arange(n, dtype=np.int64) * (f_val * B)
    return Batch(name, np.ascontiguousarray(W, dtype=np.complex64),
                 np.asarray(w_ids, dtype=np.int32), f,
                 np.ascontiguousarray(S3.reshape(-1), dtype=np.complex64), s_off)


def single_w_batch(seed: int = 1, n: int = 100) -> Batch:
    """One CN(0,1) W of 64 x 8 and n CN(0,1) S of 8 x 60."""
    rng = np.random.default_rng(seed)
    W = cn01_pool(rng, 1, 8)
    w_ids = np.zeros(n, dtype=np.int32)
    S3 = cn01(rng, (n, 8, B)).astype(np.complex64)
    return _uniform_f_batch("single-W 64x8, 100 S 8x60, CN(0,1)", W, w_ids, 8, S3)


def full_width_batch(seed: int = 2, n: int = 16384, n_w: int = 64) -> Batch:
    """Pool of n_w unit-norm W 64 x 36; n normalised 256-QAM S 36 x 60."""
    rng = np.random.default_rng(seed)
    W = unit_norm_pool(rng, n_w, F_MAX)
    w_ids = rng.integers(0, n_w, size=n).astype(np.int32)
    S3 = qam256(rng, (n, F_MAX, B)).astype(np.complex64)
    return _uniform_f_batch(f"full-width f=36, {n} S, pool {n_w} W", W, w_ids, F_MAX, S3)


def uneven_batch(seed: int = 3, n: int = 8192, n_w: int = 256) -> Batch:
    """Uneven batch: f ~ U{1..36}, pool of n_w unit-norm W 64 x 36."""
    rng = np.random.default_rng(seed)
    W = unit_norm_pool(rng, n_w, F_MAX)
    w_ids = rng.integers(0, n_w, size=n).astype(np.int32)
    f = rng.integers(1, F_MAX + 1, size=n).astype(np.int32)
    total = int(np.sum(f)) * B
    S = qam256(rng, (total,)).astype(np.complex64)
    sizes = f.astype(np.int64) * B
    s_off = np.zeros(n, dtype=np.int64)
    s_off[1:] = np.cumsum(sizes)[:-1]
    return Batch(f"uneven f~U(1..36), {n} S, pool {n_w} W", W, w_ids, f, S, s_off)


def gain_batch(seed: int = 4, n: int = 16384, n_w: int = 64) -> Batch:
    """Config-2 workload with per-request gains 10**U(-3, 3) folded into S."""
    rng = np.random.default_rng(seed)
    W = unit_norm_pool(rng, n_w, F_MAX)
    w_ids = rng.integers(0, n_w, size=n).astype(np.int32)
    S3 = qam256(rng, (n, F_MAX, B))
    gains = 10.0 ** rng.uniform(-3.0, 3.0, size=n)
    S3 = (S3 * gains[:, None, None]).astype(np.complex64)
    b = _uniform_f_batch(f"gains 1e-3..1e3, f=36, {n} S, pool {n_w} W", W, w_ids, F_MAX, S3)
    b.gains = gains
    return b


def random_batch(rng: np.random.Generator, n: int, n_w: int, f_max: int = F_MAX,
                 f_values=None, dist: str = "cn") -> Batch:
    """A small random batch for parity tests (f drawn from f_values)."""
    W = cn01_pool(rng, n_w, f_max) if dist == "cn" else unit_norm_pool(rng, n_w, f_max)
    w_ids = rng.integers(0, n_w, size=n).astype(np.int32)
    if f_values is None:
        f_values = np.arange(0, f_max + 1)
    f = np.asarray(rng.choice(np.asarray(f_values), size=n), dtype=np.int32)
    blocks = [cn01(rng, (int(ft), B)) if dist == "cn" else qam256(rng, (int(ft), B)) for ft in f]
    return _pack(f"random n={n}", W, w_ids, f, blocks)


def exact_integer_batch(rng: np.random.Generator, n: int, n_w: int, f_max: int = F_MAX) -> Batch:
    """Gaussian-integer W (|re|,|im| <= 8) and unnormalised odd-level QAM S.

    Every partial sum of a product is a Gaussian integer with parts below
    2 * 36 * 8 * 15 = 8640 < 2**14, far inside FP32's 24-bit significand, and
    every input is exactly representable in FP16 and BF16, so every summation
    order and every precision form gives the exact result.
    """
    W = gaussian_int_w(rng, n_w, f_max)
    w_ids = rng.integers(0, n_w, size=n).astype(np.int32)
    f = rng.integers(0, f_max + 1, size=n).astype(np.int32)
    blocks = [qam256_levels(rng, (int(ft), B)) for ft in f]
    return _pack(f"exact-integer n={n}", W, w_ids, f, blocks)


# ---------------------------------------------------------------------------
# Filter stage (Section III, the filter paragraph): blocks of 2048 complex
# samples and a filter sequence of 1..2048 taps.

N_FILTER = 2048


def filter_signals(rng: np.random.Generator, n: int) -> np.ndarray:
    """n blocks of 2048 CN(0,1) samples, complex64 [n, 2048]."""
    return cn01(rng, (n, N_FILTER)).astype(np.complex64)


def random_taps(rng: np.random.Generator, n_taps: int) -> np.ndarray:
    """n_taps CN(0, 1/n_taps) taps, complex64 (unit expected energy)."""
    return (cn01(rng, (n_taps,)) / math.sqrt(n_taps)).astype(np.complex64)


def lowpass_taps(n_taps: int, cutoff: float) -> np.ndarray:
    """Real windowed-sinc lowpass taps (Hamming window), complex64.

    cutoff is the passband edge as a fraction of the sample rate (0..0.5);
    the taps are normalised to unit DC gain.  A long stopband makes |H|
    span several orders of magnitude, the hard case for the error bar."""
    n = np.arange(n_taps, dtype=np.float64) - (n_taps - 1) / 2.0
    taps = 2.0 * cutoff * np.sinc(2.0 * cutoff * n)
    taps *= 0.54 - 0.46 * np.cos(2.0 * np.pi * np.arange(n_taps) / max(n_taps - 1, 1))
    taps /= np.sum(taps)
    return taps.astype(np.complex64)
