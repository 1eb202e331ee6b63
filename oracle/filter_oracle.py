"""FP64 oracle for the filter stage.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.
Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  It shares no code with the GPU library.

What it computes (Section III of the paper, the filter paragraph and its
formula): a block s of 2048 complex samples is transformed with a 2048-point
FFT, multiplied point by point with the FFT of the filter sequence, and
transformed back:

    y = IFFT(MULT(FFT(s))),   MULT(X)[k] = X[k] * H[k],   H = FFT(h zero-padded to 2048)

with the usual conventions: FFT(x)[k] = sum_n x[n] exp(-2 pi i k n / N) and
IFFT carries the factor 1/N, N = 2048.  The filter sequence h has 1..2048
taps.  The FFTs are library primitives (numpy, complex128); no blocking,
reordering or fusion beyond the formula.

``circular_convolution`` is the same result from its other definition,
y[n] = sum_j h[j] s[(n - j) mod N], written as a sum of shifted copies of
s.  It is the brute-force pin of ``filter_apply`` (the two agree by the
convolution theorem), not a second product path.

``rel_error`` is the error metric of the parity bar:
||y_gpu - y_ref||_2 / (max_k |H[k]| * ||s||_2) per block, in FP64.  Since
the FFT and IFFT are unitary up to their scale factors, ||y|| <= max|H| ||s||,
and rounding errors of the forward transform are amplified by at most
max|H|; normalising by ||y|| instead would blow up for filters whose
stopband removes most of a block's energy.

Parity status: pinned (impulse, shifts, single tones, brute-force circular
convolution, linearity), with planted mistakes those pins must reject.
``rel_error`` is pinned by three hand-worked cases (one tap, two taps, a
tap pair whose spectrum peaks away from k = 0) that separate its
denominator from ||y_ref||, from ||s|| and from max|h| ||s||.
"""
from __future__ import annotations

import numpy as np

N_FILTER = 2048


def padded_taps(h, n: int = N_FILTER) -> np.ndarray:
    h = np.asarray(h, dtype=np.complex128).reshape(-1)
    if not 1 <= h.shape[0] <= n:
        raise ValueError(f"filter needs 1..{n} taps, got {h.shape[0]}")
    out = np.zeros(n, np.complex128)
    out[: h.shape[0]] = h
    return out


def filter_spectrum(h, _mutant: int = 0) -> np.ndarray:
    """H = FFT of the zero-padded filter sequence (complex128, length 2048).

    ``_mutant`` (tests only) plants one plausible mistake:
      2 = taps reversed before the transform, 4 = inverse exponent sign."""
    hp = padded_taps(h)
    if _mutant == 2:
        hp = np.concatenate([hp[: len(np.atleast_1d(h))][::-1], hp[len(np.atleast_1d(h)):]])
    if _mutant == 4:
        return np.fft.ifft(hp) * N_FILTER
    return np.fft.fft(hp)


def filter_apply(s, h, _mutant: int = 0) -> np.ndarray:
    """y = IFFT(FFT(s) * H) for every block (last axis of length 2048).

    ``_mutant`` (tests only): 1 = forward FFT with the inverse exponent sign,
    2/4 = see filter_spectrum, 3 = multiplication by conj(H), 5 = the 1/N of
    the inverse transform left out."""
    s = np.asarray(s, dtype=np.complex128)
    if s.shape[-1] != N_FILTER:
        raise ValueError(f"blocks must have {N_FILTER} samples, got {s.shape[-1]}")
    H = filter_spectrum(h, _mutant if _mutant in (2, 4) else 0)
    if _mutant == 3:
        H = np.conj(H)
    X = np.fft.ifft(s, axis=-1) * N_FILTER if _mutant == 1 else np.fft.fft(s, axis=-1)
    y = np.fft.ifft(X * H, axis=-1)
    if _mutant == 5:
        y = y * N_FILTER
    return y


def circular_convolution(s, h) -> np.ndarray:
    """y[n] = sum_j h[j] s[(n - j) mod N]: a sum of shifted copies of s."""
    s = np.asarray(s, dtype=np.complex128)
    h = np.asarray(h, dtype=np.complex128).reshape(-1)
    y = np.zeros_like(s)
    for j, hj in enumerate(h):
        if hj != 0:
            y += hj * np.roll(s, j, axis=-1)
    return y


def rel_error(y, y_ref, s, h, _mutant: int = 0) -> np.ndarray:
    """||y - y_ref|| / (max|H| ||s||) per block (last axis).

    ``_mutant`` (tests only) plants a plausible wrong denominator:
      1 = ||y_ref||, 2 = ||s|| without max|H|, 3 = max|h| (taps, not
      spectrum) times ||s||."""
    y = np.asarray(y, dtype=np.complex128)
    y_ref = np.asarray(y_ref, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    hmax = np.max(np.abs(filter_spectrum(h)))
    if _mutant == 3:
        hmax = np.max(np.abs(np.asarray(h, dtype=np.complex128)))
    num = np.linalg.norm(y - y_ref, axis=-1)
    den = hmax * np.linalg.norm(s, axis=-1)
    if _mutant == 1:
        den = np.linalg.norm(y_ref, axis=-1)
    elif _mutant == 2:
        den = np.linalg.norm(s, axis=-1)
    return num / np.where(den > 0, den, 1.0)
