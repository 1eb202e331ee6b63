"""Pins for the FP64 oracle: checks that tie it to something other than itself.

Each pin takes ``run(W, w_ids, f, S, s_off, m, b) -> complex128 [n, m, b]``
(an oracle rendering) and raises AssertionError when the oracle disagrees
with what the mathematics fixes.  The paper prints no worked beamforming
values, so the pins are:

* exact rational brute force on tiny ragged batches (dyadic inputs make
  every double operation exact, so equality is bitwise);
* a hand-worked 2 x 2 by 2 x 3 example stored under tests/golden;
* identity W (R = [S; 0], bitwise) and f = 0 (R = 0, bitwise);
* a DFT-matrix W against numpy's FFT (closed form through a library
  routine), and Parseval for its orthonormal columns;
* linearity in S;
* Gaussian-integer W times integer QAM levels against exact int64 sums;
* numpy's complex128 matmul on the small single-W workload.

Together they reject each planted mistake of the oracle's mutant builds
(wrong sign, conjugation, dropped term, transposed operand, ignored W id).
"""
from __future__ import annotations

import json
from fractions import Fraction
from pathlib import Path

import numpy as np

from paper_1810_11451_amd import workloads as wl

GOLDEN = Path(__file__).resolve().parent / "golden"


def _dyadic(rng, shape):
    """Complex values re, im in {k/8 : |k| <= 16}: exact in FP32 and FP64."""
    re = rng.integers(-16, 17, size=shape) / 8.0
    im = rng.integers(-16, 17, size=shape) / 8.0
    return (re + 1j * im).astype(np.complex64)


def pin_fraction_bruteforce(run, seed=11):
    rng = np.random.default_rng(seed)
    m, b, ldw, n_w = 5, 7, 4, 3
    W = _dyadic(rng, (n_w, m, ldw))
    f = np.array([0, 1, 2, 3, 4, 3, 1, 4], dtype=np.int32)
    w_ids = np.array([0, 1, 2, 0, 1, 2, 1, 0], dtype=np.int32)
    sizes = f.astype(np.int64) * b
    s_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    S = _dyadic(rng, (int(sizes.sum()),))
    R = run(W, w_ids, f, S, s_off, m, b)
    for t in range(len(f)):
        ft = int(f[t])
        Wt = W[w_ids[t]]
        St = S[s_off[t]: s_off[t] + ft * b].reshape(ft, b)
        for i in range(m):
            for j in range(b):
                re = Fraction(0)
                im = Fraction(0)
                for k in range(ft):
                    a, bb = Fraction(float(Wt[i, k].real)), Fraction(float(Wt[i, k].imag))
                    c, d = Fraction(float(St[k, j].real)), Fraction(float(St[k, j].imag))
                    re += a * c - bb * d
                    im += a * d + bb * c
                got = R[t, i, j]
                assert Fraction(float(got.real)) == re and Fraction(float(got.imag)) == im, \
                    f"item {t} ({i},{j}): {got} != {re}+{im}i"


def pin_hand_example(run):
    g = json.loads((GOLDEN / "hand_example.json").read_text())
    W = np.array(g["W"], dtype=np.float64)
    S = np.array(g["S"], dtype=np.float64)
    R = np.array(g["R"], dtype=np.float64)
    W = (W[..., 0] + 1j * W[..., 1]).astype(np.complex64)[None]
    S = (S[..., 0] + 1j * S[..., 1]).astype(np.complex64).reshape(-1)
    R = R[..., 0] + 1j * R[..., 1]
    got = run(W, np.array([0], np.int32), np.array([g["f"]], np.int32), S,
              np.array([0], np.int64), g["m"], g["b"])
    assert np.array_equal(got[0], R), f"{got[0]} != {R}"


def pin_identity(run, seed=12):
    rng = np.random.default_rng(seed)
    for ft in (1, 7, 36):
        W = wl.identity_w(ft, wl.F_MAX)[None]
        S = wl.cn01(rng, (ft, wl.B)).astype(np.complex64)
        R = run(W, np.array([0], np.int32), np.array([ft], np.int32), S.reshape(-1),
                np.array([0], np.int64), wl.M, wl.B)[0]
        assert np.array_equal(R[:ft], S.astype(np.complex128)), f"identity rows differ at f={ft}"
        assert np.all(R[ft:] == 0), f"rows below f not zero at f={ft}"


def pin_f_zero(run, seed=13):
    rng = np.random.default_rng(seed)
    W = wl.cn01_pool(rng, 2, wl.F_MAX)
    S = np.zeros(0, np.complex64)
    R = run(W, np.array([1, 0], np.int32), np.array([0, 0], np.int32), S,
            np.array([0, 0], np.int64), wl.M, wl.B)
    assert R.shape == (2, wl.M, wl.B) and np.all(R == 0)


def pin_dft(run, seed=14, tol=4e-7):
    rng = np.random.default_rng(seed)
    for ft in (1, 5, 36):
        W = wl.dft_w(ft)[None]
        S = wl.qam256(rng, (ft, wl.B)).astype(np.complex64)
        R = run(W, np.array([0], np.int32), np.array([ft], np.int32), S.reshape(-1),
                np.array([0], np.int64), wl.M, wl.B)[0]
        pad = np.zeros((wl.M, wl.B), np.complex128)
        pad[:ft] = S
        ref = np.fft.fft(pad, axis=0) / 8.0
        err = np.linalg.norm(R - ref) / np.linalg.norm(ref)
        assert err < tol, f"DFT closed form off by {err:.3g} at f={ft}"


def pin_parseval(run, seed=15, tol=4e-7):
    rng = np.random.default_rng(seed)
    ft = 36
    W = wl.dft_w(ft)[None]
    S = wl.cn01(rng, (ft, wl.B)).astype(np.complex64)
    R = run(W, np.array([0], np.int32), np.array([ft], np.int32), S.reshape(-1),
            np.array([0], np.int64), wl.M, wl.B)[0]
    nr = np.linalg.norm(R)
    ns = np.linalg.norm(S.astype(np.complex128))
    assert abs(nr - ns) / ns < tol, f"Parseval: {nr} vs {ns}"


def pin_linearity(run, seed=16, tol=1e-6):
    rng = np.random.default_rng(seed)
    ft = 23
    W = wl.cn01_pool(rng, 1, wl.F_MAX)
    S1 = wl.cn01(rng, (ft, wl.B)).astype(np.complex64)
    S2 = wl.cn01(rng, (ft, wl.B)).astype(np.complex64)
    al, be = 0.7 - 1.3j, -0.4 + 0.25j
    S3 = (al * S1.astype(np.complex128) + be * S2.astype(np.complex128)).astype(np.complex64)
    S = np.concatenate([S1.reshape(-1), S2.reshape(-1), S3.reshape(-1)])
    off = np.array([0, ft * wl.B, 2 * ft * wl.B], np.int64)
    R = run(W, np.zeros(3, np.int32), np.full(3, ft, np.int32), S, off, wl.M, wl.B)
    lhs = R[2]
    rhs = al * R[0] + be * R[1]
    err = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
    assert err < tol, f"linearity off by {err:.3g}"


def pin_exact_integer(run, seed=17):
    rng = np.random.default_rng(seed)
    b = wl.exact_integer_batch(rng, 24, 3)
    R = run(b.W, b.w_ids, b.f, b.S, b.s_off, wl.M, wl.B)
    for t in range(b.n):
        Wt = b.w_block(t)
        St = b.s_block(t)
        wr, wi = Wt.real.astype(np.int64), Wt.imag.astype(np.int64)
        sr, si = St.real.astype(np.int64), St.imag.astype(np.int64)
        rr = np.zeros((wl.M, wl.B), np.int64)
        ri = np.zeros((wl.M, wl.B), np.int64)
        for k in range(int(b.f[t])):
            rr += np.outer(wr[:, k], sr[k]) - np.outer(wi[:, k], si[k])
            ri += np.outer(wr[:, k], si[k]) + np.outer(wi[:, k], sr[k])
        assert np.array_equal(R[t].real, rr) and np.array_equal(R[t].imag, ri), f"item {t}"


def pin_matmul_single_w(run, tol=1e-14):
    b = wl.single_w_batch()
    R = run(b.W, b.w_ids, b.f, b.S, b.s_off, wl.M, wl.B)
    W = b.W[0].astype(np.complex128)
    for t in range(b.n):
        ref = W @ b.s_block(t).astype(np.complex128)
        err = np.linalg.norm(R[t] - ref) / np.linalg.norm(ref)
        assert err < tol, f"item {t}: {err:.3g}"


ALL_PINS = [pin_fraction_bruteforce, pin_hand_example, pin_identity, pin_f_zero, pin_dft,
            pin_parseval, pin_linearity, pin_exact_integer, pin_matmul_single_w]


def c_runner(oracle_mod, lib=None, threads=2):
    def run(W, w_ids, f, S, s_off, m, b):
        return oracle_mod.apply_arrays(W, w_ids, f, S, s_off, m=m, b=b, threads=threads, lib=lib)
    return run


def numpy_runner(oracle_mod):
    def run(W, w_ids, f, S, s_off, m, b):
        W = np.asarray(W)
        out = np.zeros((len(w_ids), m, b), np.complex128)
        for t in range(len(w_ids)):
            ft = int(f[t])
            St = np.asarray(S)[int(s_off[t]): int(s_off[t]) + ft * b].reshape(ft, b)
            out[t] = oracle_mod.apply_numpy(W[int(w_ids[t])][:m, :], St)
        return out
    return run
