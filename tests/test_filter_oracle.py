"""CPU tests: the filter-stage oracle against closed forms, and planted mistakes.

Pins (Section III, filter paragraph: y = IFFT(FFT(s) * FFT(h))):
* impulse: h = [1] gives y = s;
* shift: h = delta at d gives y = s rotated by d samples;
* single tone: s[n] = exp(2 pi i k0 n / N) gives y = H[k0] s, with H[k0]
  summed directly from the taps;
* brute force: y equals the circular convolution sum_j h[j] s[n - j mod N]
  (convolution theorem), for 1, 7, 64 and 2048 taps;
* linearity in s.
Each planted mistake of filter_oracle (``_mutant``) must fail one of them.
"""
import numpy as np
import pytest

from oracle import filter_oracle as fo
from paper_1810_11451_amd import workloads as wl

N = fo.N_FILTER


def pin_impulse(apply, rng):
    s = wl.filter_signals(rng, 3)
    y = apply(s, np.array([1.0 + 0j]))
    assert np.max(np.abs(y - s)) <= 1e-12 * np.max(np.abs(s))


def pin_shift(apply, rng):
    s = wl.filter_signals(rng, 2)
    for d in (1, 17, 1024, N - 1):
        h = np.zeros(d + 1, np.complex128)
        h[d] = 1.0
        y = apply(s, h)
        assert np.max(np.abs(y - np.roll(s, d, axis=-1))) <= 1e-12 * np.max(np.abs(s)), d


def pin_tone(apply, rng):
    h = wl.random_taps(rng, 37).astype(np.complex128)
    n = np.arange(N)
    for k0 in (0, 3, 1024, N - 1):
        s = np.exp(2j * np.pi * k0 * n / N)
        Hk = np.sum(h * np.exp(-2j * np.pi * k0 * np.arange(h.shape[0]) / N))
        y = apply(s, h)
        assert np.max(np.abs(y - Hk * s)) <= 1e-11, k0


def pin_bruteforce(apply, rng):
    s = wl.filter_signals(rng, 2)
    for taps in (1, 7, 64, N):
        h = wl.random_taps(rng, taps)
        y = apply(s, h)
        ref = fo.circular_convolution(s, h)
        assert np.max(np.abs(y - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref))), taps


def pin_linearity(apply, rng):
    s1, s2 = wl.filter_signals(rng, 2)
    h = wl.lowpass_taps(63, 0.1)
    a, b = 0.75 - 0.5j, -1.25 + 2j
    lhs = apply(a * s1.astype(np.complex128) + b * s2.astype(np.complex128), h)
    rhs = a * apply(s1, h) + b * apply(s2, h)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


PINS = [pin_impulse, pin_shift, pin_tone, pin_bruteforce, pin_linearity]
MUTANTS = {1: "forward transform with the inverse sign", 2: "taps reversed",
           3: "multiplication by conj(H)", 4: "filter spectrum with the inverse sign",
           5: "1/N of the inverse transform left out"}


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_filter_oracle_pins(pin):
    pin(fo.filter_apply, np.random.default_rng(31))


@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=lambda k: MUTANTS[k].replace(" ", "_"))
def test_filter_pins_reject_planted_mistake(mutant):
    caught = []
    for pin in PINS:
        try:
            pin(lambda s, h: fo.filter_apply(s, h, _mutant=mutant), np.random.default_rng(31))
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"planted mistake '{MUTANTS[mutant]}' passed every pin"


def metric_pin_single_tap(rel_error):
    """Worked by hand: h = [2] gives H[k] = 2 for every k, so max|H| = 2; s is
    the unit impulse (||s|| = 1) and y_ref = 2 s.  With y = y_ref + 3 e_5 the
    error norm is 3 and the metric is 3 / (2 * 1) = 1.5 exactly."""
    s = np.zeros(N, np.complex128)
    s[0] = 1.0
    h = np.array([2.0 + 0j])
    y_ref = 2.0 * s
    y = y_ref.copy()
    y[5] += 3.0
    assert rel_error(y, y_ref, s, h)[()] == 1.5


def metric_pin_two_taps(rel_error):
    """Worked by hand: h = [1, 1] has H[k] = 1 + exp(-2 pi i k / N), largest
    at k = 0 where it is 2, so max|H| = 2.  s = [1, -1, 0, ...] has
    ||s|| = sqrt(2); the circular convolution is y_ref = [1, 0, -1, 0, ...]
    (||y_ref|| = sqrt(2), so ||y_ref|| differs from max|H| ||s|| = 2 sqrt(2)).
    With y = y_ref + 4 e_7 the metric is 4 / (2 sqrt(2)) = sqrt(2)."""
    s = np.zeros(N, np.complex128)
    s[0], s[1] = 1.0, -1.0
    h = np.array([1.0 + 0j, 1.0 + 0j])
    y_ref = np.zeros(N, np.complex128)
    y_ref[0], y_ref[2] = 1.0, -1.0
    y = y_ref.copy()
    y[7] += 4.0
    assert abs(rel_error(y, y_ref, s, h)[()] - np.sqrt(2.0)) <= 1e-15


def metric_pin_quarter_band(rel_error):
    """Worked by hand: h = [1, 1j] has |H[k]| = |1 + 1j exp(-2 pi i k / N)|,
    largest (2) where exp(-2 pi i k / N) = -1j, i.e. k = N / 4, while max|h|
    is 1.  s = unit impulse at n = 3 (||s|| = 1), y = y_ref + 1 e_0 (an error
    of norm 1): the metric is 1 / 2."""
    s = np.zeros(N, np.complex128)
    s[3] = 1.0
    h = np.array([1.0 + 0j, 1j])
    y_ref = np.zeros(N, np.complex128)
    y_ref[3], y_ref[4] = 1.0, 1j
    y = y_ref.copy()
    y[0] += 1.0
    assert abs(rel_error(y, y_ref, s, h)[()] - 0.5) <= 1e-15


METRIC_PINS = [metric_pin_single_tap, metric_pin_two_taps, metric_pin_quarter_band]
METRIC_MUTANTS = {1: "denominator ||y_ref||", 2: "denominator ||s|| without max|H|",
                  3: "max over the taps instead of the spectrum"}


@pytest.mark.parametrize("pin", METRIC_PINS, ids=lambda p: p.__name__)
def test_rel_error_hand_values(pin):
    pin(fo.rel_error)


@pytest.mark.parametrize("mutant", sorted(METRIC_MUTANTS), ids=lambda k: METRIC_MUTANTS[k].replace(" ", "_"))
def test_rel_error_pins_reject_planted_mistake(mutant):
    caught = []
    for pin in METRIC_PINS:
        try:
            pin(lambda *a: fo.rel_error(*a, _mutant=mutant))
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"planted mistake '{METRIC_MUTANTS[mutant]}' passed every metric pin"


def test_rel_error_metric():
    rng = np.random.default_rng(32)
    s = wl.filter_signals(rng, 4)
    h = wl.lowpass_taps(101, 0.05)
    y = fo.filter_apply(s, h)
    assert np.all(fo.rel_error(y, y, s, h) == 0)
    # |y| <= max|H| |s| (unitary transforms up to scale)
    H = fo.filter_spectrum(h)
    assert np.all(np.linalg.norm(y, axis=-1) <= np.max(np.abs(H)) * np.linalg.norm(s, axis=-1) * (1 + 1e-12))


def test_taps_validation():
    with pytest.raises(ValueError):
        fo.padded_taps(np.zeros(N + 1))
    with pytest.raises(ValueError):
        fo.padded_taps(np.zeros(0))
