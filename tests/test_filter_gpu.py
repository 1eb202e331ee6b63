"""GPU parity of the filter stage (bf_filter_*) against the FP64 oracle.

Bar: ||y - y_ref||_2 <= 1e-5 * max|H| * ||s||_2 per block (metric of
filter_oracle.rel_error).  Derivation: for a radix-2-based FFT with
twiddles correct to within u, the normwise relative error of one FP32
transform is at most log2(N) eta / (1 - log2(N) eta), eta = u + gamma_4
(sqrt(2) + u) ~ 6.7u (Higham, Accuracy and Stability, Thm 24.2); with u =
2^-24 and log2(N) = 11 that is 4.4e-6.  The forward transform's error is
amplified by at most max|H| through the multiply (whose own rounding adds
sqrt(2) gamma_2 ~ 1.7e-7 relative), and the inverse transform adds another
4.4e-6 of max|H| ||s||: about 9e-6 in all, hence 1e-5.  Observed errors are
about 1e-7.
"""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from oracle import filter_oracle as fo
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl

pytestmark = pytest.mark.gpu
BAR = 1e-5
N = fo.N_FILTER


def run(flt, s, torch, inplace=False):
    x = torch.from_numpy(np.ascontiguousarray(s, np.complex64)).cuda()
    if inplace:
        bf.bf_filter_apply(flt, s.shape[0], x, x)
        torch.cuda.synchronize()
        return x.cpu().numpy()
    y = torch.full_like(x, float("nan"))
    bf.bf_filter_apply(flt, s.shape[0], x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("n_taps", [1, 7, 64, 513, N])
def test_spectrum(n_taps):
    require_gpu()
    h = wl.random_taps(np.random.default_rng(40 + n_taps), n_taps)
    announce(f"filter spectrum taps={n_taps}")
    with bf.bf_filter_create(h) as flt:
        H = bf.bf_filter_spectrum(flt).astype(np.complex128)
    ref = fo.filter_spectrum(h)
    assert np.linalg.norm(H - ref) / np.linalg.norm(ref) <= BAR


@pytest.mark.parametrize("n_taps", [1, 7, 64, 513, N])
@pytest.mark.parametrize("batch", [1, 37])
def test_random_taps(n_taps, batch):
    torch = require_gpu()
    rng = np.random.default_rng(50 + n_taps + batch)
    s = wl.filter_signals(rng, batch)
    h = wl.random_taps(rng, n_taps)
    announce(f"filter random taps={n_taps} batch={batch}")
    with bf.bf_filter_create(h) as flt:
        y = run(flt, s, torch)
    err = fo.rel_error(y, fo.filter_apply(s, h), s, h)
    print(f"[filter] taps={n_taps} batch={batch} max err {err.max():.3g}", flush=True)
    assert np.all(np.isfinite(y.view(np.float32)))
    assert err.max() <= BAR


def test_lowpass_deep_stopband():
    torch = require_gpu()
    rng = np.random.default_rng(61)
    s = wl.filter_signals(rng, 24)
    h = wl.lowpass_taps(255, 0.05)
    announce("filter lowpass")
    with bf.bf_filter_create(h) as flt:
        y = run(flt, s, torch)
    err = fo.rel_error(y, fo.filter_apply(s, h), s, h)
    assert err.max() <= BAR


def test_closed_forms():
    """Impulse gives the input back, a delayed impulse rotates it."""
    torch = require_gpu()
    rng = np.random.default_rng(62)
    s = wl.filter_signals(rng, 8)
    announce("filter impulse and shift")
    with bf.bf_filter_create(np.array([1.0 + 0j])) as flt:
        y = run(flt, s, torch)
    assert fo.rel_error(y, s, s, np.array([1.0 + 0j])).max() <= BAR
    h = np.zeros(301, np.complex64)
    h[300] = 1.0
    with bf.bf_filter_create(h) as flt:
        y = run(flt, s, torch)
    assert fo.rel_error(y, np.roll(s, 300, axis=-1), s, h).max() <= BAR


def test_in_place_equals_out_of_place():
    torch = require_gpu()
    rng = np.random.default_rng(63)
    s = wl.filter_signals(rng, 300)
    h = wl.random_taps(rng, 33)
    announce("filter in place")
    with bf.bf_filter_create(h) as flt:
        a = run(flt, s, torch)
        b = run(flt, s, torch, inplace=True)
        c = run(flt, s, torch)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32)), "not deterministic"


def test_full_batch_all_blocks():
    """16384 blocks (the benchmark's launch), every block checked against
    the oracle in chunks of 1024."""
    torch = require_gpu()
    rng = np.random.default_rng(64)
    s = wl.filter_signals(rng, 16384)
    h = wl.lowpass_taps(127, 0.1)
    announce("filter full batch")
    with bf.bf_filter_create(h) as flt:
        y = run(flt, s, torch)
    assert np.all(np.isfinite(y.view(np.float32)))
    worst = 0.0
    for lo in range(0, s.shape[0], 1024):
        blk = slice(lo, lo + 1024)
        err = fo.rel_error(y[blk], fo.filter_apply(s[blk], h), s[blk], h)
        worst = max(worst, float(err.max()))
    assert worst <= BAR, f"max rel err {worst:.3g}"


def test_argument_errors():
    torch = require_gpu()
    x = torch.zeros((4, N), dtype=torch.complex64, device="cuda")
    with bf.bf_filter_create(np.ones(3, np.complex64)) as flt:
        bf.bf_filter_apply(flt, 0, 0, 0)          # empty batch: nothing to do
        with pytest.raises(bf.BfError) as ei:
            bf.bf_filter_apply(flt, 2, x.data_ptr(), x.data_ptr() + N * 8)   # partial overlap
        assert ei.value.status == bf.BF_ERR_INVALID
        with pytest.raises(bf.BfError):
            bf.bf_filter_apply(flt, -1, x, x)
    with pytest.raises(bf.BfError):
        bf.bf_filter_create(np.ones(N + 1, np.complex64))
