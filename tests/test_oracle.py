"""CPU tests: the FP64 oracle against its pins, and the pins against planted mistakes."""
import json

import numpy as np
import pytest

import pins
from paper_1810_11451_amd import workloads as wl


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_c_oracle_pins(oracle_mod, pin):
    pin(pins.c_runner(oracle_mod))


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_numpy_oracle_pins(oracle_mod, pin):
    pin(pins.numpy_runner(oracle_mod))


MUTANTS = {
    1: "wrong sign on one imaginary cross term",
    2: "conjugated W",
    3: "last flow dropped from the sum",
    4: "W indexed transposed",
    5: "S indexed transposed",
    6: "W id ignored",
    7: "wrong pairing in the imaginary part",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=lambda k: MUTANTS[k].replace(" ", "_"))
def test_pins_reject_planted_mistake(oracle_mod, tmp_path, mutant):
    """Each planted mistake in the C oracle must fail at least one pin."""
    path = oracle_mod.build(tmp_path / f"liboracle_mut{mutant}.so", mutant=mutant)
    lib = oracle_mod.load(path)
    run = pins.c_runner(oracle_mod, lib=lib)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(run)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant '{MUTANTS[mutant]}' passed every pin"


def test_c_and_numpy_agree(oracle_mod):
    rng = np.random.default_rng(21)
    b = wl.random_batch(rng, 40, 5)
    Rc = oracle_mod.apply(b, threads=3)
    for t in range(b.n):
        Rn = oracle_mod.apply_numpy(b.w_block(t), b.s_block(t))
        assert np.max(np.abs(Rc[t] - Rn)) <= 1e-13 * max(1.0, np.max(np.abs(Rn)))


def test_threads_do_not_change_result(oracle_mod):
    rng = np.random.default_rng(22)
    b = wl.random_batch(rng, 33, 4)
    assert np.array_equal(oracle_mod.apply(b, threads=1), oracle_mod.apply(b, threads=7))


def test_item_subset(oracle_mod):
    b = wl.single_w_batch()
    full = oracle_mod.apply(b)
    sub = oracle_mod.apply(b, items=[3, 0, 99])
    assert np.array_equal(sub, full[[3, 0, 99]])


def test_oracle_rejects_bad_arguments(oracle_mod):
    b = wl.single_w_batch(n=3)
    with pytest.raises(ValueError):
        oracle_mod.apply_arrays(b.W, np.array([0, 1, 0], np.int32), b.f, b.S, b.s_off)
    with pytest.raises(ValueError):
        oracle_mod.apply_arrays(b.W, b.w_ids, np.array([8, 9, 8], np.int32), b.S, b.s_off)


def test_rel_frobenius(oracle_mod):
    ref = np.ones((2, 3, 4), np.complex128)
    got = ref.copy()
    got[1] *= 1.5
    e = oracle_mod.rel_frobenius(got, ref)
    assert e[0] == 0.0 and abs(e[1] - 0.5) < 1e-15
    z = np.zeros((2, 3, 4))
    g = z.copy()
    g[1, 0, 0] = 1e-30
    e = oracle_mod.rel_frobenius(g, z)
    assert e[0] == 0.0 and np.isinf(e[1])
    e = oracle_mod.rel_frobenius(-0.0 * z, z)
    assert np.all(e == 0.0)


def test_workload_shapes_match_paper(golden_dir):
    g = json.loads((golden_dir / "paper_shapes.json").read_text())
    assert wl.M == g["antennas"] == int(np.prod(g["array"]))
    assert wl.B == g["resource_elements"]
    assert wl.F_MAX == g["f_max"]
    b = wl.full_width_batch(n=8)
    assert b.W.shape == (64, 64, 36) and b.S.shape == (8 * 36 * 60,)


def test_input_distributions():
    rng = np.random.default_rng(5)
    q = wl.qam256(rng, (200000,))
    assert abs(np.mean(np.abs(q) ** 2) - 1.0) < 0.01
    lv = wl.qam256_levels(rng, (1000,))
    assert set(np.unique(lv.real)) <= set(range(-15, 16, 2))
    W = wl.unit_norm_pool(rng, 3, 36).astype(np.complex128)
    assert np.allclose(np.linalg.norm(W, axis=1), 1.0, atol=1e-6)
    c = wl.cn01(rng, (200000,))
    assert abs(np.var(c.real) - 0.5) < 0.01 and abs(np.var(c.imag) - 0.5) < 0.01
    b4 = wl.gain_batch(n=64)
    assert np.all(b4.gains >= 1e-3) and np.all(b4.gains <= 1e3)


def test_config_seeds_are_deterministic():
    a, b = wl.uneven_batch(n=50), wl.uneven_batch(n=50)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.f, b.f) and np.array_equal(a.w_ids, b.w_ids)
    assert a.flops() == 8 * 64 * 60 * int(a.f.sum())
