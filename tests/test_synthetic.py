"""Seeded synthetic inputs: determinism and the distogram recipe's invariants."""
import numpy as np
import pytest

import synthetic as sy


def test_reference_torsions_seeded_and_wrapped():
    a = sy.reference_torsions(300, 2)
    assert np.array_equal(a, sy.reference_torsions(300, 2))
    assert not np.array_equal(a, sy.reference_torsions(300, 3))
    assert a.shape == (600,) and np.all(a > -np.pi) and np.all(a <= np.pi)
    phi = np.degrees(a[0::2])
    assert 0.80 < np.mean(phi < 0) < 1.0          # alpha_L is the minor component


def test_distogram_rows_are_distributions():
    d = np.array([1.0, 3.3, 8.0, 19.9, 20.25, 45.0, 300.0])
    for eps in (0.0, 0.1):
        y = sy.distogram(d, eps, 7)
        assert y.shape == (7, 37) and np.all(np.isfinite(y)) and np.all(y >= 0.0)
        assert np.allclose(np.exp(-y).sum(axis=1), 1.0, atol=1e-12)
    assert np.array_equal(sy.distogram(d, 0.1, 7), sy.distogram(d, 0.1, 7))
    assert not np.array_equal(sy.distogram(d, 0.1, 7), sy.distogram(d, 0.1, 8))


def test_noise_free_table_is_quadratic_in_knots():
    c = sy.bin_knots()
    y = sy.distogram(np.array([7.3]), 0.0, 0)[0]
    q = 0.5 * (c - 7.3) ** 2
    assert np.allclose(y - q, (y - q)[0], atol=1e-12)


def test_pair_index_matches_packed_row_formula():
    L = 11
    i, j = sy.pair_index(L)
    r = i * L - i * (i + 1) // 2 + (j - i - 1)
    assert np.array_equal(r, np.arange(sy.n_pairs(L)))


def test_workload_presets():
    assert sy.CFG1.L == 64 and sy.CFG1.n_chains == 1 and sy.CFG1.total_sweeps == 20000
    assert sy.CFG1.window_d == 8 and sy.CFG1.global_every == 10
    assert sy.CFG2.L == 300 and sy.CFG2.n_chains == 1024 and sy.CFG2.window_d == 12
    assert sy.CFG2.total_sweeps == 5000 and len(sy.CFG2.trace_chains) == 4
    assert sy.CFG1.sigma == pytest.approx(np.radians(10.0))


def test_ragged_and_arrivals():
    L = sy.batch_lengths(64, 50, 600, 3)
    assert L.min() >= 50 and L.max() <= 600 and np.array_equal(L, sy.batch_lengths(64, 50, 600, 3))
    t = sy.poisson_arrivals(20.0, 2000, 4)
    assert np.all(np.diff(t) > 0) and abs(2000 / t[-1] - 20.0) < 2.0
