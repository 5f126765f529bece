"""Pins of the oracle's energy: spline, full and localized distogram energies,
incremental dE, compensated sums, gradient, and the energy minimum of the
synthetic distogram.

The spline reproduces quadratics on the interior knots, which gives closed
forms: with eps = 0 the synthetic table is (c_b - d*)^2/2 + log Z, so every
pair energy is minimal at its reference distance.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as sy


def cfg_for(L, window_d=8, n_bins=37, global_every=10):
    w = sy.Workload("t", L=L, n_chains=1, total_sweeps=100, window_d=window_d,
                    global_every=global_every, n_bins=n_bins)
    return oracle.make_cfg(w)


KNOTS = sy.bin_knots()


def test_spline_hits_knots_and_clamps():
    rng = np.random.default_rng(0)
    y = rng.uniform(0.0, 9.0, 37)
    for b, c in enumerate(KNOTS):
        assert oracle.pair_energy(y, c) == pytest.approx(y[b], abs=1e-12)
    for d in (0.0, 1.0, 2.0, 2.25):
        assert oracle.pair_energy(y, d) == y[0]
    for d in (20.25, 21.0, 35.0, 1e3):
        assert oracle.pair_energy(y, d) == y[36]


@pytest.mark.parametrize("dstar", [3.1, 7.77, 12.0, 19.2])
def test_spline_reproduces_quadratic(dstar):
    y = sy.distogram(np.array([dstar]), 0.0, 0)[0]
    logZ = y.min() - ((KNOTS[np.argmin(y)] - dstar) ** 2) / 2
    for d in np.linspace(2.75, 19.75, 341):
        assert oracle.pair_energy(y, d) == pytest.approx((d - dstar) ** 2 / 2 + logZ, abs=1e-11)


def test_spline_is_c1():
    rng = np.random.default_rng(1)
    y = rng.uniform(0.0, 9.0, 37)
    h = 1e-7
    for c in list(KNOTS) + [2.25 - 1e-3, 20.25 + 1e-3]:
        left = (oracle.pair_energy(y, c) - oracle.pair_energy(y, c - h)) / h
        right = (oracle.pair_energy(y, c + h) - oracle.pair_energy(y, c)) / h
        assert left == pytest.approx(right, abs=5e-5)
    for d in np.linspace(1.0, 22.0, 97):
        fd = (oracle.pair_energy(y, d + 1e-6) - oracle.pair_energy(y, d - 1e-6)) / 2e-6
        assert oracle.pair_energy_deriv(y, d) == pytest.approx(fd, abs=1e-4)  # FD truncation ~ h E"


def test_window_pair_counts_and_global_limit():
    L = 15
    cfg = cfg_for(L, window_d=6)
    y = np.ones((sy.n_pairs(L), 37))
    at = oracle.nerf(sy.random_torsions(2 * L, 2))
    assert oracle.energy_full(cfg, y, at) == sy.n_pairs(L)
    h = 3
    for k in range(2 * L):
        c = k // 2
        lo, hi = max(0, c - h), min(L - 1, c + h)
        n = hi - lo + 1
        assert oracle.energy_window(cfg, y, at, k) == n * (n - 1) // 2
    big = cfg_for(L, window_d=2 * L)
    yr = np.random.default_rng(3).uniform(0, 5, (sy.n_pairs(L), 37))
    for k in range(2 * L):
        assert oracle.energy_window(big, yr, at, k) == pytest.approx(oracle.energy_full(big, yr, at), rel=1e-14)


def test_energy_is_sum_over_pairs_of_spline():
    L = 9
    cfg = cfg_for(L)
    y = np.random.default_rng(4).uniform(0, 6, (sy.n_pairs(L), 37))
    at = oracle.nerf(sy.random_torsions(2 * L, 4))
    cb = at[:, 3]
    i, j = sy.pair_index(L)
    ref = math.fsum(oracle.pair_energy(y[r], np.linalg.norm(cb[i[r]] - cb[j[r]])) for r in range(len(i)))
    assert oracle.energy_full(cfg, y, at) == pytest.approx(ref, rel=1e-15)


def test_rigid_body_invariance():
    L = 16
    cfg = cfg_for(L)
    y = np.random.default_rng(5).uniform(0, 6, (sy.n_pairs(L), 37))
    at = oracle.nerf(sy.random_torsions(2 * L, 6))
    q, _ = np.linalg.qr(np.random.default_rng(7).standard_normal((3, 3)))
    moved = at @ q.T + np.array([3.0, -40.0, 12.5])
    assert oracle.energy_full(cfg, y, moved) == pytest.approx(oracle.energy_full(cfg, y, at), rel=1e-12)


@pytest.mark.parametrize("L,wd", [(2, 8), (3, 2), (7, 4), (12, 8), (12, 0), (11, 30)])
def test_incremental_equals_brute(L, wd):
    cfg = cfg_for(L, window_d=wd)
    rng = np.random.default_rng(L * 100 + wd)
    y = rng.uniform(0, 7, (sy.n_pairs(L), 37))
    s = sy.random_torsions(2 * L, L + wd)
    at0 = oracle.nerf(s)
    for k in range(2 * L):
        delta = rng.normal(0, 0.4)
        for glob in (False, True):
            inc, S = oracle.delta_e(cfg, y, s, k, delta, glob, 1)
            bru, _ = oracle.delta_e(cfg, y, s, k, delta, glob, 0)
            assert inc == pytest.approx(bru, rel=1e-12, abs=1e-11)
            # brute force straight from the definitions of V and V_local
            s2 = s.copy()
            s2[k] = (s[k] + delta + math.pi) % (2 * math.pi) - math.pi
            at1 = oracle.nerf(s2)
            if glob:
                ref = oracle.energy_full(cfg, y, at1) - oracle.energy_full(cfg, y, at0)
            else:
                ref = oracle.energy_window(cfg, y, at1, k) - oracle.energy_window(cfg, y, at0, k)
            assert inc == pytest.approx(ref, rel=1e-12, abs=1e-11)
            if k in (0, 2 * L - 1):
                assert inc == 0.0 and S == 0.0


def test_neumaier_matches_fsum():
    rng = np.random.default_rng(8)
    for _ in range(20):
        x = rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 9, 5000)
        x = np.concatenate([x, -x[:2500] * (1 + 1e-12)])
        ref = math.fsum(x)
        got = oracle.neumaier_sum(x)
        assert abs(got - ref) <= 2 * np.spacing(abs(ref)) + 1e-300


def test_gradient_matches_finite_differences():
    L = 14
    cfg = cfg_for(L)
    y = sy.distogram(sy.pair_distances(oracle.cb(sy.reference_torsions(L, 9))), 0.1, 9)
    s = sy.random_torsions(2 * L, 10)
    V, g = oracle.grad(cfg, y, s)
    assert V == pytest.approx(oracle.energy(cfg, y, s), rel=1e-14)
    h = 1e-6
    for k in range(2 * L):
        sp, sm = s.copy(), s.copy()
        sp[k] += h
        sm[k] -= h
        fd = (oracle.energy(cfg, y, sp) - oracle.energy(cfg, y, sm)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-6)


@pytest.fixture(scope="module")
def exact_protein():
    """L=64 protein with a noise-free (eps=0) synthetic distogram.

    Pairs whose reference distance falls where the spline is not the quadratic
    (below 2.75 A, or within half a bin of the no-contact knot) get a flat row,
    so that every remaining pair has its closed-form minimum at d*.
    """
    L = 64
    s_ref = sy.reference_torsions(L, 1)
    dstar = sy.pair_distances(oracle.cb(s_ref))
    y = sy.distogram(dstar, 0.0, 0)
    exact = (dstar >= 2.75) & ~((dstar > 19.75) & (dstar < 20.25))
    y[~exact] = 0.0
    return L, s_ref, dstar, y, exact


def test_energy_minimum_at_reference(exact_protein):
    L, s_ref, dstar, y, exact = exact_protein
    cfg = cfg_for(L)
    dd = np.linspace(0.0, 40.0, 40001)
    V_ref = oracle.energy(cfg, y, s_ref)
    e_at = np.array([oracle.pair_energy(y[r], dstar[r]) for r in range(len(dstar))])
    # dense 1-D scan of a sample of pairs: each exact pair sits at its own minimum
    sample = np.random.default_rng(0).choice(np.flatnonzero(exact), 300, replace=False)
    for r in sample:
        assert e_at[r] <= min(oracle.pair_energy(y[r], d) for d in dd[::20]) + 1e-9
    assert V_ref == pytest.approx(e_at.sum(), rel=1e-12)
    # and the pair minimum is the normaliser log Z of its Gaussian (the closed form)
    c = sy.bin_knots()
    from scipy.special import logsumexp
    logZ = logsumexp(-0.5 * (c[None, :] - dstar[:, None]) ** 2, axis=1)
    assert np.allclose(e_at[exact & (dstar < 19.75)], logZ[exact & (dstar < 19.75)], atol=1e-10)


def test_gradient_vanishes_at_reference(exact_protein):
    L, s_ref, dstar, y, exact = exact_protein
    cfg = cfg_for(L)
    _, g = oracle.grad(cfg, y, s_ref)
    assert np.abs(g).max() < 1e-8
    h = 1e-5
    for k in range(0, 2 * L, 7):
        sp, sm = s_ref.copy(), s_ref.copy()
        sp[k] += h
        sm[k] -= h
        assert abs(oracle.energy(cfg, y, sp) - oracle.energy(cfg, y, sm)) / (2 * h) < 1e-6


def test_random_perturbations_never_lower_reference_energy(exact_protein):
    L, s_ref, dstar, y, exact = exact_protein
    cfg = cfg_for(L)
    V_ref = oracle.energy(cfg, y, s_ref)
    rng = np.random.default_rng(12)
    for _ in range(2000):
        s = s_ref + rng.normal(0.0, rng.choice([0.01, 0.1, 0.5]), 2 * L) * (rng.random(2 * L) < 0.2)
        assert oracle.energy(cfg, y, s) >= V_ref - 1e-9
