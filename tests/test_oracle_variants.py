"""Pins of the oracle's schedule variants: the proposal-width annealing, the
cascade of localization radii and the noisy restart (Sec. 2.2, Sec. 2.3 and the
second and third schemes of Sec. 3)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synthetic as sy


def test_sigma_schedule_is_geometric_between_its_ends():
    w = sy.CFG1.replace(total_sweeps=101, sigma_deg=10.0, sigma_end_deg=4.0)
    cfg = oracle.make_cfg(w)
    s = np.array([oracle.sigma_at(cfg, t) for t in range(101)])
    assert s[0] == pytest.approx(math.radians(10.0), rel=1e-15)
    assert s[-1] == pytest.approx(math.radians(4.0), rel=1e-14)
    assert np.allclose(np.diff(np.log(s)), math.log(0.4) / 100, rtol=1e-9, atol=0)
    const = oracle.make_cfg(w.replace(sigma_end_deg=0.0))
    assert all(oracle.sigma_at(const, t) == math.radians(10.0) for t in (0, 50, 100))


def test_cascade_cycles_through_the_radii():
    cfg = oracle.make_cfg(sy.CFG1.replace(window_d=10, cascade=(4, 20)))
    assert [oracle.window_at(cfg, t) for t in range(7)] == [10, 4, 20, 10, 4, 20, 10]
    cfg = oracle.make_cfg(sy.CFG1.replace(window_d=6))
    assert {oracle.window_at(cfg, t) for t in range(9)} == {6}


def _run(w, y, mode, sweeps):
    cfg = oracle.make_cfg(w)
    ch = oracle.Chains(cfg, y, np.full((2, 2 * w.L), math.pi))
    steps, acc, _ = ch.run(sweeps, mode=mode, log_steps=True)
    return ch, steps, acc


@pytest.mark.parametrize("cascade,sigma_end", [((2, 30), 0.0), ((4,), 3.0), ((), 5.0)])
def test_variant_runs_agree_between_brute_and_incremental(cascade, sigma_end):
    """With the per-sweep radius and width, the brute-force run (whole windows
    rebuilt and summed) and the incremental run take the same decisions."""
    w = sy.Workload("v", L=11, n_chains=2, total_sweeps=12, window_d=6, global_every=4,
                    sigma_deg=30.0, T0=1.0, T1=0.1, seed=77, protein_seed=1, noise_seed=2,
                    sigma_end_deg=sigma_end, cascade=cascade)
    _, y = sy.workload(w, lambda s: sy.pair_distances(oracle.cb(s)))
    a, sa, aa = _run(w, y, 0, 12)
    b, sb, ab = _run(w, y, 1, 12)
    assert np.array_equal(aa, ab)
    assert np.allclose(sa[..., 0], sb[..., 0], rtol=1e-9, atol=1e-9)
    assert np.array_equal(sa[..., 1], sb[..., 1])       # the same increments
    assert np.allclose(a.s, b.s, atol=0)
    # and the variant matters: the plain schedule takes other decisions
    plain, _, ap = _run(w.replace(cascade=(), sigma_end_deg=0.0), y, 1, 12)
    assert not np.array_equal(ap, ab)


def test_increments_follow_the_width_schedule():
    w = sy.Workload("v", L=8, n_chains=1, total_sweeps=40, window_d=4, global_every=0,
                    sigma_deg=10.0, T0=1.0, T1=1.0, seed=5, sigma_end_deg=4.0)
    cfg = oracle.make_cfg(w)
    for t in (0, 17, 39):
        d, _ = oracle.proposal(w.seed, 0, t, 3, oracle.sigma_at(cfg, t))
        d1, _ = oracle.proposal(w.seed, 0, t, 3, 1.0)
        assert d == pytest.approx(d1 * oracle.sigma_at(cfg, t), rel=1e-15)


def test_noisy_restart_is_uniform_bounded_and_reproducible():
    n = 200000
    s0 = np.zeros(n)
    a = math.radians(10.0)
    s1 = oracle.perturb(0x1234, 3, 7, a, s0)
    assert np.all(np.abs(s1) <= a)
    assert stats.kstest((s1 + a) / (2 * a), "uniform").pvalue > 1e-3
    assert np.array_equal(s1, oracle.perturb(0x1234, 3, 7, a, s0))
    assert not np.array_equal(s1, oracle.perturb(0x1234, 3, 8, a, s0))      # another tag
    assert not np.array_equal(s1, oracle.perturb(0x1234, 4, 7, a, s0))      # another chain
    assert np.array_equal(oracle.perturb(9, 0, 0, 0.0, np.full(5, 0.5)), np.full(5, 0.5))
    # wrapped into (-pi, pi]
    s2 = oracle.perturb(11, 0, 0, a, np.full(1000, math.pi))
    assert np.all(s2 <= math.pi) and np.all(s2 > -math.pi)
    d = np.angle(np.exp(1j * (s2 - math.pi)))
    assert np.all(np.abs(d) <= a + 1e-12)


def test_global_block_of_n_global_sweeps_per_cycle():
    """Algorithm 1 alternates N_global global and N_local localized sweeps: with a
    cycle of 100 and 80 global sweeps, sweeps 20..99 of every cycle are global."""
    cfg = oracle.make_cfg(sy.CFG1.replace(global_every=100, n_global=80))
    g = np.array([oracle.lib().oracle_is_global(oracle.C.byref(cfg), t) for t in range(300)])
    assert g.reshape(3, 100)[:, :20].sum() == 0 and g.reshape(3, 100)[:, 20:].all()
    one = oracle.make_cfg(sy.CFG1.replace(global_every=10, n_global=1))
    zero = oracle.make_cfg(sy.CFG1.replace(global_every=10, n_global=0))
    for t in range(40):
        expect = int((t + 1) % 10 == 0)
        assert oracle.lib().oracle_is_global(oracle.C.byref(one), t) == expect
        assert oracle.lib().oracle_is_global(oracle.C.byref(zero), t) == expect
