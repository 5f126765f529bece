"""Pins of the oracle's sampler: schedule, Metropolis rule, alternation, resume.

The Metropolis rule is pinned by detailed balance: on a two-residue chain the
only live torsions are psi_0 and phi_1, so a long global-only run at fixed
temperature must sample exp(-beta E_01(d(psi_0, phi_1))), computed here by
quadrature, and the two dead torsions must be uniform.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synthetic as sy


def test_schedule_counts_and_ends():
    cfg = oracle.make_cfg(sy.CFG1)
    g = np.array([oracle.is_global(cfg, t) for t in range(cfg.total_sweeps)])
    assert g.sum() == 2000 and (~g).sum() == 18000
    assert np.all(np.flatnonzero(g) % 10 == 9)
    assert oracle.beta(cfg, 0) == pytest.approx(1.0, rel=1e-15)
    assert oracle.beta(cfg, cfg.total_sweeps - 1) == pytest.approx(100.0, rel=1e-12)
    b = np.array([oracle.beta(cfg, t) for t in range(0, cfg.total_sweeps, 97)])
    assert np.all(np.diff(b) > 0)
    # geometric: log T is linear in t
    lt = -np.log([oracle.beta(cfg, t) for t in (0, 5000, 10000, 19999)])
    assert np.allclose(lt, np.log(0.01) * np.array([0, 5000, 10000, 19999]) / 19999, atol=1e-12)
    one = oracle.make_cfg(sy.CFG1.replace(global_every=0))
    assert not any(oracle.is_global(one, t) for t in range(100))


def _two_residue_case(T, sigma):
    w = sy.Workload("L2", L=2, n_chains=1, total_sweeps=10, window_d=2, global_every=1,
                    sigma_deg=math.degrees(sigma), T0=T, T1=T, seed=0x2222, anchor_every=1)
    c = sy.bin_knots()
    y = (1.5 * (c - 5.6) ** 2)[None, :]          # one pair, one smooth well
    return w, oracle.make_cfg(w), y


def _trajectory(cfg, y, s0, n_sweeps):
    ch = oracle.Chains(cfg, y, s0)
    log, acc, _ = ch.run(n_sweeps, log_steps=True)
    n = 2 * cfg.L
    inc = (log[0, :, 1] * acc[0]).reshape(n_sweeps, n)
    s = np.mod(s0[None, :] + np.cumsum(inc, axis=0) + np.pi, 2 * np.pi) - np.pi
    assert np.allclose(np.mod(s[-1] - ch.s[0] + np.pi, 2 * np.pi) - np.pi, 0.0, atol=1e-9)
    return s


@pytest.mark.parametrize("T", [1.0, 0.4])
def test_two_residue_chain_samples_boltzmann(T):
    w, cfg, y = _two_residue_case(T, sigma=3.0)
    s = _trajectory(cfg, y, np.zeros(4), 60000)[1000::2]
    nb = 12
    edges = np.linspace(-np.pi, np.pi, nb + 1)
    H, _, _ = np.histogram2d(s[:, 1], s[:, 2], bins=[edges, edges])
    # quadrature of exp(-E/T) over each cell (8x8 midpoints)
    sub = 8
    g = -np.pi + (np.arange(nb * sub) + 0.5) * (2 * np.pi / (nb * sub))
    E = np.empty((g.size, g.size))
    for a, psi in enumerate(g):
        for b, phi in enumerate(g):
            cb = oracle.cb(np.array([0.0, psi, phi, 0.0]))
            E[a, b] = oracle.pair_energy(y[0], float(np.linalg.norm(cb[1] - cb[0])))
    dens = np.exp(-(E - E.min()) / T).reshape(nb, sub, nb, sub).sum(axis=(1, 3))
    expected = dens / dens.sum() * H.sum()
    chi2, p = stats.chisquare(H.ravel(), expected.ravel())
    assert p > 1e-3, (chi2, p)
    # a wrong temperature is detected by the same test
    dens_wrong = np.exp(-(E - E.min()) / (2.0 * T)).reshape(nb, sub, nb, sub).sum(axis=(1, 3))
    assert stats.chisquare(H.ravel(), (dens_wrong / dens_wrong.sum() * H.sum()).ravel())[1] < 1e-6
    # dead torsions random-walk to the uniform law
    for k in (0, 3):
        assert stats.kstest((s[::5, k] + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


def test_zero_temperature_global_energy_never_rises():
    w = sy.CFG1.replace(L=24, total_sweeps=30, global_every=1, T0=1e-12, T1=1e-12, anchor_every=1)
    cfg = oracle.make_cfg(w)
    s_ref = sy.reference_torsions(24, 3)
    y = sy.distogram(sy.pair_distances(oracle.cb(s_ref)), 0.1, 3)
    ch = oracle.Chains(cfg, y, np.full(48, np.pi))
    V0 = ch.v[0, 0]
    _, _, an = ch.run(30, log_anchors=True)
    V = np.concatenate([[V0], an[0]])
    assert np.all(np.diff(V) <= 1e-9)
    assert V[-1] < V[0]


def _cfg1_small():
    w = sy.CFG1_SMALL
    s_ref = sy.reference_torsions(w.L, w.protein_seed)
    y = sy.distogram(sy.pair_distances(oracle.cb(s_ref)), w.eps, w.noise_seed)
    return w, oracle.make_cfg(w), y


def test_resume_is_exact():
    w, cfg, y = _cfg1_small()
    s0 = np.full((3, 2 * w.L), np.pi)
    a = oracle.Chains(cfg, y, s0)
    a.run(50)
    b = oracle.Chains(cfg, y, s0)
    b.run(20)
    c = oracle.Chains(cfg, y, b.s)            # restore from the saved state
    c.s_best[:] = b.s_best
    c.v[:] = b.v
    c.counters[:] = b.counters
    c.t = b.t
    c.run(30)
    assert np.array_equal(a.s, c.s) and np.array_equal(a.s_best, c.s_best)
    assert np.array_equal(a.v, c.v) and np.array_equal(a.counters, c.counters)


def test_chain_trajectory_independent_of_other_chains():
    w, cfg, y = _cfg1_small()
    alone = oracle.Chains(cfg, y, np.full((1, 2 * w.L), np.pi), chain_ids=[5])
    alone.run(30)
    mixed = oracle.Chains(cfg, y, np.full((3, 2 * w.L), np.pi), chain_ids=[3, 5, 7])
    mixed.run(30, threads=3)
    assert np.array_equal(alone.s[0], mixed.s[1])
    assert not np.array_equal(mixed.s[0], mixed.s[1])


def test_dead_torsions_always_accepted_and_state_wrapped():
    w, cfg, y = _cfg1_small()
    ch = oracle.Chains(cfg, y, np.full(2 * w.L, np.pi))
    log, acc, _ = ch.run(40, log_steps=True)
    n = 2 * w.L
    lg = log[0].reshape(40, n, 2)
    ac = acc[0].reshape(40, n)
    assert np.all(lg[:, [0, n - 1], 0] == 0.0) and np.all(ac[:, [0, n - 1]] == 1)
    assert np.all(ch.s > -np.pi) and np.all(ch.s <= np.pi)
    # every decision follows the Metropolis rule on the logged dE
    lu = np.array([[oracle.proposal(cfg.seed, 0, t, k, cfg.sigma)[1] for k in range(n)] for t in range(40)])
    beta = np.array([oracle.beta(cfg, t) for t in range(40)])[:, None]
    rule = (lg[..., 0] <= 0) | (lu < -beta * lg[..., 0])
    assert np.array_equal(rule, ac.astype(bool))


def test_alternation_local_accepts_more_than_global():
    """A localized proposal judges fewer pairs, so it is accepted more often
    (Sec. 2.2 on the radius d)."""
    w, cfg, y = _cfg1_small()
    ch = oracle.Chains(cfg, y, np.full(2 * w.L, np.pi))
    ch.run(200)
    loc, glo = ch.counters[0, 0], ch.counters[0, 1]
    assert loc / 180 > glo / 20
    assert ch.counters[0, 3] == 20          # one anchor per global sweep
    assert ch.v[0, 1] <= ch.v[0, 0]


def test_time_to_target_counter():
    w, cfg, y = _cfg1_small()
    ch = oracle.Chains(cfg, y, np.full(2 * w.L, np.pi))
    ch.run(100, target=math.inf)
    assert ch.counters[0, 2] == 10          # first anchor
    ch2 = oracle.Chains(cfg, y, np.full(2 * w.L, np.pi))
    ch2.run(100, target=-1.0)
    assert ch2.counters[0, 2] == -1
