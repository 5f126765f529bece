"""Pins of the replay checker (``oracle_replay``) that every device parity claim uses.

The checker steps its own chain through the proposals of a recorded trace and
compares each one: the Gaussian increment, dE within 1e-4 of the summed
magnitudes of the changed pair energies plus 1e-6, the decision against the
Metropolis rule min(1, exp(-beta dE)) of Sec. 2.1 applied to the trace's own dE,
and every anchored energy within 1e-4 relative.  A decision that differs from
the oracle's is a fork, allowed only where both dE values sit inside the
tolerance on either side of the acceptance threshold (a near-tie).

Here the traces come from the oracle itself (incremental and brute-force dE),
so the checker must pass them with no failure and no fork; then one error of
each kind is planted and the checker must fail exactly at the planted step,
while the same error scaled to half the tolerance must pass.  A near-tie is
built by choosing the temperature, and a flipped decision there must count as
a fork, not a failure.  All on the CPU.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as sy

REL, ABS, ANCHOR = 1e-4, 1e-6, 1e-4


def _wrap(a: float) -> float:
    if a > math.pi:
        return a - 2.0 * math.pi
    if a <= -math.pi:
        return a + 2.0 * math.pi
    return a


def _protein(w):
    return sy.workload(w, lambda s: sy.pair_distances(oracle.cb(s)))


def _logged_run(w, y, s0, n_sweeps, mode=1):
    cfg = oracle.make_cfg(w)
    ch = oracle.Chains(cfg, y, s0[None, :])
    log, acc, anc = ch.run(n_sweeps, mode=mode, log_steps=True, log_anchors=True)
    return cfg, dict(dE=log[0, :, 0].copy(), delta=log[0, :, 1].copy(), acc=acc[0].copy(),
                     anchor=anc[0].copy() if anc.shape[1] else None), ch


def _replay(cfg, y, s0, n_sweeps, tr, chain=0, t0=0):
    return oracle.replay(cfg, y, chain, s0, t0, n_sweeps, tr["dE"], tr["delta"], tr["acc"],
                         tr["anchor"], REL, ABS, ANCHOR)


def _state_before(cfg, s0, tr, q):
    """Torsions of the traced chain just before step q (its accepted increments)."""
    n = 2 * cfg.L
    s = np.array(s0, dtype=np.float64)
    for step in range(q):
        if tr["acc"][step]:
            k = step % n
            s[k] = _wrap(s[k] + tr["delta"][step])
    return s


def _step_terms(cfg, y, s0, tr, q, t0=0):
    """(dE, S, log u2, beta) of step q recomputed from its definition."""
    n = 2 * cfg.L
    t, k = t0 + q // n, q % n
    ct = oracle.Cfg.from_buffer_copy(cfg)
    ct.window_d = oracle.window_at(cfg, t)
    g = oracle.is_global(cfg, t)
    s = _state_before(cfg, s0, tr, q)
    dE, S = oracle.delta_e(ct, y, s, k, tr["delta"][q], g, 1)
    _, lu = oracle.proposal(cfg.seed, 0, t, k, oracle.sigma_at(cfg, t))
    return dE, S, lu, oracle.beta(cfg, t)


def _robust_step(cfg, y, s0, tr, global_phase, start=0):
    """First live step from `start` in a sweep of the given phase whose decision is far
    from the acceptance threshold (so that a planted error does not flip it) and whose
    changed pairs have a nonzero energy sum."""
    n = 2 * cfg.L
    for q in range(start, len(tr["acc"])):
        t, k = q // n, q % n
        if k in (0, n - 1) or oracle.is_global(cfg, t) != global_phase:
            continue
        dE, S, lu, beta = _step_terms(cfg, y, s0, tr, q)
        tol = REL * S + ABS
        if S > 0.0 and abs(lu + beta * dE) > 20.0 * beta * tol and abs(dE) > 20.0 * tol:
            assert dE == pytest.approx(tr["dE"][q], rel=1e-9, abs=1e-12)
            return q, dE, S, lu, beta
    raise AssertionError("no robust step found")


@pytest.fixture(scope="module")
def small_run():
    """The 64-residue workload, 40 sweeps from the extended chain (4 anchors)."""
    w = sy.CFG1.replace(total_sweeps=200)
    _, y = _protein(w)
    s0 = np.full(2 * w.L, math.pi)
    cfg, tr, ch = _logged_run(w, y, s0, 40)
    return w, cfg, y, s0, tr, ch


def test_own_incremental_trace_passes_exactly(small_run):
    w, cfg, y, s0, tr, ch = small_run
    rc, rep, s_out = _replay(cfg, y, s0, 40, tr)
    assert rc == 0, rep
    assert rep["n_steps"] == 40 * 2 * w.L and rep["n_anchors"] == 4
    for k in ("n_forks", "n_de_fail", "n_delta_fail", "n_logic_fail", "n_anchor_fail"):
        assert rep[k] == 0, rep
    assert rep["first_fail_step"] == -1
    # identical arithmetic on both sides: no error at all, same end state
    assert rep["max_de_abs_err"] == 0.0 and rep["max_anchor_rel_err"] == 0.0
    assert np.array_equal(s_out, ch.s[0])
    assert 0 < tr["acc"].sum() < tr["acc"].size


@pytest.mark.parametrize("L,window_d,global_every", [(40, 8, 10), (40, 12, 3), (24, 80, 1)])
def test_own_trace_from_folded_start_passes(L, window_d, global_every):
    """Folded start (the reference conformation): most changed pairs lie inside the
    last knot.  The trace of the incremental run and of the brute-force run (energies
    recomputed over the whole window or chain) both pass with no fork."""
    w = sy.Workload("replay-folded", L=L, n_chains=1, total_sweeps=60, window_d=window_d,
                    global_every=global_every, T0=0.5, T1=0.05, seed=0x7E57, protein_seed=L + 3,
                    noise_seed=L + 4)
    s_ref, y = _protein(w)
    for mode in (1, 0):
        cfg, tr, ch = _logged_run(w, y, s_ref, 30, mode=mode)
        rc, rep, s_out = _replay(cfg, y, s_ref, 30, tr)
        assert rc == 0 and rep["n_forks"] == 0, (mode, rep)
        assert rep["max_de_rel_err"] < 1e-11 and rep["max_anchor_rel_err"] < 1e-13, rep
        assert np.array_equal(s_out, ch.s[0])


@pytest.mark.parametrize("global_phase", [False, True])
def test_planted_de_error_fails_at_its_step(small_run, global_phase):
    w, cfg, y, s0, tr, _ = small_run
    q, dE, S, lu, beta = _robust_step(cfg, y, s0, tr, global_phase, start=300)
    tol = REL * S + ABS
    for sign in (1.0, -1.0):
        bad = dict(tr, dE=tr["dE"].copy())
        bad["dE"][q] = dE + sign * 2.0 * tol
        rc, rep, _ = _replay(cfg, y, s0, 40, bad)
        assert rc == 1 and rep["first_fail_step"] == q and rep["n_de_fail"] == 1, rep
        assert rep["n_logic_fail"] == 0 and rep["n_forks"] == 0, rep
        ok = dict(tr, dE=tr["dE"].copy())
        ok["dE"][q] = dE + sign * 0.5 * tol
        rc, rep, _ = _replay(cfg, y, s0, 40, ok)
        assert rc == 0 and rep["n_forks"] == 0, rep


@pytest.mark.parametrize("global_phase", [False, True])
def test_planted_decision_flip_fails_at_its_step(small_run, global_phase):
    w, cfg, y, s0, tr, _ = small_run
    q, dE, S, lu, beta = _robust_step(cfg, y, s0, tr, global_phase, start=500)
    bad = dict(tr, acc=tr["acc"].copy())
    bad["acc"][q] ^= 1
    rc, rep, _ = _replay(cfg, y, s0, 40, bad)
    assert rc == 1 and rep["first_fail_step"] == q and rep["n_logic_fail"] >= 1, rep


def test_planted_increment_error_fails_at_its_step(small_run):
    w, cfg, y, s0, tr, _ = small_run
    q, *_ = _robust_step(cfg, y, s0, tr, False, start=700)
    bad = dict(tr, delta=tr["delta"].copy())
    bad["delta"][q] += 1e-9
    rc, rep, _ = _replay(cfg, y, s0, 40, bad)
    assert rc == 1 and rep["first_fail_step"] == q and rep["n_delta_fail"] == 1, rep
    ok = dict(tr, delta=tr["delta"].copy())
    ok["delta"][q] += 1e-13          # one libm ulp apart is not an error
    rc, rep, _ = _replay(cfg, y, s0, 40, ok)
    assert rc == 0, rep


def test_planted_anchor_error_fails_at_its_anchor(small_run):
    w, cfg, y, s0, tr, _ = small_run
    n = 2 * w.L
    for ai in (0, 2):
        bad = dict(tr, anchor=tr["anchor"].copy())
        bad["anchor"][ai] *= 1.0 + 2.0 * ANCHOR
        rc, rep, _ = _replay(cfg, y, s0, 40, bad)
        # the anchor of sweep t is checked once its 2L proposals are done
        assert rc == 1 and rep["n_anchor_fail"] == 1, rep
        assert rep["first_fail_step"] == (ai + 1) * cfg.anchor_every * n, rep
        ok = dict(tr, anchor=tr["anchor"].copy())
        ok["anchor"][ai] *= 1.0 + 0.5 * ANCHOR
        rc, rep, _ = _replay(cfg, y, s0, 40, ok)
        assert rc == 0, rep


def _forced_trace(cfg, y, s0, n_sweeps, q, dE_q, acc_q):
    """Trace of a chain that follows the Metropolis rule at every step except step q,
    where the recorded dE and decision are the given ones; every other step is
    recomputed from its definition on the branch the trace takes."""
    n = 2 * cfg.L
    s = np.array(s0, dtype=np.float64)
    dEs, deltas, accs, anchors = [], [], [], []
    for t in range(n_sweeps):
        sig, beta, g = oracle.sigma_at(cfg, t), oracle.beta(cfg, t), oracle.is_global(cfg, t)
        for k in range(n):
            delta, lu = oracle.proposal(cfg.seed, 0, t, k, sig)
            dE, _ = oracle.delta_e(cfg, y, s, k, delta, g, 1)
            a = (dE <= 0.0) or (lu < -beta * dE)
            if t * n + k == q:
                dE, a = dE_q, acc_q
            dEs.append(dE)
            deltas.append(delta)
            accs.append(int(a))
            if a:
                s[k] = _wrap(s[k] + delta)
        if (t + 1) % cfg.anchor_every == 0:
            anchors.append(oracle.energy(cfg, y, s))
    return dict(dE=np.array(dEs), delta=np.array(deltas), acc=np.array(accs, dtype=np.uint8),
                anchor=np.array(anchors))


def test_flip_at_a_real_near_tie_is_a_fork():
    """Noise-free protein started at its reference conformation, the exact minimum, so
    the first live proposal (psi_0, step 1) raises V: dE > 0.  The temperature is set
    so that ln u2 + beta dE sits a quarter of the tolerance above zero (the oracle
    rejects); a trace whose dE lies half a tolerance lower accepts, correctly for its
    own dE.  That is a certified near-tie: one fork, no failure.  The same flip with
    dE two tolerances lower, or with the oracle's own dE, fails at that step."""
    base = sy.Workload("near-tie", L=12, n_chains=1, total_sweeps=3, window_d=8, global_every=1,
                       sigma_deg=10.0, eps=0.0, seed=0x7157, protein_seed=31, noise_seed=32)
    s_ref, y = _protein(base)
    q = 1
    for key in range(0x7157, 0x7157 + 64):     # a key whose first live move is well uphill
        base = base.replace(seed=key)
        cfg0 = oracle.make_cfg(base)
        delta, lu = oracle.proposal(cfg0.seed, 0, 0, q, cfg0.sigma)
        dE, S = oracle.delta_e(cfg0, y, s_ref, q, delta, True, 1)
        tol = REL * S + ABS
        if dE > 10.0 * tol:
            break
    assert dE > 10.0 * tol and lu < 0.0
    T = (dE - 0.25 * tol) / -lu           # ln u2 + dE / T = 0.25 tol / T
    w = base.replace(T0=T, T1=T)
    cfg = oracle.make_cfg(w)
    beta = oracle.beta(cfg, 0)
    assert beta == 1.0 / T
    margin = lu + beta * dE
    assert 0.0 < margin <= beta * tol      # the oracle rejects, inside the tolerance
    dev = _forced_trace(cfg, y, s_ref, 3, q, dE - 0.5 * tol, 1)
    assert dev["acc"][q] == 1 and (lu < -beta * dev["dE"][q])
    rc, rep, s_out = _replay(cfg, y, s_ref, 3, dev)
    assert rc == 0, rep
    assert rep["n_forks"] == 1 and rep["max_fork_margin"] == pytest.approx(margin, rel=1e-6), rep
    # the replay went on along the accepted branch: its end state is the trace's
    assert s_out[q] == _wrap(s_ref[q] + delta)
    # the same flip outside the tolerance, or without a dE that justifies it, fails there
    for dE_bad in (dE - 2.0 * tol, dE):
        bad = _forced_trace(cfg, y, s_ref, 3, q, dE_bad, 1)
        rc, rep, _ = _replay(cfg, y, s_ref, 3, bad)
        assert rc == 1 and rep["first_fail_step"] == q, rep
