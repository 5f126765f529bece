"""Device gradient (amh_grad), its autograd wrapper and the L-BFGS minimiser
(amh_minimize) against the oracle.

Bars: V within 1e-12 relative (float64 on both sides, the same float32 table);
dV/ds within a forward-error bound of the suffix-sum adjoint (below); L-BFGS
traces equal to the oracle's (same iteration counts and stops, values within
1e-9 over the first dozen iterations and 1e-5 over 25, where the optimiser's
own amplification of rounding differences sets the bar), Armijo-consistent
throughout, and the exact minimum reached where it is known.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synthetic as sy

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402  (an import error fails the run)
EPS = np.finfo(np.float64).eps


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grad_tol(L, s, g_or):
    """Forward-error bound of the device's adjoint: g_k is u.(T_p - a x S_p) with the
    suffix sums S_p = sum F_j and T_p = sum x_j x F_j rounded over <= L terms, each
    of size <= R |F|max, R the largest coordinate; |F|max <= sum |dV/ds|-scale terms
    is bounded here by the largest gradient plus one (forces and torques share
    the pair derivatives).  64 L eps R (|g|max + 1) covers the sums and the axis."""
    R = max(1.0, np.abs(oracle.nerf(s)).max())
    return 64.0 * L * EPS * R * (np.abs(g_or).max() + 1.0)


@pytest.mark.parametrize("L", [2, 3, 17, 64, 300, 400])
def test_grad_matches_oracle(L):
    gu.say("grad L", L)
    w = sy.CFG1.replace(L=L, protein_seed=L + 3, noise_seed=L + 4)
    s_ref, y = gu.protein(w)
    ctx = gu.context(w.replace(n_chains=1), y)
    s = np.stack([s_ref, sy.random_torsions(2 * L, L), np.full(2 * L, math.pi),
                  s_ref + 0.2 * np.random.default_rng(L).standard_normal(2 * L)])
    V, g = ctx.grad(torch.from_numpy(s).to(gu.DEV))
    V, g = V.cpu().numpy(), g.cpu().numpy()
    cfg = oracle.make_cfg(w)
    y32 = y.astype(np.float32).astype(np.float64)
    worst = 0.0
    for b in range(s.shape[0]):
        Vo, go = oracle.grad(cfg, y32, s[b])
        assert V[b] == pytest.approx(Vo, rel=1e-12)
        tol = _grad_tol(L, s[b], go)
        err = np.abs(g[b] - go).max()
        worst = max(worst, err / tol)
        assert err <= tol, (b, err, tol)
        assert g[b, 0] == 0.0 and g[b, -1] == 0.0
    gu.say("grad L", L, "worst err / tol", worst)
    ctx.close()


def test_grad_L400_512_conformations_sampled():
    """The differentiation workload's launch: 512 conformations of a 400-residue
    protein in one amh_grad call; four of them checked against the oracle."""
    L, B = 400, 512
    gu.say("grad L", L, "B", B)
    w = sy.CFG1.replace(L=L, n_chains=B, protein_seed=L + 5, noise_seed=L + 6)
    s_ref, y = gu.protein(w)
    rng = np.random.default_rng(L)
    s = s_ref[None, :] + 0.3 * rng.standard_normal((B, 2 * L))
    s = np.ascontiguousarray(np.mod(s + np.pi, 2 * np.pi) - np.pi)
    ctx = gu.context(w.replace(n_chains=1), y)
    V, g = ctx.grad(torch.from_numpy(s).to(gu.DEV))
    V, g = V.cpu().numpy(), g.cpu().numpy()
    ctx.close()
    assert np.isfinite(V).all() and np.isfinite(g).all()
    cfg = oracle.make_cfg(w)
    y32 = y.astype(np.float32).astype(np.float64)
    for b in (0, 170, 341, 511):
        Vo, go = oracle.grad(cfg, y32, s[b])
        assert V[b] == pytest.approx(Vo, rel=1e-12)
        assert np.abs(g[b] - go).max() <= _grad_tol(L, s[b], go)


def test_grad_of_current_chains_and_finite_differences():
    gu.say("grad of chains, FD")
    w = sy.CFG1.replace(L=40, n_chains=3)
    _, y = gu.protein(w)
    s0 = np.stack([sy.random_torsions(2 * w.L, 20 + c) for c in range(3)])
    ctx = gu.context(w, y, s0=s0)
    V, g = ctx.grad()
    Vs, gs = ctx.grad(torch.from_numpy(s0).to(gu.DEV))
    assert torch.equal(V, Vs) and torch.equal(g, gs)
    Ve, _, _ = ctx.energy()
    assert torch.allclose(V, Ve, rtol=1e-12, atol=0)
    # central differences of the device energy (float64) on a spread of torsions
    h = 1e-5
    ks = list(range(1, 2 * w.L - 1, 7))
    sp = np.repeat(s0[:1], 2 * len(ks), axis=0)
    for m, k in enumerate(ks):
        sp[2 * m, k] += h
        sp[2 * m + 1, k] -= h
    Vp, _, _ = ctx.energy(torch.from_numpy(sp).to(gu.DEV))
    Vp = Vp.cpu().numpy()
    fd = (Vp[0::2] - Vp[1::2]) / (2 * h)
    gk = g[0].cpu().numpy()[ks]
    assert np.allclose(gk, fd, rtol=1e-5, atol=1e-5)
    ctx.close()


def test_autograd_backward_is_the_adjoint():
    gu.say("autograd")
    w = sy.CFG1.replace(L=30, n_chains=1)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    s = torch.from_numpy(np.stack([sy.random_torsions(2 * w.L, 31 + b) for b in range(5)])).to(gu.DEV)
    s.requires_grad_(True)
    V = ctx.energy_fn()(s)
    wts = torch.linspace(0.5, 2.0, 5, dtype=torch.float64, device=gu.DEV)
    (V * wts).sum().backward()
    V2, g2 = ctx.grad(s.detach())
    assert torch.equal(V.detach(), V2)
    assert torch.allclose(s.grad, wts[:, None] * g2, rtol=1e-15, atol=0)
    ctx.close()


def _armijo_ok(tr, M):
    return all(tr[i] <= max(tr[max(0, i - M):i]) for i in range(1, len(tr)))


@pytest.mark.parametrize("M", [1, 5])
def test_minimize_replays_against_oracle_lbfgs(M):
    """Every device L-BFGS step is replayed by the oracle from the device's iterate
    (its own values, gradients and curvature pairs at the device's iterates): the
    step must match to 1e-9 of its length (gradients differ by ~1e-13 relative and
    the two-loop recursion amplifies that by the conditioning of the curvature
    pairs, ~1e-11 observed), or stop the line search one trial apart at a
    certified near-tie."""
    gu.say("minimize vs oracle, M", M)
    w = sy.CFG1.replace(L=48, n_chains=1)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    s0 = np.stack([sy.random_torsions(2 * w.L, 40 + b) for b in range(3)])
    st = torch.from_numpy(s0.copy()).to(gu.DEV)
    n_iter = 60
    opts = gu.amh.lbfgs_opts(n_iter=n_iter, nonmonotone=M)
    out = ctx.minimize(st, opts, trace=True, iterates=True)
    X = out["x"].cpu().numpy()
    tr = out["trace"].cpu().numpy()
    cfg = oracle.make_cfg(w)
    y32 = y.astype(np.float32).astype(np.float64)
    o_opts = oracle.lbfgs_opts(n_iter=n_iter, nonmonotone=M)
    for b in range(3):
        it = int(out["iters"][b])
        assert it >= 10
        rc, rep = oracle.lbfgs_replay(cfg, y32, X[b, :it + 1], o_opts, step_tol=1e-9)
        gu.say("chain", b, rep)
        assert rc == 0 and rep["n_steps"] == it and rep["n_forks"] <= 1, rep
        for k in (0, it // 2, it):
            assert tr[b, k] == pytest.approx(oracle.energy(cfg, y32, X[b, k]), rel=1e-12)
        assert float(out["V"][b]) == tr[b, it]
        s_d = st[b].cpu().numpy()
        assert np.abs(np.angle(np.exp(1j * (s_d - X[b, it])))).max() < 1e-12
        assert np.all(np.abs(s_d) <= math.pi)
        # the first iterations also coincide with the oracle's own run from the same start
        _, _, _, _, tr_or = oracle.lbfgs_protein(cfg, y32, s0[b], oracle.lbfgs_opts(n_iter=2,
                                                                                    nonmonotone=M))
        assert np.allclose(tr[b, :3], tr_or, rtol=1e-9, atol=0)
    ctx.close()


def test_minimize_long_run_properties():
    gu.say("minimize long run")
    w = sy.CFG1.replace(L=64, n_chains=1)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    B = 16
    s0 = torch.from_numpy(np.stack([sy.random_torsions(2 * w.L, 60 + b) for b in range(B)])).to(gu.DEV)
    s = s0.clone()
    out = ctx.minimize(s, gu.amh.lbfgs_opts(n_iter=300), trace=True)
    V0, _, _ = ctx.energy(s0)
    V1, _, _ = ctx.energy(s)
    tr = out["trace"].cpu().numpy()
    for b in range(B):
        it = int(out["iters"][b])
        assert _armijo_ok(tr[b, :it + 1], 5)
        assert tr[b, 0] == pytest.approx(float(V0[b]), rel=1e-12)
    assert torch.allclose(out["V"], V1, rtol=1e-12, atol=0)
    assert torch.all(V1 < V0)
    # the minimiser's end points have small gradients or stopped on a failed search
    _, g = ctx.grad(s)
    gmax = g.abs().amax(dim=1).cpu().numpy()
    status = out["status"].cpu().numpy()
    assert np.all((status == 2) | (status == 1) | (gmax <= 1e-6))
    ctx.close()


def test_minimize_reaches_exact_minimum():
    gu.say("minimize exact minimum")
    L = 24
    s_ref = sy.reference_torsions(L, 4)
    dstar = sy.pair_distances(oracle.cb(s_ref))
    y = sy.distogram(dstar, 0.0, 0)
    exact = (dstar >= 2.75) & ~((dstar > 19.75) & (dstar < 20.25))
    y[~exact] = 0.0
    w = sy.CFG1.replace(L=L, n_chains=1)
    ctx = gu.context(w, y)
    V_ref = float(ctx.energy(torch.from_numpy(s_ref[None]).to(gu.DEV))[0][0])
    rng = np.random.default_rng(11)
    s = torch.from_numpy(np.stack([s_ref + 0.03 * rng.standard_normal(2 * L) for _ in range(4)])).to(gu.DEV)
    out = ctx.minimize(s, gu.amh.lbfgs_opts(n_iter=2500, gtol=1e-7))
    V = out["V"].cpu().numpy()
    assert np.all(V - V_ref < 1e-9 * V_ref)
    ctx.close()


def test_minimize_context_chains_then_sample():
    gu.say("minimize chains in place, then sample")
    w = sy.CFG1.replace(L=32, n_chains=4, total_sweeps=40, global_every=5, anchor_every=0)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    ctx.sweep(10)
    before = ctx.get_state()
    out = ctx.minimize(None, gu.amh.lbfgs_opts(n_iter=50))
    st = ctx.get_state()
    Vc, _, _ = ctx.energy()
    assert torch.allclose(st["v"][:, 0], out["V"], rtol=0, atol=0)
    assert torch.allclose(Vc, out["V"], rtol=1e-12, atol=0)
    assert torch.all(st["v"][:, 1] <= before["v"][:, 1])
    assert torch.all(st["v"][:, 1] == torch.minimum(before["v"][:, 1], out["V"]))
    Vb, _, _ = ctx.energy(which=1)
    assert torch.allclose(Vb, st["v"][:, 1], rtol=1e-12, atol=0)
    atoms = gu.amh.conformation(st["s"]).double()
    assert torch.allclose(atoms, st["atoms"], rtol=0, atol=1e-4)
    # sampling continues from the minimised state and replays against the oracle
    s_min = st["s"].cpu().numpy()
    chains = [0, 3]
    tr = gu.traced_run(ctx, chains, 10)
    for m, c in enumerate(chains):
        rc, rep, _ = gu.replay_chain(w, y, tr, m, c, s_min[c], t0=10)
        assert rc == 0 and rep["n_de_fail"] == 0 and rep["n_forks"] <= 2, rep
    ctx.close()


def test_minimize_rejects_bad_options_and_handles_empty():
    gu.say("minimize options")
    from paper_2211_03193_amd import amh
    w = sy.CFG1.replace(L=10, n_chains=2)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    s = torch.zeros(0, 20, dtype=torch.float64, device=gu.DEV)
    assert ctx.minimize(s)["V"].numel() == 0
    for bad in (dict(m=0), dict(m=65), dict(nonmonotone=0), dict(max_ls=0), dict(c1=1.0),
                dict(shrink=0.0), dict(gtol=-1.0), dict(step0=0.0), dict(n_iter=-1)):
        with pytest.raises(amh.AmhError) as e:
            ctx.minimize(None, amh.lbfgs_opts(**bad))
        assert e.value.status == amh.E_INVAL
    with pytest.raises(ValueError):
        ctx.grad(torch.zeros(3, 19, dtype=torch.float64, device=gu.DEV))
    V, g = ctx.grad(torch.zeros(0, 20, dtype=torch.float64, device=gu.DEV))
    assert V.numel() == 0 and g.numel() == 0
    ctx.close()


def test_grad_nan_torsion_gives_nan_energy_and_a_numeric_error():
    """A NaN torsion makes that conformation's V NaN (the pairs it moves are
    evaluated with a NaN distance, which forms no table index), leaves the other
    conformations of the launch as they are alone, and amh_poll reports
    AMH_E_NUMERIC."""
    gu.say("grad NaN torsion")
    from paper_2211_03193_amd import amh
    w = sy.CFG1.replace(L=20, n_chains=1)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    s = np.stack([sy.random_torsions(2 * w.L, 70 + b) for b in range(3)])
    V_ok, g_ok = ctx.grad(torch.from_numpy(s[[0, 2]].copy()).to(gu.DEV))
    ctx.poll()
    s[1, 5] = np.nan
    V, g = ctx.grad(torch.from_numpy(s).to(gu.DEV))
    V = V.cpu().numpy()
    assert np.isnan(V[1]) and np.isfinite(V[[0, 2]]).all()
    assert np.array_equal(V[[0, 2]], V_ok.cpu().numpy())
    assert torch.equal(g[[0, 2]], g_ok)
    with pytest.raises(amh.AmhError) as e:
        ctx.poll()
    assert e.value.status == amh.E_NUMERIC
    ctx.close()


def test_grad_forces_beyond_the_integer_range_give_nan():
    """Forces that reach 2^13 within one 64 x 64 block of pairs (a finite but steep
    table: bins alternating between 0 and 1e4) would overflow the gradient's integer
    force sums: amh_grad returns V = NaN for such a conformation and amh_poll reports
    AMH_E_NUMERIC, while the energy alone (amh_energy) stays finite."""
    gu.say("grad forces beyond the integer range")
    from paper_2211_03193_amd import amh
    w = sy.CFG1.replace(L=20, n_chains=1)
    s_ref, y = gu.protein(w)
    y = np.zeros_like(y)
    y[:, 1::2] = 1.0e4
    ctx = gu.context(w, y)
    s = torch.from_numpy(np.ascontiguousarray(s_ref[None])).to(gu.DEV)
    Ve, _, _ = ctx.energy(s)
    ctx.poll()
    assert np.isfinite(Ve.cpu().numpy()).all()
    V, _ = ctx.grad(s)
    assert np.isnan(V.cpu().numpy()).all()
    with pytest.raises(amh.AmhError) as e:
        ctx.poll()
    assert e.value.status == amh.E_NUMERIC
    ctx.close()
