"""Device parity of the schedule variants: proposal-width annealing and cascaded
localization radii replayed proposal by proposal against the oracle, and the
noisy restart compared with the oracle's definition."""
import math

import numpy as np
import pytest
import torch

import oracle
import synthetic as sy

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402  (an import error fails the run)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


VAR = sy.Workload("variants", L=30, n_chains=5, total_sweeps=30, window_d=6, global_every=5,
                  sigma_deg=20.0, T0=1.5, T1=0.05, seed=0x7A7A, protein_seed=12, noise_seed=13,
                  sigma_end_deg=5.0, cascade=(2, 14))


@pytest.mark.parametrize("G,W", [(1, 4), (4, 8)])
def test_annealed_width_and_cascade_replay(G, W):
    gu.say("variants replay G", G, "W", W)
    _, y = gu.protein(VAR)
    ctx = gu.context(VAR, y, chains_per_group=G, waves_per_group=W)
    _replay_variant(ctx, VAR, y)
    ctx.close()


def test_block_of_global_sweeps_replay():
    """Cycles of 7 sweeps whose last 4 are global (Algorithm 1's N_global block)."""
    w = VAR.replace(global_every=7, n_global=4, anchor_every=7, total_sweeps=21)
    gu.say("n_global replay")
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    chains = [1, 4]
    tr = gu.traced_run(ctx, chains, w.total_sweeps, chunk=5)
    for m, c in enumerate(chains):
        rc, rep, _ = gu.replay_chain(w, y, tr, m, c, gu.extended(w))
        assert rc == 0 and rep["n_de_fail"] == 0 and rep["n_forks"] <= 2, rep
    cnt = ctx.get_state()["counters"].cpu().numpy()
    assert np.all(cnt[:, 1] > 0)          # global accepts happened
    ctx.close()


def _replay_variant(ctx, VAR, y):
    chains = [0, 2, 4]
    tr = gu.traced_run(ctx, chains, VAR.total_sweeps, chunk=7)
    for m, c in enumerate(chains):
        rc, rep, _ = gu.replay_chain(VAR, y, tr, m, c, gu.extended(VAR))
        assert rc == 0 and rep["n_delta_fail"] == 0 and rep["n_de_fail"] == 0, rep
        assert rep["n_forks"] <= 2, rep
    # the increments follow the width schedule: delta / sigma_t is the unit draw
    cfg = oracle.make_cfg(VAR)
    n = 2 * VAR.L
    for t in (0, 13, 29):
        k = 5
        d_unit, _ = oracle.proposal(VAR.seed, 2, t, k, 1.0)
        assert tr["delta"][1, t * n + k] == pytest.approx(d_unit * oracle.sigma_at(cfg, t), rel=1e-12)
    key = (tr["dE"].tobytes(), tr["acc"].tobytes())
    _KEY.setdefault("ref", key)
    assert key == _KEY["ref"]


_KEY = {}


def test_noisy_restart_matches_oracle_and_sampling_continues():
    gu.say("noisy restart")
    w = VAR.replace(sigma_end_deg=0.0, cascade=())
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    ctx.sweep(10)
    before = ctx.get_state()
    a = math.radians(10.0)
    ctx.perturb(a, 3)
    after = ctx.get_state()
    s0, s1 = before["s"].cpu().numpy(), after["s"].cpu().numpy()
    cfg = oracle.make_cfg(w)
    y32 = y.astype(np.float32).astype(np.float64)
    for c in range(w.n_chains):
        ref = oracle.perturb(w.seed, c, 3, a, s0[c])
        assert np.abs(np.angle(np.exp(1j * (s1[c] - ref)))).max() <= 1e-14
        V = oracle.energy(cfg, y32, s1[c])
        assert after["v"][c, 0].item() == pytest.approx(V, rel=1e-12)
        best = min(before["v"][c, 1].item(), after["v"][c, 0].item())
        assert after["v"][c, 1].item() == best
    assert torch.equal(after["counters"], before["counters"]) and after["t"] == before["t"]
    assert torch.allclose(gu.amh.conformation(after["s"]).double(), after["atoms"], atol=1e-4, rtol=0)
    improved = after["v"][:, 1] < before["v"][:, 1]
    assert torch.equal(after["s_best"][improved], after["s"][improved])
    assert torch.equal(after["s_best"][~improved], before["s_best"][~improved])
    # sampling continues from the perturbed state
    chains = [1, 3]
    tr = gu.traced_run(ctx, chains, 10)
    for m, c in enumerate(chains):
        rc, rep, _ = gu.replay_chain(w, y, tr, m, c, s1[c], t0=10)
        assert rc == 0 and rep["n_de_fail"] == 0 and rep["n_forks"] <= 2, rep
    ctx.close()
