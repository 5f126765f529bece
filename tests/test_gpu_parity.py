"""Per-proposal parity of the AMH hot path with the oracle at the benchmark sizes.

* one protein of 64 residues, one chain, the whole 2e4-sweep run (window 8,
  global every 10, sigma 10 deg, T 1 -> 0.01), every proposal replayed;
* one protein of 300 residues, 1024 chains in the launch shape the benchmark
  times (four chains per workgroup, eight wavefronts), chains 0, 341, 682 and
  1023 replayed over the first sweeps from the extended chain, and over 30
  sweeps from compact conformations: the reference conformation copied to every
  chain, and the device's own state at an anchor sweep late in the schedule
  (sweep 2000 of 5000, where every chain's coordinates have just been rebuilt
  from its torsions, so the oracle starts from the same geometry).  Compact
  states put many pairs inside the last knot: most rectangle tiles survive the
  sphere test and the near-pair queues fill and flush many times per proposal.
"""
import numpy as np
import pytest
import torch

import synthetic as sy

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402  (an import error fails the run)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(rep, n_steps, max_fork_frac):
    assert rep["n_steps"] == n_steps
    for k in ("n_delta_fail", "n_logic_fail", "n_de_fail", "n_anchor_fail"):
        assert rep[k] == 0, rep
    assert rep["n_forks"] <= max(2, max_fork_frac * n_steps), rep


def test_plain_L64_full_run():
    w = sy.CFG1
    gu.say("parity L64 1 chain 20000 sweeps")
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    tr = gu.traced_run(ctx, [0], w.total_sweeps, chunk=1000)
    st = ctx.get_state()
    ctx.close()
    gu.say("replay")
    rc, rep, s_out = gu.replay_chain(w, y, tr, 0, 0, gu.extended(w))
    print(rep)
    _check(rep, w.total_sweeps * 2 * w.L, 1e-4)
    assert rep["n_anchors"] == w.total_sweeps // w.global_every
    if rep["n_forks"] == 0:
        assert np.array_equal(s_out, st["s"].cpu().numpy()[0])


@pytest.mark.parametrize("n_sweeps", [20])
def test_single_L300_1024_chains_sampled(n_sweeps):
    w = sy.CFG2
    gu.say("parity L300 1024 chains", n_sweeps, "sweeps")
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    info = ctx.info()
    gu.say("launch shape", info)
    tr = gu.traced_run(ctx, w.trace_chains, n_sweeps)
    ctx.close()
    for m, c in enumerate(w.trace_chains):
        gu.say("replay chain", c)
        rc, rep, _ = gu.replay_chain(w, y, tr, m, c, gu.extended(w))
        print(c, rep)
        _check(rep, n_sweeps * 2 * w.L, 1e-4)


@pytest.mark.parametrize("start", ["reference", "late_anchor"])
def test_single_L300_1024_chains_compact(start):
    w = sy.CFG2
    n_sweeps = 30
    gu.say("parity L300 1024 chains, compact start:", start)
    s_ref, y = gu.protein(w)
    if start == "reference":
        ctx = gu.context(w, y, s0=np.tile(s_ref, (w.n_chains, 1)))
        t0, s0 = 0, {c: s_ref for c in w.trace_chains}
    else:
        ctx = gu.context(w, y)
        t0 = 2000
        ctx.sweep(t0)
        st = ctx.get_state()
        s_np = st["s"].cpu().numpy()
        s0 = {c: s_np[c].copy() for c in w.trace_chains}
        assert st["t"] == t0
    info = ctx.info()
    gu.say("launch shape", info)
    assert (info["chains_per_group"], info["waves_per_group"]) == (4, 8)
    tr = gu.traced_run(ctx, w.trace_chains, n_sweeps)
    ctx.close()
    for m, c in enumerate(w.trace_chains):
        gu.say("replay chain", c, "from sweep", t0)
        rc, rep, _ = gu.replay_chain(w, y, tr, m, c, s0[c], t0=t0)
        print(start, c, rep)
        _check(rep, n_sweeps * 2 * w.L, 1e-4)
        assert rep["n_anchors"] == n_sweeps // w.global_every
