"""The paper's run schedules (host orchestration of device calls) on small runs."""
import math

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


W = sy.Workload("sched", L=24, n_chains=6, total_sweeps=30, window_d=6, global_every=5,
                sigma_deg=10.0, T0=1.0, T1=0.05, seed=0x5C, protein_seed=21, noise_seed=22,
                sigma_end_deg=4.0)


@pytest.fixture(scope="module")
def table():
    _, y = gu.protein(W)
    return torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(gu.DEV)


def test_alt_mh_restarts(table):
    from paper_2211_03193_amd import variants
    gu.say("alt-mh restarts")
    r = variants.alt_mh_restarts(W, table, runs=4)
    assert len(r["runs"]) == 4
    bests = [h["best"] for h in r["runs"]]
    assert r["best"] == min(bests)
    # a run restarted from the previous best states ends at or below their energy;
    # after m runs without improvement the width range is 10/m -> 1/m degrees
    misses = 0
    for a, b in zip(r["runs"], r["runs"][1:]):
        misses = 0 if a["improved"] else misses + 1
        if a["improved"]:
            assert b["best"] <= a["best"] + 1e-9
        assert b["sigma_deg"] == ([10.0, 4.0] if misses == 0 else [10.0 / misses, 1.0 / misses])


def test_noisy_restart_schedule(table):
    from paper_2211_03193_amd import variants
    gu.say("mh noisy restarts")
    r = variants.mh_noisy_restarts(W, table, every=7)
    assert r["restarts"] == math.ceil(W.total_sweeps / 7) - 1 and np.isfinite(r["best"])


def test_beta_sweep_and_chain_counts(table):
    from paper_2211_03193_amd import variants
    gu.say("beta sweep, chain counts")
    r = variants.beta_sweep(W, table, betas=[0.5, 5.0], runs=4)
    for name in ("alt", "mh"):
        assert [e["beta"] for e in r[name]] == [0.5, 5.0]
        for e in r[name]:
            assert e["min"] <= e["mean"] <= e["max"]
    c = variants.chain_count_study(W, table, counts=(3, 12))
    assert c["counts"][1]["best"] <= c["counts"][0]["best"]   # the 3 chains are among the 12


def test_hybrid_lbfgs_with_localized_mh(table):
    from paper_2211_03193_amd import amh, hybrid
    gu.say("lbfgs + localized mh schedule")
    ctx = amh.Context(amh.make_config(W.replace(global_every=0, total_sweeps=40)), table)
    V0 = ctx.energy()[0].clone()
    outs = hybrid.lbfgs_with_localized_mh(ctx, cycles=2, lbfgs_iters=15, mh_sweeps=10)
    assert len(outs) == 3
    st = ctx.get_state()
    assert torch.all(st["v"][:, 1] < V0)
    assert st["t"] == 20
    ctx.close()
