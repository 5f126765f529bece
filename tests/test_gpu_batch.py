"""Batches of proteins of different lengths in one launch (amh_batch_*).

A member advanced in a batch must follow exactly the trajectory it follows
alone (same Philox counters, same arithmetic): states are compared bit for bit
against the plain per-protein launch, for every launch plan, and a traced
member is replayed by the oracle.
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


MEMBERS = [
    sy.Workload("b20", L=20, n_chains=6, total_sweeps=80, window_d=6, global_every=3, sigma_deg=20.0,
                T0=2.0, T1=0.1, seed=0xB0, protein_seed=1, noise_seed=2),
    sy.Workload("b37", L=37, n_chains=3, total_sweeps=80, window_d=8, global_every=4, sigma_deg=12.0,
                T0=1.0, T1=0.05, seed=0xB1, protein_seed=3, noise_seed=4),
    sy.Workload("b64", L=64, n_chains=9, total_sweeps=80, window_d=12, global_every=5,
                sigma_deg=10.0, T0=1.0, T1=0.01, seed=0xB2, protein_seed=5, noise_seed=6),
    sy.Workload("b150", L=150, n_chains=4, total_sweeps=80, window_d=10, global_every=2,
                sigma_deg=8.0, T0=0.5, T1=0.02, seed=0xB3, protein_seed=7, noise_seed=8),
]


@pytest.fixture(scope="module")
def tables():
    return [gu.protein(w)[1] for w in MEMBERS]


def _state(ctx):
    st = ctx.get_state()
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in st.items()}


def _alone(tables, n):
    out = []
    for w, y in zip(MEMBERS, tables):
        ctx = gu.context(w, y)
        ctx.sweep(n)
        out.append(_state(ctx))
        ctx.close()
    return out


@pytest.fixture(scope="module")
def alone12(tables):
    return _alone(tables, 12)


def _equal(a, b):
    for k in ("s", "s_best", "v", "counters", "atoms", "t"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("plan", range(6))
def test_batch_equals_plain_launches(tables, alone12, plan):
    from paper_2211_03193_amd import amh
    gu.say("batch plan", plan)
    ctxs = [gu.context(w, y) for w, y in zip(MEMBERS, tables)]
    b = amh.Batch(ctxs)
    b.set_plan(plan)
    info = b.info()
    assert info["plan"] == plan and info["launches"] >= 1
    b.sweep(5)
    b.sweep(7)
    for ctx, ref in zip(ctxs, alone12):
        _equal(_state(ctx), ref)
    b.close()
    for c in ctxs:
        c.close()


def test_per_member_sweep_counts(tables):
    from paper_2211_03193_amd import amh
    gu.say("batch per-member counts")
    counts = [12, 0, 7, 3]
    ctxs = [gu.context(w, y) for w, y in zip(MEMBERS, tables)]
    b = amh.Batch(ctxs)
    b.sweep(counts)
    for (w, y), ctx, n in zip(zip(MEMBERS, tables), ctxs, counts):
        ref = gu.context(w, y)
        ref.sweep(n)
        _equal(_state(ctx), _state(ref))
        ref.close()
    with pytest.raises(amh.AmhError):
        b.sweep([100, 0, 0, 0])      # member 0 would pass its 80 sweeps
    assert [c.info()["t"] for c in ctxs] == counts
    b.close()
    for c in ctxs:
        c.close()


def test_traced_member_replays(tables):
    from paper_2211_03193_amd import amh
    gu.say("batch traced member")
    ctxs = [gu.context(w, y) for w, y in zip(MEMBERS, tables)]
    b = amh.Batch(ctxs)
    w, y = MEMBERS[2], tables[2]
    chains = [0, 8]
    tr = ctxs[2].set_trace(chains, 10)
    b.sweep(10)
    ctxs[2].poll()
    torch.cuda.synchronize()
    trn = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in tr.items()}
    for m, c in enumerate(chains):
        rc, rep, _ = gu.replay_chain(w, y, trn, m, c, gu.extended(w))
        assert rc == 0 and rep["n_de_fail"] == 0 and rep["n_forks"] <= 2, rep
    b.close()
    for c in ctxs:
        c.close()


def test_tuner_keeps_trajectories(tables):
    from paper_2211_03193_amd import amh
    gu.say("batch tuner")
    ctxs = [gu.context(w, y) for w, y in zip(MEMBERS, tables)]
    b = amh.Batch(ctxs)
    plan, ms = b.tune(2)
    assert 0 <= plan < 6 and all(m > 0 for m in ms)
    assert b.info()["plan"] == plan
    b.sweep(3)
    ref = _alone(tables, 15)
    for ctx, r in zip(ctxs, ref):
        _equal(_state(ctx), r)
    b.close()
    for c in ctxs:
        c.close()


def test_batch_rejects_bad_use(tables):
    from paper_2211_03193_amd import amh
    gu.say("batch errors")
    ctxs = [gu.context(w, y) for w, y in zip(MEMBERS[:2], tables[:2])]
    with pytest.raises(amh.AmhError):
        amh.Batch([ctxs[0], ctxs[0]])
    with pytest.raises(amh.AmhError):
        amh.Batch([])
    b = amh.Batch(ctxs)
    ctxs[1].sweep(75)
    t0 = [c.info()["t"] for c in ctxs]
    with pytest.raises(amh.AmhError) as e:
        b.sweep(10)          # member 1 would pass its 80 sweeps
    assert e.value.status == amh.E_INVAL
    assert [c.info()["t"] for c in ctxs] == t0
    b.sweep(5)
    assert [c.info()["t"] for c in ctxs] == [5, 80]
    b.close()
    for c in ctxs:
        c.close()
