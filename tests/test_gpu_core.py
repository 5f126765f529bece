"""Device parity of the building blocks and of small AMH runs against the oracle.

Every call goes through the C ABI of libamh.so.  Bars: Philox bit-exact;
coordinates within float32 rounding of the float64 oracle; float64 energies
within 1e-9 relative; per-proposal traces replayed by the oracle with dE within
1e-4 of the summed magnitude of the changed pair energies and decisions equal
except at certified near-ties; anchors within 1e-9 relative.
"""
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


def test_philox_bit_exact():
    from paper_2211_03193_amd import amh
    gu.say("philox 2^20 counters")
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(1 << 20, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1000, 0] = np.arange(1000)
    ctr[:1000, 1:] = 0
    for key in (0, 0x414D4802, 0xFFFFFFFFFFFFFFFF):
        dev = amh.philox(torch.from_numpy(ctr.view(np.int32)).to(gu.DEV), key)
        got = dev.cpu().numpy().view(np.uint32)
        ref = oracle.philox(ctr, [key & 0xFFFFFFFF, key >> 32])
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("L", [2, 3, 17, 64, 300])
def test_conformation_matches_oracle(L):
    from paper_2211_03193_amd import amh
    gu.say("conformation L", L)
    s = sy.random_torsions((6, 2 * L), L)
    s[0] = np.pi
    atoms = amh.conformation(torch.from_numpy(s).to(gu.DEV)).cpu().numpy()
    for b in range(s.shape[0]):
        ref = oracle.nerf(s[b])
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(atoms[b] - ref).max() <= 2e-7 * scale + 1e-6


@pytest.mark.parametrize("L", [2, 5, 64, 300])
def test_energy_matches_oracle(L):
    gu.say("energy L", L)
    w = sy.CFG1.replace(L=L, protein_seed=L, noise_seed=L + 1)
    s_ref, y = gu.protein(w)
    ctx = gu.context(w.replace(n_chains=3), y)
    s = np.stack([s_ref, sy.random_torsions(2 * L, 7), np.full(2 * L, np.pi)])
    V, _, cb = ctx.energy(torch.from_numpy(s).to(gu.DEV), want_cb=True)
    V = V.cpu().numpy()
    cfg = oracle.make_cfg(w)
    y32 = y.astype(np.float32).astype(np.float64)
    for b in range(3):
        assert V[b] == pytest.approx(oracle.energy(cfg, y32, s[b]), rel=1e-9)
    # context state after init: extended chain, V(pi), counters reset
    Vc, sc, _ = ctx.energy(want_s=True)
    st = ctx.get_state()
    assert np.all(sc.cpu().numpy() == np.pi)
    assert np.allclose(st["v"].cpu().numpy(), oracle.energy(cfg, y32, np.full(2 * L, np.pi)), rtol=1e-9)
    assert np.array_equal(st["counters"].cpu().numpy(), np.tile([0, 0, -1, 0], (3, 1)))
    assert Vc.cpu().numpy() == pytest.approx(st["v"].cpu().numpy()[:, 0], rel=1e-12)
    ctx.close()


def test_nonfinite_table_rejected():
    from paper_2211_03193_amd import amh
    gu.say("non-finite table")
    w = sy.CFG1.replace(L=10)
    _, y = gu.protein(w)
    y = y.copy()
    y[7, 3] = np.nan
    with pytest.raises(amh.AmhError) as e:
        gu.context(w, y)
    assert e.value.status == amh.E_NUMERIC


def test_nonfinite_torsions_give_nan_energy():
    """A conformation with a non-finite torsion has no energy: amh_init rejects such
    a start with AMH_E_NUMERIC, and amh_energy returns NaN for that row (the other
    rows as they are alone) and reports AMH_E_NUMERIC at the next amh_poll."""
    from paper_2211_03193_amd import amh
    gu.say("non-finite torsions")
    w = sy.CFG1.replace(L=16, n_chains=3)
    _, y = gu.protein(w)
    s0 = np.stack([sy.random_torsions(2 * w.L, 90 + c) for c in range(3)])
    bad = s0.copy()
    bad[2, 9] = np.nan
    with pytest.raises(amh.AmhError) as e:
        gu.context(w, y, s0=bad)
    assert e.value.status == amh.E_NUMERIC
    ctx = gu.context(w, y, s0=s0)
    V_ok, _, _ = ctx.energy(torch.from_numpy(s0[[0, 2]].copy()).to(gu.DEV))
    ctx.poll()
    s = s0.copy()
    s[1, 4] = np.inf
    V, _, _ = ctx.energy(torch.from_numpy(s).to(gu.DEV))
    V = V.cpu().numpy()
    assert np.isnan(V[1]) and np.array_equal(V[[0, 2]], V_ok.cpu().numpy())
    with pytest.raises(amh.AmhError) as e:
        ctx.poll()
    assert e.value.status == amh.E_NUMERIC
    ctx.close()


SMALL = sy.Workload("small", L=20, n_chains=6, total_sweeps=40, window_d=6, global_every=3,
                    sigma_deg=25.0, T0=2.0, T1=0.05, seed=0x5EED01, protein_seed=5, noise_seed=6,
                    anchor_every=3)


def _replay_all(w, y, tr, chains, t0=0, s0=None):
    reps = []
    for m, c in enumerate(chains):
        rc, rep, s_out = gu.replay_chain(w, y, tr, m, c, gu.extended(w) if s0 is None else s0[c], t0)
        assert rep["n_delta_fail"] == 0, rep
        assert rep["n_logic_fail"] == 0, rep
        assert rep["n_de_fail"] == 0, rep
        assert rep["n_anchor_fail"] == 0, rep
        assert rc == 0, rep
        reps.append((rep, s_out))
    return reps


@pytest.mark.parametrize("G,W", [(1, 4), (2, 4), (4, 4), (4, 8)])
def test_small_run_replays_and_is_layout_independent(G, W):
    gu.say("small run G", G, "W", W)
    _, y = gu.protein(SMALL)
    ctx = gu.context(SMALL, y, chains_per_group=G, waves_per_group=W)
    assert ctx.info()["chains_per_group"] == G
    chains = [0, 2, 3, 5]
    tr = gu.traced_run(ctx, chains, 39, chunk=13)
    reps = _replay_all(SMALL, y, tr, chains)
    for rep, _ in reps:
        assert rep["n_forks"] <= 2
    st = ctx.get_state()
    ctx.close()
    # identical trajectories whatever the workgroup layout
    key = (tr["dE"].tobytes(), tr["acc"].tobytes(), st["s"].cpu().numpy().tobytes())
    _LAYOUT.setdefault("ref", key)
    assert key == _LAYOUT["ref"]


_LAYOUT = {}

WIDE = sy.Workload("wide", L=160, n_chains=5, total_sweeps=6, window_d=10, global_every=2,
                   sigma_deg=12.0, T0=1.0, T1=0.2, seed=0x5EED02, protein_seed=8, noise_seed=9)


@pytest.mark.parametrize("G,W", [(1, 1), (1, 4), (2, 8), (4, 8)])
def test_wide_rectangles_use_every_wave(G, W):
    """At L=160 the pair rectangle of a global proposal is split over all eight
    wavefronts, so every wave's partial sums enter the decision."""
    gu.say("wide run G", G, "W", W)
    _, y = gu.protein(WIDE)
    ctx = gu.context(WIDE, y, chains_per_group=G, waves_per_group=W)
    chains = [0, 3, 4]
    tr = gu.traced_run(ctx, chains, 6)
    ctx.close()
    if (G, W) == (1, 1):
        _replay_all(WIDE, y, tr, chains)
    key = (tr["dE"].tobytes(), tr["acc"].tobytes())
    _WIDE.setdefault("ref", key)
    assert key == _WIDE["ref"]


_WIDE = {}


@pytest.mark.parametrize("G,W", [(1, 1), (1, 4), (4, 8)])
def test_compact_start_with_more_columns_than_threads(G, W):
    """From the folded reference conformation (long-range contacts everywhere), a
    global proposal with more moved columns than workgroup threads (L = 160 at 64
    or 256 threads) must still evaluate every column: replayed by the oracle."""
    gu.say("compact wide G", G, "W", W)
    s_ref, y = gu.protein(WIDE)
    s0 = np.tile(s_ref, (WIDE.n_chains, 1))
    ctx = gu.context(WIDE, y, s0=s0, chains_per_group=G, waves_per_group=W)
    chains = [0, 4]
    tr = gu.traced_run(ctx, chains, 4)
    ctx.close()
    for m, c in enumerate(chains):
        rc, rep, _ = gu.replay_chain(WIDE, y, tr, m, c, s_ref)
        assert rc == 0 and rep["n_de_fail"] == 0 and rep["n_forks"] <= 2, rep
    key = (tr["dE"].tobytes(), tr["acc"].tobytes())
    _COMPACT.setdefault("ref", key)
    assert key == _COMPACT["ref"]


_COMPACT = {}

LONGEST = sy.Workload("longest", L=1024, n_chains=2, total_sweeps=2, window_d=12, global_every=2,
                      sigma_deg=10.0, T0=1.0, T1=0.5, seed=0x5EED03, protein_seed=10, noise_seed=11)


def test_longest_chain_replays():
    """L = 1024, the longest chain the library takes (10-bit residue indices in the
    near-pair queue, 128 blocks of 8 residues), from the folded reference
    conformation: a localized and a global sweep of both chains replayed by the
    oracle."""
    gu.say("longest chain L=1024")
    s_ref, y = gu.protein(LONGEST)
    s0 = np.tile(s_ref, (LONGEST.n_chains, 1))
    ctx = gu.context(LONGEST, y, s0=s0)
    chains = [0, 1]
    tr = gu.traced_run(ctx, chains, 2)
    ctx.close()
    for m, c in enumerate(chains):
        gu.say("replay chain", c)
        rc, rep, _ = gu.replay_chain(LONGEST, y, tr, m, c, s_ref)
        assert rc == 0 and rep["n_de_fail"] == 0 and rep["n_logic_fail"] == 0 and rep["n_forks"] <= 2, rep


def test_resume_is_bit_exact():
    gu.say("resume")
    _, y = gu.protein(SMALL)
    a = gu.context(SMALL, y)
    a.sweep(25)
    sa = a.get_state()
    b = gu.context(SMALL, y)
    b.sweep(10)
    mid = b.get_state()
    torch.cuda.synchronize()
    b.close()
    c = gu.context(SMALL, y)
    c.set_state(mid)
    c.sweep(15)
    sc = c.get_state()
    torch.cuda.synchronize()
    for k in ("s", "s_best", "v", "counters", "atoms"):
        assert torch.equal(sa[k], sc[k]), k
    assert sa["t"] == sc["t"] == 25
    # resume exactly at an anchor without the coordinates (they are rebuilt there)
    d = gu.context(SMALL, y)
    d.sweep(9)
    at_anchor = d.get_state()
    e = gu.context(SMALL, y)
    e.set_state(at_anchor, with_atoms=False)
    d.sweep(16)
    e.sweep(16)
    assert torch.equal(d.get_state()["s"], e.get_state()["s"])
    for x in (a, c, d, e):
        x.close()


def test_determinism_and_best_state():
    gu.say("determinism")
    _, y = gu.protein(SMALL)
    r = []
    for _ in range(2):
        ctx = gu.context(SMALL, y)
        ctx.sweep(40)
        st = ctx.get_state()
        Vb, sb, _ = ctx.energy(which=1, want_s=True)
        r.append((st, Vb.cpu().numpy(), sb.cpu().numpy()))
        ctx.close()
    for k in ("s", "s_best", "v", "counters", "atoms"):
        assert torch.equal(r[0][0][k], r[1][0][k]), k
    st, Vb, sb = r[0]
    v = st["v"].cpu().numpy()
    assert np.all(v[:, 1] <= v[:, 0] + 1e-12)
    assert Vb == pytest.approx(v[:, 1], rel=1e-12)
    cfg = oracle.make_cfg(SMALL)
    y32 = y.astype(np.float32).astype(np.float64)
    for c in range(SMALL.n_chains):
        assert oracle.energy(cfg, y32, sb[c]) == pytest.approx(v[c, 1], rel=1e-9)
    cnt = st["counters"].cpu().numpy()
    assert np.all(cnt[:, 3] == 40 // 3)


@pytest.mark.parametrize("case", ["L2", "L3-window0", "window-covers-chain", "local-only", "global-only"])
def test_edge_cases_replay(case):
    gu.say("edge", case)
    w = {
        "L2": SMALL.replace(L=2, n_chains=3, window_d=2),
        "L3-window0": SMALL.replace(L=3, n_chains=2, window_d=0),
        "window-covers-chain": SMALL.replace(L=9, n_chains=5, window_d=18, global_every=0),
        "local-only": SMALL.replace(L=33, n_chains=4, window_d=4, global_every=0),
        "global-only": SMALL.replace(L=31, n_chains=4, global_every=1),
    }[case]
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    chains = list(range(min(4, w.n_chains)))
    tr = gu.traced_run(ctx, chains, 30)
    reps = _replay_all(w, y, tr, chains)
    for rep, _ in reps:
        assert rep["n_forks"] <= 2
    if case == "L3-window0":
        # a one-residue window judges nothing: every local proposal is accepted
        n = 2 * w.L
        acc = tr["acc"][0, :30 * n].reshape(30, n)
        local = [t for t in range(30) if (t + 1) % w.global_every != 0]
        assert np.all(acc[local] == 1)
    ctx.close()


def test_wait_bound_reports_a_device_error():
    """A one-poll bound on the pipelined localized sweeps' wait makes them give up;
    the launch still ends and amh_poll reports the failure (error path forced from
    the host; nothing hangs)."""
    from paper_2211_03193_amd import amh
    gu.say("wait bound")
    w = SMALL.replace(global_every=0, total_sweeps=20, anchor_every=10, window_d=12, L=40)
    _, y = gu.protein(w)
    ctx = gu.context(w, y, chains_per_group=1, waves_per_group=4)
    with pytest.raises(amh.AmhError) as e:
        ctx.set_wait_bound(0)
    assert e.value.status == amh.E_INVAL
    ctx.set_wait_bound(1)
    ctx.sweep(10)
    with pytest.raises(amh.AmhError) as e:
        ctx.poll()
    assert e.value.status == amh.E_DEVICE
    ctx.close()
    ok = gu.context(w, y, chains_per_group=1, waves_per_group=4)
    ok.sweep(10)
    ok.poll()
    ok.close()


def test_launch_shapes():
    """amh_sweep's launches at L = 300 with 1024 chains: an automatically shaped
    context runs its localized sweeps in workgroups of 4 chains and 12 wavefronts
    and its global sweeps in workgroups of 2 chains and 4 wavefronts (two per CU);
    an explicit shape is kept for both kinds of launch."""
    gu.say("launch shapes")
    w = sy.CFG2.replace(total_sweeps=20)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    info = ctx.info()
    assert (info["chains_per_group"], info["waves_per_group"]) == (4, 8)
    assert (info["local_chains_per_group"], info["local_waves_per_group"]) == (4, 12)
    assert (info["global_chains_per_group"], info["global_waves_per_group"]) == (2, 4)
    assert 2 * info["global_lds_bytes"] <= 160 * 1024
    ctx.sweep(10)
    a = ctx.get_state()
    ctx.close()
    ctx = gu.context(w, y, chains_per_group=4, waves_per_group=8)
    info = ctx.info()
    assert (info["global_chains_per_group"], info["global_waves_per_group"]) == (4, 8)
    ctx.sweep(10)
    b = ctx.get_state()
    ctx.close()
    # the same trajectories whatever the grouping of the global launches
    assert np.array_equal(a["s"].cpu().numpy(), b["s"].cpu().numpy())
    assert np.array_equal(a["v"].cpu().numpy(), b["v"].cpu().numpy())
