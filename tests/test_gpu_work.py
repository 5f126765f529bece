"""The global sweeps' executed-work counters (amh_set_work_counters), which the
benchmark's roofline divides by the launch time, against an independent count:
every proposal of every chain is traced, its trial conformation rebuilt on the host
by the oracle's NeRF, and the changed pairs i < p <= j inside the last knot counted.
The device compares float32 squared distances, so its near-pair count must lie
between the counts at d2far (1 - 1e-5) and d2far (1 + 1e-5); pair tests and surviving
tiles are bounded by the near pairs and by the whole rectangles."""
import numpy as np
import pytest
import torch

import bench
import oracle
import synthetic as sy

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402  (an import error fails the run)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("L", [40, 70])
def test_work_counters_match_the_traced_proposals(L):
    """Also the same counts for three launch shapes (the work does not depend on how
    the chains are grouped)."""
    C, n_sweeps = 3, 3
    w = sy.CFG1.replace(L=L, n_chains=C, global_every=1, anchor_every=0, total_sweeps=50,
                        protein_seed=L + 11, noise_seed=L + 12)
    s_ref, y = gu.protein(w)
    rng = np.random.default_rng(L)
    s0 = np.stack([s_ref + 0.25 * rng.standard_normal(2 * L) for _ in range(C)])
    counts = []
    for G, W in ((1, 4), (2, 4), (4, 8)):
        gu.say("work counters L", L, "shape", G, W)
        ctx = gu.context(w, y, s0=s0, chains_per_group=G, waves_per_group=W)
        work = torch.zeros(3, dtype=torch.int64, device=gu.DEV)
        ctx.set_work_counters(work)
        tr = gu.traced_run(ctx, list(range(C)), n_sweeps)
        ctx.set_work_counters(None)
        counts.append(tuple(int(v) for v in work.cpu().numpy()))
        ctx.close()
    assert counts[1] == counts[0] and counts[2] == counts[0]
    tiles, tests, near = counts[0]

    dfar = w.d_min + w.bin_w * (w.n_bins - 0.5)
    lo_cut, hi_cut = dfar * dfar * (1 - 1e-5), dfar * dfar * (1 + 1e-5)
    near_lo = near_hi = 0
    iu, ju = np.triu_indices(L, 1)
    for c in range(C):
        s = s0[c].copy()
        for m in range(n_sweeps * 2 * L):
            k = m % (2 * L)
            p = (k + 1) // 2
            trial = s.copy()
            trial[k] += tr["delta"][c, m]
            x = oracle.cb(trial)
            d2 = ((x[iu] - x[ju]) ** 2).sum(axis=1)
            changed = (iu < p) & (ju >= p)
            near_lo += int(np.count_nonzero(changed & (d2 < lo_cut)))
            near_hi += int(np.count_nonzero(changed & (d2 < hi_cut)))
            if tr["acc"][c, m]:
                s = trial
    gu.say("near", near, "bounds", near_lo, near_hi, "tests", tests, "tiles", tiles)
    assert near_lo <= near <= near_hi and near > 0
    rect = C * n_sweeps * (L ** 3 - L) // 3
    cand = C * n_sweeps * bench.schedule_work(L, 8, 10)["candidate_tiles"]
    assert near <= tests <= rect
    assert -(-near // 64) <= tiles <= cand and tests <= 64 * tiles
