"""Benchmark of the AMH hot path on one MI355X.

Workload: one synthetic protein of 300 residues (37-bin distogram, eps = 0.1),
1024 independent chains, localized window d = 12, a global sweep every 10
sweeps, sigma = 10 deg, T 1 -> 0.01 geometric over 5000 sweeps, extended-chain
start.  One step = one alternation cycle (9 localized + 1 global sweep) of all
chains = 10 * 600 * 1024 proposals.  Inputs are resident in HBM before timing.

Prints one JSON line with proposals/s, the roofline of the global-sweep kernel (the
dominant one; the localized-sweep kernel's beside it) and the oracle timed on the host
cores (CPU baseline leg).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthetic as sy  # noqa: E402

PEAK_FP32_NONPACKED = 256 * 64 * 2 * 2.4e9    # FLOP/s: 256 CUs x 64 lanes x FMA x 2.4 GHz
PEAK_FP32_PUBLISHED = 157.3e12                 # FLOP/s, MI355X vector FP32 (packed)
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "sweep_kernel_L300_1024chains_traffic.json")
# algorithmic operation counts of the executed work of a sweep launch (FP32-equivalent):
FLOPS_TEST = 9.0      # squared distance of a float32 pair and its comparison with the last knot
FLOPS_SPLINE = 20.0   # square root, knot interval and fraction, Catmull-Rom cubic of one stencil
FLOPS_ROTATE = 18.0   # float64 rotation of one moved C-beta about the bond and the difference
STENCIL_BYTES = 16    # one 4-tap float32 stencil gathered from the distogram table


def code_digest(paths) -> str:
    """sha256 over the given C++/HIP sources with comments and whitespace removed, so
    that a change of the code, not of its comments, changes the digest."""
    import hashlib
    import re
    h = hashlib.sha256()
    for p in paths:
        text = open(os.path.join(ROOT, p), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the two sweep kernels ({"local": B, "global": B}) from
    the committed counter record (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None
    once the kernel code differs from the code the counters were taken on."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        if code_digest(rec["sources"]) != rec["code_sha256"]:
            return None
        return {k: rec[k]["fetch_bytes_per_launch"] + rec[k]["write_bytes_per_launch"]
                for k in ("local", "global")}
    except (OSError, ValueError, KeyError, TypeError):
        return None


def host_cores() -> int:
    for k in ("OMP_NUM_THREADS",):
        if os.environ.get(k, "").isdigit():
            return int(os.environ[k])
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def pair_evals_per_cycle(L: int, d: int, cycle: int) -> tuple[int, int]:
    """Changed pairs evaluated per chain in one cycle: (global, local)."""
    glob = sum(p * (L - p) for p in [(k + 1) // 2 for k in range(2 * L)])
    h = d // 2
    loc = 0
    for k in range(2 * L):
        c = k // 2
        p = c + 1 if k % 2 else c
        lo, hi = max(0, c - h), min(L - 1, c + h)
        loc += max(0, p - lo) * max(0, hi - p + 1)
    return glob, loc * (cycle - 1)


def schedule_work(L: int, d: int, cycle: int) -> dict:
    """Work of one chain in one alternation cycle that the schedule fixes (no
    counting needed): localized changed pairs (two stencils each), candidate tiles
    of the global rectangle (8 x 8 residue blocks), transition pairs of the psi
    proposals and the anchor's pairs."""
    nb8 = (L + 7) // 8
    cand = 0
    for k in range(2 * L):
        p = (k + 1) // 2
        if p >= 1 and L - p >= 1:
            cand += (((p - 1) >> 3) + 1) * (nb8 - (p >> 3))
    _, loc = pair_evals_per_cycle(L, d, cycle)
    return {"local_pairs": loc, "candidate_tiles": cand, "transition_pairs": L * (L - 1),
            "anchor_pairs": L * (L - 1) // 2}


def executed_work(fixed: dict, counted: dict, chains: int) -> dict:
    """Executed work of one step, split by kernel: the localized-sweep launch (the
    schedule's localized pairs: two stencils and a rotation each) and the
    global-sweep launch (the schedule's candidate tiles, transition pairs and the
    anchor's pairs, plus the counted surviving tiles, pair tests and near pairs)."""
    loc = fixed["local_pairs"] * chains
    trans = fixed["transition_pairs"] * chains
    anch = fixed["anchor_pairs"] * chains
    cand = fixed["candidate_tiles"] * chains
    tests = counted["pair_tests"]
    near = counted["near_pairs"]
    st_l = 2 * loc
    st_g = near + trans + anch
    fl_l = FLOPS_TEST * 2 * loc + FLOPS_SPLINE * st_l + FLOPS_ROTATE * loc
    fl_g = FLOPS_TEST * (tests + cand + trans + anch) + FLOPS_SPLINE * st_g
    # L2 gathers: one per localized pair (its second stencil, at the proposed distance,
    # reads the same table row right after the first and mostly the same cache line),
    # one per stencil of the global sweep
    return {
        "local": {"local_pairs": loc, "stencils": st_l, "stencil_bytes": STENCIL_BYTES * st_l,
                  "l2_gather_bytes": STENCIL_BYTES * loc, "flops": fl_l},
        "global": {"candidate_tiles": cand, "surviving_tiles": counted["tiles"], "pair_tests": tests,
                   "near_pairs": near, "transition_pairs": trans, "anchor_pairs": anch, "stencils": st_g,
                   "stencil_bytes": STENCIL_BYTES * st_g, "l2_gather_bytes": STENCIL_BYTES * st_g, "flops": fl_g},
        "step": {"stencils": st_l + st_g, "stencil_bytes": STENCIL_BYTES * (st_l + st_g), "flops": fl_l + fl_g},
    }


def gpu_leg(w, steps, warmup, G=0, W=0, target=None, count_work=True):
    import torch
    from paper_2211_03193_amd import amh

    dev = torch.device("cuda:0")
    # input: reference conformation from the library's own geometry, distogram recipe
    s_ref = sy.reference_torsions(w.L, w.protein_seed)
    atoms = amh.conformation(torch.from_numpy(s_ref[None]).to(dev))[0].cpu().numpy()
    y = sy.distogram(sy.pair_distances(atoms[:, 3, :]), w.eps, w.noise_seed)
    yt = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(dev)
    ctx = amh.Context(amh.make_config(w, chains_per_group=G, waves_per_group=W), yt)
    V_ref = ctx.energy(torch.from_numpy(s_ref[None]).to(dev))[0].item()
    # the device records, per chain, the first anchor sweep at or below the target
    target_ref = 1.05 * V_ref
    ctx.set_target(target if target is not None else target_ref)
    info = ctx.info()
    cyc = w.global_every
    # a step is one cycle: its localized sweeps (one launch of the localized-sweep
    # kernel) and then its global sweeps (one launch of the global-sweep kernel), as
    # amh_sweep(cyc) issues them; events on the launch stream around each
    n_glob = w.n_global
    n_loc = cyc - n_glob
    stream = torch.cuda.current_stream()

    def events(n):
        return [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(n)]

    def run(evs):
        for e0, e1, e2 in evs:
            e0.record(stream)
            ctx.sweep(n_loc)
            e1.record(stream)
            ctx.sweep(n_glob)
            e2.record(stream)

    wev = events(warmup)
    run(wev)
    torch.cuda.synchronize()
    work = torch.zeros(3, dtype=torch.int64, device=dev)
    if count_work:
        ctx.set_work_counters(work)
    evs = events(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_work_counters(None)
    launch_ms = np.array([e0.elapsed_time(e2) for e0, e1, e2 in evs])
    local_ms = np.array([e0.elapsed_time(e1) for e0, e1, e2 in evs])
    global_ms = np.array([e1.elapsed_time(e2) for e0, e1, e2 in evs])
    warm_ms = np.array([e0.elapsed_time(e2) for e0, e1, e2 in wev])
    ctx.poll()
    st = ctx.get_state()
    v = st["v"].cpu().numpy()
    cnt = st["counters"].cpu().numpy()
    ctx.close()
    wk = work.cpu().numpy()
    return dict(wall=wall, launch_ms=launch_ms, local_ms=local_ms, global_ms=global_ms, warm_ms=warm_ms,
                info=info, V_ref=V_ref,
                target=target, target_ref=target_ref, v=v, counters=cnt,
                counted={"tiles": int(wk[0]), "pair_tests": int(wk[1]), "near_pairs": int(wk[2])})


def batch_leg(steps, warmup, n_proteins, tune_sweeps):
    """Ragged batch (lengths uniform on [50, 600], 256 chains each): one cycle of all
    proteins in batched launches against the same cycle as one plain launch per
    protein.  Both sides start from the same state and follow the same trajectories
    (bit for bit), so equal final energies are checked exactly."""
    import torch
    from paper_2211_03193_amd import amh

    dev = torch.device("cuda:0")
    ws = sy.batch_workloads(n=n_proteins)
    cyc = ws[0].global_every
    ys, vref = [], []
    for w in ws:
        s_ref = sy.reference_torsions(w.L, w.protein_seed)
        atoms = amh.conformation(torch.from_numpy(s_ref[None]).to(dev))[0].cpu().numpy()
        y = sy.distogram(sy.pair_distances(atoms[:, 3, :]), w.eps, w.noise_seed)
        ys.append(torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(dev))
    A = [amh.Context(amh.make_config(w), y) for w, y in zip(ws, ys)]
    B = [amh.Context(amh.make_config(w), y) for w, y in zip(ws, ys)]
    for w, y, a, b in zip(ws, ys, A, B):
        s_ref = torch.from_numpy(sy.reference_torsions(w.L, w.protein_seed)[None]).to(dev)
        v = a.energy(s_ref)[0].item()
        vref.append(v)
        a.set_target(1.05 * v)
        b.set_target(1.05 * v)
    batch = amh.Batch(A)
    plan, trial_ms = batch.tune(tune_sweeps)
    for b in B:                      # the tuning sweeps, as plain launches
        b.sweep(6 * tune_sweeps)
    for _ in range(warmup):
        batch.sweep(cyc)
        for b in B:
            b.sweep(cyc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.sweep(cyc)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(steps):
        for b in B:
            b.sweep(cyc)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = True
    best_a, best_b = [], []
    for a, b in zip(A, B):
        sa, sb = a.get_state(), b.get_state()
        same &= all(torch.equal(sa[k], sb[k]) for k in ("s", "s_best", "v", "counters"))
        best_a.append(sa["v"][:, 1].min().item())
        best_b.append(sb["v"][:, 1].min().item())
    info = batch.info()
    batch.close()
    props = sum(w.n_chains * 2 * w.L for w in ws) * cyc * steps
    pairs = sum(w.n_chains * sum(pair_evals_per_cycle(w.L, w.window_d, cyc)) for w in ws) * steps
    for c in A + B:
        c.close()
    return {
        "metric": "proposals/s", "value": props / t_batch, "unit": "proposals/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": t_batch * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch-{len(ws)}proteins-L50-600-256chains",
                   "lengths": [w.L for w in ws], "chains_per_protein": ws[0].n_chains,
                   "window_d": ws[0].window_d, "global_every": cyc, "sweeps_per_step": cyc,
                   "tune_sweeps_per_plan": tune_sweeps, "plan": plan, "plan_trial_ms": trial_ms,
                   "launches_per_step": info["launches"], "workgroups": info["workgroups"]},
        "pair_evals_per_s": pairs / t_batch,
        "plain_launches": {"value": props / t_plain, "unit": "proposals/s",
                           "ms_per_step": t_plain * 1e3 / steps},
        "speedup_vs_plain": t_plain / t_batch,
        "same_trajectories_as_plain": bool(same),
        "best_energy_equal": best_a == best_b,
    }


def cpu_serve_targets(jobs, runs, cores):
    """CPU baseline of the serving workload (Sec. 3, Fig. 4E protocol): for every job,
    `runs` oracle runs of the job's own schedule and sweep budget (one chain each,
    from the extended chain); the mean of their lowest energies is the target that
    job's device chains must reach.  Jobs run in parallel over the host cores."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    def one(job):
        w, y32 = job
        ch = oracle.Chains(oracle.make_cfg(w), np.asarray(y32, dtype=np.float64),
                           np.full((runs, 2 * w.L), math.pi), chain_ids=np.arange(runs, dtype=np.uint32))
        t0 = time.perf_counter()
        ch.run(w.total_sweeps, mode=1, threads=runs)
        return float(np.mean(ch.v[:, 1])), (time.perf_counter() - t0)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=max(1, cores // runs)) as ex:
        res = list(ex.map(one, jobs))
    return [r[0] for r in res], [r[1] for r in res], time.perf_counter() - t0


def serve_leg(n_jobs, rate, sweeps, budget_gib, sweeps_per_round, plan, target_runs=3):
    """Poisson arrivals of folding jobs (L uniform on [50, 800], 64-512 chains, their
    own Philox keys), served by continuous batching and by a one-job-at-a-time queue;
    every job's best states must agree between the two.  A job ends when a chain
    reaches its target, the mean lowest energy of `target_runs` oracle runs of the
    same job on the host (the paper's time-to-solution protocol), or after its last
    sweep; 1.05 V(s_ref) is reported beside it."""
    import torch
    from paper_2211_03193_amd import amh, serving

    dev = torch.device("cuda:0")
    seed = 0x414D4805
    Ls = sy.batch_lengths(n_jobs, 50, 800, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    chains = rng.choice([64, 128, 256, 512], size=n_jobs)
    arrivals = sy.poisson_arrivals(rate, n_jobs, seed + 2)
    jobs, wl, vrefs = [], [], []
    for i, (L, C) in enumerate(zip(Ls, chains)):
        w = sy.Workload(f"job{i:02d}-L{int(L)}", L=int(L), n_chains=int(C), total_sweeps=sweeps,
                        window_d=12, seed=(seed << 16) + i, protein_seed=3000 + i, noise_seed=4000 + i)
        s_ref = sy.reference_torsions(w.L, w.protein_seed)
        atoms = amh.conformation(torch.from_numpy(s_ref[None]).to(dev))[0].cpu().numpy()
        y = np.ascontiguousarray(sy.distogram(sy.pair_distances(atoms[:, 3, :]), w.eps, w.noise_seed),
                                 dtype=np.float32)
        probe = amh.Context(amh.make_config(w.replace(n_chains=1)), torch.from_numpy(y).to(dev))
        v_ref = probe.energy(torch.from_numpy(s_ref[None]).to(dev))[0].item()
        probe.close()
        wl.append((w, y))
        vrefs.append(v_ref)
    torch.cuda.synchronize()
    cpu_targets, cpu_secs, cpu_wall = cpu_serve_targets(wl, target_runs, host_cores())
    for (w, y), tg in zip(wl, cpu_targets):
        jobs.append((amh.make_config(w), y, tg))
    out = {}
    results = {}
    # round_pairs: a job advances sweeps_per_round * clamp(5e10 / (its pair evaluations per
    # round), 1, 64) sweeps per round, so small jobs keep pace with large ones
    # continuous: the server's default, every admitted job advances sweeps_per_round per
    # round; continuous_per_job_counts: a job's sweeps per round scale with its size
    # (round_pairs); fifo: one job at a time
    modes = (("continuous", 1 << 30, 0), ("continuous_per_job_counts", 1 << 30, 50_000_000_000),
             ("fifo", 1, 0))
    for name, max_active, rp in modes:
        srv = amh.Server(int(budget_gib * 2**30), max_active=max_active,
                         sweeps_per_round=sweeps_per_round, plan=plan, round_pairs=rp)
        st = serving.run_trace(srv, jobs, arrivals)
        out[name] = serving.summarise(st)
        done = [s for s in st if s["state"] == 2]
        out[name]["jobs_per_s"] = len(done) / out[name]["makespan_s"] if done else 0.0
        props = sum(s["sweeps"] * jobs[i][0].n_chains * 2 * jobs[i][0].L for i, s in enumerate(st))
        out[name]["proposals_per_s"] = props / out[name]["makespan_s"] if done else 0.0
        results[name] = [srv.job(s["id"], want_state=True) if s["state"] == 2 else None for s in st]
        out[name]["reached_1.05_V_ref"] = int(sum(
            1 for r, v in zip(results[name], vrefs) if r is not None and r["v"][:, 1].min() <= 1.05 * v))
        srv.close()
    same = all(a is not None and b is not None and np.array_equal(a["s_best"], b["s_best"])
               and np.array_equal(a["v"], b["v"])
               for a, b in zip(results["continuous"], results["fifo"]))
    per_job = out["continuous_per_job_counts"]
    c, f = out["continuous"], out["fifo"]
    return {
        "metric": "p99 time-to-target", "value": c["p99_time_to_target_s"], "unit": "s",
        "n_gpus": 1, "steps": n_jobs, "warmup": 0, "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serve-{n_jobs}jobs-poisson{rate:g}-L50-800-64to512chains",
                   "sweeps_per_job": sweeps, "sweeps_per_round": sweeps_per_round, "plan": plan,
                   "hbm_budget_gib": budget_gib,
                   "target": f"mean lowest energy of {target_runs} oracle runs of the job (same "
                             "schedule and sweep budget, one chain each)",
                   "round_pairs": {"continuous": 0, "continuous_per_job_counts": 5e10, "fifo": 0},
                   "time_to_target": "submit to the first anchor with a chain at or below the target"},
        "continuous": c, "fifo": f, "continuous_per_job_counts": per_job,
        "p99_time_to_target_speedup_vs_fifo": (f["p99_time_to_target_s"] / c["p99_time_to_target_s"]
                                               if c["p99_time_to_target_s"] and f["p99_time_to_target_s"]
                                               else None),
        "p99_time_to_done_speedup_vs_fifo": (f["p99_time_to_done_s"] / c["p99_time_to_done_s"]
                                             if c["p99_time_to_done_s"] else None),
        "same_results_alone_and_in_mix": bool(same),
        "cpu_baseline": {"kind": "oracle", "cores": host_cores(), "runs_per_job": target_runs,
                         "seconds_per_job_run_mean": float(np.mean(cpu_secs)),
                         "wall_s": cpu_wall, "targets": cpu_targets, "V_ref": vrefs},
    }


def variants_leg(samples, chains):
    """The paper's schemes (Sec. 3, Fig. 3 columns 1-5, and the Sec. 2.3 restart
    procedure) on one synthetic 100-residue protein, `samples` samples each (a
    sweep for MH schemes, an iteration for L-BFGS), `chains` independent chains;
    then the beta sweep of Fig. 5 and the chain-count study of Fig. 4C."""
    import torch
    from paper_2211_03193_amd import amh, hybrid, variants

    dev = torch.device("cuda:0")
    # Alt-MH as benchmarked in Sec. 3: cycles of 20 localized (d = 5) and 80 global
    # sweeps, width 10 -> 4 degrees; every scheme anneals 0.1 < beta < 1
    w = sy.Workload("variants-L100", L=100, n_chains=chains, total_sweeps=samples, window_d=5,
                    global_every=100, n_global=80, sigma_deg=10.0, sigma_end_deg=4.0,
                    T0=10.0, T1=1.0, seed=0x414D4806, protein_seed=6, noise_seed=106)
    s_ref = sy.reference_torsions(w.L, w.protein_seed)
    atoms = amh.conformation(torch.from_numpy(s_ref[None]).to(dev))[0].cpu().numpy()
    y = torch.from_numpy(np.ascontiguousarray(
        sy.distogram(sy.pair_distances(atoms[:, 3, :]), w.eps, w.noise_seed), dtype=np.float32)).to(dev)
    probe = amh.Context(amh.make_config(w.replace(n_chains=1)), y)
    V_ref = probe.energy(torch.from_numpy(s_ref[None]).to(dev))[0].item()
    probe.close()
    res, secs = {}, {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res[name] = fn()
        torch.cuda.synchronize()
        secs[name] = time.perf_counter() - t0

    mh_w = w.replace(sigma_end_deg=0.0)
    timed("1_mh_annealed", lambda: variants.mh_noisy_restarts(mh_w, y, every=samples + 1))
    timed("2_mh_noisy_restarts", lambda: variants.mh_noisy_restarts(mh_w, y, every=100))

    def alt():
        ctx = amh.Context(amh.make_config(w), y)
        ctx.sweep(samples)
        v = ctx.energy(which=1)[0].min().item()
        ctx.close()
        return {"best": v}
    timed("3_alt_mh", alt)

    def col5():
        # its localized-MH phases (20 sweeps per batch of 100 samples) anneal over their own run
        ctx = amh.Context(amh.make_config(w.replace(global_every=0, n_global=1,
                                                    total_sweeps=samples // 100 * 20)), y)
        hybrid.lbfgs_with_localized_mh(ctx, cycles=samples // 100, lbfgs_iters=80, mh_sweeps=20,
                                       final_lbfgs=False)
        v = ctx.energy(which=1)[0].min().item()
        ctx.close()
        return {"best": v}
    timed("5_lbfgs_localized_mh", col5)
    timed("alt_mh_10_restarts", lambda: variants.alt_mh_restarts(w.replace(total_sweeps=samples // 10), y, runs=10))
    props82k = 82000 // (2 * w.L)
    timed("beta_sweep", lambda: variants.beta_sweep(w.replace(total_sweeps=props82k, sigma_end_deg=0.0), y,
                                                     betas=[0.01, 0.1, 1.0, 10.0, 100.0], runs=25))
    timed("chain_counts", lambda: variants.chain_count_study(w.replace(total_sweeps=props82k), y,
                                                              counts=(10, 1000)))
    best = {k: v["best"] for k, v in res.items() if "best" in v}
    return {
        "metric": "lowest energy", "value": best["3_alt_mh"], "unit": "nats", "n_gpus": 1,
        "steps": samples, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "variants-L100", "chains": chains, "samples": samples,
                   "window_d": 5, "cycle": [20, 80], "sigma_deg": [10.0, 4.0], "beta": [0.1, 1.0],
                   "beta_sweep_proposals_per_run": props82k * 2 * w.L},
        "V_ref": V_ref, "best": best, "seconds": secs,
        "alt_mh_gain_vs_mh": (best["1_mh_annealed"] - best["3_alt_mh"]) / best["1_mh_annealed"],
        "alt_mh_gain_vs_noisy_restarts": (best["2_mh_noisy_restarts"] - best["3_alt_mh"]) / best["2_mh_noisy_restarts"],
        "restarts": res["alt_mh_10_restarts"]["runs"], "beta_sweep": res["beta_sweep"],
        "chain_counts": res["chain_counts"]["counts"],
    }


def tts_leg(cpu_runs, chains):
    """Time to solution as in Sec. 3 (Fig. 4E): the oracle runs one chain for 1e5
    proposals `cpu_runs` times (one host core each); the target is the mean of those
    runs' lowest energies; the GPU runs `chains` chains of the same schedule until one
    chain's anchored energy reaches the target.  Synthetic 100-residue protein."""
    import torch
    import oracle
    from paper_2211_03193_amd import amh

    dev = torch.device("cuda:0")
    L = 100
    S = 100000 // (2 * L)          # 1e5 proposals
    w = sy.Workload("tts-L100", L=L, n_chains=1, total_sweeps=S, window_d=12, sigma_deg=10.0,
                    sigma_end_deg=4.0, T0=10.0, T1=1.0, seed=0x414D4807, protein_seed=6,
                    noise_seed=106)
    s_ref = sy.reference_torsions(w.L, w.protein_seed)
    atoms = amh.conformation(torch.from_numpy(s_ref[None]).to(dev))[0].cpu().numpy()
    y64 = sy.distogram(sy.pair_distances(atoms[:, 3, :]), w.eps, w.noise_seed)
    y32 = np.ascontiguousarray(y64, dtype=np.float32)
    cfg = oracle.make_cfg(w)
    cpu_t, cpu_min = [], []
    for r in range(cpu_runs):
        ch = oracle.Chains(cfg, y32.astype(np.float64), np.full((1, 2 * L), math.pi),
                           chain_ids=np.array([r], dtype=np.uint32))
        t0 = time.perf_counter()
        ch.run(S, mode=1, threads=1)
        cpu_t.append(time.perf_counter() - t0)
        cpu_min.append(float(ch.v[0, 1]))
    target = float(np.mean(cpu_min))
    yt = torch.from_numpy(y32).to(dev)
    # warm-up on a throwaway context of the same shape (loads the kernels' code
    # objects), so that the timed run holds the sampling only, like the CPU runs
    warm = amh.Context(amh.make_config(w.replace(n_chains=chains)), yt)
    warm.sweep(w.anchor_period)
    warm.get_state()
    torch.cuda.synchronize()
    warm.close()
    ctx = amh.Context(amh.make_config(w.replace(n_chains=chains)), yt)
    ctx.set_target(target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reached_at, done = None, 0
    while done < S:
        ctx.sweep(w.anchor_period)
        done += w.anchor_period
        cnt = ctx.get_state()["counters"][:, 2]
        if bool((cnt >= 0).any()):
            reached_at = done
            break
    t_polled = time.perf_counter() - t0
    ctx.close()
    # the same run again without the host looking in every cycle: the device records
    # the sweep at which a chain reached the target, so one launch of that many sweeps
    # and one read of the counters at the end give the same trajectory and the answer
    t_gpu = None
    if reached_at:
        ctx = amh.Context(amh.make_config(w.replace(n_chains=chains)), yt)
        ctx.set_target(target)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.sweep(reached_at)
        ok = bool((ctx.get_state()["counters"][:, 2] >= 0).any())
        t_gpu = time.perf_counter() - t0
        ctx.close()
        assert ok, "the repeated run must reach the target at the same sweep"
    return {
        "metric": "time-to-target-energy speedup", "value": (float(np.mean(cpu_t)) / t_gpu
                                                            if reached_at else None),
        "unit": "x", "n_gpus": 1, "steps": S, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tts-L100", "proposals_per_cpu_run": S * 2 * L, "cpu_runs": cpu_runs,
                   "gpu_chains": chains, "window_d": 12, "global_every": 10,
                   "sigma_deg": [10.0, 4.0], "beta": [0.1, 1.0]},
        "target": target, "cpu_seconds_mean": float(np.mean(cpu_t)), "cpu_min_energies": cpu_min,
        "gpu_seconds": t_gpu, "gpu_seconds_polled_every_cycle": t_polled,
        "gpu_sweeps_to_target": reached_at,
        "note": "paper: 7.5x to 26.5x (P100 GPU vs an Intel i3-10100 core, CASP proteins); "
                "here an MI355X against one core of the host running the float64 oracle",
    }


# float64 operations of one pair of the gradient's force pass: distance (3 sub, 3 mul,
# 2 add, sqrt), spline value and derivative (~24), force and torque accumulation (~15)
FLOPS_GRAD_PAIR = 48.0


def hybrid_leg(cycles=2, lbfgs_iters=200, amh_sweeps=500, chains=512, L=400):
    """Differentiation + hybrid: L-BFGS phases (amh_minimize, the adjoint gradient in
    every line-search trial) interleaved with AMH phases on the same chains, against
    plain AMH over the same sweeps.  Synthetic 400-residue protein, 512 chains.  The
    time-to-target is the time the hybrid needs to reach plain AMH's final lowest
    energy.  The gradient kernel's force pass is also timed alone for its roofline."""
    import torch
    from paper_2211_03193_amd import amh, hybrid

    dev = torch.device("cuda:0")
    w = sy.Workload("hybrid-L400", L=L, n_chains=chains, total_sweeps=cycles * amh_sweeps, window_d=12,
                    global_every=10, sigma_deg=10.0, T0=1.0, T1=0.01, seed=0x414D4804,
                    protein_seed=4, noise_seed=104)
    s_ref = sy.reference_torsions(w.L, w.protein_seed)
    atoms = amh.conformation(torch.from_numpy(s_ref[None]).to(dev))[0].cpu().numpy()
    y = torch.from_numpy(np.ascontiguousarray(
        sy.distogram(sy.pair_distances(atoms[:, 3, :]), w.eps, w.noise_seed), dtype=np.float32)).to(dev)
    st = torch.cuda.current_stream()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(st)
        return e

    # plain AMH over the whole schedule
    plain = amh.Context(amh.make_config(w), y)
    V_ref = plain.energy(torch.from_numpy(s_ref[None]).to(dev))[0].item()
    e0 = ev()
    plain.sweep(w.total_sweeps)
    e1 = ev()
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) * 1e-3
    best_plain = plain.energy(which=1)[0].min().item()
    plain.close()
    # hybrid: AMH phase, then L-BFGS phase, repeated
    ctx = amh.Context(amh.make_config(w), y)
    opts = amh.lbfgs_opts(n_iter=lbfgs_iters)
    phases, t_total, t_target = [], 0.0, None
    for c in range(cycles):
        for kind in ("amh", "lbfgs"):
            e0 = ev()
            if kind == "amh":
                ctx.sweep(amh_sweeps)
            else:
                out = hybrid.lbfgs_with_localized_mh(ctx, cycles=1, lbfgs_iters=lbfgs_iters, mh_sweeps=0,
                                                     opts=opts, final_lbfgs=False)[0]
            e1 = ev()
            torch.cuda.synchronize()
            dt = e0.elapsed_time(e1) * 1e-3
            t_total += dt
            vb = ctx.energy(which=1)[0]
            rec = {"cycle": c, "phase": kind, "seconds": dt, "best_min": vb.min().item(),
                   "best_median": vb.median().item()}
            if kind == "lbfgs":
                rec["iterations_mean"] = out["iters"].double().mean().item()
                rec["status_counts"] = {str(k): int((out["status"] == k).sum().item()) for k in (0, 1, 2)}
            else:
                rec["proposals_per_s"] = chains * amh_sweeps * 2 * L / dt
            phases.append(rec)
            if t_target is None and rec["best_min"] <= best_plain:
                t_target = t_total
    best_hybrid = ctx.energy(which=1)[0].min().item()
    # the adjoint gradient alone: V and dV/ds of the 512 current conformations
    s_now = ctx.get_state()["s"].contiguous()
    ctx.grad(s_now)
    reps = 20
    e0 = ev()
    for _ in range(reps):
        ctx.grad(s_now)
    e1 = ev()
    torch.cuda.synchronize()
    g_s = e0.elapsed_time(e1) * 1e-3 / reps
    ctx.close()
    pairs = chains * L * (L - 1) // 2
    achieved = FLOPS_GRAD_PAIR * pairs / g_s
    return {
        "metric": "time-to-target-energy vs plain AMH", "value": (t_plain / t_target) if t_target else None,
        "unit": "x", "n_gpus": 1, "steps": cycles, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hybrid-L{L}-{chains}chains", "cycles": cycles, "amh_sweeps": amh_sweeps,
                   "lbfgs_iterations": lbfgs_iters, "window_d": 12, "global_every": 10,
                   "sigma_deg": 10.0, "T": [1.0, 0.01], "lbfgs": {"m": opts.m, "nonmonotone": opts.nonmonotone,
                                                                "c1": opts.c1, "max_ls": opts.max_ls},
                   "orientation_terms": "not built (the paper does not define them)"},
        "target": best_plain, "target_kind": "plain AMH's lowest energy after the same sweeps",
        "V_ref": V_ref, "plain_seconds": t_plain, "hybrid_seconds": t_total,
        "hybrid_seconds_to_target": t_target, "best_plain": best_plain, "best_hybrid": best_hybrid,
        "phases": phases,
        "gradient": {"conformations": chains, "ms_per_call": g_s * 1e3, "pairs_per_call": pairs,
                     "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": 78.6432,
                                  "unit": "TFLOP/s (float64)", "frac": achieved / 78.6432e12,
                                  "flops_per_pair": FLOPS_GRAD_PAIR}},
    }


def cpu_leg(w, cores, sweeps, one_core_sweeps=200, target_runs=10, target_proposals=100000):
    """The float64 oracle on the host: (a) all `cores` threads, two chains each, for
    `sweeps` sweeps of the workload from the extended chain; (b) one thread, two
    chains, `one_core_sweeps` sweeps; (c) the paper's time-to-solution target (Sec. 3,
    Fig. 4E): `target_runs` runs of `target_proposals` proposals each (the workload's
    schedule compressed to that many sweeps), whose mean lowest energy is the target
    the device chains must reach."""
    import oracle
    from oracle import build as obuild
    s_ref = sy.reference_torsions(w.L, w.protein_seed)
    y = sy.distogram(sy.pair_distances(oracle.cb(s_ref)), w.eps, w.noise_seed)
    y32 = np.asarray(y, dtype=np.float32).astype(np.float64)
    cfg = oracle.make_cfg(w)

    def rate(n_chains, n_sweeps, threads):
        ch = oracle.Chains(cfg, y32, np.full((n_chains, 2 * w.L), math.pi),
                           chain_ids=np.arange(n_chains, dtype=np.uint32))
        t0 = time.perf_counter()
        ch.run(n_sweeps, mode=1, threads=threads)
        return n_chains * n_sweeps * 2 * w.L / (time.perf_counter() - t0), time.perf_counter() - t0

    flags = " ".join(obuild.FLAGS)
    v_all, t_all = rate(2 * cores, sweeps, cores)
    v_one, t_one = rate(2, one_core_sweeps, 1)
    S = -(-target_proposals // (2 * w.L))
    wt = w.replace(total_sweeps=S)
    ch = oracle.Chains(oracle.make_cfg(wt), y32, np.full((target_runs, 2 * w.L), math.pi),
                       chain_ids=np.arange(target_runs, dtype=np.uint32))
    t0 = time.perf_counter()
    ch.run(S, mode=1, threads=min(cores, target_runs))
    t_target = time.perf_counter() - t0
    lows = [float(x) for x in ch.v[:, 1]]
    return dict(value=v_all, unit="proposals/s", cores=cores, kind="oracle",
                sample=f"{2 * cores} chains x {sweeps} sweeps ({sweeps // w.global_every} alternation "
                       f"cycles) of the same workload from the extended chain, incremental FP64 "
                       f"oracle, OpenMP over chains; {t_all:.1f} s wall; gcc {flags}",
                one_core={"value": v_one, "unit": "proposals/s", "cores": 1,
                          "sample": f"2 chains x {one_core_sweeps} sweeps, one thread; {t_one:.1f} s wall"},
                target_runs={"runs": target_runs, "proposals_per_run": S * 2 * w.L, "sweeps": S,
                             "lowest_energies": lows, "mean_lowest": float(np.mean(lows)),
                             "seconds_per_run_one_core": t_target * min(cores, target_runs) / target_runs})


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=495)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--chains", type=int, default=0,
                    help="chains of the single-protein workload (default 1024; 128 is one GPU's "
                         "share when 1024 chains are split over 8 GPUs)")
    ap.add_argument("--chains-per-group", type=int, default=0)
    ap.add_argument("--waves-per-group", type=int, default=0)
    ap.add_argument("--cpu-sweeps", type=int, default=800,
                    help="sweeps of the oracle CPU-baseline sample (2 chains per core)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU-baseline leg")
    ap.add_argument("--no-yardsticks", action="store_true",
                    help="skip the achievable-bandwidth yardsticks of the roofline")
    ap.add_argument("--workload", choices=["single", "batch", "serve", "variants", "tts", "hybrid"],
                    default="single",
                    help="single: one L=300 protein, 1024 chains (default); batch: 64 proteins "
                         "of lengths 50-600, 256 chains each, batched vs plain launches; serve: "
                         "Poisson arrivals of jobs, continuous batching vs one job at a time")
    ap.add_argument("--jobs", type=int, default=40, help="jobs in the serve workload")
    ap.add_argument("--rate", type=float, default=20.0, help="mean arrivals per second (serve)")
    ap.add_argument("--job-sweeps", type=int, default=100, help="sweeps per job at most (serve)")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="device-memory budget (serve)")
    ap.add_argument("--samples", type=int, default=10000, help="samples per scheme (variants)")
    ap.add_argument("--variant-chains", type=int, default=64, help="chains per scheme (variants)")
    ap.add_argument("--proteins", type=int, default=64, help="proteins in the batch workload")
    ap.add_argument("--tune-sweeps", type=int, default=10, help="sweeps per autotuner trial")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer (reference kernel for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy * 2**18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); chains shard across "
              "GPUs with no per-step communication, see the design notes.", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.workload in ("batch", "serve", "variants", "tts", "hybrid"):
        if args.workload == "tts":
            out = tts_leg(10, 1024)
        elif args.workload == "hybrid":
            out = hybrid_leg()
        elif args.workload == "batch":
            out = batch_leg(args.steps, args.warmup, args.proteins, args.tune_sweeps)
        elif args.workload == "serve":
            out = serve_leg(args.jobs, args.rate, args.job_sweeps, args.budget_gib, 10, 3)
        else:
            out = variants_leg(args.samples, args.variant_chains)
        if rank == 0:
            print(json.dumps(out), flush=True)
        return
    w = sy.CFG2
    if args.chains:
        w = w.replace(n_chains=args.chains, name=f"single-L300-{args.chains}chains")
    cyc = w.global_every
    if (args.warmup + args.steps) * cyc > w.total_sweeps:
        sys.exit(f"warmup + steps must fit the {w.total_sweeps}-sweep schedule "
                 f"({w.total_sweeps // cyc} steps)")
    cpu = None
    if rank == 0 and not args.no_cpu:
        cpu = cpu_leg(w, host_cores(), args.cpu_sweeps)
    target = cpu["target_runs"]["mean_lowest"] if cpu else None
    yard = None
    if not args.no_yardsticks:
        from paper_2211_03193_amd import amh as _amh
        yard = _amh.yardsticks()
    r = gpu_leg(w, args.steps, args.warmup, args.chains_per_group, args.waves_per_group, target=target)
    props_step = w.n_chains * cyc * 2 * w.L
    ms_step = r["wall"] * 1e3 / args.steps
    value = props_step * args.steps / r["wall"]
    glob, loc = pair_evals_per_cycle(w.L, w.window_d, cyc)
    dense_pairs = (glob + loc) * w.n_chains
    # rooflines on the work each kernel executes per launch (a step = one launch of the
    # localized-sweep kernel and one of the global-sweep kernel): the schedule's fixed
    # part plus the counted global-sweep part, averaged over the timed steps, over the
    # kernel's average launch duration (HIP events on the launch stream)
    per_launch = {k: v / args.steps for k, v in r["counted"].items()}
    ex = executed_work(schedule_work(w.L, w.window_d, cyc), per_launch, w.n_chains)
    glob_s = float(np.mean(r["global_ms"])) * 1e-3
    loc_s = float(np.mean(r["local_ms"])) * 1e-3
    step_s = float(np.mean(r["launch_ms"])) * 1e-3
    Gg, Gl = r["info"]["global_chains_per_group"], r["info"]["local_chains_per_group"]
    l2y = yard["l2_gather_16B"]["GB_per_s"] * 1e9 if yard else None

    def roof(work, secs, kernel, traffic):
        a = work["flops"] / secs
        gb = work["l2_gather_bytes"] / secs
        return {"bound": "alu", "achieved": a / 1e12, "peak": PEAK_FP32_NONPACKED / 1e12, "unit": "TFLOP/s",
                "frac": a / PEAK_FP32_NONPACKED, "traffic": traffic, "traffic_unit": "bytes per launch (HBM)",
                "kernel": kernel, "avg_launch_ms": secs * 1e3,
                "work": "executed per launch (fixed by the schedule, plus counted in the kernel)",
                "executed_per_launch": work,
                "flops_per": {"pair_test": FLOPS_TEST, "stencil_spline": FLOPS_SPLINE,
                              "local_rotation": FLOPS_ROTATE},
                "frac_of_published_fp32": a / PEAK_FP32_PUBLISHED,
                "gather": {"achieved_GB_per_s": gb / 1e9, "yardstick": "l2_gather_16B",
                           "yardstick_GB_per_s": l2y / 1e9 if l2y else None,
                           "frac": gb / l2y if l2y else None}}

    traffic = measured_traffic() if w.name == sy.CFG2.name else None
    roof_g = roof(ex["global"], glob_s, f"sweep_kernel<{Gg}, 2> (global sweeps)",
                  traffic.get("global") if traffic else None)
    roof_g["dense_equivalent"] = {"pairs_per_launch": glob * w.n_chains,
                                  "note": "every changed pair of the rectangle counted, culled or not; "
                                          "not executed work"}
    roof_l = roof(ex["local"], loc_s, f"sweep_kernel<{Gl}, 1> (localized sweeps)",
                  traffic.get("local") if traffic else None)
    a_step = ex["step"]["flops"] / step_s
    cnt = r["counters"]
    ttt = cnt[:, 2]
    reached = ttt[ttt >= 0]
    all_ms = np.concatenate([r["warm_ms"], r["launch_ms"]])
    first = int(reached.min()) if reached.size else None
    out = {
        "metric": "proposals/s", "value": value, "unit": "proposals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "L": w.L, "chains": w.n_chains, "window_d": w.window_d,
                   "global_every": cyc, "sigma_deg": w.sigma_deg, "T": [w.T0, w.T1],
                   "total_sweeps": w.total_sweeps, "sweeps_per_step": cyc,
                   "seed": hex(w.seed), "protein_seed": w.protein_seed,
                   "noise_seed": w.noise_seed, "eps": w.eps, "accum_dtype": "f64",
                   "coord_dtype": "f64", "launch": r["info"]},
        "pair_evals_per_s": dense_pairs * args.steps / r["wall"],
        "roofline": roof_g,
        "roofline_local": roof_l,
        "step_work": {"flops": ex["step"]["flops"], "stencil_bytes": ex["step"]["stencil_bytes"],
                      "avg_step_ms": step_s * 1e3, "achieved_TFLOP_per_s": a_step / 1e12,
                      "frac": a_step / PEAK_FP32_NONPACKED},
        "yardsticks": yard,
        "energy": {"V_ref": r["V_ref"], "target_1.05_V_ref": r["target_ref"],
                   "best_min": float(r["v"][:, 1].min()), "best_median": float(np.median(r["v"][:, 1])),
                   "chains_reaching_1.05_V_ref": int((r["v"][:, 1] <= r["target_ref"]).sum())},
    }
    if target is not None:
        step = -(-first // cyc) if first is not None else None
        out["time_to_target"] = {
            "target": target, "target_kind": "mean lowest energy of the oracle runs (cpu_baseline)",
            "chains_reaching": int(reached.size), "first_sweep": first,
            "gpu_seconds": float(all_ms[:step].sum()) * 1e-3 if step else None,
            "oracle_seconds_per_run_one_core": cpu["target_runs"]["seconds_per_run_one_core"],
            "speedup_vs_one_core_run": (cpu["target_runs"]["seconds_per_run_one_core"]
                                        / (float(all_ms[:step].sum()) * 1e-3)) if step else None}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
