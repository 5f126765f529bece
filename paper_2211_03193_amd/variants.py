"""The paper's run schedules built from the library's device calls.

Host code only: each function decides which contexts to create and in what
order to call amh_sweep / amh_batch_sweep / amh_perturb / amh_energy; every
proposal, energy and restart runs on the device.  Energies are in nats.

* ``alt_mh_restarts`` -- Alt-MH with the proposal width reduced from 10 to 4
  degrees over each run, repeated from the best state found so far, with the
  width range falling to 10/m -> 1/m degrees after the m-th run without
  improvement (Sec. 2.3);
* ``mh_noisy_restarts`` -- plain MH (every sweep global) annealed over
  0.1 < beta < 1 with a uniform [-10, 10] degree kick to every torsion every 100
  sweeps (the second scheme of Sec. 3);
* ``beta_sweep`` -- Alt-MH and plain MH at fixed beta over a range of beta, many
  independent runs each (Fig. 5);
* ``chain_count_study`` -- the best energy found by few and by many chains
  (Fig. 4C).

The fourth scheme of Sec. 3, L-BFGS with noisy restarts, is one of the paper's
comparison systems and is not built; the fifth, L-BFGS interleaved with
localized MH, is ``hybrid.lbfgs_with_localized_mh``.
"""
from __future__ import annotations

import math

import torch

from . import amh


def _ctx(w, y: torch.Tensor, s0: torch.Tensor | None = None, **over) -> amh.Context:
    return amh.Context(amh.make_config(w, **over), y, s0)


def alt_mh_restarts(w, y: torch.Tensor, runs: int = 10, sigma_deg=(10.0, 4.0)) -> dict:
    """Alt-MH repeated `runs` times.  Run r starts every chain from its best state of
    the previous run (the extended chain for r = 0) with Philox key seed + r.  A run
    counts as an improvement when the lowest best energy over the chains drops;
    after the m-th run without one the width range becomes 10/m -> 1/m degrees."""
    s0 = None
    best = math.inf
    misses = 0
    hist = []
    for r in range(runs):
        lo, hi = (sigma_deg if misses == 0 else (10.0 / misses, 1.0 / misses))
        ctx = _ctx(w, y, s0, seed=w.seed + r, sigma=math.radians(lo),
                   sigma_end=math.radians(hi))
        ctx.sweep(w.total_sweeps)
        Vb, sb, _ = ctx.energy(which=1, want_s=True)
        ctx.poll()
        m = float(Vb.min())
        improved = m < best
        hist.append({"run": r, "sigma_deg": [lo, hi], "best": m, "improved": improved})
        if improved:
            best = m
            misses = 0
            s0 = sb.contiguous()
        else:
            misses += 1
        ctx.close()
    return {"best": best, "runs": hist}


def mh_noisy_restarts(w, y: torch.Tensor, every: int = 100, amplitude_deg: float = 10.0,
                      beta=(0.1, 1.0)) -> dict:
    """Plain MH (every sweep global), T from 1/beta[0] to 1/beta[1] geometrically, with
    a noisy restart of every chain after each `every` sweeps (except the last)."""
    ctx = _ctx(w.replace(global_every=1, n_global=1), y, T0=1.0 / beta[0], T1=1.0 / beta[1])
    done, tag = 0, 0
    while done < w.total_sweeps:
        n = min(every, w.total_sweeps - done)
        ctx.sweep(n)
        done += n
        if done < w.total_sweeps:
            ctx.perturb(math.radians(amplitude_deg), tag)
            tag += 1
    Vb, _, _ = ctx.energy(which=1)
    ctx.poll()
    out = {"best": float(Vb.min()), "restarts": tag}
    ctx.close()
    return out


def beta_sweep(w, y: torch.Tensor, betas, runs: int = 25) -> dict:
    """For every beta: `runs` independent chains of Alt-MH (w's alternation) and of
    plain MH, at constant temperature 1/beta, all advanced in one batch.  Returns the
    mean, min and max over runs of each run's lowest energy."""
    ctxs, keys = [], []
    for i, b in enumerate(betas):
        T = 1.0 / b
        for name, ge, ng in (("alt", w.global_every, w.n_global), ("mh", 1, 1)):
            ctxs.append(_ctx(w.replace(n_chains=runs, global_every=ge, n_global=ng), y, T0=T, T1=T,
                             seed=w.seed + 2 * i + (name == "mh")))
            keys.append((name, b))
    batch = amh.Batch(ctxs)
    batch.sweep(w.total_sweeps)
    batch.close()
    out = {"alt": [], "mh": []}
    for (name, b), c in zip(keys, ctxs):
        Vb, _, _ = c.energy(which=1)
        c.poll()
        v = Vb.cpu().numpy()
        out[name].append({"beta": b, "mean": float(v.mean()), "min": float(v.min()),
                          "max": float(v.max())})
        c.close()
    return out


def chain_count_study(w, y: torch.Tensor, counts=(10, 1000)) -> dict:
    """Best energy found by each number of independent chains (same schedule; the
    chains of the smaller run are the first chains of the larger one)."""
    out = []
    for n in counts:
        ctx = _ctx(w.replace(n_chains=n), y)
        ctx.sweep(w.total_sweeps)
        Vb, _, _ = ctx.energy(which=1)
        ctx.poll()
        out.append({"chains": n, "best": float(Vb.min()), "median": float(Vb.median())})
        ctx.close()
    return {"counts": out}


def summary_gain(a: float, b: float) -> float:
    """Relative energy improvement of a over b (positive when a is lower)."""
    return (b - a) / abs(b) if b else float("nan")


__all__ = ["alt_mh_restarts", "mh_noisy_restarts", "beta_sweep", "chain_count_study",
           "summary_gain"]
