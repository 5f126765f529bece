"""Helpers shared by the GPU tests: seeded proteins, contexts, traced runs, replays."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import oracle
import synthetic as sy
from paper_2211_03193_amd import amh

DEV = "cuda:0"


def say(*a):
    """Name the case before each GPU step (flushed), so a failed run shows it."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def protein(w: sy.Workload):
    """(s_ref, y float64) of a workload, reference distances from the oracle's NeRF."""
    return sy.workload(w, lambda s: sy.pair_distances(oracle.cb(s)))


def context(w: sy.Workload, y64, s0=None, **over) -> amh.Context:
    cfg = amh.make_config(w, **over)
    y = torch.from_numpy(np.ascontiguousarray(y64, dtype=np.float32)).to(DEV)
    s0t = None if s0 is None else torch.from_numpy(np.ascontiguousarray(s0, dtype=np.float64)).to(DEV)
    return amh.Context(cfg, y, s0t)


def traced_run(ctx: amh.Context, chains, n_sweeps: int, chunk: int | None = None):
    """Run n_sweeps with the given chains traced; returns numpy trace arrays."""
    tr = ctx.set_trace(chains, n_sweeps)
    chunk = chunk or n_sweeps
    done = 0
    while done < n_sweeps:
        m = min(chunk, n_sweeps - done)
        ctx.sweep(m)
        done += m
    ctx.poll()
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in tr.items()}
    ctx.clear_trace()
    return out


def replay_chain(w: sy.Workload, y64, tr, slot: int, chain: int, s0, t0: int = 0,
                 rel_tol: float = 1e-4, abs_tol: float = 1e-6, anchor_rel_tol: float = 1e-4):
    cfg = oracle.make_cfg(w)
    n = tr["n_sweeps"] * 2 * w.L
    A = cfg.anchor_every
    na = (t0 + tr["n_sweeps"]) // A - t0 // A
    y32 = np.asarray(y64, dtype=np.float32).astype(np.float64)   # the table the device sees
    rc, rep, s_out = oracle.replay(cfg, y32, chain, s0, t0, tr["n_sweeps"], tr["dE"][slot, :n],
                                   tr["delta"][slot, :n], tr["acc"][slot, :n],
                                   tr["anchor"][slot, :na] if na > 0 else None,
                                   rel_tol, abs_tol, anchor_rel_tol)
    return rc, rep, s_out


def extended(w: sy.Workload) -> np.ndarray:
    return np.full(2 * w.L, math.pi)
