"""Replay an arrival trace against a Server and summarise latencies.

Host driver only: jobs are submitted when the wall clock passes their arrival
time, the server is stepped in between, and the per-job clocks recorded by the
library (steady clock, seconds) give time-to-target and time-to-completion.
"""
from __future__ import annotations

import time

import numpy as np

from . import amh


def run_trace(server: amh.Server, jobs, arrivals, max_wall: float = 600.0) -> list[dict]:
    """jobs: list of (amh_config, y float32 host array, target); arrivals: seconds from
    the start, non-decreasing.  Returns the final status of every job (with its
    handle under "id"), in arrival order."""
    t0 = time.monotonic()
    ids = []
    i, n = 0, len(jobs)
    active = pending = 0
    while True:
        now = time.monotonic() - t0
        if now > max_wall:
            raise TimeoutError(f"trace not drained after {max_wall} s")
        submitted = False
        while i < n and arrivals[i] <= now:
            cfg, y, target = jobs[i]
            ids.append(server.submit(cfg, y, target))
            i += 1
            submitted = True
        if submitted or active or pending:
            active, pending = server.step()
            continue
        if i == n:
            break
        time.sleep(max(0.0, min(arrivals[i] - now, 0.05)))
    return [dict(server.job(j), id=j) for j in ids]


def summarise(status: list[dict]) -> dict:
    done = [s for s in status if s["state"] == 2]
    lat_done = np.array([s["t_done"] - s["t_submit"] for s in done])
    lat_tgt = np.array([s["t_target"] - s["t_submit"] for s in done if s["reached"]])
    span = max(s["t_done"] for s in done) - min(s["t_submit"] for s in status) if done else 0.0

    def pct(a, q):
        return float(np.percentile(a, q)) if a.size else None

    return {"jobs": len(status), "done": len(done), "failed": sum(s["state"] == 3 for s in status),
            "reached_target": int(lat_tgt.size),
            "p50_time_to_target_s": pct(lat_tgt, 50), "p99_time_to_target_s": pct(lat_tgt, 99),
            "p50_time_to_done_s": pct(lat_done, 50), "p99_time_to_done_s": pct(lat_done, 99),
            "makespan_s": span}
