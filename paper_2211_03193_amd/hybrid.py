"""Host schedules that alternate the library's device phases.

Only the order of calls is decided here; every step (sampling sweeps, L-BFGS
iterations, energies, best-state tracking) runs in libamh.so's kernels.
"""
from __future__ import annotations

from . import amh


def lbfgs_with_localized_mh(ctx: amh.Context, cycles: int, lbfgs_iters: int = 80,
                            mh_sweeps: int = 20, opts: amh.LbfgsOpts | None = None,
                            final_lbfgs: bool = True) -> list[dict]:
    """L-BFGS interleaved with localized MH (the paper's fifth scheme in Sec. 3:
    each batch of 100 samples is 80 L-BFGS iterations followed by 20 localized MH
    sweeps in place of a noisy restart).

    The context's chains are minimised in place (amh_minimize with no torsion
    buffer keeps their V, best state and coordinates current), then swept
    `mh_sweeps` times by the context's own schedule; a context configured with
    global_every = 0 runs localized sweeps only.  Returns the per-phase outputs of
    amh_minimize.
    """
    base = opts or amh.lbfgs_opts()
    o = amh.LbfgsOpts(**{f: getattr(base, f) for f, _ in amh.LbfgsOpts._fields_})
    o.n_iter = lbfgs_iters
    out = []
    for _ in range(cycles):
        out.append(ctx.minimize(None, o))
        ctx.sweep(mh_sweeps)
    if final_lbfgs:
        out.append(ctx.minimize(None, o))
    return out
