"""ctypes wrapper of the FP64 AMH oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU
baseline leg of ``bench.py``; never by the product package.  All arrays are
numpy float64 / uint32 / uint8 in C order.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")


class Cfg(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("n_bins", C.c_int32), ("d_min", C.c_double), ("bin_w", C.c_double),
        ("window_d", C.c_int32), ("global_every", C.c_int32), ("anchor_every", C.c_int32),
        ("n_global", C.c_int32), ("sigma", C.c_double), ("T0", C.c_double), ("T1", C.c_double),
        ("total_sweeps", C.c_int64), ("seed", C.c_uint64), ("sigma_end", C.c_double),
        ("n_cascade", C.c_int32), ("cascade_d", C.c_int32 * 3),
    ]


class LbfgsOpts(C.Structure):
    _fields_ = [
        ("n_iter", C.c_int32), ("m", C.c_int32), ("nonmonotone", C.c_int32), ("max_ls", C.c_int32),
        ("c1", C.c_double), ("shrink", C.c_double), ("gtol", C.c_double), ("step0", C.c_double),
    ]


def lbfgs_opts(n_iter=200, m=8, nonmonotone=5, max_ls=30, c1=1e-4, shrink=0.5, gtol=1e-6,
               step0=0.1) -> LbfgsOpts:
    return LbfgsOpts(n_iter=n_iter, m=m, nonmonotone=nonmonotone, max_ls=max_ls, c1=c1,
                     shrink=shrink, gtol=gtol, step0=step0)


class LbfgsReplayReport(C.Structure):
    _fields_ = [("n_steps", C.c_int64), ("n_forks", C.c_int64), ("n_fail", C.c_int64),
                ("first_fail", C.c_int64), ("max_step_err", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


FG_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                    C.POINTER(C.c_double))


class ReplayReport(C.Structure):
    _fields_ = [
        ("n_steps", C.c_int64), ("n_forks", C.c_int64), ("n_de_fail", C.c_int64),
        ("n_delta_fail", C.c_int64), ("n_logic_fail", C.c_int64), ("first_fail_step", C.c_int64),
        ("n_anchors", C.c_int64), ("n_anchor_fail", C.c_int64),
        ("max_de_abs_err", C.c_double), ("max_de_rel_err", C.c_double),
        ("max_anchor_rel_err", C.c_double), ("max_fork_margin", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_U32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def _opt(nd):
    """ndpointer that also accepts None."""
    class _P(nd):  # type: ignore[misc, valid-type]
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return super().from_param(obj)
    return _P


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(_LIB_PATH)
    P = C.POINTER
    L.oracle_philox4x32_10.argtypes = [_U32, _U32, _U32]
    L.oracle_philox_batch.argtypes = [C.c_int64, _U32, _U32, _U32]
    L.oracle_proposal.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int32, C.c_double,
                                  P(C.c_double), P(C.c_double)]
    L.oracle_beta.argtypes = [P(Cfg), C.c_int64]
    L.oracle_beta.restype = C.c_double
    L.oracle_is_global.argtypes = [P(Cfg), C.c_int64]
    L.oracle_is_global.restype = C.c_int32
    L.oracle_sigma.argtypes = [P(Cfg), C.c_int64]
    L.oracle_sigma.restype = C.c_double
    L.oracle_window_d.argtypes = [P(Cfg), C.c_int64]
    L.oracle_window_d.restype = C.c_int32
    L.oracle_perturb.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_double, C.c_int32, _D]
    L.oracle_nerf.argtypes = [C.c_int32, _D, _D]
    L.oracle_geometry_constants.argtypes = [_D]
    L.oracle_pair_energy.argtypes = [_D, C.c_int32, C.c_double, C.c_double, C.c_double]
    L.oracle_pair_energy.restype = C.c_double
    L.oracle_pair_energy_deriv.argtypes = [_D, C.c_int32, C.c_double, C.c_double, C.c_double]
    L.oracle_pair_energy_deriv.restype = C.c_double
    L.oracle_energy_full.argtypes = [P(Cfg), _D, _D]
    L.oracle_energy_full.restype = C.c_double
    L.oracle_energy_window.argtypes = [P(Cfg), _D, _D, C.c_int32]
    L.oracle_energy_window.restype = C.c_double
    L.oracle_neumaier_sum.argtypes = [C.c_int64, _D]
    L.oracle_neumaier_sum.restype = C.c_double
    L.oracle_delta_e.argtypes = [P(Cfg), _D, _D, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                 P(C.c_double)]
    L.oracle_delta_e.restype = C.c_double
    L.oracle_grad.argtypes = [P(Cfg), _D, _D, P(C.c_double), _D]
    L.oracle_lbfgs_direction.argtypes = [C.c_int32, C.c_int32, _D, _D, _D, C.c_double, _D]
    L.oracle_lbfgs.argtypes = [C.c_int32, _D, P(LbfgsOpts), FG_FN, C.c_void_p, P(C.c_double),
                               P(C.c_int32), _opt(_D), _opt(_D)]
    L.oracle_lbfgs.restype = C.c_int32
    L.oracle_lbfgs_protein.argtypes = [P(Cfg), _D, _D, P(LbfgsOpts), P(C.c_double), P(C.c_int32),
                                       _opt(_D), _opt(_D)]
    L.oracle_lbfgs_protein.restype = C.c_int32
    L.oracle_lbfgs_replay.argtypes = [P(Cfg), _D, C.c_int32, _D, P(LbfgsOpts), C.c_double,
                                      C.c_double, P(LbfgsReplayReport)]
    L.oracle_lbfgs_replay.restype = C.c_int32
    L.oracle_chain_init.argtypes = [P(Cfg), _D, C.c_int32, _D, _D, _D]
    L.oracle_run.argtypes = [P(Cfg), _D, C.c_int32, _opt(_U32), C.c_int64, C.c_int64, C.c_int32,
                             C.c_int32, _D, _D, _D, _I64, C.c_double, _opt(_D), _opt(_U8),
                             _opt(_D)]
    L.oracle_run.restype = C.c_int32
    L.oracle_replay.argtypes = [P(Cfg), _D, C.c_uint32, _D, C.c_int64, C.c_int64, _D, _D, _U8,
                                _opt(_D), C.c_double, C.c_double, C.c_double, _D,
                                P(ReplayReport)]
    L.oracle_replay.restype = C.c_int32
    _lib = L
    return L


def make_cfg(w) -> Cfg:
    """Oracle config from a synthetic.Workload."""
    casc = list(getattr(w, "cascade", ()))
    return Cfg(L=w.L, n_bins=w.n_bins, d_min=w.d_min, bin_w=w.bin_w, window_d=w.window_d,
               global_every=w.global_every, anchor_every=w.anchor_period,
               n_global=getattr(w, "n_global", 1),
               sigma=w.sigma, T0=w.T0, T1=w.T1, total_sweeps=w.total_sweeps, seed=w.seed,
               sigma_end=math.radians(getattr(w, "sigma_end_deg", 0.0)), n_cascade=len(casc),
               cascade_d=(C.c_int32 * 3)(*(casc + [0] * (3 - len(casc)))))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- #
def philox(ctr, key) -> np.ndarray:
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    key = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.empty_like(ctr)
    lib().oracle_philox_batch(ctr.shape[0], ctr, key, out)
    return out


def sigma_at(cfg: Cfg, t: int) -> float:
    return lib().oracle_sigma(C.byref(cfg), t)


def window_at(cfg: Cfg, t: int) -> int:
    return lib().oracle_window_d(C.byref(cfg), t)


def perturb(seed: int, chain: int, tag: int, amplitude: float, s) -> np.ndarray:
    """Noisy restart of one chain's torsions (a copy is returned)."""
    s = _f64(s).copy()
    lib().oracle_perturb(seed, chain, tag, amplitude, s.size, s)
    return s


def proposal(seed: int, chain: int, t: int, k: int, sigma: float) -> tuple[float, float]:
    d, lu = C.c_double(), C.c_double()
    lib().oracle_proposal(seed, chain, t, k, sigma, C.byref(d), C.byref(lu))
    return d.value, lu.value


def beta(cfg: Cfg, t: int) -> float:
    return lib().oracle_beta(C.byref(cfg), t)


def is_global(cfg: Cfg, t: int) -> bool:
    return bool(lib().oracle_is_global(C.byref(cfg), t))


def nerf(s) -> np.ndarray:
    s = _f64(s)
    L = s.shape[-1] // 2
    out = np.empty((L, 4, 3))
    lib().oracle_nerf(L, s, out)
    return out


def cb(s) -> np.ndarray:
    return nerf(s)[:, 3, :].copy()


def geometry_constants() -> np.ndarray:
    out = np.empty(10)
    lib().oracle_geometry_constants(out)
    return out


def pair_energy(y_row, d: float, d_min: float = 2.0, bin_w: float = 0.5) -> float:
    y_row = _f64(y_row)
    return lib().oracle_pair_energy(y_row, y_row.shape[0], d_min, bin_w, d)


def pair_energy_deriv(y_row, d: float, d_min: float = 2.0, bin_w: float = 0.5) -> float:
    y_row = _f64(y_row)
    return lib().oracle_pair_energy_deriv(y_row, y_row.shape[0], d_min, bin_w, d)


def energy_full(cfg: Cfg, y, atoms) -> float:
    return lib().oracle_energy_full(C.byref(cfg), _f64(y), _f64(atoms))


def energy(cfg: Cfg, y, s) -> float:
    return energy_full(cfg, y, nerf(s))


def energy_window(cfg: Cfg, y, atoms, k: int) -> float:
    return lib().oracle_energy_window(C.byref(cfg), _f64(y), _f64(atoms), k)


def neumaier_sum(x) -> float:
    x = _f64(x)
    return lib().oracle_neumaier_sum(x.shape[0], x)


def delta_e(cfg: Cfg, y, s, k: int, delta: float, global_: bool, mode: int) -> tuple[float, float]:
    S = C.c_double()
    dE = lib().oracle_delta_e(C.byref(cfg), _f64(y), _f64(s), k, delta, int(global_), mode,
                              C.byref(S))
    return dE, S.value


def grad(cfg: Cfg, y, s) -> tuple[float, np.ndarray]:
    s = _f64(s)
    g = np.empty_like(s)
    V = C.c_double()
    lib().oracle_grad(C.byref(cfg), _f64(y), s, C.byref(V), g)
    return V.value, g


def lbfgs_direction(S, Y, g, gamma: float) -> np.ndarray:
    """-H g by the two-loop recursion over the rows of S, Y (oldest first)."""
    g = _f64(g)
    n = g.size
    S = _f64(np.asarray(S).reshape(-1, n))
    Y = _f64(np.asarray(Y).reshape(-1, n))
    d = np.empty_like(g)
    lib().oracle_lbfgs_direction(n, S.shape[0], S.ravel() if S.size else np.zeros(1), Y.ravel()
                                 if Y.size else np.zeros(1), g, gamma, d)
    return d


def lbfgs(fg, x0, opts: LbfgsOpts | None = None):
    """Minimise a Python callable fg(x) -> (f, g); returns (x, f, iters, status, f_trace)."""
    opts = opts or lbfgs_opts()
    x = _f64(x0).copy()
    n = x.size

    def _cb(_ctx, xp, fp, gp):
        xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        f, g = fg(xv)
        fp[0] = float(f)
        np.ctypeslib.as_array(gp, shape=(n,))[:] = g

    cb = FG_FN(_cb)
    f, it = C.c_double(), C.c_int32()
    tr = np.full(opts.n_iter + 1, np.nan)
    st = lib().oracle_lbfgs(n, x, C.byref(opts), cb, None, C.byref(f), C.byref(it), tr, None)
    return x, f.value, it.value, st, tr[: it.value + 1]


def lbfgs_protein(cfg: Cfg, y, s0, opts: LbfgsOpts | None = None, iterates: bool = False):
    """L-BFGS on V(s); returns (s wrapped, V, iters, status, f_trace[, x_trace])."""
    opts = opts or lbfgs_opts()
    s = _f64(s0).copy()
    V, it = C.c_double(), C.c_int32()
    tr = np.full(opts.n_iter + 1, np.nan)
    xt = np.full((opts.n_iter + 1, s.size), np.nan) if iterates else None
    st = lib().oracle_lbfgs_protein(C.byref(cfg), _f64(y), s, C.byref(opts), C.byref(V),
                                    C.byref(it), tr, xt)
    out = (s, V.value, it.value, st, tr[: it.value + 1])
    return out + (xt[: it.value + 1],) if iterates else out


def lbfgs_replay(cfg: Cfg, y, X, opts: LbfgsOpts | None = None, step_tol: float = 1e-6,
                 tie_tol: float = 1e-9) -> tuple[int, dict]:
    """Check device L-BFGS iterates X [n_it + 1][2L] step by step (see oracle.c)."""
    opts = opts or lbfgs_opts()
    X = _f64(X)
    rep = LbfgsReplayReport()
    rc = lib().oracle_lbfgs_replay(C.byref(cfg), _f64(y), X.shape[0] - 1, X.ravel(), C.byref(opts),
                                   step_tol, tie_tol, C.byref(rep))
    return rc, rep.as_dict()


class Chains:
    """State of a set of oracle chains (s, s_best, V_anchor, V_best, counters)."""

    def __init__(self, cfg: Cfg, y, s0, chain_ids=None):
        self.cfg = cfg
        self.y = _f64(y)
        s0 = np.atleast_2d(_f64(s0))
        self.C = s0.shape[0]
        self.s = s0.copy()
        self.s_best = s0.copy()
        self.v = np.empty((self.C, 2))
        lib().oracle_chain_init(C.byref(cfg), self.y, self.C, self.s, self.s_best, self.v)
        self.counters = np.zeros((self.C, 4), dtype=np.int64)
        self.counters[:, 2] = -1
        self.ids = (np.arange(self.C, dtype=np.uint32) if chain_ids is None
                    else np.ascontiguousarray(chain_ids, dtype=np.uint32))
        self.t = 0

    def run(self, n_sweeps: int, mode: int = 1, threads: int = 1, target: float = -math.inf,
            log_steps: bool = False, log_anchors: bool = False):
        n = 2 * self.cfg.L
        A = self.cfg.anchor_every
        na = (self.t + n_sweeps) // A - self.t // A
        step_log = np.empty((self.C, n_sweeps * n, 2)) if log_steps else None
        acc_log = np.empty((self.C, n_sweeps * n), dtype=np.uint8) if log_steps else None
        anchor_log = np.empty((self.C, na)) if log_anchors else None
        rc = lib().oracle_run(C.byref(self.cfg), self.y, self.C, self.ids, self.t, n_sweeps, mode,
                              threads, self.s, self.s_best, self.v, self.counters, target,
                              step_log, acc_log, anchor_log)
        if rc != 0:
            raise ValueError("oracle_run rejected its input")
        self.t += n_sweeps
        return step_log, acc_log, anchor_log


def replay(cfg: Cfg, y, chain_id: int, s0, t_begin: int, n_sweeps: int, gpu_dE, gpu_delta,
           gpu_acc, gpu_anchor=None, rel_tol: float = 1e-4, abs_tol: float = 1e-6,
           anchor_rel_tol: float = 1e-4):
    s_out = np.empty(2 * cfg.L)
    rep = ReplayReport()
    rc = lib().oracle_replay(C.byref(cfg), _f64(y), chain_id, _f64(s0), t_begin, n_sweeps,
                             _f64(gpu_dE), _f64(gpu_delta),
                             np.ascontiguousarray(gpu_acc, dtype=np.uint8),
                             None if gpu_anchor is None else _f64(gpu_anchor),
                             rel_tol, abs_tol, anchor_rel_tol, s_out, C.byref(rep))
    return rc, rep.as_dict(), s_out
