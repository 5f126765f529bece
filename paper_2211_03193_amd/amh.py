"""Thin ctypes binding of libamh.so (C ABI in include/amh.h).

Argument marshalling only: every step of the sampler runs in the HIP kernels of
libamh.so.  PyTorch provides device memory and the stream.  There is no CPU
fallback: if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamh.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NUMERIC, E_UNSUPPORTED, E_BUSY = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "AMH_OK", -1: "AMH_E_INVAL", -2: "AMH_E_NOMEM", -3: "AMH_E_DEVICE",
          -4: "AMH_E_NUMERIC", -5: "AMH_E_UNSUPPORTED", -6: "AMH_E_BUSY"}


class AmhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class AmhConfig(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("n_chains", C.c_int32), ("n_bins", C.c_int32), ("window_d", C.c_int32),
        ("d_min", C.c_double), ("bin_w", C.c_double), ("global_every", C.c_int32),
        ("anchor_every", C.c_int32), ("sigma", C.c_double), ("T0", C.c_double), ("T1", C.c_double),
        ("total_sweeps", C.c_int64), ("seed", C.c_uint64), ("chain_offset", C.c_uint32),
        ("chains_per_group", C.c_int32), ("waves_per_group", C.c_int32), ("n_global", C.c_int32),
        ("sigma_end", C.c_double), ("n_cascade", C.c_int32), ("cascade_d", C.c_int32 * 3),
    ]


class LbfgsOpts(C.Structure):
    _fields_ = [
        ("n_iter", C.c_int32), ("m", C.c_int32), ("nonmonotone", C.c_int32), ("max_ls", C.c_int32),
        ("c1", C.c_double), ("shrink", C.c_double), ("gtol", C.c_double), ("step0", C.c_double),
    ]


def lbfgs_opts(n_iter=200, m=8, nonmonotone=5, max_ls=30, c1=1e-4, shrink=0.5, gtol=1e-6,
               step0=0.1) -> LbfgsOpts:
    """amh_lbfgs_opts with the defaults used throughout (see include/amh.h)."""
    return LbfgsOpts(n_iter=n_iter, m=m, nonmonotone=nonmonotone, max_ls=max_ls, c1=c1,
                     shrink=shrink, gtol=gtol, step0=step0)


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_active", C.c_int32),
                ("sweeps_per_round", C.c_int32), ("plan", C.c_int32), ("reserved", C.c_int32),
                ("round_pairs", C.c_int64)]


class JobTrace(C.Structure):
    _fields_ = [("chain", C.c_int32), ("reserved", C.c_int32), ("dE_dev", C.c_void_p),
                ("delta_dev", C.c_void_p), ("acc_dev", C.c_void_p), ("capacity", C.c_int64),
                ("anchor_dev", C.c_void_p), ("anchor_capacity", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("cfg", AmhConfig), ("y_host", C.c_void_p), ("target", C.c_double),
                ("trace", C.POINTER(JobTrace))]


class JobStatus(C.Structure):
    _fields_ = [("state", C.c_int32), ("reached", C.c_int32), ("sweeps", C.c_int64),
                ("sweeps_to_target", C.c_int64), ("best_V", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_target", C.c_double), ("t_done", C.c_double),
                ("bytes", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_P = C.c_void_p


def lib():
    """Load libamh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2211_03193_amd/build.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    sig = {
        "amh_init": [C.POINTER(AmhConfig), _P, _P, _P, C.POINTER(_P)],
        "amh_sweep": [_P, C.c_int64],
        "amh_energy": [_P, _P, C.c_int32, C.c_int32, _P, _P, _P],
        "amh_conformation": [_P, C.c_int32, C.c_int32, _P, _P],
        "amh_get_state": [_P, _P, _P, _P, _P, _P, C.POINTER(C.c_int64)],
        "amh_set_state": [_P, _P, _P, _P, _P, _P, C.c_int64],
        "amh_set_target": [_P, C.c_double],
        "amh_perturb": [_P, C.c_double, C.c_uint32],
        "amh_set_wait_bound": [_P, C.c_int32],
        "amh_set_trace": [_P, C.c_int32, C.POINTER(C.c_int32), _P, _P, _P, C.c_int64, _P, C.c_int64],
        "amh_poll": [_P],
        "amh_set_work_counters": [_P, _P],
        "amh_info": [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                     C.POINTER(C.c_int64)],
        "amh_info_launches": [_P] + [C.POINTER(C.c_int32)] * 6,
        "amh_grad": [_P, _P, C.c_int32, _P, _P],
        "amh_minimize": [_P, _P, C.c_int32, C.POINTER(LbfgsOpts), _P, _P, _P, _P, _P],
        "amh_minimize_noalloc": [_P, _P, C.c_int32, C.POINTER(LbfgsOpts), _P, _P, _P, _P, _P],
        "amh_batch_create": [C.POINTER(_P), C.c_int32, C.POINTER(_P)],
        "amh_batch_sweep": [_P, C.c_int64],
        "amh_batch_sweep_each": [_P, C.POINTER(C.c_int64)],
        "amh_batch_tune": [_P, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_int32)],
        "amh_batch_set_plan": [_P, C.c_int32],
        "amh_batch_info": [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
        "amh_batch_destroy": [_P],
        "amh_server_create": [C.POINTER(ServerOpts), _P, C.POINTER(_P)],
        "amh_server_step": [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
        "amh_server_job": [_P, C.c_uint64, C.POINTER(JobStatus), _P, _P],
        "amh_server_destroy": [_P],
        "amh_submit": [_P, _P, C.POINTER(C.c_uint64)],
        "amh_destroy": [_P],
        "amh_philox": [_P, C.c_int64, C.c_uint64, _P, _P],
        "amh_yard_stream": [_P, C.c_int64, C.c_int32, _P, _P],
        "amh_yard_gather": [_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P],
        "amh_yard_lds": [C.c_int32, C.c_int32, _P, _P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.amh_last_error.argtypes = []
    L.amh_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != OK:
        raise AmhError(status, lib().amh_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_config(w, **over) -> AmhConfig:
    """amh_config from a workload description (synthetic.Workload or any object
    with the same attribute names)."""
    cfg = AmhConfig(L=w.L, n_chains=w.n_chains, n_bins=w.n_bins, window_d=w.window_d,
                    d_min=w.d_min, bin_w=w.bin_w, global_every=w.global_every,
                    anchor_every=w.anchor_period, sigma=math.radians(w.sigma_deg), T0=w.T0,
                    T1=w.T1, total_sweeps=w.total_sweeps, seed=w.seed, chain_offset=0,
                    chains_per_group=0, waves_per_group=0, n_global=getattr(w, "n_global", 1),
                    sigma_end=math.radians(getattr(w, "sigma_end_deg", 0.0)))
    casc = list(getattr(w, "cascade", ()))
    cfg.n_cascade = len(casc)
    for i, d in enumerate(casc):
        cfg.cascade_d[i] = d
    for k, v in over.items():
        setattr(cfg, k, v)
    return cfg


class Context:
    """A sampler on the current GPU: C chains of one protein (amh_init .. amh_destroy)."""

    def __init__(self, cfg: AmhConfig, y: torch.Tensor, s0: torch.Tensor | None = None,
                 stream=None):
        if not y.is_cuda or y.dtype != torch.float32 or not y.is_contiguous():
            raise ValueError("y must be a contiguous float32 CUDA tensor [P][n_bins]")
        P = cfg.L * (cfg.L - 1) // 2
        if tuple(y.shape) != (P, cfg.n_bins):
            raise ValueError(f"y has shape {tuple(y.shape)}, expected {(P, cfg.n_bins)}")
        if s0 is not None:
            if not s0.is_cuda or s0.dtype != torch.float64 or not s0.is_contiguous():
                raise ValueError("s0 must be a contiguous float64 CUDA tensor [C][2L]")
            if tuple(s0.shape) != (cfg.n_chains, 2 * cfg.L):
                raise ValueError(f"s0 has shape {tuple(s0.shape)}, expected {(cfg.n_chains, 2 * cfg.L)}")
        self.cfg = cfg
        self.device = y.device
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream(y.device)
        self._h = C.c_void_p()
        self._trace_keep = None
        check(lib().amh_init(C.byref(cfg), _ptr(y), _ptr(s0), _stream(self._stream_obj),
                             C.byref(self._h)))

    @property
    def L(self) -> int:
        return self.cfg.L

    @property
    def C(self) -> int:
        return self.cfg.n_chains

    def sweep(self, n: int) -> None:
        check(lib().amh_sweep(self._h, n))

    def energy(self, s: torch.Tensor | None = None, which: int = 0, want_s: bool = False,
               want_cb: bool = False):
        B = self.C if s is None else s.shape[0]
        if s is not None and (s.dtype != torch.float64 or not s.is_contiguous() or s.shape[1] != 2 * self.L):
            raise ValueError("s must be a contiguous float64 tensor [B][2L]")
        V = torch.empty(B, dtype=torch.float64, device=self.device)
        so = torch.empty(B, 2 * self.L, dtype=torch.float64, device=self.device) if want_s else None
        cb = torch.empty(B, self.L, 3, dtype=torch.float32, device=self.device) if want_cb else None
        check(lib().amh_energy(self._h, _ptr(s), B, which, _ptr(V), _ptr(so), _ptr(cb)))
        return V, so, cb

    def _check_s(self, s):
        if s is not None and (s.dtype != torch.float64 or not s.is_contiguous() or s.dim() != 2
                              or s.shape[1] != 2 * self.L or not s.is_cuda):
            raise ValueError("s must be a contiguous float64 CUDA tensor [B][2L]")

    def grad(self, s: torch.Tensor | None = None):
        """(V [B], dV/ds [B][2L]) in float64 of s [B][2L], or of the current chains."""
        self._check_s(s)
        B = self.C if s is None else s.shape[0]
        V = torch.empty(B, dtype=torch.float64, device=self.device)
        g = torch.empty(B, 2 * self.L, dtype=torch.float64, device=self.device)
        if B > 0:   # an empty tensor has no address; NULL would mean the context's chains
            check(lib().amh_grad(self._h, _ptr(s), B, _ptr(V), _ptr(g)))
        return V, g

    def minimize(self, s: torch.Tensor | None = None, opts: LbfgsOpts | None = None,
                 trace: bool = False, iterates: bool = False, no_alloc: bool = False) -> dict:
        """L-BFGS on V (amh_minimize, or amh_minimize_noalloc with no_alloc: the
        library's fixed scratch as workspace).  s [B][2L] is minimised in place; with s
        None the context's current chains are (and their V, best state and coordinates
        follow)."""
        self._check_s(s)
        opts = opts or lbfgs_opts()
        B = self.C if s is None else s.shape[0]
        d = self.device
        out = {"V": torch.empty(B, dtype=torch.float64, device=d),
               "iters": torch.empty(B, dtype=torch.int32, device=d),
               "status": torch.empty(B, dtype=torch.int32, device=d),
               "trace": torch.full((B, opts.n_iter + 1), float("nan"), dtype=torch.float64, device=d)
               if trace else None,
               "x": torch.full((B, opts.n_iter + 1, 2 * self.L), float("nan"), dtype=torch.float64,
                               device=d) if iterates else None}
        if B > 0:   # an empty tensor has no address; NULL would mean the context's chains
            fn = lib().amh_minimize_noalloc if no_alloc else lib().amh_minimize
            check(fn(self._h, _ptr(s), B, C.byref(opts), _ptr(out["V"]), _ptr(out["iters"]),
                     _ptr(out["status"]), _ptr(out["trace"]), _ptr(out["x"])))
        return out

    def energy_fn(self):
        """V(s) as a differentiable function of s [B][2L] (torch.autograd)."""
        return lambda s: _Energy.apply(s, self)

    def set_work_counters(self, counters: torch.Tensor | None) -> None:
        """Count the executed work of later global sweeps into an int64[3] device tensor
        (amh_set_work_counters): surviving tiles, pair tests, near pairs; None stops."""
        if counters is not None and (counters.dtype != torch.int64 or counters.numel() < 3
                                     or not counters.is_cuda):
            raise ValueError("counters must be an int64 CUDA tensor of 3 elements")
        self._work_keep = counters
        check(lib().amh_set_work_counters(self._h, _ptr(counters)))

    def get_state(self) -> dict:
        n, Cc, L = 2 * self.L, self.C, self.L
        d = self.device
        st = {"s": torch.empty(Cc, n, dtype=torch.float64, device=d),
              "s_best": torch.empty(Cc, n, dtype=torch.float64, device=d),
              "v": torch.empty(Cc, 2, dtype=torch.float64, device=d),
              "counters": torch.empty(Cc, 4, dtype=torch.int64, device=d),
              "atoms": torch.empty(Cc, L, 4, 3, dtype=torch.float64, device=d)}
        t = C.c_int64()
        check(lib().amh_get_state(self._h, _ptr(st["s"]), _ptr(st["s_best"]), _ptr(st["v"]),
                                  _ptr(st["counters"]), _ptr(st["atoms"]), C.byref(t)))
        st["t"] = t.value
        return st

    def set_state(self, st: dict, with_atoms: bool = True) -> None:
        check(lib().amh_set_state(self._h, _ptr(st.get("s")), _ptr(st.get("s_best")),
                                  _ptr(st.get("v")), _ptr(st.get("counters")),
                                  _ptr(st.get("atoms")) if with_atoms else None, int(st["t"])))

    def set_target(self, target: float) -> None:
        check(lib().amh_set_target(self._h, target))

    def set_wait_bound(self, polls: int) -> None:
        check(lib().amh_set_wait_bound(self._h, polls))

    def perturb(self, amplitude: float, tag: int) -> None:
        """Noisy restart of every chain (amh_perturb): uniform in [-amplitude, amplitude] rad."""
        check(lib().amh_perturb(self._h, amplitude, tag))

    def set_trace(self, chain_ids, n_sweeps: int) -> dict:
        """Trace every proposal of the given chains (<= 4) over the next n_sweeps sweeps."""
        ids = list(chain_ids)
        n = len(ids)
        cap = n_sweeps * 2 * self.L
        A = self.cfg.anchor_every
        t = self.info()["t"]
        acap = (t + n_sweeps) // A - t // A
        d = self.device
        rows = max(n, 1)
        tr = {"dE": torch.zeros(rows, cap, dtype=torch.float64, device=d),
              "delta": torch.zeros(rows, cap, dtype=torch.float64, device=d),
              "acc": torch.zeros(rows, cap, dtype=torch.uint8, device=d),
              "anchor": torch.zeros(rows, max(acap, 1), dtype=torch.float64, device=d),
              "chains": ids, "t0": t, "n_sweeps": n_sweeps}
        arr = (C.c_int32 * 4)(*(ids + [-1] * (4 - n)))
        self._trace_keep = tr
        check(lib().amh_set_trace(self._h, n, arr, _ptr(tr["dE"]), _ptr(tr["delta"]),
                                  _ptr(tr["acc"]), cap, _ptr(tr["anchor"]), acap))
        return tr

    def clear_trace(self) -> None:
        check(lib().amh_set_trace(self._h, 0, None, None, None, None, 0, None, 0))
        self._trace_keep = None

    def poll(self) -> None:
        check(lib().amh_poll(self._h))

    def info(self) -> dict:
        g, w, l = C.c_int32(), C.c_int32(), C.c_int32()
        t = C.c_int64()
        check(lib().amh_info(self._h, C.byref(g), C.byref(w), C.byref(l), C.byref(t)))
        sh = [C.c_int32() for _ in range(6)]
        check(lib().amh_info_launches(self._h, *[C.byref(v) for v in sh]))
        out = {"chains_per_group": g.value, "waves_per_group": w.value, "lds_bytes": l.value, "t": t.value}
        for i, kind in enumerate(("local", "global")):
            out[f"{kind}_chains_per_group"] = sh[3 * i].value
            out[f"{kind}_waves_per_group"] = sh[3 * i + 1].value
            out[f"{kind}_lds_bytes"] = sh[3 * i + 2].value
        return out

    def close(self) -> None:
        if self._h:
            check(lib().amh_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several contexts (proteins of any lengths) advanced together (amh_batch_*)."""

    N_PLANS = 6

    def __init__(self, contexts):
        self.members = list(contexts)
        arr = (_P * len(self.members))(*[c._h for c in self.members])
        self._h = C.c_void_p()
        check(lib().amh_batch_create(arr, len(self.members), C.byref(self._h)))

    def sweep(self, n) -> None:
        """n sweeps for every member, or a sequence of per-member counts."""
        if isinstance(n, int):
            check(lib().amh_batch_sweep(self._h, n))
        else:
            arr = (C.c_int64 * len(self.members))(*[int(v) for v in n])
            check(lib().amh_batch_sweep_each(self._h, arr))

    def tune(self, sweeps_per_trial: int) -> tuple[int, list[float]]:
        ms = (C.c_float * self.N_PLANS)()
        plan = C.c_int32()
        check(lib().amh_batch_tune(self._h, sweeps_per_trial, ms, C.byref(plan)))
        return plan.value, list(ms)

    def set_plan(self, plan: int) -> None:
        check(lib().amh_batch_set_plan(self._h, plan))

    def info(self) -> dict:
        p, nl, wg = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().amh_batch_info(self._h, C.byref(p), C.byref(nl), C.byref(wg)))
        return {"plan": p.value, "launches": nl.value, "workgroups": wg.value}

    def close(self) -> None:
        if self._h:
            check(lib().amh_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (amh_server_* and amh_submit)."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 1 << 30, sweeps_per_round: int = 10,
                 plan: int = 0, round_pairs: int = 0, stream=None):
        self.opts = ServerOpts(hbm_budget_bytes=int(hbm_budget_bytes), max_active=int(max_active),
                               sweeps_per_round=int(sweeps_per_round), plan=int(plan), reserved=0,
                               round_pairs=int(round_pairs))
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream()
        self._h = C.c_void_p()
        self._cfg = {}
        self._traces = {}
        check(lib().amh_server_create(C.byref(self.opts), _stream(self._stream_obj), C.byref(self._h)))

    def submit(self, cfg: AmhConfig, y, target: float, trace_chain: int | None = None) -> int:
        """Queue a job: cfg (amh_config), y [L(L-1)/2][n_bins] float32 host array, target V.
        With trace_chain, that chain's proposals are traced from the job's first sweep
        (buffers sized for all its sweeps; read them with trace(job_id))."""
        import numpy as np
        y = np.ascontiguousarray(y, dtype=np.float32)
        if y.shape != (cfg.L * (cfg.L - 1) // 2, cfg.n_bins):
            raise ValueError(f"y has shape {y.shape}")
        job = Job(cfg=cfg, y_host=y.ctypes.data, target=float(target))
        bufs = None
        if trace_chain is not None:
            dev = torch.cuda.current_device()
            cap = int(cfg.total_sweeps) * 2 * cfg.L
            acap = max(1, int(cfg.total_sweeps) // max(1, cfg.anchor_every))
            bufs = {"dE": torch.full((cap,), float("nan"), dtype=torch.float64, device=dev),
                    "delta": torch.full((cap,), float("nan"), dtype=torch.float64, device=dev),
                    "acc": torch.full((cap,), 255, dtype=torch.uint8, device=dev),
                    "anchor": torch.full((acap,), float("nan"), dtype=torch.float64, device=dev),
                    "chain": int(trace_chain)}
            tr = JobTrace(chain=int(trace_chain), reserved=0, dE_dev=_ptr(bufs["dE"]),
                          delta_dev=_ptr(bufs["delta"]), acc_dev=_ptr(bufs["acc"]), capacity=cap,
                          anchor_dev=_ptr(bufs["anchor"]), anchor_capacity=acap)
            job.trace = C.pointer(tr)
        jid = C.c_uint64()
        check(lib().amh_submit(self._h, C.byref(job), C.byref(jid)))
        self._cfg[jid.value] = (cfg.n_chains, cfg.L)
        if bufs is not None:
            self._traces[jid.value] = bufs
        return jid.value

    def trace(self, jid: int) -> dict:
        """The trace buffers of a traced job (device tensors; valid once it is done)."""
        return self._traces[jid]

    def step(self) -> tuple[int, int]:
        a, p = C.c_int32(), C.c_int32()
        check(lib().amh_server_step(self._h, C.byref(a), C.byref(p)))
        return a.value, p.value

    def job(self, jid: int, want_state: bool = False) -> dict:
        import numpy as np
        st = JobStatus()
        out = None
        if want_state:
            Cn, L = self._cfg[jid]
            sb = np.empty((Cn, 2 * L))
            v = np.empty((Cn, 2))
            check(lib().amh_server_job(self._h, jid, C.byref(st), sb.ctypes.data, v.ctypes.data))
            out = {"s_best": sb, "v": v}
        else:
            check(lib().amh_server_job(self._h, jid, C.byref(st), None, None))
        d = st.as_dict()
        if out:
            d.update(out)
        return d

    def close(self) -> None:
        if self._h:
            check(lib().amh_server_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Energy(torch.autograd.Function):
    """V(s) with the hand-written adjoint of amh_grad as its backward."""

    @staticmethod
    def forward(ctx, s, sampler):
        V, g = sampler.grad(s.detach().contiguous())
        ctx.save_for_backward(g)
        return V

    @staticmethod
    def backward(ctx, gV):
        (g,) = ctx.saved_tensors
        return gV[:, None] * g, None


def conformation(s: torch.Tensor, stream=None) -> torch.Tensor:
    """G(s): atoms [B][L][4][3] float32 (N, CA, C, C-beta) of s [B][2L] float64."""
    if not s.is_cuda or s.dtype != torch.float64 or not s.is_contiguous() or s.dim() != 2:
        raise ValueError("s must be a contiguous float64 CUDA tensor [B][2L]")
    B, n = s.shape
    out = torch.empty(B, n // 2, 4, 3, dtype=torch.float32, device=s.device)
    check(lib().amh_conformation(_ptr(s), B, n // 2, _ptr(out), _stream(stream)))
    return out


def philox(ctr: torch.Tensor, key: int, stream=None) -> torch.Tensor:
    """Philox4x32-10 blocks of counters ctr [n][4] (int32 view of uint32) with a 64-bit key."""
    if not ctr.is_cuda or ctr.dtype != torch.int32 or not ctr.is_contiguous():
        raise ValueError("ctr must be a contiguous int32 CUDA tensor [n][4]")
    out = torch.empty_like(ctr)
    check(lib().amh_philox(_ptr(ctr), ctr.shape[0], key, _ptr(out), _stream(stream)))
    return out


def yardsticks(device="cuda:0", table_rows=44850, table_stride=40, max_bin=35, repeats=3) -> dict:
    """Achievable bandwidths of the access patterns of the sweep kernel on this GPU
    (include/amh_yardstick.h): HBM streaming read of 2 GiB, 16-byte gathers from an
    L2-resident table of the given padded shape (the 300-residue distogram by
    default), LDS float4 reads.  Best of `repeats` timed launches each, GB/s."""
    dev = torch.device(device)
    st = torch.cuda.current_stream(dev)
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    out = {}

    def best(fn, nbytes):
        fn()   # warm
        ms = []
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            torch.cuda.synchronize(dev)
            ms.append(e0.elapsed_time(e1))
        return nbytes / (min(ms) * 1e-3) / 1e9, min(ms)

    nf4 = (2 << 30) // 16
    src = torch.ones(nf4 * 4, dtype=torch.float32, device=dev)
    blocks = 16 * n_cu
    sink = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    gbs, ms = best(lambda: check(lib().amh_yard_stream(_ptr(src), nf4, blocks, _ptr(sink), _stream(st))),
                   16 * nf4)
    out["hbm_stream_read"] = {"GB_per_s": gbs, "bytes": 16 * nf4, "ms": ms}
    del src
    table = torch.rand(table_rows * table_stride, dtype=torch.float32, device=dev)
    per_thread, gblocks = 256, 32 * n_cu
    sink = torch.empty(gblocks * 256, dtype=torch.float32, device=dev)
    nbytes = 16 * gblocks * 256 * per_thread
    gbs, ms = best(lambda: check(lib().amh_yard_gather(_ptr(table), table_rows, table_stride, max_bin,
                                                       per_thread, gblocks, _ptr(sink), _stream(st))), nbytes)
    out["l2_gather_16B"] = {"GB_per_s": gbs, "gathers_per_s": gbs * 1e9 / 16,
                            "table_bytes": table_rows * table_stride * 4, "ms": ms}
    lblocks, lper = 2 * n_cu, 4096
    sink = torch.empty(lblocks * 512, dtype=torch.float32, device=dev)
    nbytes = 16 * lblocks * 512 * lper
    gbs, ms = best(lambda: check(lib().amh_yard_lds(lper, lblocks, _ptr(sink), _stream(st))), nbytes)
    out["lds_read_16B"] = {"GB_per_s": gbs, "ms": ms}
    return out

