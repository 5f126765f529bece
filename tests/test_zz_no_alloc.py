"""amh_minimize_noalloc (the L-BFGS entry point whose workspace is the library's
fixed scratch array) against amh_minimize, both called through the C ABI.

The two share the kernel and its fixed-order reductions, so their outputs must be
identical: final torsions, V, iteration counts, stop codes and value traces, on
consecutive calls that reuse the scratch with a smaller input each time, and for
the context's own chains.  Sizes beyond the scratch are rejected on the host.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synthetic as sy

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402  (an import error fails the run)
from paper_2211_03193_amd import amh  # noqa: E402

SCRATCH_DOUBLES = 8 << 20


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _call(fn_name, ctx, s, B, opts, n_iter):
    d = gu.DEV
    out = {"V": torch.full((B,), float("nan"), dtype=torch.float64, device=d),
           "iters": torch.full((B,), -7, dtype=torch.int32, device=d),
           "status": torch.full((B,), -7, dtype=torch.int32, device=d),
           "trace": torch.full((B, n_iter + 1), float("nan"), dtype=torch.float64, device=d)}
    fn = getattr(amh.lib(), fn_name)
    st = fn(ctx._h, None if s is None else C.c_void_p(s.data_ptr()), B, C.byref(opts),
            C.c_void_p(out["V"].data_ptr()), C.c_void_p(out["iters"].data_ptr()),
            C.c_void_p(out["status"].data_ptr()), C.c_void_p(out["trace"].data_ptr()), None)
    amh.check(st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    for k in ("V", "iters", "status", "trace"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def _starts(w, s_ref, B, seed):
    rng = np.random.default_rng(seed)
    s = s_ref[None, :] + 0.3 * rng.standard_normal((B, 2 * w.L))
    s[: B // 2] = np.stack([sy.random_torsions(2 * w.L, seed + b) for b in range(B // 2)])
    return torch.from_numpy(np.ascontiguousarray(s)).to(gu.DEV)


def test_noalloc_equals_minimize_on_consecutive_calls():
    n_iter = 60
    opts = amh.lbfgs_opts(n_iter=n_iter)
    cases = [(64, 40), (64, 12), (24, 8)]   # each call smaller than the one before
    ctxs = {}
    for L, B in cases:
        gu.say("minimize_noalloc vs minimize: L", L, "B", B)
        w = sy.CFG1.replace(L=L, n_chains=2, protein_seed=L + 11, noise_seed=L + 12)
        if L not in ctxs:
            s_ref, y = gu.protein(w)
            ctxs[L] = (gu.context(w, y), s_ref)
        ctx, s_ref = ctxs[L]
        s0 = _starts(w, s_ref, B, 100 * L + B)
        s_a, s_b = s0.clone(), s0.clone()
        ra = _call("amh_minimize_noalloc", ctx, s_a, B, opts, n_iter)
        rb = _call("amh_minimize", ctx, s_b, B, opts, n_iter)
        _same(ra, rb)
        assert torch.equal(s_a, s_b)
        assert np.all(ra["iters"] >= 1) and np.all(np.isfinite(ra["V"]))
        assert np.all(ra["V"] <= ra["trace"][:, 0])
    for ctx, _ in ctxs.values():
        ctx.close()


def test_noalloc_on_context_chains():
    gu.say("minimize_noalloc on the context's chains")
    n_iter = 40
    opts = amh.lbfgs_opts(n_iter=n_iter)
    w = sy.CFG1.replace(L=48, n_chains=6, total_sweeps=40, global_every=5)
    _, y = gu.protein(w)
    a, b = gu.context(w, y), gu.context(w, y)
    a.sweep(10)
    b.sweep(10)
    for rnd in range(2):
        ra = _call("amh_minimize_noalloc", a, None, w.n_chains, opts, n_iter)
        rb = _call("amh_minimize", b, None, w.n_chains, opts, n_iter)
        _same(ra, rb)
        sa, sb = a.get_state(), b.get_state()
        for k in ("s", "s_best", "v", "atoms"):
            assert torch.equal(sa[k], sb[k]), (rnd, k)
        a.sweep(5)
        b.sweep(5)
    a.close()
    b.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    gu.say("minimize_noalloc size limit")
    w = sy.CFG1.replace(L=64, n_chains=1)
    _, y = gu.protein(w)
    ctx = gu.context(w, y)
    m = 64
    per = (5 + 2 * m) * 2 * w.L
    B_max = SCRATCH_DOUBLES // per
    s = torch.zeros(B_max + 1, 2 * w.L, dtype=torch.float64, device=gu.DEV)
    opts = amh.lbfgs_opts(n_iter=1, m=m)
    V = torch.full((B_max + 1,), -1.0, dtype=torch.float64, device=gu.DEV)
    st = amh.lib().amh_minimize_noalloc(ctx._h, C.c_void_p(s.data_ptr()), B_max + 1, C.byref(opts),
                                        C.c_void_p(V.data_ptr()), None, None, None, None)
    assert st == amh.E_INVAL
    assert b"scratch" in amh.lib().amh_last_error()
    torch.cuda.synchronize()
    assert torch.all(V == -1.0)   # nothing was launched
    # the largest size that fits runs
    r = _call("amh_minimize_noalloc", ctx, s[:B_max].clone(), B_max, opts, 1)
    assert np.all(np.isfinite(r["V"]))
    ctx.close()
