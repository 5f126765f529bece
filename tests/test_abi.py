"""The C ABI without a GPU: the library loads, exports every declared entry point,
and rejects invalid configurations on the host before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("amh.h", "amh_yardstick.h")]


def declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:amh_status|const char\*)\s+(amh_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def amh():
    from paper_2211_03193_amd import amh
    return amh


def test_library_exports_every_declared_symbol(amh):
    names = declared()
    assert len(names) >= 14
    lib = amh.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_config_struct_layout(amh):
    # the ctypes mirror must match the C layout (static_assert in the library): 120 bytes
    assert C.sizeof(amh.AmhConfig) == 120
    assert amh.AmhConfig.seed.offset == 72 and amh.AmhConfig.chain_offset.offset == 80
    assert amh.AmhConfig.sigma_end.offset == 96 and amh.AmhConfig.cascade_d.offset == 108


def _good():
    import synthetic as sy
    from paper_2211_03193_amd import amh
    return amh.make_config(sy.CFG2)


@pytest.mark.parametrize("field,value", [
    ("L", 1), ("L", 1025), ("n_chains", 0), ("n_bins", 3), ("n_bins", 65), ("window_d", -1),
    ("bin_w", 0.0), ("global_every", -2), ("anchor_every", 0), ("sigma", -0.1),
    ("sigma", float("nan")), ("T0", 0.0), ("T1", -1.0), ("total_sweeps", 0),
    ("total_sweeps", 2**32), ("chains_per_group", 3), ("waves_per_group", 9),
    ("d_min", float("inf")), ("sigma_end", -1.0), ("sigma_end", float("inf")), ("n_cascade", 4),
    ("n_cascade", -1),
])
def test_invalid_config_rejected_on_host(amh, field, value):
    cfg = _good()
    setattr(cfg, field, value)
    h = C.c_void_p()
    st = amh.lib().amh_init(C.byref(cfg), C.c_void_p(16), None, None, C.byref(h))
    assert st == amh.E_INVAL
    assert h.value is None
    assert amh.lib().amh_last_error()


def test_lds_budget_rejected(amh):
    cfg = _good()
    cfg.L, cfg.chains_per_group, cfg.waves_per_group = 1000, 4, 8
    h = C.c_void_p()
    assert amh.lib().amh_init(C.byref(cfg), C.c_void_p(16), None, None, C.byref(h)) == amh.E_INVAL
    assert b"LDS" in amh.lib().amh_last_error()


def test_null_arguments_rejected(amh):
    h = C.c_void_p()
    assert amh.lib().amh_init(None, C.c_void_p(16), None, None, C.byref(h)) == amh.E_INVAL
    cfg = _good()
    assert amh.lib().amh_init(C.byref(cfg), None, None, None, C.byref(h)) == amh.E_INVAL
    assert amh.lib().amh_sweep(None, 1) == amh.E_INVAL
    assert amh.lib().amh_energy(None, None, 1, 0, None, None, None) == amh.E_INVAL
    assert amh.lib().amh_poll(None) == amh.E_INVAL
    assert amh.lib().amh_destroy(None) == amh.OK
    assert amh.lib().amh_conformation(None, 1, 10, None, None) == amh.E_INVAL
    assert amh.lib().amh_philox(None, 4, 0, None, None) == amh.E_INVAL
    assert amh.lib().amh_grad(None, None, 1, None, None) == amh.E_INVAL
    opts = amh.lbfgs_opts()
    assert amh.lib().amh_minimize(None, None, 1, C.byref(opts), None, None, None, None, None) == amh.E_INVAL
    assert amh.lib().amh_minimize_noalloc(None, None, 1, C.byref(opts), None, None, None, None,
                                          None) == amh.E_INVAL


def test_lbfgs_opts_layout(amh):
    assert C.sizeof(amh.LbfgsOpts) == 48 and amh.LbfgsOpts.c1.offset == 16


def test_server_calls_reject_null_arguments(amh):
    assert amh.lib().amh_submit(None, None, None) == amh.E_INVAL
    h = C.c_void_p()
    assert amh.lib().amh_server_create(None, None, C.byref(h)) == amh.E_INVAL
    for bad in (dict(hbm_budget_bytes=0), dict(max_active=0), dict(sweeps_per_round=0), dict(plan=6),
                dict(round_pairs=-1)):
        o = amh.ServerOpts(hbm_budget_bytes=1 << 30, max_active=4, sweeps_per_round=10, plan=0)
        for k, v in bad.items():
            setattr(o, k, v)
        assert amh.lib().amh_server_create(C.byref(o), None, C.byref(h)) == amh.E_INVAL
    assert amh.lib().amh_server_step(None, None, None) == amh.E_INVAL
    st = amh.JobStatus()
    assert amh.lib().amh_server_job(None, 1, C.byref(st), None, None) == amh.E_INVAL
    assert amh.lib().amh_server_destroy(None) == amh.OK
    arr = (C.c_void_p * 1)(None)
    assert amh.lib().amh_batch_create(arr, 1, C.byref(h)) == amh.E_INVAL
    assert amh.lib().amh_batch_create(arr, 0, C.byref(h)) == amh.E_INVAL
    assert amh.lib().amh_batch_sweep(None, 1) == amh.E_INVAL
    assert amh.lib().amh_batch_sweep_each(None, None) == amh.E_INVAL
    assert amh.lib().amh_batch_destroy(None) == amh.OK


def test_server_struct_layouts(amh):
    assert C.sizeof(amh.ServerOpts) == 32 and amh.ServerOpts.round_pairs.offset == 24
    assert C.sizeof(amh.Job) == 120 + 8 + 8 + 8 and amh.Job.target.offset == 128
    assert amh.Job.trace.offset == 136 and C.sizeof(amh.JobTrace) == 56
    assert amh.JobTrace.capacity.offset == 32 and amh.JobTrace.anchor_capacity.offset == 48
    assert C.sizeof(amh.JobStatus) == 72 and amh.JobStatus.best_V.offset == 24


def test_missing_library_fails_loudly(amh, monkeypatch, tmp_path):
    monkeypatch.setattr(amh, "_lib", None)
    monkeypatch.setattr(amh, "LIB_PATH", str(tmp_path / "libamh.so"))
    with pytest.raises(ImportError):
        amh.lib()
