"""Pins of the oracle's random numbers: Philox4x32-10 and the Box-Muller increment.

Philox is pinned against an independent implementation (rocRAND's host-side
engine, compiled from its installed header and run here; no GPU needed) and
by uniformity; the Gaussian increment against the normal law.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference probe")
    exe = str(tmp_path_factory.mktemp("probe") / "probe")
    subprocess.run([hipcc, os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(seed, subseq, count):
        out = subprocess.run([exe, str(seed), str(subseq), str(count)], check=True,
                             capture_output=True, text=True).stdout
        return np.array([list(map(int, l.split())) for l in out.strip().splitlines()],
                        dtype=np.uint64).astype(np.uint32)
    return run


@pytest.mark.parametrize("seed", [0, 0x414D4801, 0x414D4802, 0x0123456789ABCDEF, 2**64 - 1])
@pytest.mark.parametrize("subseq", [0, 7, 0xFFFFFFFF, 0x100000003])
def test_philox_matches_rocrand(rocrand_probe, seed, subseq):
    n = 4096
    ref = rocrand_probe(seed, subseq, n)
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint64).astype(np.uint32)
    ctr[:, 2] = subseq & 0xFFFFFFFF
    ctr[:, 3] = subseq >> 32
    got = oracle.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])
    assert np.array_equal(got, ref)


def test_philox_uniformity():
    n = 1 << 18
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32) % 600
    ctr[:, 1] = np.arange(n, dtype=np.uint32) // 600
    ctr[:, 2] = 17
    x = oracle.philox(ctr, [0x414D4802, 0]).reshape(-1)
    counts = np.bincount(x >> 24, minlength=256)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-3
    # low bits too
    counts = np.bincount(x & 0xFF, minlength=256)
    assert stats.chisquare(counts)[1] > 1e-3


def test_box_muller_increment_is_normal():
    sigma = math.radians(10.0)
    d = np.array([oracle.proposal(0x414D4801, c, t, k, sigma)[0]
                  for c in range(4) for t in range(50) for k in range(128)])
    z = d / sigma
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_accept_uniform_log():
    lu = np.array([oracle.proposal(7, 3, t, k, 0.1)[1] for t in range(40) for k in range(200)])
    u = np.exp(lu)
    assert np.all(lu < 0.0)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_proposal_counter_layout():
    # the increment of (k, t, chain) is fixed by Philox at counter (k, t, chain, 0), key = seed
    seed, chain, t, k, sigma = 0x414D4802, 341, 1234, 577, 0.2
    x = oracle.philox([[k, t, chain, 0]], [seed & 0xFFFFFFFF, seed >> 32])[0].astype(np.float64)
    u = (x + 0.5) / 2.0**32
    delta, lu = oracle.proposal(seed, chain, t, k, sigma)
    assert delta == pytest.approx(sigma * math.sqrt(-2 * math.log(u[0])) * math.cos(2 * math.pi * u[1]), rel=1e-14)
    assert lu == pytest.approx(math.log(u[2]), rel=1e-14)
