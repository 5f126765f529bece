"""Seeded synthetic inputs for the Alternating Metropolis-Hastings (AMH) sampler.

This module is the only code that both the FP64 oracle (``oracle/``) and the HIP
path (``paper_2211_03193_amd/``) receive data from.  It holds random draws and the
synthetic-workload recipe only; none of the sampler's arithmetic (geometry,
spline energy, proposals, Metropolis rule) lives here.  Reference distances are
an *input* to :func:`distogram`: callers obtain them from whichever side they
are exercising (the oracle in tests, the library's conformation call on the
device in the benchmark).

The paper evaluates on AlphaFold1 CASP13 distograms (Sec. 2.3, Eq. of the
distogram energy), which are not available; the recipe below stands in for them
with the same shapes:

* reference torsions per residue from a Ramachandran-like Gaussian mixture
  (alpha_R (-63, -43) deg w=0.55, beta (-120, 130) w=0.40, alpha_L (57, 47)
  w=0.05, each angle N(mu, 15 deg));
* per residue pair a 37-bin distogram: 36 bins of 0.5 A over [2, 20) plus a
  no-contact bin, knots at bin centres 2.25 + 0.5 b (the no-contact knot at
  20.25); p = (1-eps) softmax(-(c_b - d*)^2 / 2) + eps q with
  q ~ Dirichlet(0.5 * 1_37) and d* the reference C-beta distance; the table
  handed to the sampler is y = -ln p.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

__all__ = [
    "N_BINS", "D_MIN", "BIN_W", "bin_knots", "n_pairs", "pair_index",
    "reference_torsions", "dirichlet_log_noise", "distogram",
    "pair_distances", "Workload", "CFG1", "CFG2", "CFG1_SMALL", "workload",
    "batch_lengths", "poisson_arrivals", "random_torsions",
]

N_BINS = 37
D_MIN = 2.0
BIN_W = 0.5

# Ramachandran-like mixture: (weight, mu_phi deg, mu_psi deg)
_RAMA = ((0.55, -63.0, -43.0), (0.40, -120.0, 130.0), (0.05, 57.0, 47.0))
_RAMA_SD_DEG = 15.0


def bin_knots(n_bins: int = N_BINS, d_min: float = D_MIN, bin_w: float = BIN_W) -> np.ndarray:
    """Knot positions (bin centres) in Angstrom; the last bin is no-contact."""
    return d_min + bin_w * (np.arange(n_bins, dtype=np.float64) + 0.5)


def n_pairs(L: int) -> int:
    return L * (L - 1) // 2


def pair_index(L: int) -> tuple[np.ndarray, np.ndarray]:
    """(i, j) of every packed row, i < j, row r(i,j) = i*L - i*(i+1)/2 + (j-i-1)."""
    i, j = np.triu_indices(L, k=1)
    return i.astype(np.int64), j.astype(np.int64)


def _wrap(a: np.ndarray) -> np.ndarray:
    """Wrap angles to (-pi, pi]."""
    w = np.mod(a + np.pi, 2.0 * np.pi) - np.pi
    w[w <= -np.pi] += 2.0 * np.pi
    return w


def reference_torsions(L: int, seed: int) -> np.ndarray:
    """Seeded reference torsions s_ref[2L] (radians): s[2c]=phi_c, s[2c+1]=psi_c."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.array([m[0] for m in _RAMA])
    comp = rng.choice(len(_RAMA), size=L, p=w / w.sum())
    mu = np.radians(np.array([[m[1], m[2]] for m in _RAMA]))[comp]  # [L,2]
    s = mu + np.radians(_RAMA_SD_DEG) * rng.standard_normal((L, 2))
    return _wrap(s.reshape(-1))


def random_torsions(shape, seed: int) -> np.ndarray:
    """Uniform torsions on (-pi, pi] (for invariance tests and random starts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _wrap(rng.uniform(-np.pi, np.pi, size=shape))


def dirichlet_log_noise(P: int, n_bins: int, seed: int, alpha: float = 0.5) -> np.ndarray:
    """log q for q ~ Dirichlet(alpha * 1) per row, [P][n_bins] float64.

    Drawn as normalised Gamma(alpha) variates; returned in log space so that
    components far below double precision's normal range stay finite.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_gamma(alpha, size=(P, n_bins))
    g = np.maximum(g, np.finfo(np.float64).tiny)
    lg = np.log(g)
    m = lg.max(axis=1, keepdims=True)
    return lg - (m + np.log(np.exp(lg - m).sum(axis=1, keepdims=True)))


def distogram(d_star: np.ndarray, eps: float, noise_seed: int, n_bins: int = N_BINS,
              d_min: float = D_MIN, bin_w: float = BIN_W) -> np.ndarray:
    """Synthetic -ln p table [P][n_bins] (float64) around reference distances d_star[P].

    p = (1-eps) * softmax(-(c_b - d*)^2/2) + eps * q, computed in log space.
    With eps == 0 the table is exactly (c_b - d*)^2/2 + log Z, a quadratic in the
    knot position, which the invariant tests rely on.
    """
    d_star = np.asarray(d_star, dtype=np.float64)
    c = bin_knots(n_bins, d_min, bin_w)
    logit = -0.5 * (c[None, :] - d_star[:, None]) ** 2
    m = logit.max(axis=1, keepdims=True)
    log_g = logit - (m + np.log(np.exp(logit - m).sum(axis=1, keepdims=True)))
    if eps == 0.0:
        return -log_g
    log_q = dirichlet_log_noise(d_star.shape[0], n_bins, noise_seed)
    log_p = np.logaddexp(math.log1p(-eps) + log_g, math.log(eps) + log_q)
    return -log_p


def pair_distances(cb: np.ndarray) -> np.ndarray:
    """Packed i<j distances between rows of cb[L][3] (any float dtype -> float64)."""
    cb = np.asarray(cb, dtype=np.float64)
    i, j = pair_index(cb.shape[0])
    return np.sqrt(((cb[j] - cb[i]) ** 2).sum(axis=1))


@dataclass
class Workload:
    """One AMH run configuration (radians, Angstrom, nats)."""
    name: str
    L: int
    n_chains: int
    total_sweeps: int
    window_d: int
    global_every: int = 10
    sigma_deg: float = 10.0
    T0: float = 1.0
    T1: float = 0.01
    seed: int = 0x414D4801        # Philox key
    protein_seed: int = 1         # reference torsions
    noise_seed: int = 101         # Dirichlet noise
    eps: float = 0.1
    n_bins: int = N_BINS
    d_min: float = D_MIN
    bin_w: float = BIN_W
    anchor_every: int = 0         # 0 -> same as global_every (or 10 when local-only)
    trace_chains: list = field(default_factory=list)
    sigma_end_deg: float = 0.0    # > 0: proposal width decays geometrically to this
    n_global: int = 1             # global sweeps per cycle of global_every (the last ones)
    cascade: tuple = ()           # extra localization radii taken in turn with window_d

    @property
    def sigma(self) -> float:
        return math.radians(self.sigma_deg)

    @property
    def anchor_period(self) -> int:
        if self.anchor_every > 0:
            return self.anchor_every
        return self.global_every if self.global_every > 0 else 10

    def replace(self, **kw) -> "Workload":
        d = asdict(self)
        d.update(kw)
        return Workload(**d)


# One synthetic protein, L=64, one chain, 2e4 sweeps, window 8, global every 10.
CFG1 = Workload("plain-L64-1chain", L=64, n_chains=1, total_sweeps=20000, window_d=8,
                seed=0x414D4801, protein_seed=1, noise_seed=101, trace_chains=[0])
# One protein at scale: L=300, 1024 chains, window 12, 5e3 sweeps, 4 sampled chains.
CFG2 = Workload("single-L300-1024chains", L=300, n_chains=1024, total_sweeps=5000, window_d=12,
                seed=0x414D4802, protein_seed=2, noise_seed=102,
                trace_chains=[0, 341, 682, 1023])
# A reduced twin of CFG1 that the oracle finishes in well under a second.
CFG1_SMALL = CFG1.replace(name="plain-L64-1chain-200sweeps", total_sweeps=200)


def workload(w: Workload, d_star_fn) -> tuple[np.ndarray, np.ndarray]:
    """(s_ref, y) for a workload; d_star_fn(s_ref) -> packed reference distances."""
    s_ref = reference_torsions(w.L, w.protein_seed)
    y = distogram(d_star_fn(s_ref), w.eps, w.noise_seed, w.n_bins, w.d_min, w.bin_w)
    return s_ref, y


def batch_lengths(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Protein lengths uniform on [lo, hi] (ragged batches)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=n)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given mean rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def batch_workloads(n: int = 64, lo: int = 50, hi: int = 600, chains: int = 256,
                    sweeps: int = 5000, seed: int = 0x414D4803) -> list[Workload]:
    """Ragged batch of proteins (lengths uniform on [lo, hi]), each with its own
    protein/noise seeds and its own Philox key, window 12, global every 10 sweeps."""
    Ls = batch_lengths(n, lo, hi, seed)
    return [Workload(f"batch{i:02d}-L{int(L)}", L=int(L), n_chains=chains, total_sweeps=sweeps,
                     window_d=12, seed=(seed << 16) + i, protein_seed=1000 + i,
                     noise_seed=2000 + i) for i, L in enumerate(Ls)]
