"""Pins of the oracle's L-BFGS (the minimiser the paper pairs with its sampler).

The two-loop recursion is checked against the dense BFGS inverse-Hessian update
it stands for; the minimiser against closed-form minima (a quadratic, the
Rosenbrock valley, and the noise-free synthetic protein whose reference
conformation is an exact minimum of V); the line search against the Armijo rule
it states.
"""
import numpy as np
import pytest

import oracle
import synthetic as sy


def _dense_bfgs(S, Y, gamma):
    n = S.shape[1]
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("k", [0, 1, 3, 7])
def test_two_loop_equals_dense_bfgs_update(k):
    rng = np.random.default_rng(k)
    n = 9
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    S = rng.standard_normal((k, n))
    Y = S @ A.T + 0.1 * rng.standard_normal((k, n))     # s.y > 0 for these
    assert np.all(np.einsum("ij,ij->i", S, Y) > 0)
    g = rng.standard_normal(n)
    gamma = 0.37
    d = oracle.lbfgs_direction(S, Y, g, gamma)
    ref = -_dense_bfgs(S, Y, gamma) @ g
    assert np.allclose(d, ref, rtol=1e-12, atol=1e-12)


def _armijo_trace_ok(tr, M):
    """Each accepted value lies at or below the largest of the previous M (the Armijo
    term is negative, but it can round away next to a minimum)."""
    for i in range(1, len(tr)):
        ref = max(tr[max(0, i - M):i])
        if not tr[i] <= ref:
            return False
    return True


@pytest.mark.parametrize("M", [1, 5])
def test_quadratic_reaches_closed_form_minimum(M):
    rng = np.random.default_rng(3)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + np.eye(n)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    fs = -0.5 * b @ xs
    x, f, it, st, tr = oracle.lbfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(n),
                                    oracle.lbfgs_opts(n_iter=500, m=8, nonmonotone=M, gtol=1e-7))
    assert st == 0
    assert np.allclose(x, xs, atol=1e-6)
    assert f == pytest.approx(fs, rel=1e-12)
    assert _armijo_trace_ok(tr, M)
    if M == 1:
        assert np.all(np.diff(tr) <= 0)


def test_rosenbrock_valley():
    def fg(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        return f, np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
    x, f, it, st, tr = oracle.lbfgs(fg, np.array([-1.2, 1.0]),
                                    oracle.lbfgs_opts(n_iter=1000, m=5, nonmonotone=1, gtol=1e-9,
                                                      step0=1.0))
    assert st == 0
    assert np.allclose(x, [1.0, 1.0], atol=1e-6)
    assert f < 1e-12


def test_zero_iterations_and_converged_start():
    A = np.eye(3)
    x, f, it, st, tr = oracle.lbfgs(lambda x: (0.5 * x @ A @ x, A @ x), np.zeros(3))
    assert (it, st) == (0, 0) and f == 0.0
    x, f, it, st, tr = oracle.lbfgs(lambda x: (0.5 * x @ A @ x, A @ x), np.ones(3),
                                    oracle.lbfgs_opts(n_iter=0))
    assert (it, st) == (0, 1) and f == 1.5


@pytest.fixture(scope="module")
def exact_small():
    """Noise-free (eps = 0) synthetic protein whose reference torsions are an
    exact minimum of V: pairs outside the band where the spline reproduces the
    quadratic get flat rows (the same construction as the energy-minimum pin)."""
    L = 24
    s_ref = sy.reference_torsions(L, 4)
    dstar = sy.pair_distances(oracle.cb(s_ref))
    y = sy.distogram(dstar, 0.0, 0)
    exact = (dstar >= 2.75) & ~((dstar > 19.75) & (dstar < 20.25))
    y[~exact] = 0.0
    cfg = oracle.make_cfg(sy.CFG1.replace(L=L))
    return cfg, y, s_ref


@pytest.mark.parametrize("M", [1, 5])
def test_protein_returns_to_exact_minimum(exact_small, M):
    cfg, y, s_ref = exact_small
    V_ref = oracle.energy(cfg, y, s_ref)
    rng = np.random.default_rng(11)
    s0 = s_ref + 0.03 * rng.standard_normal(s_ref.size)
    V0 = oracle.energy(cfg, y, s0)
    s, V, it, st, tr = oracle.lbfgs_protein(cfg, y, s0,
                                            oracle.lbfgs_opts(n_iter=2500, nonmonotone=M, gtol=1e-7))
    assert V0 > V_ref + 1.0
    assert V - V_ref < 1e-9 * V_ref
    assert V == pytest.approx(oracle.energy(cfg, y, s), rel=1e-12)
    assert np.all(np.abs(s) <= np.pi)
    assert tr[0] == pytest.approx(V0, rel=1e-14)
    assert _armijo_trace_ok(tr, M)
    # V is a function of the Cbeta distances only: the reached conformation matches
    # the reference up to a rigid motion
    d_ref = sy.pair_distances(oracle.cb(s_ref))
    d = sy.pair_distances(oracle.cb(s))
    assert np.abs(d - d_ref).max() < 1e-4


def test_protein_status_and_trace_length():
    w = sy.CFG1.replace(L=16)
    s_ref = sy.reference_torsions(w.L, 2)
    y = sy.distogram(sy.pair_distances(oracle.cb(s_ref)), 0.1, 3)
    cfg = oracle.make_cfg(w)
    s0 = sy.random_torsions(2 * w.L, 5)
    s, V, it, st, tr = oracle.lbfgs_protein(cfg, y, s0, oracle.lbfgs_opts(n_iter=7))
    assert st == 1 and it == 7 and len(tr) == 8
    assert V == pytest.approx(tr[-1]) and V < tr[0]


def test_replay_accepts_its_own_iterates_and_catches_a_planted_step():
    w = sy.CFG1.replace(L=20)
    s_ref = sy.reference_torsions(w.L, 6)
    y = sy.distogram(sy.pair_distances(oracle.cb(s_ref)), 0.1, 7)
    cfg = oracle.make_cfg(w)
    opts = oracle.lbfgs_opts(n_iter=30)
    s, V, it, st, tr, X = oracle.lbfgs_protein(cfg, y, sy.random_torsions(2 * w.L, 8), opts,
                                               iterates=True)
    assert X.shape == (it + 1, 2 * w.L) and it == 30
    assert tr[-1] == pytest.approx(oracle.energy(cfg, y, X[-1]), rel=1e-14)
    rc, rep = oracle.lbfgs_replay(cfg, y, X, opts)
    assert rc == 0 and rep["n_steps"] == it and rep["n_fail"] == 0 and rep["n_forks"] == 0
    assert rep["max_step_err"] < 1e-10         # only the rounding of x + a d remains
    # a wrong step (a small error in one coordinate of one iterate) is caught there
    Xb = X.copy()
    Xb[12, 5] += 1e-4 * np.abs(X[12] - X[11]).max()
    rc, rep = oracle.lbfgs_replay(cfg, y, Xb, opts)
    assert rc == 1 and rep["first_fail"] == 11
    # so is a step taken at another trial length without a near-tie
    Xc = X.copy()
    Xc[8:] += -0.5 * (X[8] - X[7])
    rc, rep = oracle.lbfgs_replay(cfg, y, Xc, opts)
    assert rc == 1 and rep["first_fail"] == 7
