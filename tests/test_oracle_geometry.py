"""Pins of the oracle's geometry x = G(s) (NeRF chain, virtual C-beta).

Checked against what geometry fixes independently of the construction:
recomputed bond lengths, bond angles and dihedrals, planarity of the extended
chain, screw symmetry of constant torsions, the handedness and CA-CA spacing of
the alpha helix, and the rigid motion of everything past a turned bond.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as sy

B_NCA, B_CAC, B_CN, B_CACB = 1.458, 1.525, 1.329, 1.53
A_NCAC, A_CACN, A_CNCA, A_NCACB = 111.2, 116.2, 121.7, 110.5
T_CB = -122.5


def dihedral(a, b, c, d):
    """Signed dihedral (deg) by the atan2 formula, IUPAC sign convention."""
    b0, b1, b2 = a - b, c - b, d - c
    b1n = b1 / np.linalg.norm(b1)
    v = b0 - np.dot(b0, b1n) * b1n
    w = b2 - np.dot(b2, b1n) * b1n
    return math.degrees(math.atan2(np.dot(np.cross(b1n, v), w), np.dot(v, w)))


def angle(a, b, c):
    u, v = a - b, c - b
    return math.degrees(math.acos(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v)))


def wrapdeg(x):
    return (x + 180.0) % 360.0 - 180.0


def test_constants_table():
    g = oracle.geometry_constants()
    assert np.allclose(g, [B_NCA, B_CAC, B_CN, B_CACB, A_NCAC, A_CACN, A_CNCA, A_NCACB, 180.0, T_CB])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_internal_coordinates_recovered(seed):
    L = 40
    s = sy.random_torsions(2 * L, seed)
    at = oracle.nerf(s)
    N, CA, C, CB = at[:, 0], at[:, 1], at[:, 2], at[:, 3]
    for c in range(L):
        assert np.linalg.norm(CA[c] - N[c]) == pytest.approx(B_NCA, abs=1e-12)
        assert np.linalg.norm(C[c] - CA[c]) == pytest.approx(B_CAC, abs=1e-12)
        assert np.linalg.norm(CB[c] - CA[c]) == pytest.approx(B_CACB, abs=1e-12)
        assert angle(N[c], CA[c], C[c]) == pytest.approx(A_NCAC, abs=1e-9)
        assert angle(N[c], CA[c], CB[c]) == pytest.approx(A_NCACB, abs=1e-9)
        assert dihedral(C[c], N[c], CA[c], CB[c]) == pytest.approx(T_CB, abs=1e-9)
        if c + 1 < L:
            assert np.linalg.norm(N[c + 1] - C[c]) == pytest.approx(B_CN, abs=1e-12)
            assert angle(CA[c], C[c], N[c + 1]) == pytest.approx(A_CACN, abs=1e-9)
            assert angle(C[c], N[c + 1], CA[c + 1]) == pytest.approx(A_CNCA, abs=1e-9)
            psi = dihedral(N[c], CA[c], C[c], N[c + 1])
            omega = dihedral(CA[c], C[c], N[c + 1], CA[c + 1])
            phi = dihedral(C[c], N[c + 1], CA[c + 1], C[c + 1])
            assert wrapdeg(psi - math.degrees(s[2 * c + 1])) == pytest.approx(0.0, abs=1e-8)
            assert wrapdeg(omega - 180.0) == pytest.approx(0.0, abs=1e-8)
            assert wrapdeg(phi - math.degrees(s[2 * c + 2])) == pytest.approx(0.0, abs=1e-8)


def test_extended_chain_is_planar():
    at = oracle.nerf(np.full(2 * 30, math.pi))
    assert np.abs(at[:, :3, 2]).max() < 1e-12       # backbone in the xy-plane
    assert np.abs(at[:, 3, 2]).min() > 1.0          # C-beta off the plane


def test_dead_torsions_move_nothing():
    L = 12
    s = sy.random_torsions(2 * L, 5)
    a0 = oracle.nerf(s)
    for k in (0, 2 * L - 1):
        s2 = s.copy()
        s2[k] += 0.7
        assert np.array_equal(oracle.nerf(s2), a0)


@pytest.mark.parametrize("phi,psi", [(-57.0, -47.0), (-120.0, 130.0), (60.0, 45.0)])
def test_screw_symmetry(phi, psi):
    L = 30
    s = np.radians(np.tile([phi, psi], L))
    cb = oracle.cb(s)
    for m in (1, 2, 3, 5, 8):
        d = np.linalg.norm(cb[m:] - cb[:-m], axis=1)
        assert np.ptp(d[1:-1]) < 1e-9


def test_alpha_helix_right_handed():
    L = 20
    at = oracle.nerf(np.radians(np.tile([-57.0, -47.0], L)))
    ca = at[:, 1]
    assert np.linalg.norm(ca[1] - ca[0]) == pytest.approx(3.80, abs=0.01)
    v = np.diff(ca, axis=0)
    triple = np.einsum("ij,ij->i", np.cross(v[:-2], v[1:-1]), v[2:])
    assert np.all(triple > 0.0)                      # right-handed
    # 3.6 residues per turn: CA(i)-CA(i+4) is short (about 6.2 A), CA(i)-CA(i+2) about 5.4 A
    assert np.linalg.norm(ca[8] - ca[4]) < 6.5


def rodrigues(x, a, u, t):
    v = x - a
    return a + v * math.cos(t) + np.cross(u, v) * math.sin(t) + np.outer(np.dot(v, u), u) * (1 - math.cos(t))


@pytest.mark.parametrize("k", [1, 2, 7, 10, 17, 22])
def test_turning_a_torsion_is_a_rigid_rotation(k):
    """Turning s_k by delta rotates every atom past the bond about the bond axis
    by +delta and leaves the rest fixed (Sec. 2.4, proposal generation)."""
    L = 12
    s = sy.random_torsions(2 * L, 11)
    delta = 0.37
    a0 = oracle.nerf(s)
    s2 = s.copy()
    s2[k] += delta
    a1 = oracle.nerf(s2)
    c = k // 2
    flat0 = a0.reshape(-1, 3)
    if k % 2 == 0:      # phi_c: axis N_c -> CA_c, moves C_c, CB_c and residues > c
        A, B = a0[c, 0], a0[c, 1]
        moved = [(c, 2), (c, 3)] + [(r, a) for r in range(c + 1, L) for a in range(4)]
    else:               # psi_c: axis CA_c -> C_c, moves residues > c
        A, B = a0[c, 1], a0[c, 2]
        moved = [(r, a) for r in range(c + 1, L) for a in range(4)]
    u = (B - A) / np.linalg.norm(B - A)
    idx = [r * 4 + a for r, a in moved]
    rot = rodrigues(flat0[idx], A, u, delta)
    assert np.allclose(a1.reshape(-1, 3)[idx], rot, atol=1e-10)
    fixed = sorted(set(range(4 * L)) - set(idx))
    assert np.array_equal(a1.reshape(-1, 3)[fixed], flat0[fixed])


def test_rotating_preceding_side_gives_same_distances():
    L = 10
    s = sy.random_torsions(2 * L, 3)
    at = oracle.nerf(s)
    k, delta = 9, -0.6                           # psi_4
    c = k // 2
    A, B = at[c, 1], at[c, 2]
    u = (B - A) / np.linalg.norm(B - A)
    cb = at[:, 3].copy()
    down = cb.copy()
    down[c + 1:] = rodrigues(cb[c + 1:], A, u, delta)
    up = cb.copy()
    up[:c + 1] = rodrigues(cb[:c + 1], A, u, -delta)
    d1 = np.linalg.norm(down[:, None] - down[None], axis=2)
    d2 = np.linalg.norm(up[:, None] - up[None], axis=2)
    assert np.allclose(d1, d2, atol=1e-10)
    d3 = np.linalg.norm(oracle.cb(np.where(np.arange(2 * L) == k, s + delta, s))[:, None]
                        - oracle.cb(np.where(np.arange(2 * L) == k, s + delta, s))[None], axis=2)
    assert np.allclose(d1, d3, atol=1e-10)
