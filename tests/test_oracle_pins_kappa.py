"""Pins of the oracle's operator-error metric and of its two condition numbers.

operator_error is the gate of the metric's operator-error bound (per particle
and stencil, |c - c_ref|_2 / |c_ref|_2 over the row): it is pinned by a
hand-worked two-row case, by exact zeros, and by a planted perturbation that it
must report with its size and position.

The condition numbers of the local least-squares problem of
Eq. (GFDM_Definition), kappa_1(R) of the QR factor and kappa_1(G) of the Gram
matrix G = M^T W M, are pinned on particles whose neighbourhood is a symmetric
lattice patch: there the odd moments vanish, G is block diagonal and its
blocks are written here from the moments by symmetry (no QR, no Gram product),
so kappa_1(G) follows from a closed-form inverse and kappa_1(R) from the
Cholesky factor of that G (R is unique up to the signs of its rows, which a
1-norm condition number does not see).  The support weight is the reading of
the oracle (w(q) = (e^{-a q^2} - e^{-a}) / (1 - e^{-a}), a = 8): the paper does
not give it, and these pins take it as an input.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13165_amd import workloads as W


def _w(q, a=oracle.ALPHA_W):
    return (math.exp(-a * q * q) - math.exp(-a)) / (1.0 - math.exp(-a))


def _kappa1(G):
    return np.abs(G).sum(0).max() * np.abs(np.linalg.inv(G)).sum(0).max()


# --------------------------------------------------------------------------- operator error
def test_operator_error_hand_case():
    # row 0: two entries; row 1: one entry.  Stencil columns dx, dy, dz, lap.
    rp = np.array([0, 2, 3])
    ref = np.array([[3.0, 0.0, 1.0, 6.0],
                    [4.0, 0.0, 0.0, 8.0],
                    [2.0, 0.0, -5.0, 0.0]])
    w = ref.copy()
    w[0, 0] += 0.3; w[1, 0] += 0.4          # row 0, dx: |(0.3, 0.4)| / |(3, 4)| = 0.1
    w[1, 3] -= 1.0                          # row 0, lap: 1 / |(6, 8)| = 0.1
    w[0, 1] = 1e-3                          # row 0, dy: reference zero -> absolute norm 1e-3
    w[2, 2] = -5.5                          # row 1, dz: 0.5 / 5 = 0.1
    e = oracle.operator_error(w, ref, rp)
    expect = np.array([[0.1, 1e-3, 0.0, 0.1],
                       [0.0, 0.0, 0.1, 0.0]])
    assert e.shape == (2, 4)
    assert np.allclose(e, expect, rtol=1e-12, atol=1e-15)


def test_operator_error_detects_a_planted_perturbation():
    d = W.plain_cube(n_axis=8)
    rp, col = oracle.neighbours(d)
    w, st, _ = oracle.gfdm_weights(d, rp, col)
    assert np.all(oracle.operator_error(w, w, rp) == 0.0)
    row = 200
    k = rp[row] + 3
    norm = np.linalg.norm(w[rp[row]:rp[row + 1], 3])
    wp = w.copy()
    wp[k, 3] += 2e-6 * norm                 # a 2e-6 relative error in one Laplacian entry
    e = oracle.operator_error(wp, w, rp)
    assert abs(e[row, 3] - 2e-6) < 1e-12
    e[row, 3] = 0.0
    assert np.all(e == 0.0)


# --------------------------------------------------------------------------- condition numbers
def _film_patch(a=1.0):
    # film particle at the origin (normal +z: tangent frame t1 = x, t2 = y) with
    # a 3x3 lattice patch of spacing a around it, h = 3a everywhere
    g = np.array([-a, 0.0, a])
    X, Y = np.meshgrid(g, g, indexing="ij")
    x, y = X.ravel(), Y.ravel()
    n = x.size
    d = dict(x=x, y=y, z=np.zeros(n), h=np.full(n, 3 * a), model=np.ones(n, np.int8),
             kind=np.full(n, 2, np.int8), nx=np.zeros(n), ny=np.zeros(n), nz=np.ones(n))
    centre = int(np.flatnonzero((x == 0) & (y == 0))[0])
    return d, centre


def _film_gram():
    # scaled coordinates U = d/h: axis points at 1/3, diagonal points at (1/3, 1/3)
    s = 1.0 / 3.0
    w1, w2 = _w(s), _w(math.sqrt(2) * s)          # q = |d| / h
    M00 = 1.0 + 4 * w1 + 4 * w2
    M20 = 2 * s ** 2 * w1 + 4 * s ** 2 * w2
    M40 = 2 * s ** 4 * w1 + 4 * s ** 4 * w2
    M22 = 4 * s ** 4 * w2
    # basis [1, U, V, U^2, V^2, UV]: odd moments vanish by symmetry
    G = np.zeros((6, 6))
    G[0, 0] = M00
    G[0, 3] = G[3, 0] = G[0, 4] = G[4, 0] = M20
    G[1, 1] = G[2, 2] = M20
    G[3, 3] = G[4, 4] = M40
    G[3, 4] = G[4, 3] = M22
    G[5, 5] = M22
    return G, (M00, M20, M40, M22)


def test_gram_kappa_film_closed_form():
    d, c = _film_patch()
    rp, col = oracle.neighbours(d)
    assert rp[c + 1] - rp[c] == 9
    kg = oracle.gram_kappa(d, rp, col)[c]
    G, (p, q, r, t) = _film_gram()
    # closed-form inverse of the {1, U^2, V^2} block [[p, q, q], [q, r, t], [q, t, r]]
    # (split into the symmetric pair (U^2 + V^2) and the antisymmetric U^2 - V^2)
    D = p * (r + t) - 2 * q * q
    b11, b12 = (r + t) / D, -q / D
    b22, b23 = p / (2 * D) + 1 / (2 * (r - t)), p / (2 * D) - 1 / (2 * (r - t))
    norm_g = max(p + 2 * q, q, q + r + t, t)
    norm_inv = max(abs(b11) + 2 * abs(b12), abs(b12) + abs(b22) + abs(b23), 1 / q, 1 / t)
    closed = norm_g * norm_inv
    assert abs(kg - closed) <= 1e-12 * closed
    assert abs(closed - _kappa1(G)) <= 1e-10 * closed
    # kappa_1(R): R is the Cholesky factor of G up to row signs
    R = np.linalg.cholesky(G).T
    kr = oracle.gfdm_weights(d, rp, col)[2][c]
    assert abs(kr - _kappa1(R)) <= 1e-10 * kr
    # the two are different quantities: a planted swap would show
    assert kg > 1.5 * kr


def test_gram_kappa_3d_lattice_closed_form():
    # 3x3x3 lattice patch around a 3D particle, spacing 1, h = 3 (all 26 within the support)
    g = np.array([-1.0, 0.0, 1.0])
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    n = x.size
    d = dict(x=x, y=y, z=z, h=np.full(n, 3.0), model=np.zeros(n, np.int8), kind=np.zeros(n, np.int8),
             nx=np.zeros(n), ny=np.zeros(n), nz=np.zeros(n))
    c = int(np.flatnonzero((x == 0) & (y == 0) & (z == 0))[0])
    rp, col = oracle.neighbours(d)
    assert rp[c + 1] - rp[c] == 27
    s = 1.0 / 3.0
    w1, w2, w3 = _w(s), _w(math.sqrt(2) * s), _w(math.sqrt(3) * s)
    # moments sum w X^a Y^b Z^c by symmetry: 6 axis, 12 face-diagonal, 8 corner neighbours
    M0 = 1 + 6 * w1 + 12 * w2 + 8 * w3
    M2 = s ** 2 * (2 * w1 + 8 * w2 + 8 * w3)       # sum w X^2
    M4 = s ** 4 * (2 * w1 + 8 * w2 + 8 * w3)       # sum w X^4
    M22 = s ** 4 * (4 * w2 + 8 * w3)               # sum w X^2 Y^2
    # basis [1, X, Y, Z, X^2, Y^2, Z^2, XY, XZ, YZ]
    G = np.zeros((10, 10))
    G[0, 0] = M0
    for a in (4, 5, 6):
        G[0, a] = G[a, 0] = M2
        G[a, a] = M4
        for b in (4, 5, 6):
            if b != a:
                G[a, b] = M22
    for a in (1, 2, 3):
        G[a, a] = M2
    for a in (7, 8, 9):
        G[a, a] = M22
    kg = oracle.gram_kappa(d, rp, col)[c]
    assert abs(kg - _kappa1(G)) <= 1e-10 * kg
    kr = oracle.gfdm_weights(d, rp, col)[2][c]
    assert abs(kr - _kappa1(np.linalg.cholesky(G).T)) <= 1e-10 * kr


def test_gram_kappa_invariances_and_degenerate_rows():
    d = W.plain_cube(n_axis=7)
    rp, col = oracle.neighbours(d)
    k0 = oracle.gram_kappa(d, rp, col)
    assert np.all(np.isfinite(k0)) and np.all(k0 >= 1.0)
    # translation and uniform scaling (positions and supports together) leave the
    # scaled local problem unchanged
    q = dict(d)
    q["x"], q["y"], q["z"], q["h"] = 3.0 * d["x"] + 5.0, 3.0 * d["y"] - 2.0, 3.0 * d["z"] + 1.0, 3.0 * d["h"]
    assert np.allclose(oracle.gram_kappa(q, rp, col), k0, rtol=1e-9)
    # fewer neighbours than monomials -> 0; an exactly coplanar 3D row -> inf
    z = dict(x=np.array([0.0, 1.0, 0.0, 1.0, 0.5, 0.2, 0.8, 0.3, 0.6, 0.9, 0.1]),
             y=np.array([0.0, 0.0, 1.0, 1.0, 0.5, 0.7, 0.3, 0.1, 0.9, 0.6, 0.4]))
    m = z["x"].size
    z.update(z=np.zeros(m), h=np.full(m, 4.0), model=np.zeros(m, np.int8), kind=np.zeros(m, np.int8),
             nx=np.zeros(m), ny=np.zeros(m), nz=np.zeros(m))
    rpz, colz = oracle.neighbours(z)
    assert np.all(np.diff(rpz) == m)
    assert np.all(np.isinf(oracle.gram_kappa(z, rpz, colz)))
    few = {k: (v[:5] if isinstance(v, np.ndarray) else v) for k, v in z.items()}
    rpf, colf = oracle.neighbours(few)
    assert np.all(oracle.gram_kappa(few, rpf, colf) == 0.0)
