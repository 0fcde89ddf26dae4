"""Pins of the oracle for the coupling layer: the film height of the droplet
model (Eq. Height), the 2D->3D transition (Sec. 5.2, Eq. psi~, Eq. gamma,
Alg. 4), the ghost particles of the buffer zone (Sec. 6.1, Alg. 5) and
derivatives and implicit solves over extended neighbourhoods (Sec. 6.2).

Each check rests on something other than the oracle's own code: closed forms
(the droplet kernel integrates to the droplet volume), hand-worked examples,
brute-force pair tests, conservation laws, the exactness of second-order
stencils, and the equivalence of two formulations of the implicit split.
"""
import numpy as np
import pytest

import oracle
from paper_2405_13165_amd import workloads as W


def _film_lattice(m, s, hfun, dfun):
    jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    x = (ii.ravel() + 0.5) * s
    y = (jj.ravel() + 0.5) * s
    n = x.size
    p = dict(x=x, y=y, z=np.zeros(n), h=hfun(x, y), model=np.ones(n, np.int8),
             kind=np.full(n, 2, np.int8), nx=np.zeros(n), ny=np.zeros(n), nz=np.ones(n))
    return p, dfun(x, y)


# --------------------------------------------------------------------------- Eq. (Height)
def test_film_height_isolated_droplet():
    # one droplet alone in its support: H = alpha/(pi h^2) * pi d^3/6
    p = dict(x=np.array([0.0, 10.0]), y=np.zeros(2), z=np.zeros(2), h=np.array([0.5, 0.25]),
             model=np.ones(2, np.int8), kind=np.full(2, 2, np.int8), nx=np.zeros(2),
             ny=np.zeros(2), nz=np.ones(2))
    rp, col = oracle.neighbours(p)
    d = np.array([0.1, 0.2])
    for alpha in (3.0, 8.0):
        H = oracle.film_height(p, rp, col, d, alpha)
        expect = alpha * d ** 3 / (6.0 * p["h"] ** 2)
        assert np.allclose(H, expect, rtol=1e-15, atol=0)


def test_film_height_integrates_to_droplet_volume():
    # The kernel of droplet j, alpha/(pi h_j^2) exp(-alpha r^2/h_j^2), has unit
    # integral over the plane, so on a lattice of spacing s the heights carry
    # the droplet volumes: s^2 sum_i H_i = sum_j V_j when every droplet's
    # kernel lies well inside the lattice.  h varies by 50% across the patch,
    # which tells h_j (the droplet's own width) from h_i apart.
    s = 1.0 / 64
    alpha = 40.0
    rng = np.random.default_rng(5)

    def hfun(x, y):
        return 12 * s * (1.0 + 0.5 * x)

    def dfun(x, y):
        inner = (np.abs(x - 0.5) < 0.2) & (np.abs(y - 0.5) < 0.2)
        return np.where(inner, rng.uniform(0.5, 1.5, x.size) * s, 0.0)

    p, d = _film_lattice(64, s, hfun, dfun)
    rp, col = oracle.neighbours(p)
    H = oracle.film_height(p, rp, col, d, alpha)
    vol = np.pi * d ** 3 / 6.0
    assert abs(s * s * H.sum() - vol.sum()) <= 1e-7 * vol.sum()
    # the same sum with the receiver's h in place of h_j misses by far more
    X = np.stack([p["x"], p["y"]], 1)
    rid = np.repeat(np.arange(X.shape[0]), np.diff(rp))
    r2 = ((X[col] - X[rid]) ** 2).sum(1)
    hi = p["h"][rid]
    wrong = np.bincount(rid, alpha / (np.pi * hi ** 2) * np.exp(-alpha * r2 / hi ** 2) * vol[col])
    assert abs(s * s * wrong.sum() - vol.sum()) > 1e-4 * vol.sum()


def test_film_height_of_bulk_particles_is_zero():
    p = W.mixed_block_film(factor=10)
    rp, col = oracle.neighbours(p)
    H = oracle.film_height(p, rp, col, np.full(p["x"].size, 1e-3))
    assert np.all(H[p["model"] == 0] == 0.0) and np.all(H[p["model"] == 1] > 0.0)


# --------------------------------------------------------------------------- 2D -> 3D
def _film_points(X, N):
    n = len(X)
    X = np.asarray(X, float); N = np.asarray(N, float)
    return dict(x=X[:, 0], y=X[:, 1], z=X[:, 2], h=np.full(n, 0.1), model=np.ones(n, np.int8),
                kind=np.full(n, 2, np.int8), nx=N[:, 0], ny=N[:, 1], nz=N[:, 2])


def test_2d_to_3d_hand_cases():
    # psi~ = (0.2 h3 + 0.3 h3)/2 = 0.25 for h3 = 1.
    #  a: H = 0.75 -> gamma = 3, psi = 0.25, normal +z
    #  b: H = 0.8  -> gamma = ceil(3.2) = 4, psi = 0.2, normal (0.6, 0, 0.8)
    #  c: H = 0    -> gamma = 0 (only the particle itself, now 3D wall)
    p = _film_points([[0, 0, 0], [1, 2, 3], [5, 5, 5]], [[0, 0, 1], [0.6, 0, 0.8], [0, 1, 0]])
    H = np.array([0.75, 0.8, 0.0])
    m = np.array([4.0, 10.0, 3.0])
    rho = np.array([1000.0, 990.0, 980.0])
    phi = np.array([[1.0, 2.0, 3.0], [-1.0, -2.0, -3.0]])
    o = oracle.transition_2d_to_3d(p, np.array([0, 1, 2]), H, np.ones(3), m, rho, phi, 0.2, 0.3)
    assert o["off"].tolist() == [0, 4, 9, 10]
    assert o["src"].tolist() == [0] * 4 + [1] * 5 + [2]
    assert o["kind"].tolist() == [2, 0, 0, 1, 2, 0, 0, 0, 1, 2]
    assert np.all(o["model"] == 0)
    assert o["z"][:4].tolist() == [0.0, 0.25, 0.5, 0.75]
    exp_b = np.array([[1.0, 2.0, 3.0]]) + np.array([0.0, 0.2, 0.4, 0.6, 0.8])[:, None] * [0.6, 0.0, 0.8]
    assert np.allclose(np.stack([o["x"], o["y"], o["z"]], 1)[4:9], exp_b, rtol=0, atol=1e-15)
    assert o["mass"].tolist() == [1.0] * 4 + [2.0] * 5 + [3.0]
    assert o["rho"].tolist() == [1000.0] * 4 + [990.0] * 5 + [980.0]
    assert o["phi"][1].tolist() == [-1.0] * 4 + [-2.0] * 5 + [-3.0]
    assert np.all(o["h"] == 1.0)
    assert o["x"][9] == 5 and o["y"][9] == 5 and o["z"][9] == 5


def test_2d_to_3d_depth_spacing_and_mass():
    # random heights: the added column reaches depth H exactly (gamma psi = H),
    # spacing psi lies in ((gamma-1)/gamma psi~, psi~], mass is conserved
    rng = np.random.default_rng(3)
    n = 300
    N = rng.normal(size=(n, 3)); N /= np.linalg.norm(N, axis=1)[:, None]
    p = _film_points(rng.uniform(-1, 1, (n, 3)), N)
    H = rng.uniform(0, 0.3, n); H[:10] = 0.0
    h3 = rng.uniform(0.05, 0.1, n)
    m = rng.uniform(1, 2, n)
    o = oracle.transition_2d_to_3d(p, np.arange(n), H, h3, m, np.ones(n))
    X = np.stack([p["x"], p["y"], p["z"]], 1)
    O = np.stack([o["x"], o["y"], o["z"]], 1)
    assert abs(o["mass"].sum() - m.sum()) <= 1e-13 * m.sum()
    psit = 0.5 * (oracle.R_MIN + oracle.R_MAX) * h3
    for i in range(n):
        a, b = o["off"][i], o["off"][i + 1]
        gam = b - a - 1
        assert (gam == 0) == (H[i] == 0)
        assert np.array_equal(O[a], X[i])
        if gam:
            depth = (O[b - 1] - X[i]) @ N[i]
            assert abs(depth - H[i]) <= 1e-14
            psi = H[i] / gam
            assert psi <= psit[i] * (1 + 1e-15) and psi > psit[i] * (gam - 1) / gam
            steps = np.diff(O[a:b], axis=0) @ N[i]
            assert np.allclose(steps, psi, rtol=1e-12)


# --------------------------------------------------------------------------- Alg. 5
def test_buffer_flags_brute_force():
    p = W.mixed_block_film(factor=8)
    rp, col = oracle.neighbours(p, cross=True)
    flag = oracle.buffer_flags(p, rp, col)
    X = np.stack([p["x"], p["y"], p["z"]], 1)
    n = X.shape[0]
    expect = np.zeros(n, np.uint8)
    for a in range(0, n, 512):          # all pairs, in blocks of rows
        D = X[a:a + 512, None, :] - X[None, :, :]
        d2 = (D[..., 0] ** 2 + D[..., 1] ** 2) + D[..., 2] ** 2
        r = 0.5 * (p["h"][a:a + 512, None] + p["h"][None, :])
        other = p["model"][a:a + 512, None] != p["model"][None, :]
        expect[a:a + 512] = np.any((d2 <= r * r) & other, axis=1)
    assert np.array_equal(flag, expect)
    assert 0 < flag.sum() < X.shape[0] // 4
    assert np.any(flag[p["model"] == 0]) and np.any(flag[p["model"] == 1])


def _hand_cloud():
    # 3D column at the origin: wall P0 (z=0, normal +z), interior P1 (z=0.1),
    # free surface P2 (z=0.2); a far 3D particle P3; film F0 at (0.1,0,0) and
    # a far film particle F1.  h = 0.25 everywhere.
    X = np.array([[0, 0, 0], [0, 0, 0.1], [0, 0, 0.2], [-5, 0, 0.1], [0.1, 0, 0], [5, 0, 0]], float)
    n = 6
    p = dict(x=X[:, 0], y=X[:, 1], z=X[:, 2], h=np.full(n, 0.25),
             model=np.array([0, 0, 0, 0, 1, 1], np.int8), kind=np.array([2, 0, 1, 0, 2, 2], np.int8),
             nx=np.zeros(n), ny=np.zeros(n), nz=np.array([1.0, 0, 0, 0, 1, 1]))
    mass = np.array([1.0, 2.0, 3.0, 9.0, 4.0, 9.0])
    rho = np.array([1000.0, 1010.0, 1020.0, 1.0, 990.0, 1.0])
    phi = np.array([[1.0, 2.0, 3.0, 9.0, 7.0, 9.0]])
    film_h = np.array([0, 0, 0, 0, 0.5, 0.5])
    h_other = np.array([0.05, 0.05, 0.05, 0.05, 1.0, 1.0])
    return p, mass, rho, phi, film_h, h_other


def test_buffer_zone_hand_example():
    # Cross pairs within 0.25: F0-P0 (0.1), F0-P1 (0.141), F0-P2 (0.224): so
    # P0, P1, P2, F0 are flagged.  The 3D ghosts of P0..P2 transition to 2D:
    # P1 and P2 map onto the wall ghost P0 -> one 2D ghost at the origin with
    # mass 6, averaged rho and phi, height 0.2.  The 2D ghost of F0 transitions
    # to 3D: psi~ = 0.25, gamma = 2 -> ghosts at z = 0, 0.25, 0.5, mass 4/3 each.
    p, mass, rho, phi, film_h, h_other = _hand_cloud()
    rp, col = oracle.neighbours(p, cross=True)
    flag, g = oracle.buffer_zone(p, rp, col, film_h, h_other, mass, rho, phi, r_min=0.2, r_max=0.3)
    assert flag.tolist() == [1, 1, 1, 0, 1, 0]
    assert g["src"].tolist() == [0, 4, 4, 4]
    assert g["model"].tolist() == [1, 0, 0, 0]
    assert g["kind"].tolist() == [2, 2, 0, 1]
    assert g["x"].tolist() == [0.0, 0.1, 0.1, 0.1]
    assert g["z"].tolist() == [0.0, 0.0, 0.25, 0.5]
    assert g["h"].tolist() == [0.05, 1.0, 1.0, 1.0]
    assert g["mass"][0] == 6.0 and np.allclose(g["mass"][1:], 4.0 / 3.0, rtol=1e-15)
    assert g["rho"].tolist() == [1010.0, 990.0, 990.0, 990.0]
    assert g["phi"][0].tolist() == [2.0, 7.0, 7.0, 7.0]
    assert g["height"][0] == 0.2 and np.all(g["height"][1:] == 0)
    assert abs(g["diam"][0] ** 3 - 36.0 / (np.pi * 1010.0)) <= 1e-15
    assert np.all(g["nz"] == 1.0)


def test_buffer_zone_without_other_model_is_empty():
    p = W.plain_cube(6)
    n = p["x"].size
    rp, col = oracle.neighbours(p, cross=True)
    flag, g = oracle.buffer_zone(p, rp, col, np.zeros(n), np.full(n, 0.1), np.ones(n), np.ones(n))
    assert flag.sum() == 0 and g["x"].size == 0


def test_buffer_zone_mass_accounting_mixed_cloud():
    # every 3D ghost maps to a 2D ghost (nearest wall ghost within its support);
    # each 2D ghost carries its source's mass split over 1 + gamma 3D ghosts
    p = W.mixed_block_film(factor=4)
    n = p["x"].size
    rp, col = oracle.neighbours(p, cross=True)
    mass, rho = np.ones(n), np.full(n, 1000.0)
    flag, g = oracle.buffer_zone(p, rp, col, p["film_height"], p["h3d"], mass, rho)
    src = g["src"]
    from_bulk = p["model"][src] == 0
    from_film = ~from_bulk
    assert np.all(g["model"][from_bulk] == 1) and np.all(g["model"][from_film] == 0)
    for i in np.unique(src[from_film]):
        sel = src == i
        assert abs(g["mass"][sel].sum() - mass[i]) <= 1e-15 * mass[i] * sel.sum()
    # 2D ghosts: sources are flagged 3D walls; the mass they carry equals the
    # number of flagged 3D particles that map onto them (unit masses)
    assert np.all(p["kind"][src[from_bulk]] == W.WALL)
    flagged_bulk = np.nonzero((flag == 1) & (p["model"] == 0))[0]
    assert g["mass"][from_bulk].sum() <= flagged_bulk.size
    assert g["mass"][from_bulk].sum() >= from_bulk.sum()


# --------------------------------------------------------------------------- Sec. 6.2
def _extended(factor=8):
    p = W.mixed_block_film(factor=factor)
    n = p["x"].size
    rp, col = oracle.neighbours(p, cross=True)
    flag, g = oracle.buffer_zone(p, rp, col, p["film_height"], p["h3d"], np.ones(n),
                                 np.full(n, 1000.0))
    return p, g, oracle.extend_cloud(p, g)


def test_extended_neighbourhoods_brute_force():
    p, g, e = _extended()
    n = p["x"].size
    m = e["x"].size
    rp, col = oracle.neighbours_rows(e, n)
    assert m > n
    # ghost rows hold only themselves
    for i in range(n, m):
        assert col[rp[i]:rp[i + 1]].tolist() == [i]
    # regular rows: Eq. (Nbd) over regular and ghost particles of the same model
    X = np.stack([e["x"], e["y"], e["z"]], 1)
    rng = np.random.default_rng(2)
    for i in rng.choice(n, 200, replace=False):
        D = X - X[i]
        d2 = (D[:, 0] ** 2 + D[:, 1] ** 2) + D[:, 2] ** 2
        r = 0.5 * (e["h"] + e["h"][i])
        expect = np.nonzero((d2 <= r * r) & (e["model"] == e["model"][i]))[0]
        assert col[rp[i]:rp[i + 1]].tolist() == expect.tolist()


def test_stencils_with_ghost_neighbours_reproduce_quadratics():
    from test_oracle_pins import _poly_checks
    p, g, e = _extended()
    n = p["x"].size
    rp, col = oracle.neighbours_rows(e, n)
    w, st, _ = oracle.gfdm_weights(e, rp, col)
    assert np.all(st[:n] == 0) and np.all(st[n:] == 3)
    # rows that gained ghost neighbours
    rid = np.repeat(np.arange(e["x"].size), np.diff(rp))
    touched = np.unique(rid[(col >= n) & (rid < n)])
    assert touched.size > 0
    bulk = touched[e["model"][touched] == 0]
    film = touched[e["model"][touched] == 1]
    assert bulk.size and film.size
    _poly_checks(e, rp, col, w, bulk)
    _poly_checks(e, rp, col, w, film, film=True)


def test_implicit_split_equals_pinned_ghost_rows():
    # Sec. 6.2: regular unknowns only, ghost terms on the right-hand side.
    # The same solution comes from the full system in which every ghost row is
    # an identity row whose right-hand side is the known ghost value.
    p, g, e = _extended(factor=10)
    n = p["x"].size
    m = e["x"].size
    rp, col = oracle.neighbours_rows(e, n)
    w, st, _ = oracle.gfdm_weights(e, rp, col)
    rt = np.zeros(m, np.int8)
    rt[:n][p["kind"] == W.WALL] = 2
    rt[:n][p["kind"] == W.FREE_SURFACE] = 1
    # film rows: Laplacian inside, Dirichlet on the outer edge of the film
    # (its wall rows alone would leave the constants in the null space)
    film = p["model"] == 1
    rt[:n][film] = 0
    edge = film & ((p["x"] > 0.9) | (p["y"] < 0.1) | (p["y"] > 0.9))
    rt[:n][edge] = 1
    rt[n:] = 1
    rng = np.random.default_rng(4)
    rhs = rng.uniform(-1, 1, m)
    pg = rng.uniform(-1, 1, m - n)
    x_split = oracle.poisson_split_solve(e, rp, col, w, rt, n, rhs, pg)
    val = oracle.poisson_matrix(e, rp, col, w, rt)
    full_rhs = np.concatenate([rhs[:n], pg])
    x_full = oracle.poisson_solve(rp, col, val, full_rhs)
    assert np.allclose(x_full[n:], pg, rtol=0, atol=1e-12)
    assert np.abs(x_full[:n] - x_split).max() <= 1e-9 * max(1.0, np.abs(x_split).max())
    # and the ghost values matter: without them the solution changes
    x0 = oracle.poisson_split_solve(e, rp, col, w, rt, n, rhs, np.zeros_like(pg))
    assert np.abs(x0 - x_split).max() > 1e-6


# --------------------------------------------------------------------------- Alg. 3, whole cloud
def test_transition_cloud_hand_example():
    # the hand example of Sec. 5.1 (walls A, B flagged; p, q -> A, r -> B; s kept)
    X = np.array([[0, 0, 0], [1, 0, 0], [3, 0, 0], [0.2, 0, 0.3], [0.5, 0, 0.4], [0.9, 0, 0.3],
                  [2.4, 0, 0.2]], float)
    n = X.shape[0]
    p = dict(x=X[:, 0], y=X[:, 1], z=X[:, 2], h=np.full(n, 3.2), model=np.zeros(n, np.int8),
             kind=np.array([2, 2, 2, 0, 0, 0, 1], np.int8), nx=np.zeros(n), ny=np.zeros(n),
             nz=np.array([1.0, 1.0, 1.0, 0, 0, 0, 0]))
    rp, col = oracle.neighbours(p)
    flag = np.array([1, 1, 0, 0, 0, 0, 0], np.uint8)
    m = np.array([1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0])
    rho = np.array([1000.0, 1000, 1000, 900, 1100, 1000, 1000])
    phi = np.array([[1.0, 2, 3, 4, 5, 6, 7], [10.0, 20, 30, 40, 50, 60, 70]])
    o = oracle.transition_3d_to_2d_cloud(p, rp, col, flag, m, rho, phi, h_film=np.full(n, 0.5))
    assert o["src"].tolist() == [0, 1, 2, 6]          # p, q, r deleted
    assert o["model"].tolist() == [1, 1, 0, 0]
    assert o["kind"].tolist() == [2, 2, 2, 1]
    assert o["h"].tolist() == [0.5, 0.5, 3.2, 3.2]
    assert o["mass"].tolist() == [25.0, 34.0, 4.0, 64.0]
    assert o["phi"][0].tolist() == [(1 + 4 + 5) / 3, (2 + 6) / 2, 3.0, 7.0]
    assert o["phi"][1].tolist() == [(10 + 40 + 50) / 3, (20 + 60) / 2, 30.0, 70.0]
    assert o["height"].tolist() == [0.4, 0.3, 0.0, 0.0]
    assert o["x"].tolist() == [0.0, 1.0, 3.0, 2.4]


def test_transition_cloud_conserves_mass_and_counts():
    p = W.shallow_cylinder()
    rp, col = oracle.neighbours(p)
    lam, w3, eps = oracle.pca(p, rp, col)
    flag = oracle.classify(p, rp, col, eps, w3, cross=oracle.neighbours(p, cross=True))
    n = p["x"].shape[0]
    o = oracle.transition_3d_to_2d_cloud(p, rp, col, flag, p["mass"], p["rho"],
                                         np.stack([p["x"], p["z"]]))
    assert abs(o["mass"].sum() - p["mass"].sum()) <= 1e-13 * p["mass"].sum()
    moved = (flag == 1)
    assert (o["model"] == 1).sum() == moved.sum() + (p["model"] == 1).sum()
    # every deleted particle was an interior / free-surface bulk particle
    gone = np.setdiff1d(np.arange(n), o["src"])
    assert gone.size > 0 and np.all(p["kind"][gone] != W.WALL) and np.all(p["model"][gone] == 0)
    # a field that is the same everywhere stays the same after averaging
    o2 = oracle.transition_3d_to_2d_cloud(p, rp, col, flag, p["mass"], p["rho"], np.full((1, n), 7.25))
    assert np.all(o2["phi"] == 7.25)


# --------------------------------------------------------------------------- Sec. 7.2 analogue
def _advdiff_errors(h, kappa=5e-3, t_end=0.5, factor=0.25, ghost_scale=1.0):
    d = W.advdiff_plate(h)
    steps = int(np.ceil(t_end / (factor * 0.05 * h * h / kappa)))
    T = oracle.advdiff_run(d, W.advdiff_rows(d, h), kappa, t_end, steps, ghost_scale=ghost_scale)
    ex = W.advdiff_exact(d["x"], d["y"], t_end, kappa)
    e2 = np.sqrt(((T - ex) ** 2).sum() / (ex ** 2).sum())
    einf = np.abs(T - ex).max() / ex.max()
    return e2, einf


def test_advdiff_converges_at_second_order():
    # against the exact heat-kernel solution of the Gaussian (constant in
    # depth), the coupled 2D / 3D / ghost discretisation converges at about
    # second order, as the paper reports for its analogue (Table 2)
    e_c = _advdiff_errors(0.12)
    e_f = _advdiff_errors(0.06)
    order2 = np.log2(e_c[0] / e_f[0])
    orderi = np.log2(e_c[1] / e_f[1])
    assert e_f[0] < 1e-2 and order2 > 1.7 and orderi > 1.5, (e_c, e_f, order2, orderi)


def test_advdiff_needs_the_ghost_data():
    # without the ghost values the block and the film do not exchange heat:
    # the error grows several-fold (about 5x at h = 0.06)
    e_g = _advdiff_errors(0.06)
    e_0 = _advdiff_errors(0.06, ghost_scale=0.0)
    assert e_0[0] > 4 * e_g[0]


def _advect_cloud(d):
    c = {k: np.asarray(d[k]).copy() for k in ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz", "mass", "rho")}
    c["T"], c["H"], c["edge"] = d["T0"].copy(), d["film_height"].copy(), d["edge"].copy()
    return c


def test_model_adaptive_advection_round_trip():
    # the plate moves through the 3D window [1, 2] and out again: every film
    # particle that entered became a column (Sec. 5.2) and every column came
    # back as one film particle (Sec. 5.1); the mass is conserved by both
    # transitions, the film thickness is recovered from the columns, the
    # edge marker stays 0 / 1, and the Gaussian carried through the 3D
    # region matches the exact advected and diffused solution (about 3% at
    # h = 0.12; about 0.8% at h = 0.06, i.e. close to second order)
    h, kappa, t_end = 0.12, 5e-3, 2.0
    d = W.advect_plate(h)
    c = _advect_cloud(d)
    n0, m0 = c["x"].size, c["mass"].sum()
    steps = int(np.ceil(t_end / (0.25 * 0.05 * h * h / kappa)))
    saw3d = 0
    for _ in range(steps):
        c = oracle.advect_step(c, h, kappa, t_end / steps)
        saw3d = max(saw3d, int((c["model"] == 0).sum()))
        assert abs(c["mass"].sum() / m0 - 1.0) < 1e-13
    assert saw3d > n0 and np.all(c["model"] == 1) and c["x"].size == n0
    assert np.allclose(c["H"], d["depth"], rtol=1e-12, atol=0)
    assert np.all((c["edge"] == 0.0) | (c["edge"] == 1.0))
    ex = W.advdiff_exact(c["x"], c["y"], t_end, kappa, x0=0.6 + t_end)
    e2 = np.sqrt(((c["T"] - ex) ** 2).sum() / (ex ** 2).sum())
    einf = np.abs(c["T"] - ex).max() / ex.max()
    assert e2 < 0.04 and einf < 0.07, (e2, einf)


def test_pure_advection_transfers_data_exactly():
    # kappa = 0 (Sec. 7.2, pure advection): the plate [0,3]x[0,1] passes the
    # 3D window [1,2]; since the field is constant in depth, the transitions
    # in both directions move it without loss, and at t = 2 it equals the
    # initial field moved by 2: exactly for the disc of Eq. (AdvDiff_IC)
    # (values 0 / 1), to rounding of the moved positions for a Gaussian
    for ic, tol in (("disc", 0.0), ("gauss", 1e-12)):
        d = W.advect_plate(0.1, lx=3.0, ly=1.0, ic=ic, center=(0.5, 0.5))
        c = _advect_cloud(d)
        saw3d = 0
        for _ in range(40):
            c = oracle.advect_step(c, 0.1, 0.0, 2.0 / 40)
            saw3d = max(saw3d, int((c["model"] == 0).sum()))
        assert saw3d > d["x"].size and c["x"].size == d["x"].size and np.all(c["model"] == 1)
        r2 = (c["x"] - 2.5) ** 2 + (c["y"] - 0.5) ** 2
        ex = (r2 <= 0.04).astype(np.float64) if ic == "disc" else np.exp(-r2 / (2 * 0.1 ** 2))
        assert np.abs(c["T"] - ex).max() <= tol, ic
        assert np.allclose(c["H"], d["depth"], rtol=1e-12, atol=0)
