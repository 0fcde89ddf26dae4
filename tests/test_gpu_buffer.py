"""Parity of the coupling layer with the FP64 oracle: buffer flags and ghost
particles (Sec. 6.1, Alg. 5), film height (Eq. Height), the 2D->3D
transition (Sec. 5.2), extended neighbourhoods, stencils over regular and
ghost neighbours and the implicit ghost split (Sec. 6.2).

Integer results (flags, counts, kinds, models, sources, neighbour lists) and
positions are compared bit for bit: both sides evaluate them in FP64 with the
same operations and no fused multiply-adds.  Averages and lumped masses are
summed in the same order on both sides; the droplet diameter goes through a
cube root, whose last bit may differ between math libraries (1e-15).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2405_13165_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    from paper_2405_13165_amd import gfdm
    gfdm.load_library()
    return gfdm


@pytest.fixture(scope="module")
def ctx(g):
    c = g.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def _lists(ctx, g, d):
    p = g.Particles.from_dict(ctx, d)
    same = g.build_neighbours(ctx, p)
    cross = g.build_neighbours(ctx, p, cross_model=True)
    return p, same, cross


def _hand_cloud():
    X = np.array([[0, 0, 0], [0, 0, 0.1], [0, 0, 0.2], [-5, 0, 0.1], [0.1, 0, 0], [5, 0, 0]], float)
    n = 6
    d = dict(x=X[:, 0], y=X[:, 1], z=X[:, 2], h=np.full(n, 0.25),
             model=np.array([0, 0, 0, 0, 1, 1], np.int8), kind=np.array([2, 0, 1, 0, 2, 2], np.int8),
             nx=np.zeros(n), ny=np.zeros(n), nz=np.array([1.0, 0, 0, 0, 1, 1]),
             mass=np.array([1.0, 2.0, 3.0, 9.0, 4.0, 9.0]),
             rho=np.array([1000.0, 1010.0, 1020.0, 1.0, 990.0, 1.0]),
             film_height=np.array([0, 0, 0, 0, 0.5, 0.5]),
             h_other=np.array([0.05, 0.05, 0.05, 0.05, 1.0, 1.0]))
    return d


def _compare_new(got, exp, what):
    k = exp["x"].size
    assert got["x"].shape[0] == k, (what, got["x"].shape[0], k)
    for key in ("model", "kind", "src"):
        assert np.array_equal(_np(got[key]), exp[key]), (what, key)
    for key in ("x", "y", "z", "h", "nx", "ny", "nz", "mass", "rho", "height"):
        assert np.array_equal(_np(got[key]), exp[key]), (what, key)
    assert np.array_equal(_np(got["phi"]), exp["phi"]), (what, "phi")
    dg, de = _np(got["diam"]), exp["diam"]
    assert np.all(np.abs(dg - de) <= 1e-15 * np.abs(de)), (what, "diam")


# --------------------------------------------------------------------------- flags and ghosts
@pytest.mark.parametrize("case", ["hand", "mixed4", "mixed2", "jet_small"])
def test_buffer_zone_matches_oracle(ctx, g, case):
    print(f"\n[buffer] {case}", flush=True)
    if case == "hand":
        d = _hand_cloud()
        r_min, r_max = 0.2, 0.3
    elif case == "jet_small":
        d = W.jet_impact(n_bulk=60_000, n_film=60_000)
        r_min, r_max = g.R_MIN, g.R_MAX
    else:
        d = W.mixed_block_film(factor=int(case[-1]))
        r_min, r_max = g.R_MIN, g.R_MAX
    n = d["x"].size
    rng = np.random.default_rng(n)
    phi = rng.uniform(-1, 1, (2, n))
    p, same, cross = _lists(ctx, g, d)
    flag, gh = g.buffer_zone(ctx, p, same, cross, d["film_height"], d["h_other"], d["mass"], d["rho"],
                             phi, r_min, r_max)
    rp_c, col_c = oracle.neighbours(d, cross=True)
    flag_o, gh_o = oracle.buffer_zone(d, rp_c, col_c, d["film_height"], d["h_other"], d["mass"],
                                      d["rho"], phi, r_min, r_max)
    assert np.array_equal(_np(flag), flag_o)
    print(f"[buffer] {case}: {int(flag_o.sum())} flagged, {gh_o['x'].size} ghosts", flush=True)
    _compare_new(gh, gh_o, case)
    # the flags alone
    assert np.array_equal(_np(g.buffer_flags(ctx, p, same, cross)), flag_o)


def test_buffer_zone_empty_and_capacity(ctx, g):
    # a single-model cloud has no buffer zone
    d = W.plain_cube(8)
    n = d["x"].size
    p, same, cross = _lists(ctx, g, d)
    flag, gh = g.buffer_zone(ctx, p, same, cross, np.zeros(n), np.full(n, 0.1), np.ones(n), np.ones(n))
    assert int(flag.sum()) == 0 and gh["x"].shape[0] == 0
    # capacity too small: GF_ECAPACITY with the needed count, nothing written
    d = _hand_cloud()
    p, same, cross = _lists(ctx, g, d)
    dev = ctx.device
    tens = {k: torch.as_tensor(d[k], device=dev) for k in ("film_height", "h_other", "mass", "rho")}
    o, st = g._new_buffers(dev, 2, 0)
    o["x"].fill_(-7.0)
    cnt = ctypes.c_int64(-1)
    ctx._sync_stream()
    status = ctx.lib.gf_buffer_zone(ctx.handle, ctypes.byref(p.s), same.handle, cross.handle,
                                    g._ptr(tens["film_height"]), g._ptr(tens["h_other"]), 0.2, 0.3,
                                    g._ptr(tens["mass"]), g._ptr(tens["rho"]), None, 0, ctypes.byref(st),
                                    ctypes.byref(cnt), None)
    assert status == g.GF_ECAPACITY and cnt.value == 4
    assert torch.all(o["x"] == -7.0)
    # argument errors are rejected before any kernel runs
    status = ctx.lib.gf_buffer_zone(ctx.handle, ctypes.byref(p.s), cross.handle, same.handle,
                                    g._ptr(tens["film_height"]), g._ptr(tens["h_other"]), 0.2, 0.3,
                                    g._ptr(tens["mass"]), g._ptr(tens["rho"]), None, 0, ctypes.byref(st),
                                    ctypes.byref(cnt), None)
    assert status == g.GF_EINVAL
    status = ctx.lib.gf_buffer_zone(ctx.handle, ctypes.byref(p.s), same.handle, cross.handle,
                                    g._ptr(tens["film_height"]), g._ptr(tens["h_other"]), 0.3, 0.2,
                                    g._ptr(tens["mass"]), g._ptr(tens["rho"]), None, 0, ctypes.byref(st),
                                    ctypes.byref(cnt), None)
    assert status == g.GF_EINVAL


# --------------------------------------------------------------------------- Eq. (Height)
@pytest.mark.parametrize("case", ["mixed2", "jet_small"])
def test_film_height_matches_oracle(ctx, g, case):
    d = W.mixed_block_film(factor=2) if case == "mixed2" else W.jet_impact(n_bulk=60_000, n_film=60_000)
    p = g.Particles.from_dict(ctx, d)
    same = g.build_neighbours(ctx, p)
    rp, col = oracle.neighbours(d)
    for alpha in (g.ALPHA_FILM, 20.0):
        H = _np(g.film_height(ctx, p, same, d["diam"], alpha))
        H_o = oracle.film_height(d, rp, col, d["diam"], alpha)
        assert np.all(H[d["model"] == 0] == 0.0)
        assert np.all(np.abs(H - H_o) <= 1e-13 * H_o), case


# --------------------------------------------------------------------------- 2D -> 3D
def test_transition_2d_to_3d_matches_oracle(ctx, g):
    d = W.mixed_block_film(factor=2)
    n = d["x"].size
    rng = np.random.default_rng(7)
    flag = np.zeros(n, np.uint8)
    film = np.nonzero(d["model"] == 1)[0]
    bulk = np.nonzero(d["model"] == 0)[0]
    flag[rng.choice(film, film.size // 3, replace=False)] = 2
    flag[rng.choice(film, 50, replace=False)] = 1          # other flag value: ignored
    flag[rng.choice(bulk, 50, replace=False)] = 2          # not film: ignored
    H = d["film_height"] * rng.uniform(0.0, 20.0, n)       # 0 .. ~15 layers
    H[film[:100]] = 0.0
    phi = rng.uniform(-1, 1, (3, n))
    p = g.Particles.from_dict(ctx, d)
    o = g.transition_2d_to_3d(ctx, p, flag, H, d["h3d"], d["mass"], d["rho"], phi)
    sel = np.nonzero((flag == 2) & (d["model"] == 1))[0]
    o_o = oracle.transition_2d_to_3d(d, sel, H, d["h3d"], d["mass"], d["rho"], phi)
    o_o.pop("off")
    _compare_new(o, o_o, "2d->3d")
    assert o_o["x"].size > 2 * sel.size
    # nothing flagged
    o = g.transition_2d_to_3d(ctx, p, np.zeros(n, np.uint8), H, d["h3d"], d["mass"], d["rho"])
    assert o["x"].shape[0] == 0
    # too many layers for one particle -> GF_EINVAL
    Hbad = H.copy()
    Hbad[sel[0]] = 1e9
    with pytest.raises(g.GfdmError) as e:
        g.transition_2d_to_3d(ctx, p, flag, Hbad, d["h3d"], d["mass"], d["rho"])
    assert e.value.status == g.GF_EINVAL


# --------------------------------------------------------------------------- Sec. 6.2
def _extended(ctx, g, factor):
    d = W.mixed_block_film(factor=factor)
    n = d["x"].size
    p, same, cross = _lists(ctx, g, d)
    flag, gh = g.buffer_zone(ctx, p, same, cross, d["film_height"], d["h_other"], d["mass"], d["rho"])
    pe = g.extend_particles(ctx, p, gh)
    de = oracle.extend_cloud(d, {k: _np(v) for k, v in gh.items()})
    return d, n, pe, de


@pytest.mark.parametrize("factor", [4, 2])
def test_extended_neighbourhoods_and_stencils(ctx, g, factor):
    d, n, pe, de = _extended(ctx, g, factor)
    m = pe.n
    nb = g.build_neighbours(ctx, pe, n_rows=n)
    rp_o, col_o = oracle.neighbours_rows(de, n)
    rp, col = nb.export()
    assert np.array_equal(_np(rp), rp_o) and np.array_equal(_np(col), col_o)
    w_o, st_o, _ = oracle.gfdm_weights(de, rp_o, col_o)
    assert np.all(st_o[n:] == 3)
    for wtype, tol in ((g.GF_F32, 1e-6), (g.GF_F64, 1e-10)):
        status = torch.empty(m, dtype=torch.int8, device=ctx.device)
        w = g.gfdm_weights(ctx, pe, nb, g.GF_BATCHED, wtype, status=status)
        st = _np(status)
        assert np.array_equal(np.where(st == 1, 0, st), st_o)
        e = oracle.operator_error(_np(w).astype(np.float64)[: rp_o[n]], w_o[: rp_o[n]], rp_o[: n + 1])
        assert e.max() <= tol, (wtype, e.max())
    # applied with ghost values u^(n) (explicit step, Eq. GhostDerivatives)
    f, *_ = W.test_field(de["x"], de["y"], de["z"])
    u = torch.as_tensor(f, device=ctx.device)
    _, y = g.gfdm_weights_apply(ctx, pe, nb, u, wtype=g.GF_F64, store_weights=False)
    y_o = oracle.apply(rp_o, col_o, w_o, f)
    assert np.abs(_np(y)[:, :n] - y_o[:, :n]).max() <= 1e-8 * (1 + np.abs(y_o).max())
    assert np.all(_np(y)[:, n:] == 0.0)


def test_position_adjoint_over_extended_neighbourhoods(ctx, g):
    # ghost neighbours have no rows of their own, so the entries (i, g) have
    # no twin (g, i); x_i still loses every dbar(i, j).  The regular
    # particles' gradients match the oracle's definition (Laplacian-only and
    # a general operator set), and a second call accumulates onto the first.
    d, n, pe, de = _extended(ctx, g, 4)
    m = pe.n
    nb = g.build_neighbours(ctx, pe, n_rows=n)
    rp, col = (a.cpu().numpy() for a in nb.export())
    rid = np.repeat(np.arange(m), np.diff(rp))
    assert np.any((col >= n) & (rid < n))   # rows with ghost neighbours
    f, *_ = W.test_field(de["x"], de["y"], de["z"])
    u = torch.as_tensor(f, device=ctx.device)
    yb = np.random.default_rng(17).uniform(-1, 1, (2, m))
    for mask, k in ((g.OP_LAP, 1), (g.OP_LAP | g.OP_DX, 2)):
        xb_o = oracle.weights_adjoint_x(de, rp, col, f, yb[:k], op_mask=mask)
        ybt = torch.as_tensor(yb[:k], device=ctx.device)
        xbar = g.gfdm_weights_adjoint(ctx, pe, nb, u, ybt, op_mask=mask)
        first = _np(xbar).copy()
        err = np.abs(first[:n] - xb_o[:n]).max() / np.abs(xb_o[:n]).max()
        print(f"[adjoint, ghosts] mask {mask}: rel err {err:.2e}", flush=True)
        assert err <= 1e-9
        g.gfdm_weights_adjoint(ctx, pe, nb, u, ybt, op_mask=mask, xbar=xbar)
        assert np.abs(_np(xbar) - 2 * first).max() <= 1e-12 * np.abs(first).max()
    # the application adjoint likewise: u_i loses c_ig ybar_i for ghost neighbours g
    w64 = g.gfdm_weights(ctx, pe, nb, g.GF_BATCHED, g.GF_F64)
    yb4 = np.random.default_rng(18).uniform(-1, 1, (4, m))
    ub = _np(g.apply_stencil_adjoint(ctx, nb, w64, torch.as_tensor(yb4, device=ctx.device)))
    ub_o = oracle.apply_adjoint(rp, col, _np(w64), yb4)
    assert np.abs(ub[:n] - ub_o[:n]).max() <= 1e-12 * np.abs(ub_o[:n]).max()


def test_implicit_split_with_ghost_rows(ctx, g):
    d, n, pe, de = _extended(ctx, g, 4)
    m = pe.n
    nb = g.build_neighbours(ctx, pe, n_rows=n)
    rp, col = (a.cpu().numpy() for a in nb.export())
    # bulk: Laplacian inside, Neumann rows on the bottom wall, Dirichlet on the
    # free surface (the block's top and sides); film rows Dirichlet; ghost rows
    # pinned.  (On this thin block the combined PDE + zeta*BC wall rows make
    # the Jacobi-preconditioned operator indefinite and BiCGStab diverges, with
    # or without ghosts; pure Neumann rows do not.)
    rt = np.zeros(m, np.int8)
    rt[:n][d["kind"] == W.WALL] = 3
    rt[:n][d["kind"] == W.FREE_SURFACE] = 1
    rt[:n][d["model"] == 1] = 1
    rt[n:] = 1
    rid = np.repeat(np.arange(m), np.diff(rp))
    assert np.any((col >= n) & (rid < n) & (rt[rid] != 1))   # the split acts on some rows
    rng = np.random.default_rng(9)
    rhs = rng.uniform(-1, 1, m)
    pg = rng.uniform(-1, 1, m - n)
    rhs[n:] = pg
    x0 = np.zeros(m)
    x0[n:] = pg
    # the oracle's stencils over the extended neighbourhoods, uploaded: the GPU
    # solve then works on the oracle's matrix, whose reduced system the oracle
    # solves directly (sparse LU)
    w_o, _, _ = oracle.gfdm_weights(de, rp, col)
    val = oracle.poisson_matrix(de, rp, col, w_o, rt)
    x_o = oracle.poisson_split_solve(de, rp, col, w_o, rt, n, rhs, pg)
    w64 = g.gfdm_weights(ctx, pe, nb, g.GF_BATCHED, g.GF_F64)
    for label, wsolve in (("oracle stencils", torch.as_tensor(w_o, device=ctx.device)), ("own stencils", w64)):
        x, st = g.poisson_solve(ctx, pe, nb, wsolve, rt, torch.as_tensor(rhs, device=ctx.device),
                                x0=torch.as_tensor(x0, device=ctx.device), params=g.solve_params(rtol=1e-13))
        xs = _np(x)
        assert st["converged"] == 1
        assert np.array_equal(xs[n:], pg)          # ghost unknowns never move
        # the regular part solves the reduced system A_rr x_r = rhs_r - A_rg p_g
        res = rhs - oracle.csr_matvec(rp, col, val, xs)
        rel = np.linalg.norm(res[:n]) / np.linalg.norm(rhs)
        dx = np.linalg.norm(xs[:n] - x_o) / np.linalg.norm(x_o)
        print(f"[split] {label}: its {st['inner_its_total']}, reduced-system residual {rel:.2e}, "
              f"solution difference {dx:.2e}", flush=True)
        if label == "oracle stencils":
            assert rel <= 1.5e-13
            assert dx <= 1e-10
        else:
            # the library's FP64 stencils differ from the oracle's in the last digits
            assert rel <= 1e-10
            assert dx <= 1e-9


# --------------------------------------------------------------------------- Alg. 3 on the cloud
@pytest.mark.parametrize("case", ["mixed2_walls", "cylinder_pca"])
def test_transition_cloud_matches_oracle(ctx, g, case):
    if case == "cylinder_pca":
        d = W.shallow_cylinder()
        rp, col = oracle.neighbours(d)
        lam, w3, eps = oracle.pca(d, rp, col)
        flag = oracle.classify(d, rp, col, eps, w3, cross=oracle.neighbours(d, cross=True))
    else:
        # every bulk wall flagged: the layers above the bottom are deleted
        d = W.mixed_block_film(factor=2)
        rp, col = oracle.neighbours(d)
        flag = ((d["model"] == 0) & (d["kind"] == W.WALL)).astype(np.uint8)
    n = d["x"].size
    rng = np.random.default_rng(n)
    phi = rng.uniform(-1, 1, (3, n))
    fh = d.get("film_height", np.zeros(n))
    dm = d.get("diam", np.zeros(n))
    hf = np.full(n, 0.004)
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    o = g.transition_3d_to_2d_cloud(ctx, p, nb, flag, d["mass"], d["rho"], phi, fh, dm, hf)
    o_o = oracle.transition_3d_to_2d_cloud(d, rp, col, flag, d["mass"], d["rho"], phi, fh, dm, hf)
    print(f"[cloud] {case}: {n} -> {o_o['x'].size} particles, {int((flag == 1).sum())} to film", flush=True)
    assert o_o["x"].size < n
    _compare_new(o, o_o, case)
