"""Parity at the full workload sizes, in the launch configuration the bench
times (autotuned team sizes, batched FP32 stencils), against the FP64 oracle.

 - mixed bulk/film cloud, 503,944 particles: every neighbour list, every
   stored stencil and every applied value; every PCA output and flag, and
   every output of the transition with all bulk wall particles flagged;
 - jet impact, 2.0M particles with uneven supports (13..228 neighbours):
   every neighbour list, stencils of 20,000 sampled rows;
 - differentiation cube, 10^6 particles: gradients with respect to field
   values and positions at 100 sampled coordinates against central finite
   differences of the oracle (local re-evaluation of the affected rows);
 - projection cylinder, 4.0M rows: FP64 and mixed solves of a seeded
   right-hand side, residual re-evaluated by the oracle on sampled rows.
"""
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


def test_full_mixed_workload(ctx, g):
    print("\n[full] mixed 503,944", flush=True)
    d = W.mixed_block_film()
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    rp_o, col_o = oracle.neighbours(d)
    rp, col = nb.export()
    assert np.array_equal(_np(rp), rp_o) and np.array_equal(_np(col), col_o)
    g.autotune(ctx, p, nb, g.GF_F32)
    f, *_ = W.test_field(d["x"], d["y"], d["z"])
    u = torch.as_tensor(f, device=ctx.device)
    status = torch.empty(p.n, dtype=torch.int8, device=ctx.device)
    w32 = g.gfdm_weights(ctx, p, nb, g.GF_BATCHED, g.GF_F32, status=status)
    y32 = g.apply_stencil(ctx, nb, w32, u)
    w_o, st_o, _ = oracle.gfdm_weights(d, rp_o, col_o)
    st = _np(status)
    assert np.array_equal(np.where(st == 1, 0, st), st_o)
    e = oracle.operator_error(_np(w32).astype(np.float64), w_o, rp_o)
    print(f"[full] mixed FP32 operator error max {e.max():.3e}", flush=True)
    assert e.max() <= 1e-6
    y_o = oracle.apply(rp_o, col_o, w_o, f)
    rid = np.repeat(np.arange(p.n), np.diff(rp_o))
    du = np.abs(f[col_o] - f[rid])
    y = _np(y32)
    for s in range(4):
        mag = np.bincount(rid, np.abs(w_o[:, s]) * du, minlength=p.n).max()
        assert np.abs(y[s] - y_o[s]).max() <= 1e-6 * mag
    # FP64 batched on the same launch configuration
    w64 = g.gfdm_weights(ctx, p, nb, g.GF_BATCHED, g.GF_F64)
    assert oracle.operator_error(_np(w64), w_o, rp_o).max() <= 1e-10
    # fused call, stencils not stored
    _, yf = g.gfdm_weights_apply(ctx, p, nb, u, wtype=g.GF_F32, store_weights=False)
    assert (yf - y32).abs().max().item() <= 1e-9 * (y32.abs().max().item() + 1)


def test_full_mixed_pca_and_transition(ctx, g):
    # a3 and a7 on the full mixed cloud as the bench times them: PCA with the
    # cross-model smoothing lists, film heights and h_3D; the transition with
    # every bulk wall particle flagged (which deletes the layers above the
    # bottom).  Every output against the oracle.
    import math
    print("\n[full] mixed 503,944: PCA + transition", flush=True)
    d = W.mixed_block_film()
    n = d["x"].size
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    xnb = g.build_neighbours(ctx, p, cross_model=True)
    rp, col = oracle.neighbours(d)
    xr, xc = oracle.neighbours(d, cross=True)
    lam, w3, eps, flag = g.classify_pca(ctx, p, nb, xnb, film_height=d["film_height"], h3d=d["h3d"])
    lam_o, w3_o, eps_o = oracle.pca(d, rp, col)
    flag_o = oracle.classify(d, rp, col, eps_o, w3_o, cross=(xr, xc), film_height=d["film_height"], h3d=d["h3d"])
    lam, w3, eps, flag = _np(lam), _np(w3), _np(eps), _np(flag)
    scale = np.maximum(lam_o[:, :1], 1e-300)
    assert np.all(np.abs(lam - lam_o) <= 1e-10 * scale)
    fin = np.isfinite(eps_o)
    assert np.array_equal(np.isfinite(eps), fin)
    assert np.all(np.abs(eps[fin] - eps_o[fin]) <= 1e-10)
    gap = (lam_o[:, 1] - lam_o[:, 2]) > 1e-8 * lam_o[:, 0]
    assert np.all(np.abs((w3 * w3_o).sum(1))[gap] >= 1 - 1e-10)
    # flags: identical away from the thresholds (where rounding may decide)
    nd = np.abs(w3_o[:, 0] * d["nx"] + w3_o[:, 1] * d["ny"] + w3_o[:, 2] * d["nz"])
    band = (np.abs(eps_o - oracle.EPS_LAMBDA_MAX) <= 1e-8) | (np.abs(nd - math.cos(oracle.THETA_STAR)) <= 1e-8)
    print(f"[full] flags {np.bincount(flag_o, minlength=3).tolist()}, {int(band.sum())} in the threshold band",
          flush=True)
    assert np.array_equal(flag[~band], flag_o[~band])
    tflag = ((d["model"] == 0) & (d["kind"] == W.WALL)).astype(np.uint8)
    mass = np.ones(n)
    rho = np.full(n, 1000.0)
    phi, *_ = W.test_field(d["x"], d["y"], d["z"])
    t = g.transition_3d_to_2d(ctx, p, nb, tflag, mass, rho, phi)
    t_o = oracle.transition_3d_to_2d(d, rp, col, tflag, mass, rho, phi)
    for k in ("keep", "owner", "mass", "rho", "phi", "height"):
        assert np.array_equal(_np(t[k]), t_o[k]), k
    assert np.allclose(_np(t["diam"]), t_o["diam"], rtol=1e-15, atol=0)
    deleted = int((t_o["keep"] == 0).sum())
    print(f"[full] transition: {int(tflag.sum())} flagged, {deleted} deleted", flush=True)
    assert deleted > 0
    assert abs(_np(t["mass"]).sum() - mass.sum()) <= 1e-12 * mass.sum()


def test_full_jet_uneven(ctx, g):
    print("\n[full] jet 2.0M", flush=True)
    d = W.jet_impact()
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    rp_o, col_o = oracle.neighbours(d)
    rp, col = nb.export()
    assert np.array_equal(_np(rp), rp_o) and np.array_equal(_np(col), col_o)
    g.autotune(ctx, p, nb, g.GF_F32)
    status = torch.empty(p.n, dtype=torch.int8, device=ctx.device)
    w32, stats = g.gfdm_weights(ctx, p, nb, g.GF_BATCHED, g.GF_F32, status=status, stats=True)
    print(f"[full] jet stats {stats}", flush=True)
    rows = np.sort(np.random.default_rng(11).choice(p.n, 20000, replace=False))
    w_o, st_o, _ = oracle.gfdm_weights(d, rp_o, col_o, rows=rows)
    st = _np(status)[rows]
    assert np.array_equal(np.where(st == 1, 0, st), st_o[rows])
    sel = np.concatenate([np.arange(rp_o[i], rp_o[i + 1]) for i in rows])
    sub_rp = np.concatenate([[0], np.cumsum(np.diff(rp_o)[rows])])
    e = oracle.operator_error(_np(w32)[sel].astype(np.float64), w_o[sel], sub_rp)
    print(f"[full] jet FP32 operator error max {e.max():.3e} on {rows.size} rows", flush=True)
    assert e.max() <= 1e-6


def test_full_differentiation_fd(ctx, g):
    print("\n[full] differentiation 1e6", flush=True)
    d = W.diff_cube()
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    # the oracle works on its own neighbour lists, which the library's must equal
    rp, col = oracle.neighbours(d)
    rp_g, col_g = nb.export()
    assert np.array_equal(_np(rp_g), rp) and np.array_equal(_np(col_g), col)
    dev = ctx.device
    u = torch.as_tensor(d["u"], device=dev)
    x = torch.as_tensor(d["x"], device=dev)
    y = torch.as_tensor(d["y"], device=dev)
    z = torch.as_tensor(d["z"], device=dev)
    gt = torch.as_tensor(d["g"], device=dev)
    ur = u.clone().requires_grad_(True)
    xr, yr, zr = (t.clone().requires_grad_(True) for t in (x, y, z))
    out = g.stencil_op(ctx, p, nb, ur, xr, yr, zr, op_mask=g.OP_LAP, wtype=g.GF_F32)
    loss = ((out[0] - gt) ** 2).sum()
    gu, gx, gy, gz = torch.autograd.grad(loss, (ur, xr, yr, zr))
    grads = {"u": _np(gu), "x": _np(gx), "y": _np(gy), "z": _np(gz)}
    # oracle: central differences of the local loss (only rows whose stencil
    # contains the perturbed particle change), eps = 1e-6, FP64
    rng = np.random.default_rng(21)
    X = np.stack([d["x"], d["y"], d["z"]], 1)
    eps = 1e-6
    checked = 0
    for t in range(100):
        i = int(rng.integers(p.n))
        key = "u" if t < 50 else "xyz"[t % 3]
        rows = np.unique(np.concatenate([[i], col[rp[i]:rp[i + 1]]]))
        nbs = col[rp[i]:rp[i + 1]]
        dist = np.sqrt(((X[nbs] - X[i]) ** 2).sum(1))
        if np.any(np.abs(dist - 0.5 * (d["h"][i] + d["h"][nbs])) < 10 * eps):
            continue

        def local_loss(dd, uu):
            # oracle stencils of the affected rows, applied in differenced form
            w, _, _ = oracle.gfdm_weights(dd, rp, col, rows=rows)
            tot = 0.0
            for r in rows:
                seg = slice(rp[r], rp[r + 1])
                cj = col[seg]
                yv = (w[seg, 3] * (uu[cj] - uu[r]))[cj != r].sum()
                tot += (yv - d["g"][r]) ** 2
            return tot

        if key == "u":
            up = d["u"].copy(); up[i] += eps
            um = d["u"].copy(); um[i] -= eps
            fd = (local_loss(d, up) - local_loss(d, um)) / (2 * eps)
        else:
            dp = dict(d); dp[key] = d[key].copy(); dp[key][i] += eps
            dm = dict(d); dm[key] = d[key].copy(); dm[key][i] -= eps
            fd = (local_loss(dp, d["u"]) - local_loss(dm, d["u"])) / (2 * eps)
        got = grads[key][i]
        scale = np.abs(grads[key]).max()
        assert abs(got - fd) <= 1e-6 * scale + 1e-4 * abs(fd), (key, i, got, fd)
        checked += 1
    assert checked >= 90


def test_full_buffer_zone_and_extended_stencils(ctx, g):
    print("\n[full] buffer zone, mixed 503,944", flush=True)
    d = W.mixed_block_film()
    n = d["x"].size
    p = g.Particles.from_dict(ctx, d)
    same = g.build_neighbours(ctx, p)
    cross = g.build_neighbours(ctx, p, cross_model=True)
    flag, gh = g.buffer_zone(ctx, p, same, cross, d["film_height"], d["h_other"], d["mass"], d["rho"],
                             d["film_height"][None, :])
    rp_c, col_c = oracle.neighbours(d, cross=True)
    flag_o, gh_o = oracle.buffer_zone(d, rp_c, col_c, d["film_height"], d["h_other"], d["mass"], d["rho"],
                                      d["film_height"][None, :])
    assert np.array_equal(_np(flag), flag_o)
    for key in ("model", "kind", "src", "x", "y", "z", "h", "mass", "rho", "height", "phi"):
        assert np.array_equal(_np(gh[key]), gh_o[key]), key
    assert np.all(np.abs(_np(gh["diam"]) - gh_o["diam"]) <= 1e-15 * gh_o["diam"])
    # film height over the whole cloud
    rp_s, col_s = oracle.neighbours(d)
    H = _np(g.film_height(ctx, p, same, d["diam"]))
    assert np.all(np.abs(H - oracle.film_height(d, rp_s, col_s, d["diam"])) <= 1e-13 * H)
    # extended neighbourhoods and FP32 stencils in the batched launch configuration
    pe = g.extend_particles(ctx, p, gh)
    de = oracle.extend_cloud(d, gh_o)
    nb = g.build_neighbours(ctx, pe, n_rows=n)
    rp_o, col_o = oracle.neighbours_rows(de, n)
    rp, col = nb.export()
    assert np.array_equal(_np(rp), rp_o) and np.array_equal(_np(col), col_o)
    g.autotune(ctx, pe, nb, g.GF_F32)
    w32 = g.gfdm_weights(ctx, pe, nb, g.GF_BATCHED, g.GF_F32)
    rid = np.repeat(np.arange(pe.n), np.diff(rp_o))
    touched = np.unique(rid[(col_o >= n) & (rid < n)])
    rows = np.unique(np.concatenate([touched, np.random.default_rng(41).choice(n, 5000, replace=False)]))
    w_o, _, _ = oracle.gfdm_weights(de, rp_o, col_o, rows=rows)
    sel = np.concatenate([np.arange(rp_o[i], rp_o[i + 1]) for i in rows])
    sub_rp = np.concatenate([[0], np.cumsum(np.diff(rp_o)[rows])])
    e = oracle.operator_error(_np(w32)[sel].astype(np.float64), w_o[sel], sub_rp)
    print(f"[full] {touched.size} rows with ghost neighbours; FP32 operator error {e.max():.3e}", flush=True)
    assert e.max() <= 1e-6


@pytest.mark.parametrize("mixed", [0, 1, 2])
def test_full_projection_solve(ctx, g, mixed):
    print(f"\n[full] projection 4.0M mixed={mixed}", flush=True)
    d = W.projection_cylinder()
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    # the oracle works on its own neighbour lists, which the library's must equal
    rp, col = oracle.neighbours(d)
    rp_g, col_g = nb.export()
    assert np.array_equal(_np(rp_g), rp) and np.array_equal(_np(col_g), col)
    del rp_g, col_g
    w64 = g.gfdm_weights(ctx, p, nb, g.GF_BATCHED, g.GF_F64)
    rhs = np.random.default_rng(31).uniform(-1.0, 1.0, p.n)   # seeded, independent of the device
    x, st = g.poisson_solve(ctx, p, nb, w64, d["row_type"], torch.as_tensor(rhs, device=ctx.device),
                            params=g.solve_params(mixed=mixed))
    print(f"[full] projection stats {st}", flush=True)
    assert st["converged"] == 1 and st["final_rel_res"] <= 1e-8
    xs = _np(x)
    # residual of 3,000 sampled rows under the oracle's own stencils: the sample
    # estimates ||b - A x||_2 (n / 3000 times the sampled sum of squares)
    rows = np.sort(np.random.default_rng(32).choice(p.n, 3000, replace=False))
    w_o, _, _ = oracle.gfdm_weights(d, rp, col, rows=rows)
    val = oracle.poisson_matrix(d, rp, col, w_o, d["row_type"])
    r = np.array([rhs[i] - (val[rp[i]:rp[i + 1]] * xs[col[rp[i]:rp[i + 1]]]).sum() for i in rows])
    scale = np.array([abs(rhs[i]) + np.abs(val[rp[i]:rp[i + 1]] * xs[col[rp[i]:rp[i + 1]]]).sum() for i in rows])
    est = np.sqrt(p.n / rows.size * (r ** 2).sum()) / np.linalg.norm(rhs)
    print(f"[full] sampled residual estimate {est:.2e}; largest row residual / row scale "
          f"{(np.abs(r) / scale).max():.2e}", flush=True)
    assert est <= 1.5e-8
    assert np.all(np.abs(r) <= 1e-6 * scale)
    # the manufactured solution p*: b = A p* on the library's matrix, solved back
    val_g = g.poisson_assemble(ctx, p, nb, w64, d["row_type"])
    A = torch.sparse_csr_tensor(torch.as_tensor(rp, device=ctx.device), torch.as_tensor(col, device=ctx.device).long(),
                                val_g, size=(p.n, p.n))
    ps = torch.as_tensor(d["pstar"], device=ctx.device)
    b = (A @ ps.unsqueeze(1)).squeeze(1)
    del A, val_g
    x, st = g.poisson_solve(ctx, p, nb, w64, d["row_type"], b, params=g.solve_params(mixed=mixed))
    err = ((x - ps).norm() / ps.norm()).item()
    print(f"[full] manufactured solution: {st['inner_its_total']} iterations, error {err:.2e}", flush=True)
    assert st["converged"] == 1 and err <= 1e-6
