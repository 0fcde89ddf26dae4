"""Seeded synthetic particle clouds shaped like the paper's workloads.

This module only lays out particles: positions, support radii h, the model
(3D bulk or 2D film) of each particle, its kind (interior, free surface, wall),
wall/film normals, film heights and smooth test fields.  It performs none of
the method's arithmetic (no neighbourhoods, no PCA, no stencils), so it can
feed both the FP64 oracle and the GPU library from the same bytes.

Shapes follow the paper's test cases: a jittered cubic lattice (plain GFDM
check), a bulk block beside a flat film (Sec. 2.2-2.4, Sec. 4), a jet hitting a
plate and spreading as a film (cleaning jet, Sec. 7.3), and a shallow cylinder
(Sec. 7.1).  The paper's own point clouds are not available; these stand in
for them.

Kinds: 0 interior, 1 free surface, 2 wall (Sec. 2.3).  Models: 0 = 3D bulk,
1 = 2D film.  Film particles are wall particles (Sec. 4.2).
"""
from __future__ import annotations

import numpy as np

INTERIOR, FREE_SURFACE, WALL = 0, 1, 2
BULK, FILM = 0, 1


def rng_for(config_id: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng([2405, 13165, int(config_id), int(extra)])


def _pack(x, y, z, h, model, kind, nx=None, ny=None, nz=None, **extra):
    n = x.shape[0]
    d = dict(
        x=np.ascontiguousarray(x, dtype=np.float64),
        y=np.ascontiguousarray(y, dtype=np.float64),
        z=np.ascontiguousarray(z, dtype=np.float64),
        h=np.ascontiguousarray(h, dtype=np.float64),
        model=np.ascontiguousarray(model, dtype=np.int8),
        kind=np.ascontiguousarray(kind, dtype=np.int8),
        nx=np.ascontiguousarray(np.zeros(n) if nx is None else nx, dtype=np.float64),
        ny=np.ascontiguousarray(np.zeros(n) if ny is None else ny, dtype=np.float64),
        nz=np.ascontiguousarray(np.zeros(n) if nz is None else nz, dtype=np.float64),
    )
    d.update(extra)
    return d


def concat(a: dict, b: dict) -> dict:
    out = {}
    for k in a:
        if isinstance(a[k], np.ndarray) and k in b and isinstance(b[k], np.ndarray) \
                and a[k].shape[:1] == (a["x"].shape[0],):
            out[k] = np.concatenate([a[k], b[k]])
    return out


def _droplets(model, film_height, spacing, rho0=1000.0):
    """Droplet diameters, masses and densities: a film particle that stands for
    an area spacing^2 of film of thickness film_height holds the volume
    film_height * spacing^2 (diameter from V = pi d^3 / 6); a bulk particle
    holds spacing^3."""
    film = model == FILM
    vol = np.where(film, film_height * spacing ** 2, spacing ** 3)
    diam = np.where(film, np.cbrt(6.0 * vol / np.pi), 0.0)
    rho = np.full(model.shape[0], rho0)
    return dict(diam=diam, mass=rho * vol, rho=rho)


def jittered_cube(n_axis: int, s: float, rng, jitter: float = 0.2):
    """n_axis^3 lattice with centres (i+1/2)s, each coordinate jittered by U(+-jitter*s)."""
    i = np.arange(n_axis)
    kk, jj, ii = np.meshgrid(i, i, i, indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.float64)
    pos = (base + 0.5) * s + rng.uniform(-jitter * s, jitter * s, size=base.shape)
    return pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy()


def plain_cube(n_axis: int = 27, s: float = 0.01, seed_extra: int = 0):
    """Jittered lattice in a cube, h = 3 s, every particle 3D interior.

    27^3 = 19,683 particles at s = 0.01 is the 20k-particle plain FP64 case.
    """
    rng = rng_for(1, seed_extra)
    x, y, z = jittered_cube(n_axis, s, rng)
    n = x.shape[0]
    return _pack(x, y, z, np.full(n, 3.0 * s), np.zeros(n), np.zeros(n),
                 spacing=s)


def test_field(x, y, z):
    """f = 1 + x + 2 y^2 - 3 x z with its exact gradient and Laplacian."""
    f = 1.0 + x + 2.0 * y * y - 3.0 * x * z
    gx = 1.0 - 3.0 * z
    gy = 4.0 * y
    gz = -3.0 * x
    lap = np.full_like(x, 4.0)
    return f, gx, gy, gz, lap


def _bulk_block(nx_, ny_, nz_, s, x0, rng, jitter=0.2):
    """Jittered lattice block; bottom layer exactly on z = 0 is wall (normal +z),
    top and lateral outer layers are free surface, the rest interior."""
    i = np.arange(nx_); j = np.arange(ny_); k = np.arange(nz_)
    kk, jj, ii = np.meshgrid(k, j, i, indexing="ij")
    ii = ii.ravel(); jj = jj.ravel(); kk = kk.ravel()
    x = x0 + (ii + 0.5) * s + rng.uniform(-jitter * s, jitter * s, ii.shape)
    y = (jj + 0.5) * s + rng.uniform(-jitter * s, jitter * s, ii.shape)
    z = kk * s + rng.uniform(-jitter * s, jitter * s, ii.shape)
    wall = kk == 0
    z[wall] = 0.0
    kind = np.zeros(ii.shape, np.int8)
    side = (ii == 0) | (ii == nx_ - 1) | (jj == 0) | (jj == ny_ - 1) | (kk == nz_ - 1)
    kind[side] = FREE_SURFACE
    kind[wall] = WALL
    nz = np.where(wall, 1.0, 0.0)
    return x, y, z, kind, nz


def mixed_block_film(factor: int = 1, seed_extra: int = 0):
    """Half a 3D block of height ~0.2 beside half a flat 2D film on z = 0.

    factor = 1: bulk 68 x 136 x 28 = 258,944 lattice particles (s_b = 1/136) on
    [0,0.5]x[0,1]x[0,0.2] and film 350 x 700 = 245,000 jittered 2D lattice
    particles (s_f = 1/700) on [0.5,1]x[0,1]; 503,944 in total.  Larger factors
    coarsen both lattices by that factor (same geometry).  h = 3 x local spacing.
    Film thickness uniform in [1e-3, 5e-3]; h_3D = 3 s_b is the bulk resolution
    used by the 2D->3D test.
    """
    rng = rng_for(2, seed_extra)
    nby = 136 // factor
    nbx = nby // 2
    nbz = max(3, int(round(28 / factor)))
    sb = 1.0 / nby
    xb, yb, zb, kb, nzb = _bulk_block(nbx, nby, nbz, sb, 0.0, rng)
    nb = xb.shape[0]
    nfy = 700 // factor
    nfx = nfy // 2
    sf = 1.0 / nfy
    j = np.arange(nfy); i = np.arange(nfx)
    jj, ii = np.meshgrid(j, i, indexing="ij")
    ii = ii.ravel(); jj = jj.ravel()
    xf = 0.5 + (ii + 0.5) * sf + rng.uniform(-0.2 * sf, 0.2 * sf, ii.shape)
    yf = (jj + 0.5) * sf + rng.uniform(-0.2 * sf, 0.2 * sf, ii.shape)
    nf = xf.shape[0]
    x = np.concatenate([xb, xf]); y = np.concatenate([yb, yf])
    z = np.concatenate([zb, np.zeros(nf)])
    h = np.concatenate([np.full(nb, 3.0 * sb), np.full(nf, 3.0 * sf)])
    model = np.concatenate([np.zeros(nb, np.int8), np.ones(nf, np.int8)])
    kind = np.concatenate([kb, np.full(nf, WALL, np.int8)])
    nzv = np.concatenate([nzb, np.ones(nf)])
    film_height = np.concatenate([np.zeros(nb), rng.uniform(1e-3, 5e-3, nf)])
    h3d = np.full(nb + nf, 3.0 * sb)
    h_other = np.concatenate([np.full(nb, 3.0 * sf), h3d[nb:]])
    spacing = np.concatenate([np.full(nb, sb), np.full(nf, sf)])
    return _pack(x, y, z, h, model, kind, None, None, nzv,
                 film_height=film_height, h3d=h3d, h_other=h_other, n_bulk=nb, n_film=nf,
                 spacing_bulk=sb, spacing_film=sf, **_droplets(model, film_height, spacing))


def advdiff_plate(h: float = 0.06, layers: int = 4, seed_extra: int = 0):
    """Plate for the advection-diffusion analogue (Sec. 7.2): film particles
    on [0,2]x[0,1.5] outside x in (0.75, 1.25) and a 3D block of `layers`
    lattice layers on [0.75,1.25]x[0,1.5] (bottom layer wall, normal +z; top
    layer free surface, normal -z, both pointing into the fluid), spacing
    s = h/3, jitter U(+-0.2 s) in the plane, support h everywhere.  The film
    thickness is the block's height, so the 2D->3D ghost columns match it.
    T0 is a Gaussian of width 0.1 around (1.0, 0.75), constant in depth."""
    rng = rng_for(7, seed_extra)
    s = h / 3.0
    nxf = int(round(2.0 / s)); nyf = int(round(1.5 / s))
    jj, ii = np.meshgrid(np.arange(nyf), np.arange(nxf), indexing="ij")
    xf = (ii.ravel() + 0.5) * s; yf = (jj.ravel() + 0.5) * s
    keep = (xf < 0.75) | (xf > 1.25)
    xf, yf = xf[keep], yf[keep]
    xf = xf + rng.uniform(-0.2 * s, 0.2 * s, xf.size); yf = yf + rng.uniform(-0.2 * s, 0.2 * s, yf.size)
    nbx = int(round(0.5 / s))
    kk, jb, ib = np.meshgrid(np.arange(layers), np.arange(nyf), np.arange(nbx), indexing="ij")
    xb = 0.75 + (ib.ravel() + 0.5) * s; yb = (jb.ravel() + 0.5) * s; zb = kk.ravel() * s
    xb = xb + rng.uniform(-0.2 * s, 0.2 * s, xb.size); yb = yb + rng.uniform(-0.2 * s, 0.2 * s, yb.size)
    kind_b = np.where(kk.ravel() == 0, WALL, np.where(kk.ravel() == layers - 1, FREE_SURFACE, INTERIOR))
    nb, nf = xb.size, xf.size
    x = np.concatenate([xb, xf]); y = np.concatenate([yb, yf]); z = np.concatenate([zb, np.zeros(nf)])
    model = np.concatenate([np.zeros(nb, np.int8), np.ones(nf, np.int8)])
    kind = np.concatenate([kind_b.astype(np.int8), np.full(nf, WALL, np.int8)])
    nzv = np.concatenate([np.where(kind_b == WALL, 1.0, np.where(kind_b == FREE_SURFACE, -1.0, 0.0)), np.ones(nf)])
    depth = (layers - 1) * s
    film_height = np.concatenate([np.zeros(nb), np.full(nf, depth)])
    hh = np.full(nb + nf, h)
    T0 = np.exp(-((x - 1.0) ** 2 + (y - 0.75) ** 2) / (2 * 0.1 ** 2))
    spacing = np.full(nb + nf, s)
    return _pack(x, y, z, hh, model, kind, None, None, nzv, film_height=film_height, h3d=hh.copy(),
                 h_other=hh.copy(), T0=T0, n_bulk=nb, n_film=nf, spacing=s, depth=depth,
                 **_droplets(model, film_height, spacing))


def advdiff_rows(d, h):
    """Row roles of the plate's regular particles (the problem's boundary
    conditions): 3 (zero normal flux) on the 3D block's top and bottom
    layers, 1 (held at zero) within h/2 of the plate's outer edge, 4 (implicit
    diffusion row) elsewhere.  Ghost rows are appended as 1 (known values)."""
    x, y = d["x"], d["y"]
    rt = np.full(x.shape[0], 4, np.int8)
    rt[(np.asarray(d["model"]) == BULK) & (np.asarray(d["kind"]) != INTERIOR)] = 3
    rt[(x < 0.5 * h) | (x > 2 - 0.5 * h) | (y < 0.5 * h) | (y > 1.5 - 0.5 * h)] = 1
    return rt


def advect_plate(h: float = 0.06, layers: int = 4, seed_extra: int = 0, lx: float = 2.5, ly: float = 1.5,
                 ic: str = "gauss", center=(0.6, 0.75), radius: float = 0.2, sigma: float = 0.1):
    """Initial cloud of the model-adaptive advection(-diffusion) case
    (Sec. 7.2): a film of particles on [0,lx]x[0,ly] (spacing s = h/3, jitter
    U(+-0.2 s)), all 2D at t = 0, film thickness (layers-1) s, support h.
    T0, constant in depth, is a Gaussian of width sigma around `center`
    (ic="gauss") or 1 inside the disc of the given radius around it and 0
    outside (ic="disc", Eq. (AdvDiff_IC)).  `edge` marks the particles within
    h/2 of the plate's outer edge (they carry it as they move and change
    model)."""
    rng = rng_for(8, seed_extra)
    s = h / 3.0
    nx_ = int(round(lx / s)); ny_ = int(round(ly / s))
    jj, ii = np.meshgrid(np.arange(ny_), np.arange(nx_), indexing="ij")
    x = (ii.ravel() + 0.5) * s + rng.uniform(-0.2 * s, 0.2 * s, ii.size)
    y = (jj.ravel() + 0.5) * s + rng.uniform(-0.2 * s, 0.2 * s, ii.size)
    n = x.size
    depth = (layers - 1) * s
    film_height = np.full(n, depth)
    model = np.ones(n, np.int8)
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2
    if ic == "disc":
        T0 = (r2 <= radius * radius).astype(np.float64)
    else:
        T0 = np.exp(-r2 / (2 * sigma ** 2))
    edge = ((x < 0.5 * h) | (x > lx - 0.5 * h) | (y < 0.5 * h) | (y > ly - 0.5 * h)).astype(np.float64)
    return _pack(x, y, np.zeros(n), np.full(n, h), model, np.full(n, WALL, np.int8), None, None, np.ones(n),
                 film_height=film_height, T0=T0, edge=edge, spacing=s, depth=depth,
                 **_droplets(model, film_height, np.full(n, s)))


def advdiff_exact(x, y, t, kappa, sigma0=0.1, x0=1.0, y0=0.75):
    """Heat equation in the plane from a Gaussian of width sigma0: the width
    grows to sqrt(sigma0^2 + 2 kappa t) and the peak falls accordingly."""
    s2 = sigma0 ** 2 + 2.0 * kappa * t
    return sigma0 ** 2 / s2 * np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / (2.0 * s2))


def _truncated_normal(rng, n, clip=2.0):
    zeta = rng.standard_normal(n)
    bad = np.abs(zeta) > clip
    while bad.any():
        zeta[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(zeta) > clip
    return zeta


def _jet_cylinder(n_target, rng, radius=0.05, height=0.2, jitter=0.2):
    """Jittered lattice clipped to a vertical cylinder; bottom layer is wall on
    z = 0, outer lateral ring and top layer are free surface."""
    vol = np.pi * radius ** 2 * height
    s = (vol / n_target) ** (1.0 / 3.0)
    nxy = int(np.ceil(2 * radius / s))
    nzl = int(np.floor(height / s)) + 1
    c = (np.arange(nxy) + 0.5) * s - nxy * s / 2
    kk, jj, ii = np.meshgrid(np.arange(nzl), np.arange(nxy), np.arange(nxy), indexing="ij")
    cx = c[ii.ravel()]; cy = c[jj.ravel()]; k = kk.ravel()
    r0 = np.hypot(cx, cy)
    keep = r0 <= radius
    cx = cx[keep]; cy = cy[keep]; k = k[keep]; r0 = r0[keep]
    n = cx.shape[0]
    x = cx + rng.uniform(-jitter * s, jitter * s, n)
    y = cy + rng.uniform(-jitter * s, jitter * s, n)
    z = k * s + rng.uniform(-jitter * s, jitter * s, n)
    wall = k == 0
    z[wall] = 0.0
    kind = np.zeros(n, np.int8)
    kind[(r0 > radius - s) | (k == nzl - 1)] = FREE_SURFACE
    kind[wall] = WALL
    return x, y, z, kind, s


def jet_impact(n_bulk: int = 1_000_000, n_film: int = 1_000_000, seed_extra: int = 0):
    """Jet-on-plate layout with uneven neighbourhoods (cleaning-jet shape).

    Bulk: jittered lattice in the cylinder r <= 0.05, 0 <= z <= 0.2; wall at
    z = 0.  Film: z = 0, r ~ U(0.05, 0.5), theta ~ U(0, 2 pi), so the areal
    density falls as 1/r; local spacing s_f(r) = sqrt(2 pi 0.45 r / N_f); film
    thickness 5e-3 * 0.05 / r.  h_i = base * exp(0.3 zeta), zeta ~ N(0,1)
    truncated to |zeta| <= 2, base = 2.56 s_b (bulk) or 4.74 s_f(r) (film), so
    neighbour counts span roughly 20..250.
    """
    rng = rng_for(3, seed_extra)
    xb, yb, zb, kb, sb = _jet_cylinder(n_bulk, rng)
    nb = xb.shape[0]
    r = rng.uniform(0.05, 0.5, n_film)
    th = rng.uniform(0.0, 2 * np.pi, n_film)
    xf = r * np.cos(th); yf = r * np.sin(th)
    sf = np.sqrt(2 * np.pi * 0.45 * r / n_film)
    hb = 2.56 * sb * np.exp(0.3 * _truncated_normal(rng, nb))
    hf = 4.74 * sf * np.exp(0.3 * _truncated_normal(rng, n_film))
    x = np.concatenate([xb, xf]); y = np.concatenate([yb, yf])
    z = np.concatenate([zb, np.zeros(n_film)])
    model = np.concatenate([np.zeros(nb, np.int8), np.ones(n_film, np.int8)])
    kind = np.concatenate([kb, np.full(n_film, WALL, np.int8)])
    nzv = np.concatenate([np.where(kb == WALL, 1.0, 0.0), np.ones(n_film)])
    film_height = np.concatenate([np.zeros(nb), 5e-3 * 0.05 / r])
    h3d = np.full(nb + n_film, 3.0 * sb)
    # film resolution at the jet's foot: the film's own h there
    h_other = np.concatenate([np.full(nb, 4.74 * np.sqrt(2 * np.pi * 0.45 * 0.05 / n_film)), h3d[nb:]])
    spacing = np.concatenate([np.full(nb, sb), sf])
    return _pack(x, y, z, np.concatenate([hb, hf]), model, kind, None, None, nzv,
                 film_height=film_height, h3d=h3d, h_other=h_other, n_bulk=nb, n_film=n_film,
                 spacing_bulk=sb, **_droplets(model, film_height, spacing))


def fourier_field(x, y, z, rng, modes: int = 8):
    """Sum of `modes` unit-amplitude cosines cos(2 pi k.x + phase),
    k in {-3..3}^3 without 0, phase ~ U(0, 2 pi)."""
    ks = []
    while len(ks) < modes:
        k = rng.integers(-3, 4, size=3)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    ph = rng.uniform(0, 2 * np.pi, modes)
    f = np.zeros_like(x)
    for m in range(modes):
        f += np.cos(2 * np.pi * (ks[m, 0] * x + ks[m, 1] * y + ks[m, 2] * z) + ph[m])
    return f


def diff_cube(n_axis: int = 100, s: float = 0.01, seed_extra: int = 0):
    """Jittered lattice for the differentiation case: n_axis^3 particles,
    h = 3 s, all 3D interior, plus two independent smooth Fourier fields u, g."""
    rng = rng_for(4, seed_extra)
    x, y, z = jittered_cube(n_axis, s, rng)
    n = x.shape[0]
    u = fourier_field(x, y, z, rng_for(4, 1000 + seed_extra))
    g = fourier_field(x, y, z, rng_for(4, 2000 + seed_extra))
    return _pack(x, y, z, np.full(n, 3.0 * s), np.zeros(n), np.zeros(n), u=u, g=g,
                 spacing=s)


# Row types of the pressure system.
ROW_INTERIOR, ROW_DIRICHLET, ROW_NEUMANN_COMBINED, ROW_NEUMANN_PLAIN = 0, 1, 2, 3


def projection_cylinder(n_target: int = 4_000_000, seed_extra: int = 0,
                        wall_rows: int = ROW_NEUMANN_PLAIN):
    """Bulk-only jet cylinder for the pressure-Poisson solve, uniform h = 3 s_b.

    Bottom wall rows are Neumann rows (plain n.grad rows by default, or the
    combined PDE + zeta BC rows), free-surface rows are Dirichlet, the rest
    interior.  The wall normal of the boundary condition is the outward one
    (-z on the bottom plate).  p*(x) = sin(20x + 1) cos(20y) (1 + 5z) is the
    manufactured solution.
    """
    rng = rng_for(5, seed_extra)
    x, y, z, kind, s = _jet_cylinder(n_target, rng)
    n = x.shape[0]
    row_type = np.full(n, ROW_INTERIOR, np.int8)
    row_type[kind == FREE_SURFACE] = ROW_DIRICHLET
    row_type[kind == WALL] = wall_rows
    nzv = np.where(kind == WALL, -1.0, 0.0)
    pstar = np.sin(20 * x + 1) * np.cos(20 * y) * (1 + 5 * z)
    return _pack(x, y, z, np.full(n, 3.0 * s), np.zeros(n), kind, None, None, nzv,
                 row_type=row_type, pstar=pstar, spacing=s)


def shallow_cylinder(s: float = 0.15, h_factor: float = 4.0, seed_extra: int = 0):
    """Analogue of the steady shallow-cylinder case (Sec. 7.1): unit-radius
    cylinder filled to 0.15, two lattice layers (z = 0 and z = s).

    Base layer: wall, normal +z.  Upper layer: outer ring is the vertical wall
    (horizontal radial normal), the rest free surface.  The representative
    mass is rho * s^3 with rho = 1000.
    """
    rng = rng_for(6, seed_extra)
    nxy = int(np.ceil(2.0 / s)) + 1
    c = (np.arange(nxy) - (nxy - 1) / 2.0) * s
    pts = []
    for k in range(2):
        cx, cy = np.meshgrid(c, c, indexing="ij")
        cx = cx.ravel(); cy = cy.ravel()
        keep = np.hypot(cx, cy) <= 1.0
        cx = cx[keep]; cy = cy[keep]
        jx = rng.uniform(-0.1 * s, 0.1 * s, cx.shape)
        jy = rng.uniform(-0.1 * s, 0.1 * s, cx.shape)
        pts.append((cx + jx, cy + jy, np.full(cx.shape, k * s), np.full(cx.shape, k)))
    x = np.concatenate([p[0] for p in pts]); y = np.concatenate([p[1] for p in pts])
    z = np.concatenate([p[2] for p in pts]); k = np.concatenate([p[3] for p in pts])
    r = np.hypot(x, y)
    n = x.shape[0]
    kind = np.full(n, FREE_SURFACE, np.int8)
    nx = np.zeros(n); ny = np.zeros(n); nz = np.zeros(n)
    base = k == 0
    kind[base] = WALL; nz[base] = 1.0
    rim = (k == 1) & (r > 1.0 - 0.75 * s)
    kind[rim] = WALL; nx[rim] = x[rim] / r[rim]; ny[rim] = y[rim] / r[rim]
    mass = np.full(n, 1000.0 * s ** 3)
    return _pack(x, y, z, np.full(n, h_factor * s), np.zeros(n), kind, nx, ny, nz,
                 mass=mass, rho=np.full(n, 1000.0), base=base, rim=rim)


def subset(d: dict, idx) -> dict:
    n = d["x"].shape[0]
    out = {}
    for k, v in d.items():
        if isinstance(v, np.ndarray) and v.shape[:1] == (n,):
            out[k] = np.ascontiguousarray(v[idx])
        else:
            out[k] = v
    return out
