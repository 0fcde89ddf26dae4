"""Diffusion analogue of the advection-diffusion test (Sec. 7.2) on the
library: a static plate of film particles with a 3D block in its middle
(fixed interfaces), so the ghost particles of the buffer zone keep their
places and only their data is recomputed each step (Sec. 6.2).  Each step:
gf_buffer_zone maps the current field onto the ghosts (Alg. 5 data mapping),
then gf_poisson_solve performs one implicit Euler step (I - dt kappa Lap)
T^{n+1} = T^n over the extended neighbourhoods (GF_ROW_IMPLICIT rows), with
zero-flux rows on the block's top and bottom, zero on the plate's outer edge
and the ghost rows pinned to their values.  Every step runs in the
library's kernels; this module only chains the calls and moves buffers.
"""
from __future__ import annotations

import time

import torch

from . import gfdm as g


class DiffusionPlate:
    def __init__(self, ctx, d, rows, kappa, dt, rtol=1e-12):
        self.ctx = ctx
        self.d = d
        self.kappa = kappa
        self.dt = dt
        dev = ctx.device
        self.p = g.Particles.from_dict(ctx, d)
        self.n = self.p.n
        self.same = g.build_neighbours(ctx, self.p)
        self.cross = g.build_neighbours(ctx, self.p, cross_model=True)
        self.H = torch.as_tensor(d["film_height"], device=dev)
        self.h_other = torch.as_tensor(d["h_other"], device=dev)
        self.mass = torch.as_tensor(d["mass"], device=dev)
        self.rho = torch.as_tensor(d["rho"], device=dev)
        T0 = torch.as_tensor(d["T0"], device=dev)
        _, gh = g.buffer_zone(ctx, self.p, self.same, self.cross, self.H, self.h_other, self.mass, self.rho,
                              T0[None, :])
        self.n_ghosts = int(gh["x"].shape[0])
        self.pe = g.extend_particles(ctx, self.p, gh)
        self.nb = g.build_neighbours(ctx, self.pe, n_rows=self.n)
        self.w = g.gfdm_weights(ctx, self.pe, self.nb, g.GF_BATCHED, g.GF_F64)
        rt = torch.ones(self.pe.n, dtype=torch.int8)
        rt[: self.n] = torch.as_tensor(rows)
        self.rt = rt.to(dev)
        self.bc = self.rt[: self.n] != g.ROW_IMPLICIT
        self.params = g.solve_params(implicit_a=dt * kappa, rtol=rtol)

    def step(self, T):
        ctx = self.ctx
        _, gh = g.buffer_zone(ctx, self.p, self.same, self.cross, self.H, self.h_other, self.mass, self.rho,
                              T[None, :])
        gT = gh["phi"][0]
        rhs = torch.cat([torch.where(self.bc, torch.zeros_like(T), T), gT])
        x0 = torch.cat([T, gT])
        x, st = g.poisson_solve(ctx, self.pe, self.nb, self.w, self.rt, rhs, x0=x0, params=self.params)
        return x[: self.n].clone(), st

    def run(self, steps):
        T = torch.as_tensor(self.d["T0"], device=self.ctx.device).clone()
        its = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            T, st = self.step(T)
            its += st["inner_its_total"]
        torch.cuda.synchronize()
        return T, {"seconds": time.perf_counter() - t0, "steps": steps, "bicgstab_its": its}


_FIELDS = ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz", "mass", "rho")


class AdvectPlate:
    """The model-adaptive case of the advection-diffusion test (Sec. 7.2): a
    film plate moves with v = (1, 0, 0) through the window x0 <= x <= x1.
    Film particles that enter the window turn into 3D columns (Sec. 5.2),
    3D wall particles that leave it collapse back onto the film with their
    columns (Sec. 5.1, Alg. 3); the ghosts (Alg. 5), the extended
    neighbourhoods and the stencils are rebuilt at every step, since every
    particle has moved, and one implicit Euler diffusion step follows
    (zero normal flux on 3D walls and free surfaces, zero on the plate's
    outer edge); with kappa = 0 (pure advection) a step ends after the
    transitions.  The temperature and a 0/1 marker of the plate's edge are
    carried through both transitions as mapped fields; the film thickness is
    carried by the film particles.  Each transition, build and solve runs in
    the library's kernels; this class moves the particles, selects the
    flagged ones and concatenates buffers."""

    def __init__(self, ctx, d, kappa, dt, x0=1.0, x1=2.0, rtol=1e-12):
        # (x0, x1) = (-inf, inf) turns the whole plate into 3D at the first
        # step and keeps it there: the full-3D run of the same case
        self.ctx = ctx
        self.kappa, self.dt, self.x0, self.x1 = kappa, dt, x0, x1
        dev = ctx.device
        c = {k: torch.as_tensor(d[k], device=dev) for k in _FIELDS}
        c["model"] = c["model"].to(torch.int8)
        c["kind"] = c["kind"].to(torch.int8)
        c["T"] = torch.as_tensor(d["T0"], device=dev, dtype=torch.float64).clone()
        c["H"] = torch.as_tensor(d["film_height"], device=dev, dtype=torch.float64).clone()
        c["edge"] = torch.as_tensor(d["edge"], device=dev, dtype=torch.float64).clone()
        self.c = c
        self.params = g.solve_params(implicit_a=dt * kappa, rtol=rtol)
        self.stats = {"bicgstab_its": 0, "to_3d": 0, "to_2d": 0, "max_n": 0, "max_ghosts": 0}

    def _particles(self):
        return g.Particles.from_dict(self.ctx, self.c)

    def _rows(self):
        c = self.c
        rt = torch.full_like(c["model"], g.ROW_IMPLICIT)
        rt[(c["model"] == 0) & (c["kind"] != 0)] = g.ROW_NEUMANN
        rt[c["edge"] > 0.5] = g.ROW_DIRICHLET
        return rt

    def step(self):
        ctx, c = self.ctx, self.c
        c["x"] = c["x"] + self.dt
        # film particles inside the window -> 3D columns
        f2 = (c["model"] == 1) & (c["x"] >= self.x0) & (c["x"] <= self.x1)
        if bool(f2.any()):
            p = self._particles()
            o = g.transition_2d_to_3d(ctx, p, f2.to(torch.uint8) * 2, c["H"], c["h"], c["mass"], c["rho"],
                                      torch.stack([c["T"], c["edge"]]))
            new = {k: o[k] for k in _FIELDS}
            new["T"], new["edge"] = o["phi"][0], o["phi"][1]
            new["H"] = torch.zeros_like(o["x"])
            keep = ~f2
            c = {k: torch.cat([c[k][keep], new[k].to(c[k].dtype)]) for k in c}
            self.stats["to_3d"] += int(f2.sum())
        # 3D wall particles past the window -> film particles
        f1 = (c["model"] == 0) & (c["kind"] == 2) & (c["x"] > self.x1)
        if bool(f1.any()):
            self.c = c
            p = self._particles()
            same = g.build_neighbours(ctx, p)
            o = g.transition_3d_to_2d_cloud(ctx, p, same, f1.to(torch.uint8), c["mass"], c["rho"],
                                            torch.stack([c["T"], c["edge"]]), film_height=c["H"], h_film=c["h"])
            c = {k: o[k] for k in _FIELDS}
            c["T"], c["edge"], c["H"] = o["phi"][0], o["phi"][1], o["height"]
            self.stats["to_2d"] += int(f1.sum())
        self.c = c
        if self.kappa == 0.0:
            return
        # ghosts, extended neighbourhoods, stencils, one implicit step
        p = self._particles()
        n = p.n
        same = g.build_neighbours(ctx, p)
        cross = g.build_neighbours(ctx, p, cross_model=True)
        _, gh = g.buffer_zone(ctx, p, same, cross, c["H"], c["h"], c["mass"], c["rho"], c["T"][None, :])
        pe = g.extend_particles(ctx, p, gh)
        nb = g.build_neighbours(ctx, pe, n_rows=n)
        w = g.gfdm_weights(ctx, pe, nb, g.GF_BATCHED, g.GF_F64)
        rt = torch.cat([self._rows(), torch.full((pe.n - n,), g.ROW_DIRICHLET, dtype=torch.int8, device=ctx.device)])
        gT = gh["phi"][0]
        T = c["T"]
        rhs = torch.cat([torch.where(rt[:n] == g.ROW_IMPLICIT, T, torch.zeros_like(T)), gT])
        x, st = g.poisson_solve(ctx, pe, nb, w, rt, rhs, x0=torch.cat([T, gT]), params=self.params)
        c["T"] = x[:n].clone()
        self.stats["bicgstab_its"] += st["inner_its_total"]
        self.stats["max_n"] = max(self.stats["max_n"], n)
        self.stats["max_ghosts"] = max(self.stats["max_ghosts"], pe.n - n)
        for o in (same, cross, nb):
            o.close()

    def run(self, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        return self.c, dict(self.stats, seconds=time.perf_counter() - t0, steps=steps)
