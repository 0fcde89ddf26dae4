"""Diffusion analogue of the advection-diffusion test (Sec. 7.3) on the
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
