#!/usr/bin/env python3
"""Throughput of the GFDM hot path on one MI355X.

Metric: particles/s for GFDM stencil weights + application (all four
stencils d/dx, d/dy, d/dz, Laplacian applied to one scalar field), on the
mixed bulk/film cloud of 503,944 particles (258,944 jittered-lattice bulk
particles beside 245,000 film particles on z = 0, h = 3 x local spacing).
value = N / t_step for the batched path: one gf_gfdm_weights_apply call that
computes every stencil (FP64 moments and solves, QR fallback), stores it in
FP32 and applies it to the field.  The same work as two calls (weights, then
apply), the plain FP64 path and the other steps of the hot path are timed
beside it.

A step is one weights + apply pass over the resident cloud; K steps are timed
with HIP events on the library's stream after W warm-up steps.  The FP64 CPU
oracle is timed on the same workload (weights + apply, every particle) and
its stencils are the reference for the stated operator error.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector
BANDS = (24, 48, 128)        # neighbour-count bands of the batched kernels (bands 0-2 are tiled)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--factor", type=int, default=1, help="coarsen the workload (parity/debug only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip timing the other hot-path steps")
    ap.add_argument("--poisson", type=int, default=0,
                    help="also solve the pressure system on a jet cylinder of this many particles")
    ap.add_argument("--jet", action="store_true",
                    help="also time the fused step on the 2.0M-particle jet cloud (uneven neighbourhoods)")
    ap.add_argument("--diff", action="store_true",
                    help="also time forward + backward of the stencil operator on the 1e6-particle cube")
    ap.add_argument("--advdiff", action="store_true",
                    help="also run the diffusion analogue of the advection-diffusion test (Sec. 7.3) at "
                         "h = 0.06, 0.03, 0.015, and its model-adaptive moving-plate case at h = 0.12, 0.06, 0.03, "
                         "against the exact solutions (convergence study)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warm-up plus a few steps of the metric path and exit (for rocprofv3)")
    return ap.parse_args()


KERNEL_SOURCES = ("weights.hip", "stencil_common.h", "internal.h", "apply.hip")


def measure_hbm(dev):
    """Achievable HBM bandwidth of this GPU, for reference beside the published
    peak: a 1 GiB device-to-device copy (1 GiB read + 1 GiB written) and a
    4 GiB streaming read (a sum), each the mean of 10 runs between events after
    2 warm-ups.  Outside every timed region; the buffers are freed after."""
    import torch
    x = torch.ones(1 << 29, dtype=torch.float64, device=dev)
    y = torch.empty(1 << 27, dtype=torch.float64, device=dev)

    def ms(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 10

    copy_ms = ms(lambda: y.copy_(x[: y.numel()]))
    read_ms = ms(lambda: x.sum())
    out = {"copy_GBs": round(2 * 8 * y.numel() / (copy_ms * 1e-3) / 1e9, 1),
           "read_GBs": round(8 * x.numel() / (read_ms * 1e-3) / 1e9, 1),
           "method": "1 GiB device copy (read + write) and 4 GiB sum, torch ops timed with events"}
    del x, y
    torch.cuda.empty_cache()
    return out


def measured_traffic(launch, team):
    """HBM bytes per launch of `launch` at team size `team`, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (already scaled by the copy
    calibration), or None when no summary covers it or the kernel sources
    have changed since the counters were taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_13165_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic_json: "):
                    continue
                rec = json.loads(line[len("traffic_json: "):])
                if (rec.get("launch") == launch and rec.get("team") == team
                        and rec.get("source_sha256_16") == digest and rec.get("bytes_per_launch")):
                    return float(rec["bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def band_of(n):
    for b, hi in enumerate(BANDS):
        if n <= hi:
            return b
    return len(BANDS)


def algorithmic_costs(rp, model, fused):
    """Per (model, band) launch of the stencil kernels: rows, nnz, FP64 flops
    and unique bytes of the FP32-output path.
    flops/row: Gram n m(m+1) + weighted monomials n m + targets 8 n m
               + factorisation and inverse ~ m^3/3 + 2 m^3 (+ 8 n applied)
    bytes/row: 2 n (tile slots) + 16 n (FP32 stencils) + 32 (own x, y, z, h)
               (+ 8 field value + 32 four results when fused)."""
    import numpy as np
    n_i = np.diff(rp)
    out = {}
    bands = np.searchsorted(np.array(BANDS), n_i, side="left")
    # launch units: the tiled bands 0-2 of a model run as one launch ("tiles"), band 3 alone
    for m in (0, 1):
        M = 10 if m == 0 else 6
        for unit, sel in (("tiles", bands <= 2), ("b3", bands == 3)):
            nn = n_i[(model == m) & sel]
            if nn.size == 0:
                continue
            flops = float((nn * (M * (M + 1) + M + 8 * M + (8 if fused else 0))).sum()
                          + nn.size * (M ** 3 / 3 + 2 * M ** 3))
            byts = float((18 * nn + (72 if fused else 32)).sum())
            out[(m, unit)] = dict(rows=int(nn.size), nnz=int(nn.sum()), flops=flops, bytes=byts)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the stencil path runs on a single MI355X "
              "(sharding over several GPUs is not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_13165_amd import gfdm as g
    from paper_2405_13165_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t0 = time.time()
    d = W.mixed_block_film(factor=args.factor)
    N = d["x"].shape[0]
    print(f"[bench] workload generated: {N} particles ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)

    ctx = g.Context(0)
    p = g.Particles.from_dict(ctx, d)
    f, *_ = W.test_field(d["x"], d["y"], d["z"])
    u = torch.as_tensor(f, device=ctx.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb = g.build_neighbours(ctx, p)
    torch.cuda.synchronize()
    t_nbr_first = time.perf_counter() - t0
    nnz = nb.nnz
    rp_d, col_d = nb.export()
    rp = rp_d.cpu().numpy()
    print(f"[bench] neighbours: nnz={nnz} max_row={nb.max_row}", file=sys.stderr, flush=True)

    w32 = torch.empty((nnz, 4), dtype=torch.float32, device=ctx.device)
    w64 = torch.empty((nnz, 4), dtype=torch.float64, device=ctx.device)
    y32 = torch.empty((4, N), dtype=torch.float64, device=ctx.device)
    y64 = torch.empty((4, N), dtype=torch.float64, device=ctx.device)
    yf = torch.empty((4, N), dtype=torch.float64, device=ctx.device)
    status = torch.empty(N, dtype=torch.int8, device=ctx.device)

    def step_batched():
        g.gfdm_weights(ctx, p, nb, g.GF_BATCHED, g.GF_F32, out=w32, status=status)
        g.apply_stencil(ctx, nb, w32, u, 0xF, out=y32)

    def step_plain():
        g.gfdm_weights(ctx, p, nb, g.GF_PLAIN_F64, g.GF_F64, out=w64)
        g.apply_stencil(ctx, nb, w64, u, 0xF, out=y64)

    def step_fused():
        g.gfdm_weights_apply(ctx, p, nb, u, 0xF, g.GF_F32, w_out=w32, out=yf, status=status)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    t0 = time.perf_counter()
    teams = g.autotune(ctx, p, nb, g.GF_F32)
    print(f"[bench] autotune {time.perf_counter() - t0:.2f}s: {teams}", file=sys.stderr, flush=True)

    if args.profile_only:
        timed(step_fused, max(args.steps, 1), args.warmup)
        timed(step_batched, 2, 1)
        timed(step_plain, 2, 1)
        # a plain device copy of known size: calibrates the HBM byte counters
        # (FETCH_SIZE / WRITE_SIZE) read by rocprofv3 for the same run
        src = torch.ones(1 << 27, dtype=torch.float64, device=ctx.device)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] profile run done (copy calibration: 1 GiB read + 1 GiB written)",
              file=sys.stderr, flush=True)
        return

    ms_eager = timed(step_fused, args.steps, args.warmup)
    ms_batched = timed(step_batched, args.steps, args.warmup)
    ms_plain = timed(step_plain, args.steps, args.warmup)
    # the same fused step captured once in a HIP graph and replayed; the
    # replay must reproduce the eager outputs exactly
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step_fused()
    step_fused()
    torch.cuda.synchronize()
    w_ref, y_ref = w32.clone(), yf.clone()
    w32.zero_()
    yf.zero_()
    graph.replay()
    torch.cuda.synchronize()
    graph_ok = bool(torch.equal(w32, w_ref) and torch.equal(yf, y_ref))
    del w_ref, y_ref
    ms_graph = timed(graph.replay, args.steps, args.warmup)
    use_graph = graph_ok and ms_graph < ms_eager
    ms_fused = ms_graph if use_graph else ms_eager
    print(f"[bench] fused eager {ms_eager:.3f} ms  graph {ms_graph:.3f} ms (replay exact: {graph_ok})  "
          f"separate calls {ms_batched:.3f} ms  plain {ms_plain:.3f} ms", file=sys.stderr, flush=True)

    # per-kernel times of the metric step (HIP events around each launch)
    ctx.profile(True)
    reps = max(3, min(args.steps, 10))
    for _ in range(reps):
        step_fused()
    prof = ctx.profile_read()
    for _ in range(reps):
        step_batched()
    prof_sep = ctx.profile_read()
    for _ in range(reps):
        step_plain()
    prof_plain = ctx.profile_read()
    ctx.profile(False)
    costs = algorithmic_costs(rp, d["model"], fused=True)
    kernels = {}
    for name, (cnt, tot) in prof.items():
        kernels[name] = {"launches": cnt, "avg_us": 1000.0 * tot / cnt}
    # dominant kernel: the (model, band) stencil launch with the largest time
    weights_kernels = {k: v for k, v in kernels.items() if k.startswith("weights_apply_")}
    dom = max(weights_kernels, key=lambda k: weights_kernels[k]["avg_us"] * weights_kernels[k]["launches"])
    m_dom = 0 if "_3d_" in dom else 1
    b_dom = dom.rsplit("_", 1)[1]
    per_launch_s = kernels[dom]["avg_us"] * 1e-6
    flops_l = costs[(m_dom, b_dom)]["flops"]
    bytes_l = costs[(m_dom, b_dom)]["bytes"]
    tflops = flops_l / per_launch_s / 1e12
    gbs = bytes_l / per_launch_s / 1e9
    frac_alu = tflops / PEAK_FP64_TFLOPS
    frac_hbm = gbs / PEAK_HBM_GBS
    if frac_alu >= frac_hbm:
        roof = {"kernel": dom, "bound": "alu", "achieved": round(tflops, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(frac_alu, 4), "traffic": None}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(frac_hbm, 4), "traffic": None}
    team_dom = teams["fused"][4 * m_dom + (2 if b_dom == "tiles" else 3)]
    traffic, traffic_src = measured_traffic(dom, team_dom)
    roof["traffic"] = round(traffic) if traffic is not None else None
    if traffic is not None:
        roof["traffic_note"] = (f"HBM bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated) "
                                f"from {traffic_src}; algorithmic bytes {bytes_l}")
    roof["other_roof"] = {"hbm_GBs": round(gbs, 1), "hbm_frac": round(frac_hbm, 4),
                          "fp64_TFLOPs": round(tflops, 3), "fp64_frac": round(frac_alu, 4)}
    roof["algorithmic_per_launch"] = {"flops": flops_l, "bytes": bytes_l, "avg_launch_us": round(per_launch_s * 1e6, 2),
                                      "rows": costs[(m_dom, b_dom)]["rows"], "nnz": costs[(m_dom, b_dom)]["nnz"]}

    # whole-step HBM view: unique bytes of the fused step (slots, FP32
    # stencils written, positions, field, four results)
    step_bytes = float(nnz) * (2 + 16) + N * (32 + 8 + 32)
    step_hbm_frac = step_bytes / (ms_fused * 1e-3) / 1e9 / PEAK_HBM_GBS

    # ---- outputs of the metric step (stencils stored by the fused call and
    # its results), of the separate calls, and of the plain FP64 path
    step_batched()
    torch.cuda.synchronize()
    y32n = y32.cpu().numpy()
    step_fused(); step_plain()
    torch.cuda.synchronize()
    w32n = w32.double().cpu().numpy()
    w64n = w64.cpu().numpy()
    yfn = yf.cpu().numpy()

    result = {
        "metric": "particles/s for GFDM weights+apply; batched-FP32 vs plain-FP64 @1e-6 rel err",
        "value": N / (ms_fused * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fused,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "weights_storage": "f32",
        "data": "synthetic",
        "config": {"workload": "mixed bulk/film cloud: 258,944 jittered-lattice bulk particles beside "
                               "245,000 film particles on z=0, h = 3 x spacing (10 / 6 monomials)",
                   "n_particles": N, "nnz": nnz, "factor": args.factor},
        "step": ("gf_gfdm_weights_apply: batched stencils stored in FP32 and applied (one call), "
                 + ("replayed from a HIP graph" if use_graph else "eager launches (faster than the graph replay)")),
        "fused_eager": {"value": N / (ms_eager * 1e-3), "ms_per_step": ms_eager},
        "fused_graph": {"value": N / (ms_graph * 1e-3), "ms_per_step": ms_graph, "replay_exact": graph_ok},
        "plain_f64": {"value": N / (ms_plain * 1e-3), "ms_per_step": ms_plain,
                      "step": "gf_gfdm_weights(GF_PLAIN_F64) + gf_apply_stencil"},
        "separate_calls_f32": {"value": N / (ms_batched * 1e-3), "ms_per_step": ms_batched,
                               "step": "gf_gfdm_weights(GF_BATCHED, FP32) + gf_apply_stencil"},
        "speedup_batched_vs_plain": ms_plain / ms_fused,
        "team_sizes": teams,
        "step_hbm_frac": round(step_hbm_frac, 4),
        "kernels_batched": kernels,
        "kernels_separate_calls": {k: {"launches": c, "avg_us": 1000.0 * t / c} for k, (c, t) in prof_sep.items()},
        "kernels_plain": {k: {"launches": c, "avg_us": 1000.0 * t / c} for k, (c, t) in prof_plain.items()},
        "roofline": roof,
    }
    hbm_meas = measure_hbm(ctx.device)
    result["hbm_measured"] = hbm_meas
    roof["other_roof"]["hbm_frac_of_measured_copy"] = round(gbs / hbm_meas["copy_GBs"], 4)

    # ---- other hot-path steps (timed once each after a warm-up call)
    if not args.no_rows:
        rows = {"build_neighbours_first_ms": t_nbr_first * 1e3}

        kern = {}

        def once(fn, key=None):
            """Wall time of one call after a warm-up call; with key, also the
            library's own per-kernel times of that call."""
            fn()
            torch.cuda.synchronize()
            if key:
                ctx.profile(True)
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            el = (time.perf_counter() - t) * 1e3
            if key:
                kern[key] = {k: round(1000.0 * tt / c, 1) for k, (c, tt) in ctx.profile_read().items()}
                ctx.profile(False)
            return el, r

        rows["build_neighbours_ms"], nb2 = once(lambda: g.build_neighbours(ctx, p), "build_neighbours")
        del nb2
        xnb = g.build_neighbours(ctx, p, cross_model=True)
        rows["classify_pca_ms"], cl = once(lambda: g.classify_pca(ctx, p, nb, xnb, film_height=d["film_height"],
                                                                 h3d=d["h3d"]), "classify_pca")
        flag = cl[3]
        mass = torch.ones(N, dtype=torch.float64, device=ctx.device)
        rho = torch.full((N,), 1000.0, dtype=torch.float64, device=ctx.device)
        # this cloud flags no particle (its bottom walls see interior neighbours only): the transition is
        # timed with every bulk wall particle flagged, which deletes the layers above the bottom
        tflag = torch.as_tensor(((d["model"] == 0) & (d["kind"] == W.WALL)).astype(np.uint8), device=ctx.device)
        rows["transition_ms"], _ = once(lambda: g.transition_3d_to_2d(ctx, p, nb, tflag, mass, rho, u), "transition")
        rows["apply_ms"], _ = once(lambda: g.apply_stencil(ctx, nb, w32, u, 0xF, out=y32), "apply")
        ybar = torch.ones((1, N), dtype=torch.float64, device=ctx.device)
        rows["apply_adjoint_ms"], _ = once(lambda: g.apply_stencil_adjoint(ctx, nb, w32, ybar, g.OP_LAP),
                                           "apply_adjoint")
        rows["weights_adjoint_ms"], _ = once(lambda: g.gfdm_weights_adjoint(ctx, p, nb, u, ybar, g.OP_LAP),
                                             "weights_adjoint")
        # coupling layer: film height (Eq. Height), ghost particles of the buffer zone (Alg. 5), and the
        # stencils over the extended neighbourhoods (regular + ghost particles, Sec. 6.2)
        rows["film_height_ms"], _ = once(lambda: g.film_height(ctx, p, nb, d["diam"]), "film_height")
        rows["buffer_zone_ms"], bz = once(lambda: g.buffer_zone(ctx, p, nb, xnb, d["film_height"], d["h_other"],
                                                                d["mass"], d["rho"]), "buffer_zone")
        ghosts = bz[1]
        pe = g.extend_particles(ctx, p, ghosts)
        rows["extended_build_ms"], nbe = once(lambda: g.build_neighbours(ctx, pe, n_rows=N), "extended_build")
        ue = torch.cat([u, torch.as_tensor(W.test_field(ghosts["x"].cpu().numpy(), ghosts["y"].cpu().numpy(),
                                                        ghosts["z"].cpu().numpy())[0], device=ctx.device)])
        rows["extended_weights_apply_ms"], _ = once(
            lambda: g.gfdm_weights_apply(ctx, pe, nbe, ue, wtype=g.GF_F32, store_weights=False),
            "extended_weights_apply")
        rows["buffer_zone_counts"] = {"flagged": int(bz[0].sum().item()), "ghosts": int(ghosts["x"].shape[0]),
                                      "ghosts_3d": int((ghosts["model"] == 0).sum().item()),
                                      "extended_nnz": nbe.nnz}
        del nbe, pe
        result["rows"] = rows
        result["rows_kernels_us"] = kern
        # algorithmic bytes of each row: per particle (N) and per neighbour entry (nnz) the bytes a
        # row must read or write at least once
        film_nnz = float((np.diff(rp)[d["model"] == 1]).sum())
        row_bytes = {"build_neighbours": 4.0 * nnz + 41.0 * N, "classify_pca": 4.0 * nnz + 106.0 * N,
                     "apply": 18.0 * nnz + 40.0 * N, "transition": 4.0 * nnz + 48.0 * N,
                     "apply_adjoint": 48.0 * nnz + 16.0 * N, "weights_adjoint": 80.0 * nnz + 56.0 * N,
                     "film_height": 4.0 * film_nnz + 60.0 * float((d["model"] == 1).sum()) + 13.0 * N,
                     "buffer_zone": 60.0 * N}
        roof_rows = {}
        for key, byts in row_bytes.items():
            us = sum(kern.get(key, {}).values())
            if us > 0:
                roof_rows[key] = {"kernel_us": round(us, 1), "algorithmic_bytes": byts,
                                  "GBs": round(byts / (us * 1e-6) / 1e9, 1),
                                  "hbm_frac": round(byts / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                                  "frac_of_measured_copy": round(byts / (us * 1e-6) / 1e9 / hbm_meas["copy_GBs"], 4)}
        result["rows_roofline"] = roof_rows
        result["flags"] = {"bulk_to_film": int((flag == 1).sum().item()), "film_to_bulk": int((flag == 2).sum().item())}

    if args.poisson:
        dp = W.projection_cylinder(args.poisson)
        pp = g.Particles.from_dict(ctx, dp)
        nbp = g.build_neighbours(ctx, pp)
        wp = g.gfdm_weights(ctx, pp, nbp, g.GF_BATCHED, g.GF_F64)
        val = g.poisson_assemble(ctx, pp, nbp, wp, dp["row_type"])
        rpp, colp = nbp.export()
        A = torch.sparse_csr_tensor(rpp, colp.long(), val, size=(pp.n, pp.n))
        b = (A @ torch.as_tensor(dp["pstar"], device=ctx.device).unsqueeze(1)).squeeze(1)
        ps = {}
        ps_n, ps_nnz = pp.n, nbp.nnz
        for mixed in (0, 1):
            # one untimed solve, one timed solve, one profiled solve (per-iteration launch times)
            g.poisson_solve(ctx, pp, nbp, wp, dp["row_type"], b, params=g.solve_params(mixed=mixed),
                            raise_on_fail=False)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, st = g.poisson_solve(ctx, pp, nbp, wp, dp["row_type"], b, params=g.solve_params(mixed=mixed),
                                    raise_on_fail=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            ctx.profile(True)
            g.poisson_solve(ctx, pp, nbp, wp, dp["row_type"], b, params=g.solve_params(mixed=mixed),
                            raise_on_fail=False)
            prof_p = ctx.profile_read()
            ctx.profile(False)
            err = ((x - torch.as_tensor(dp["pstar"], device=ctx.device)).norm() /
                   torch.as_tensor(dp["pstar"], device=ctx.device).norm()).item()
            rec = dict(seconds=el, err_vs_pstar=err, **st)
            # one Jacobi-BiCGStab iteration: two SpMV on the neighbour tiles (value + 2-byte slot
            # per entry; the vector is staged per tile) and the vector updates (26 vector passes)
            for name, vb in (("bicgstab_iter_f64", 8), ("bicgstab_iter_f32", 4)):
                if name in prof_p:
                    cnt, tot = prof_p[name]
                    it_s = tot / cnt * 1e-3
                    byts = 2.0 * ps_nnz * (vb + 2) + 26.0 * vb * ps_n
                    rec[name] = {"iterations": cnt, "avg_us": round(it_s * 1e6, 1),
                                 "algorithmic_bytes": byts, "GBs": round(byts / it_s / 1e9, 1),
                                 "hbm_frac": round(byts / it_s / 1e9 / PEAK_HBM_GBS, 4),
                                 "frac_of_measured_copy": round(byts / it_s / 1e9 / hbm_meas["copy_GBs"], 4)}
            ps["mixed" if mixed else "plain_f64"] = rec
            print(f"[bench] poisson mixed={mixed}: {el:.3f}s {rec}", file=sys.stderr, flush=True)
        result["poisson"] = {"n": ps_n, "nnz": ps_nnz, **ps}
        del dp, pp, nbp, wp, val, A, b, x

    if args.advdiff:
        from paper_2405_13165_amd.advdiff import DiffusionPlate
        kappa, t_end = 5e-3, 0.5
        study = []
        for hh in (0.06, 0.03, 0.015):
            da = W.advdiff_plate(hh)
            steps = int(np.ceil(t_end / (0.25 * 0.05 * hh * hh / kappa)))
            plate = DiffusionPlate(ctx, da, W.advdiff_rows(da, hh), kappa, t_end / steps)
            Ta, info = plate.run(steps)
            Ta = Ta.cpu().numpy()
            ex = W.advdiff_exact(da["x"], da["y"], t_end, kappa)
            rec = {"h": hh, "n_3d": int(da["n_bulk"]), "n_2d": int(da["n_film"]), "ghosts": plate.n_ghosts,
                   "steps": steps, "eps2": float(np.sqrt(((Ta - ex) ** 2).sum() / (ex ** 2).sum())),
                   "epsinf": float(np.abs(Ta - ex).max() / ex.max()), "seconds": round(info["seconds"], 3),
                   "ms_per_step": round(1e3 * info["seconds"] / steps, 3), "bicgstab_its": info["bicgstab_its"]}
            if study:
                rec["order_eps2"] = round(float(np.log2(study[-1]["eps2"] / rec["eps2"])), 2)
                rec["order_epsinf"] = round(float(np.log2(study[-1]["epsinf"] / rec["epsinf"])), 2)
            study.append(rec)
            print(f"[bench] advdiff {rec}", file=sys.stderr, flush=True)
            del plate
        # the moving plate: both transitions, ghosts, stencils and solve every step
        from paper_2405_13165_amd.advdiff import AdvectPlate
        t_adv = 2.0
        moving = []
        for hh in (0.12, 0.06, 0.03):
            da = W.advect_plate(hh)
            steps = int(np.ceil(t_adv / (0.25 * 0.05 * hh * hh / kappa)))
            c, info = AdvectPlate(ctx, da, kappa, t_adv / steps).run(steps)
            Ta = c["T"].cpu().numpy()
            ex = W.advdiff_exact(c["x"].cpu().numpy(), c["y"].cpu().numpy(), t_adv, kappa, x0=0.6 + t_adv)
            rec = {"h": hh, "n_start": int(da["x"].size), "max_n": info["max_n"], "max_ghosts": info["max_ghosts"],
                   "to_3d": info["to_3d"], "to_2d": info["to_2d"], "steps": steps,
                   "eps2": float(np.sqrt(((Ta - ex) ** 2).sum() / (ex ** 2).sum())),
                   "epsinf": float(np.abs(Ta - ex).max() / ex.max()), "seconds": round(info["seconds"], 3),
                   "ms_per_step": round(1e3 * info["seconds"] / steps, 3), "bicgstab_its": info["bicgstab_its"]}
            if moving:
                rec["order_eps2"] = round(float(np.log2(moving[-1]["eps2"] / rec["eps2"])), 2)
                rec["order_epsinf"] = round(float(np.log2(moving[-1]["epsinf"] / rec["epsinf"])), 2)
            moving.append(rec)
            print(f"[bench] advect {rec}", file=sys.stderr, flush=True)
        # the paper's configuration (Sec. 7.3, Table 2): plate [0,4]x[0,3], disc of radius 0.2 at
        # (0.5, 0.5), errors against a fine full-3D run of the same case at the nearest particle
        from scipy.spatial import cKDTree
        geo = dict(lx=4.0, ly=3.0, ic="disc", center=(0.5, 0.5))
        h_ref = 0.025
        dref = W.advect_plate(h_ref, **geo)
        steps = int(np.ceil(t_adv / (0.25 * 0.05 * h_ref * h_ref / kappa)))
        cref, iref = AdvectPlate(ctx, dref, kappa, t_adv / steps, x0=-np.inf, x1=np.inf).run(steps)
        print(f"[bench] advect full-3D reference h={h_ref}: {iref}", file=sys.stderr, flush=True)
        tree = cKDTree(np.stack([cref[k].cpu().numpy() for k in ("x", "y", "z")], 1))
        Tref_all = cref["T"].cpu().numpy()
        table2 = {0.2: (6.61e-2, 7.79e-2), 0.1: (2.35e-2, 3.67e-2), 0.05: (1.14e-2, 1.68e-2)}
        paper_cfg = []
        for hh in (0.2, 0.1, 0.05):
            da = W.advect_plate(hh, **geo)
            steps = int(np.ceil(t_adv / (0.25 * 0.05 * hh * hh / kappa)))
            ap = AdvectPlate(ctx, da, kappa, t_adv / steps)
            ap.step()
            n3, n2 = int((ap.c["model"] == 0).sum()), int((ap.c["model"] == 1).sum())
            c, info = ap.run(steps - 1)
            Ta = c["T"].cpu().numpy()
            _, I = tree.query(np.stack([c[k].cpu().numpy() for k in ("x", "y", "z")], 1))
            Tr = Tref_all[I]
            ms = ((Ta - Tr) ** 2).sum() / (Tr ** 2).sum()
            rec = {"h": hh, "n_3d_after_first_step": n3, "n_2d_after_first_step": n2, "steps": steps,
                   "eps2": float(np.sqrt(ms)), "eps2_no_sqrt": float(ms),
                   "epsinf": float(np.abs(Ta - Tr).max() / np.abs(Tr).max()),
                   "paper_eps2": table2[hh][0], "paper_epsinf": table2[hh][1],
                   "seconds": round(info["seconds"], 3), "bicgstab_its": info["bicgstab_its"]}
            if paper_cfg:
                rec["order_eps2"] = round(float(np.log2(paper_cfg[-1]["eps2"] / rec["eps2"])), 2)
                rec["order_epsinf"] = round(float(np.log2(paper_cfg[-1]["epsinf"] / rec["epsinf"])), 2)
            paper_cfg.append(rec)
            print(f"[bench] advect paper configuration {rec}", file=sys.stderr, flush=True)
        result["advdiff"] = {"kappa": kappa, "t_end": t_end, "study": study,
                             "moving": {"t_end": t_adv, "window": [1.0, 2.0], "study": moving},
                             "paper_configuration": {"reference": {"h": h_ref, "n": int(dref["x"].size),
                                                                   "n_3d": iref["max_n"],
                                                                   "seconds": round(iref["seconds"], 3)},
                                                     "study": paper_cfg}}

    if args.jet:
        dj = W.jet_impact()
        pj = g.Particles.from_dict(ctx, dj)
        nbj = g.build_neighbours(ctx, pj)
        teams_j = g.autotune(ctx, pj, nbj, g.GF_F32)
        uj = torch.as_tensor(W.test_field(dj["x"], dj["y"], dj["z"])[0], device=ctx.device)
        wj = torch.empty((nbj.nnz, 4), dtype=torch.float32, device=ctx.device)
        yj = torch.empty((4, pj.n), dtype=torch.float64, device=ctx.device)
        stj = torch.empty(pj.n, dtype=torch.int8, device=ctx.device)
        ms_j = timed(lambda: g.gfdm_weights_apply(ctx, pj, nbj, uj, 0xF, g.GF_F32, w_out=wj, out=yj, status=stj),
                     args.steps, args.warmup)
        ctx.profile(True)
        g.gfdm_weights_apply(ctx, pj, nbj, uj, 0xF, g.GF_F32, w_out=wj, out=yj, status=stj)
        prof_j = ctx.profile_read()
        ctx.profile(False)
        counts = np.bincount(stj.cpu().numpy().astype(np.int64), minlength=4)
        # neighbour builds (same and cross model), wall time of one build after a warm-up
        build_ms = {}
        for cross in (False, True):
            g.build_neighbours(ctx, pj, cross_model=cross).close()
            best = float("inf")
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                nbx = g.build_neighbours(ctx, pj, cross_model=cross)
                torch.cuda.synchronize()
                best = min(best, (time.perf_counter() - t0) * 1e3)
                nbx.close()
            build_ms["cross_model" if cross else "same_model"] = round(best, 3)
        result["jet"] = {"n": pj.n, "nnz": nbj.nnz, "max_row": nbj.max_row, "ms_per_step": ms_j,
                         "build_neighbours_ms": build_ms, "team_sizes": teams_j,
                         "value": pj.n / (ms_j * 1e-3), "unit": "particles/s",
                         "status_counts": {"ok": int(counts[0]), "qr_fallback": int(counts[1]),
                                           "rank_deficient": int(counts[2]), "too_few": int(counts[3])},
                         "kernels": {k: {"launches": c, "avg_us": 1000.0 * t / c} for k, (c, t) in prof_j.items()}}
        print(f"[bench] jet: {ms_j:.3f} ms per fused step", file=sys.stderr, flush=True)
        del dj, pj, nbj, uj, wj, yj, stj

    if args.diff:
        dd = W.diff_cube()
        pd = g.Particles.from_dict(ctx, dd)
        nbd = g.build_neighbours(ctx, pd)
        ud = torch.as_tensor(dd["u"], device=ctx.device)
        gd = torch.as_tensor(dd["g"], device=ctx.device)
        xs = [torch.as_tensor(dd[k], device=ctx.device) for k in ("x", "y", "z")]

        def fwd_bwd():
            ur = ud.clone().requires_grad_(True)
            xr, yr, zr = (t.clone().requires_grad_(True) for t in xs)
            out = g.stencil_op(ctx, pd, nbd, ur, xr, yr, zr, op_mask=g.OP_LAP, wtype=g.GF_F32)
            loss = ((out[0] - gd) ** 2).sum()
            return torch.autograd.grad(loss, (ur, xr, yr, zr))

        ms_d = timed(fwd_bwd, max(3, args.steps // 4), 1)
        result["differentiation"] = {"n": pd.n, "nnz": nbd.nnz, "ms_forward_backward": ms_d,
                                     "value": pd.n / (ms_d * 1e-3), "unit": "particles/s"}
        print(f"[bench] differentiation: {ms_d:.3f} ms forward+backward", file=sys.stderr, flush=True)
        del dd, pd, nbd

    # ---- CPU oracle baseline and operator error (oracle inputs never come from the device)
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        rp_o, col_o = oracle.neighbours(d)
        t_nbr_o = time.perf_counter() - t0
        assert np.array_equal(rp_o, rp) and np.array_equal(col_o, col_d.cpu().numpy()), "neighbour lists differ"
        # repeat the full pass until about 10 s of wall time have been spent
        passes, t_all = 0, 0.0
        while passes < 1 or (t_all < 10.0 and passes < 40):
            t0 = time.perf_counter()
            w_o, st_o, _ = oracle.gfdm_weights(d, rp_o, col_o)
            y_o = oracle.apply(rp_o, col_o, w_o, f)
            t_all += time.perf_counter() - t0
            passes += 1
        t_o = t_all / passes
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # the other rows, once each on the same cloud (same inputs as the GPU rows above)
        orows = {"build_neighbours_s": t_nbr_o}
        if not args.no_rows:
            xr_o, xc_o = oracle.neighbours(d, cross=True)   # input of the classification, not timed
            t0 = time.perf_counter()
            lam_o, w3_o, eps_o = oracle.pca(d, rp_o, col_o)
            oracle.classify(d, rp_o, col_o, eps_o, w3_o, cross=(xr_o, xc_o), film_height=d["film_height"],
                            h3d=d["h3d"])
            orows["classify_pca_s"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.apply(rp_o, col_o, w_o, f)
            orows["apply_s"] = time.perf_counter() - t0
            tflag_o = ((d["model"] == 0) & (d["kind"] == W.WALL)).astype(np.uint8)
            t0 = time.perf_counter()
            oracle.transition_3d_to_2d(d, rp_o, col_o, tflag_o, np.ones(N), np.full(N, 1000.0), f)
            orows["transition_s"] = time.perf_counter() - t0
            yb_o = np.ones((1, N))
            t0 = time.perf_counter()
            oracle.apply_adjoint(rp_o, col_o, w_o, yb_o, 8)
            orows["apply_adjoint_s"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.weights_adjoint_x(d, rp_o, col_o, f, yb_o, 8)
            orows["weights_adjoint_s"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.film_height(d, rp_o, col_o, d["diam"])
            orows["film_height_s"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.buffer_zone(d, xr_o, xc_o, d["film_height"], d["h_other"], d["mass"], d["rho"])
            orows["buffer_zone_s"] = time.perf_counter() - t0
            for key in ("classify_pca", "apply", "transition", "apply_adjoint", "weights_adjoint",
                        "film_height", "buffer_zone"):
                if key in result.get("rows_roofline", {}):
                    rr = result["rows_roofline"][key]
                    rr["oracle_s"] = round(orows[key + "_s"], 4)
                    rr["speedup_vs_oracle"] = round(orows[key + "_s"] / (rr["kernel_us"] * 1e-6), 1)
            if "build_neighbours" in result.get("rows_roofline", {}):
                rr = result["rows_roofline"]["build_neighbours"]
                rr["oracle_s"] = round(t_nbr_o, 4)
                rr["speedup_vs_oracle"] = round(t_nbr_o / (rr["kernel_us"] * 1e-6), 1)
        result["oracle_rows_s"] = orows
        e32 = oracle.operator_error(w32n, w_o, rp_o)
        e64 = oracle.operator_error(w64n, w_o, rp_o)
        result["cpu_baseline"] = {"value": N / t_o, "unit": "particles/s", "cores": cores, "kind": "oracle",
                                  "sample": f"all {N} particles of the workload, weights + apply, mean of "
                                            f"{passes} passes ({t_o:.2f} s each; neighbour search "
                                            f"{t_nbr_o:.1f} s not included)"}
        result["operator_error"] = {
            "batched_f32_max": float(e32.max()), "batched_f32_p9999": float(np.quantile(e32, 0.9999)),
            "plain_f64_max": float(e64.max()),
            "fused_apply_max_abs_rel": float(np.max(np.abs(yfn - y_o)) / np.max(np.abs(y_o))),
            "separate_apply_max_abs_rel": float(np.max(np.abs(y32n - y_o)) / np.max(np.abs(y_o))),
        }
        print(f"[bench] oracle {t_o:.1f}s; f32 err max {e32.max():.2e}, f64 err max {e64.max():.2e}",
              file=sys.stderr, flush=True)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
