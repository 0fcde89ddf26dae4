#!/usr/bin/env python3
"""Throughput of the GFDM hot path on one MI355X.

Metric: particles/s for GFDM stencil weights + application (all four
stencils d/dx, d/dy, d/dz, Laplacian applied to one scalar field), on the
mixed bulk/film cloud of 503,944 particles (258,944 jittered-lattice bulk
particles beside 245,000 film particles on z = 0, h = 3 x local spacing).
value = N / t_step for the batched path: one gf_gfdm_weights_apply call that
computes every stencil (FP64 moments and solves, FP64 QR fallback), stores it
in FP32 and applies it to the field.  The plain FP64 path (one work-item per
particle, FP64 stencils, then the application) and the same batched work as
two calls are timed beside it.

A step is one weights + apply pass over the resident cloud.  Each of the K
timed steps is bracketed by HIP events on the library's stream; before it,
1 GiB is written to one scratch buffer and 1 GiB read from another, so that
the caches (L2, the 256 MB Infinity Cache) hold nothing of the step's inputs
and no write-back is pending; ms_per_step is the mean.  The same steps back
to back are reported beside it.

The default run also reports the other workloads of the path: the uneven
2.0M-particle jet-on-plate cloud (fused step), the 10^6-particle
differentiation cube (forward + backward through the adjoints) and the
4.0M-row pressure-Poisson solve (FP64 and the two mixed-precision forms);
per-output errors against the FP64 oracle; the roofline of the dominant
kernel; and the oracle timed on the host's cores.
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
FLUSH_BYTES = 1 << 30        # written before every timed step (> 256 MB Infinity Cache)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--factor", type=int, default=1, help="coarsen the workload (parity/debug only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip timing the other hot-path steps")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline workload (no jet, differentiation or pressure-solve records)")
    ap.add_argument("--records", default="jet,diff,poisson",
                    help="comma list of the further records to run: jet, diff, poisson (default: all)")
    ap.add_argument("--poisson-n", type=int, default=4_000_000,
                    help="particles of the projection cylinder of the pressure-solve record")
    ap.add_argument("--advdiff", action="store_true",
                    help="also run the diffusion analogue of the advection-diffusion test (Sec. 7.2) at "
                         "h = 0.06, 0.03, 0.015, and its model-adaptive moving-plate case at h = 0.12, 0.06, 0.03, "
                         "against the exact solutions (convergence study)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warm-up plus a few steps of the metric path and exit (for rocprofv3)")
    ap.add_argument("--profile-jet", action="store_true",
                    help="with --profile-only: the jet cloud's fused step instead of the headline cloud")
    ap.add_argument("--profile-graph", action="store_true",
                    help="with --profile-only: 30 eager fused steps, then 30 replays of the step captured in a "
                         "HIP graph (for a kernel trace comparing the two)")
    return ap.parse_args()


# the translation unit of the fused stencil kernel (sources relative to csrc/)
KERNEL_SOURCES = ("weights.hip", "stencil_common.h", "internal.h", "../../include/gfdm.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def unit_costs(rp, model):
    """Algorithmic cost of each launch unit of the fused stencil step (per
    model: the tiled rows with at most 128 neighbours, "tiles", and the rows
    with more, "b3"), by the per-particle figures of the step's roofline:
      bytes = 40 n + 52   (FP32 stencils: 4 n index + 16 n stencils written by
                           the weights, 4 n + 16 n read again by the application,
                           32 B position and support, 4 B field value, 16 B
                           for the four results)
      flops = 2 n m^2 + 4 S n m + 2 S n   (Gram accumulation, stencil
                           evaluation, application; m monomials, S stencils)
    with n = |S_i| (self included), m = 10 / 6 and S = 4 / 3 (3D / film)."""
    import numpy as np
    n_i = np.diff(rp)
    bands = np.searchsorted(np.array(BANDS), n_i, side="left")
    out = {}
    for m in (0, 1):
        M, S = (10, 4) if m == 0 else (6, 3)
        for unit, sel in (("tiles", bands <= 2), ("b3", bands == 3)):
            nn = n_i[(model == m) & sel].astype(np.float64)
            if nn.size == 0:
                continue
            out[(m, unit)] = dict(rows=int(nn.size), nnz=int(nn.sum()),
                                  bytes=float((40.0 * nn + 52.0).sum()),
                                  flops=float((2 * nn * M * M + 4 * S * nn * M + 2 * S * nn).sum()))
    return out


def per_output_errors(y, y_ref, rp, col, w_ref, u, model, rows=None):
    """Error of every applied output by the condition-aware metric:
    max_i |y_i - y_i^ref| / max_i sum_j |c_ij^ref (u_j - u_i)|, per output and
    model (bulk: gx, gy, gz, lap; film: gt1, gt2 (= gx, gy on a film in the
    z = 0 plane, whose tangent frame is (e_x, e_y)) and the surface Laplacian).
    rows: the rows of a sampled record; then y, y_ref [4, len(rows)] hold those
    rows' outputs and (rp, col, w_ref) their CSR (rp from 0, global columns)."""
    import numpy as np
    ids = np.arange(rp.shape[0] - 1) if rows is None else np.asarray(rows)
    nr = ids.size
    loc = np.repeat(np.arange(nr), np.diff(rp))
    own = ids[loc]
    du = np.where(col == own, 0.0, u[col] - u[own])
    out = {}
    names = {0: ("gx", "gy", "gz", "lap"), 1: ("gt1", "gt2", None, "lap_s")}
    mrow = model[ids]
    for m, label in ((0, "bulk"), (1, "film")):
        rsel = mrow == m
        if not rsel.any():
            continue
        rec = {}
        for s in range(4):
            name = names[m][s]
            if name is None:
                continue
            scale = np.bincount(loc, np.abs(w_ref[:, s] * du), minlength=nr)[rsel].max()
            err = np.abs(y[s][rsel] - y_ref[s][rsel]).max()
            rec[name] = float(err / scale) if scale > 0 else float(err)
        out[label] = rec
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
    t_start = time.time()
    records = set() if args.quick else {r.strip() for r in args.records.split(",") if r.strip()}
    t0 = time.time()
    d = W.mixed_block_film(factor=args.factor)
    N = d["x"].shape[0]
    log(f"workload generated: {N} particles ({time.time() - t0:.1f}s)")

    ctx = g.Context(0)
    dev = ctx.device
    flush_buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
    flush_src = torch.ones(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)

    def flush():
        # 1 GiB written, then another 1 GiB read: the caches (L2, 256 MB Infinity Cache) then hold
        # clean lines of the read buffer, none of the step's inputs, and no write-back is pending
        flush_buf.fill_(1.0)
        flush_src.sum()

    def timed(fn, steps, warmup, flushed=True, kernels=False):
        """Mean ms of one call over `steps` calls after `warmup` untimed ones.
        flushed: each call bracketed by its own events, after the cache flush.
        kernels: also return the library's HIP-event times of each of its kernels
        ({name: {launches, avg_us}}), taken in a second pass of as many calls
        under the same protocol (the events the library records around each
        launch are not part of the timed step)."""
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        if kernels:
            ms = timed(fn, steps, 0, flushed)
            ctx.profile(True)
            timed(fn, steps, 0, flushed)
            prof = ctx.profile_read()
            ctx.profile(False)
            return ms, {k: {"launches": c, "avg_us": 1000.0 * t / c} for k, (c, t) in prof.items()}
        if not flushed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(steps):
                fn()
            e1.record(s)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps
        evs = []
        for _ in range(steps):
            flush()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in evs) / steps

    def kernels_of(fn, reps):
        """The library's own HIP-event times of each kernel over `reps` calls."""
        ctx.profile(True)
        for _ in range(reps):
            fn()
        prof = ctx.profile_read()
        ctx.profile(False)
        return {k: {"launches": c, "avg_us": 1000.0 * t / c} for k, (c, t) in prof.items()}

    p = g.Particles.from_dict(ctx, d)
    f, *_ = W.test_field(d["x"], d["y"], d["z"])
    u = torch.as_tensor(f, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb = g.build_neighbours(ctx, p)
    torch.cuda.synchronize()
    t_nbr_first = time.perf_counter() - t0
    nnz = nb.nnz
    rp_d, col_d = nb.export()
    rp = rp_d.cpu().numpy()
    col_np = col_d.cpu().numpy()
    log(f"neighbours: nnz={nnz} max_row={nb.max_row}")

    w32 = torch.empty((nnz, 4), dtype=torch.float32, device=dev)
    w64 = torch.empty((nnz, 4), dtype=torch.float64, device=dev)
    y32 = torch.empty((4, N), dtype=torch.float64, device=dev)
    y64 = torch.empty((4, N), dtype=torch.float64, device=dev)
    yf = torch.empty((4, N), dtype=torch.float64, device=dev)
    status = torch.empty(N, dtype=torch.int8, device=dev)

    def step_batched():
        g.gfdm_weights(ctx, p, nb, g.GF_BATCHED, g.GF_F32, out=w32, status=status)
        g.apply_stencil(ctx, nb, w32, u, 0xF, out=y32)

    def step_plain():
        g.gfdm_weights(ctx, p, nb, g.GF_PLAIN_F64, g.GF_F64, out=w64)
        g.apply_stencil(ctx, nb, w64, u, 0xF, out=y64)

    def step_fused():
        g.gfdm_weights_apply(ctx, p, nb, u, 0xF, g.GF_F32, w_out=w32, out=yf, status=status)

    t0 = time.perf_counter()
    teams = g.autotune(ctx, p, nb, g.GF_F32)
    log(f"autotune {time.perf_counter() - t0:.2f}s: {teams}")

    if args.profile_only and args.profile_graph:
        for _ in range(3):
            step_fused()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step_fused()
        torch.cuda.synchronize()
        marker = torch.empty(1 << 20, device=dev)
        marker.fill_(0)          # separates the eager steps from the replays in the trace
        for _ in range(30):
            step_fused()
        torch.cuda.synchronize()
        marker.fill_(1)
        for _ in range(30):
            graph.replay()
        torch.cuda.synchronize()
        marker.fill_(2)
        torch.cuda.synchronize()
        log("profile run done (30 eager steps, 30 graph replays)")
        return

    if args.profile_only:
        if args.profile_jet:
            dj = W.jet_impact()
            pj = g.Particles.from_dict(ctx, dj)
            nbj = g.build_neighbours(ctx, pj)
            g.autotune(ctx, pj, nbj, g.GF_F32)
            uj = torch.as_tensor(W.test_field(dj["x"], dj["y"], dj["z"])[0], device=dev)
            wj = torch.empty((nbj.nnz, 4), dtype=torch.float32, device=dev)
            yj = torch.empty((4, pj.n), dtype=torch.float64, device=dev)
            timed(lambda: g.gfdm_weights_apply(ctx, pj, nbj, uj, 0xF, g.GF_F32, w_out=wj, out=yj),
                  max(args.steps, 1), args.warmup, flushed=False)
        else:
            # the fused step under the metric's protocol (cache flushed before each
            # step), so that its launches here time as in the bench line
            timed(step_fused, max(args.steps, 1), args.warmup)
            timed(step_batched, 2, 1, flushed=False)
            timed(step_plain, 2, 1, flushed=False)
        # a plain device copy of known size: calibrates the HBM byte counters
        # (FETCH_SIZE / WRITE_SIZE) read by rocprofv3 for the same run
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("profile run done (copy calibration: 1 GiB read + 1 GiB written)")
        return

    ms_fused, kernels = timed(step_fused, args.steps, args.warmup, kernels=True)
    ms_fused_b2b = timed(step_fused, args.steps, args.warmup, flushed=False)
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
    ms_graph_b2b = timed(graph.replay, args.steps, args.warmup, flushed=False)
    del graph
    log(f"fused {ms_fused:.3f} ms (back to back {ms_fused_b2b:.3f}); graph {ms_graph:.3f} "
        f"(b2b {ms_graph_b2b:.3f}, replay exact: {graph_ok}); separate calls {ms_batched:.3f}; plain {ms_plain:.3f}")

    reps = max(3, min(args.steps, 10))
    kernels_b2b = kernels_of(step_fused, reps)
    kernels_sep = kernels_of(step_batched, reps)
    kernels_plain = kernels_of(step_plain, reps)

    # ---- roofline of the dominant kernel (the largest fused stencil launch)
    costs = unit_costs(rp, d["model"])

    def roofline(kern, costs_, team_of, kern_b2b=None):
        wk = {k: v for k, v in kern.items() if k.startswith("weights_apply_")}
        dom = max(wk, key=lambda k: wk[k]["avg_us"] * wk[k]["launches"])
        m_dom = 0 if "_3d_" in dom else 1
        unit = dom.rsplit("_", 1)[1]
        c = costs_[(m_dom, unit)]
        sec = wk[dom]["avg_us"] * 1e-6
        gbs = c["bytes"] / sec / 1e9
        tfl = c["flops"] / sec / 1e12
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None}
        traffic, src = measured_traffic(dom, team_of(m_dom, unit))
        if traffic is not None:
            roof["traffic"] = round(traffic)
            roof["traffic_note"] = (f"HBM bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated) "
                                    f"from {src}")
        roof["algorithmic_per_launch"] = {"bytes": c["bytes"], "flops": c["flops"], "rows": c["rows"],
                                          "nnz": c["nnz"], "avg_launch_us": round(sec * 1e6, 2),
                                          "bytes_per_particle": "40 n + 52",
                                          "flops_per_particle": "2 n m^2 + 4 S n m + 2 S n"}
        roof["other_roof"] = {"fp64_TFLOPs": round(tfl, 3), "fp64_frac": round(tfl / PEAK_FP64_TFLOPS, 4)}
        roof["timing"] = ("HIP events around each launch, over a second pass of the same number of "
                          "cache-flushed steps")
        if kern_b2b and dom in kern_b2b:
            sec_b = kern_b2b[dom]["avg_us"] * 1e-6
            roof["other_roof"]["back_to_back"] = {"avg_launch_us": round(sec_b * 1e6, 2),
                                                  "GBs": round(c["bytes"] / sec_b / 1e9, 1),
                                                  "hbm_frac": round(c["bytes"] / sec_b / 1e9 / PEAK_HBM_GBS, 4)}
        return roof

    roof = roofline(kernels, costs, lambda m, unit: teams["fused"][4 * m + (2 if unit == "tiles" else 3)], kernels_b2b)
    step_bytes = sum(c["bytes"] for c in costs.values())
    step_hbm_frac = step_bytes / (ms_fused * 1e-3) / 1e9 / PEAK_HBM_GBS

    # ---- outputs of the metric step, the separate calls and the plain path
    step_batched()
    torch.cuda.synchronize()
    y32n = y32.cpu().numpy()
    step_fused(); step_plain()
    torch.cuda.synchronize()
    w32n = w32.double().cpu().numpy()
    w64n = w64.cpu().numpy()
    yfn = yf.cpu().numpy()
    y64n = y64.cpu().numpy()

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
        "step": "gf_gfdm_weights_apply: batched stencils stored in FP32 and applied (one call), eager launches",
        "timing": "mean of the per-step HIP-event times; before each step 1 GiB is written and another 1 GiB read "
                  "(Infinity Cache and L2 evicted, no write-back pending)",
        "fused_back_to_back": {"value": N / (ms_fused_b2b * 1e-3), "ms_per_step": ms_fused_b2b},
        "fused_graph": {"value": N / (ms_graph * 1e-3), "ms_per_step": ms_graph, "replay_exact": graph_ok,
                        "ms_per_step_back_to_back": ms_graph_b2b},
        "plain_f64": {"value": N / (ms_plain * 1e-3), "ms_per_step": ms_plain,
                      "step": "gf_gfdm_weights(GF_PLAIN_F64) + gf_apply_stencil"},
        "separate_calls_f32": {"value": N / (ms_batched * 1e-3), "ms_per_step": ms_batched,
                               "step": "gf_gfdm_weights(GF_BATCHED, FP32) + gf_apply_stencil"},
        "speedup_batched_vs_plain": ms_plain / ms_fused,
        "team_sizes": teams,
        "step_roofline": {"algorithmic_bytes": step_bytes, "GBs": round(step_bytes / (ms_fused * 1e-3) / 1e9, 1),
                          "hbm_frac": round(step_hbm_frac, 4), "bytes_per_particle": "40 n + 52"},
        "kernels_batched": kernels,
        "kernels_batched_back_to_back": kernels_b2b,
        "kernels_separate_calls": kernels_sep,
        "kernels_plain": kernels_plain,
        "roofline": roof,
    }
    hbm_meas = measure_hbm(dev)
    result["hbm_measured"] = hbm_meas
    roof["other_roof"]["hbm_frac_of_measured_copy"] = round(roof["achieved"] / hbm_meas["copy_GBs"], 4)
    log(f"roofline {roof['kernel']}: {roof['achieved']} GB/s = {roof['frac']:.3f} of HBM; step {step_hbm_frac:.3f}")

    # ---- other hot-path steps on the same cloud (timed once each after a warm-up call)
    if not args.no_rows:
        rows = {"build_neighbours_first_ms": t_nbr_first * 1e3}
        kern = {}

        def once(fn, key=None):
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
        mass = torch.ones(N, dtype=torch.float64, device=dev)
        rho = torch.full((N,), 1000.0, dtype=torch.float64, device=dev)
        # this cloud flags no particle (its bottom walls see interior neighbours only): the transition is
        # timed with every bulk wall particle flagged, which deletes the layers above the bottom
        tflag = torch.as_tensor(((d["model"] == 0) & (d["kind"] == W.WALL)).astype(np.uint8), device=dev)
        rows["transition_ms"], _ = once(lambda: g.transition_3d_to_2d(ctx, p, nb, tflag, mass, rho, u), "transition")
        rows["apply_ms"], _ = once(lambda: g.apply_stencil(ctx, nb, w32, u, 0xF, out=y32), "apply")
        ybar = torch.ones((1, N), dtype=torch.float64, device=dev)
        rows["apply_adjoint_ms"], _ = once(lambda: g.apply_stencil_adjoint(ctx, nb, w32, ybar, g.OP_LAP),
                                           "apply_adjoint")
        rows["weights_adjoint_ms"], _ = once(lambda: g.gfdm_weights_adjoint(ctx, p, nb, u, ybar, g.OP_LAP),
                                             "weights_adjoint")
        rows["film_height_ms"], _ = once(lambda: g.film_height(ctx, p, nb, d["diam"]), "film_height")
        rows["buffer_zone_ms"], bz = once(lambda: g.buffer_zone(ctx, p, nb, xnb, d["film_height"], d["h_other"],
                                                                d["mass"], d["rho"]), "buffer_zone")
        ghosts = bz[1]
        pe = g.extend_particles(ctx, p, ghosts)
        rows["extended_build_ms"], nbe = once(lambda: g.build_neighbours(ctx, pe, n_rows=N), "extended_build")
        ue = torch.cat([u, torch.as_tensor(W.test_field(ghosts["x"].cpu().numpy(), ghosts["y"].cpu().numpy(),
                                                        ghosts["z"].cpu().numpy())[0], device=dev)])
        rows["extended_weights_apply_ms"], _ = once(
            lambda: g.gfdm_weights_apply(ctx, pe, nbe, ue, wtype=g.GF_F32, store_weights=False),
            "extended_weights_apply")
        rows["buffer_zone_counts"] = {"flagged": int(bz[0].sum().item()), "ghosts": int(ghosts["x"].shape[0]),
                                      "ghosts_3d": int((ghosts["model"] == 0).sum().item()),
                                      "extended_nnz": nbe.nnz}
        del nbe, pe
        result["rows"] = rows
        result["rows_kernels_us"] = kern
        # algorithmic bytes of each row (per particle N and per neighbour entry nnz, each byte a row
        # must read or write at least once)
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
        log(f"rows {rows}")

    # ---- jet-on-plate cloud: uneven neighbourhoods (20-250), the fused step
    jet_eval = None
    if "jet" in records:
        dj = W.jet_impact()
        pj = g.Particles.from_dict(ctx, dj)
        nbj = g.build_neighbours(ctx, pj)
        rpj = nbj.export()[0].cpu().numpy()
        teams_j = g.autotune(ctx, pj, nbj, g.GF_F32)
        fj = W.test_field(dj["x"], dj["y"], dj["z"])[0]
        uj = torch.as_tensor(fj, device=dev)
        wj = torch.empty((nbj.nnz, 4), dtype=torch.float32, device=dev)
        yj = torch.empty((4, pj.n), dtype=torch.float64, device=dev)
        stj = torch.empty(pj.n, dtype=torch.int8, device=dev)
        step_j = lambda: g.gfdm_weights_apply(ctx, pj, nbj, uj, 0xF, g.GF_F32, w_out=wj, out=yj, status=stj)
        ms_j, kern_j = timed(step_j, args.steps, args.warmup, kernels=True)
        w64j = torch.empty((nbj.nnz, 4), dtype=torch.float64, device=dev)
        y64j = torch.empty((4, pj.n), dtype=torch.float64, device=dev)

        def step_jp():
            g.gfdm_weights(ctx, pj, nbj, g.GF_PLAIN_F64, g.GF_F64, out=w64j)
            g.apply_stencil(ctx, nbj, w64j, uj, 0xF, out=y64j)

        ms_jp = timed(step_jp, max(3, args.steps // 2), 1)
        costs_j = unit_costs(rpj, dj["model"])
        roof_j = roofline(kern_j, costs_j, lambda m, unit: teams_j["fused"][4 * m + (2 if unit == "tiles" else 3)])
        step_j()
        torch.cuda.synchronize()
        counts = np.bincount(stj.cpu().numpy().astype(np.int64), minlength=4)
        nrow = np.diff(rpj)
        result["jet"] = {
            "workload": "jet impact: 1.0M bulk particles in a cylinder (r 0.05, height 0.2) above 1.0M film "
                        "particles on z = 0 (density ~ 1/r), lognormal h (sigma 0.3)",
            "n": pj.n, "nnz": nbj.nnz, "neighbours_min_p50_max": [int(nrow.min()), int(np.median(nrow)),
                                                                  int(nrow.max())],
            "ms_per_step": ms_j, "value": pj.n / (ms_j * 1e-3), "unit": "particles/s",
            "plain_f64": {"ms_per_step": ms_jp, "value": pj.n / (ms_jp * 1e-3)},
            "speedup_batched_vs_plain": ms_jp / ms_j,
            "step_hbm_frac": round(sum(c["bytes"] for c in costs_j.values()) / (ms_j * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "roofline": roof_j, "team_sizes": teams_j,
            "status_counts": {"ok": int(counts[0]), "qr_fallback": int(counts[1]),
                              "rank_deficient": int(counts[2]), "too_few": int(counts[3])},
            "kernels": kern_j}
        # a sample of 20,000 rows for the errors against the oracle (their stencils and outputs)
        samp = np.sort(np.random.default_rng(13).choice(pj.n, 20000, replace=False))
        sel = torch.as_tensor(np.concatenate([np.arange(rpj[i], rpj[i + 1]) for i in samp]), device=dev)
        si = torch.as_tensor(samp, device=dev)
        jet_eval = (dj, fj, samp, rpj, wj[sel].double().cpu().numpy(), yj[:, si].cpu().numpy(),
                    w64j[sel].cpu().numpy(), y64j[:, si].cpu().numpy())
        del sel, si
        log(f"jet: {ms_j:.3f} ms per fused step (plain {ms_jp:.3f}); {roof_j['kernel']} {roof_j['frac']:.3f} of HBM")
        del pj, nbj, uj, wj, yj, stj, w64j, y64j

    # ---- differentiation cube: forward + backward of the Laplacian loss
    if "diff" in records:
        dd = W.diff_cube()
        pd = g.Particles.from_dict(ctx, dd)
        nbd = g.build_neighbours(ctx, pd)
        ud = torch.as_tensor(dd["u"], device=dev)
        gd = torch.as_tensor(dd["g"], device=dev)
        xs = [torch.as_tensor(dd[k], device=dev) for k in ("x", "y", "z")]

        def fwd_bwd():
            ur = ud.clone().requires_grad_(True)
            xr, yr, zr = (t.clone().requires_grad_(True) for t in xs)
            out = g.stencil_op(ctx, pd, nbd, ur, xr, yr, zr, op_mask=g.OP_LAP, wtype=g.GF_F32)
            loss = ((out[0] - gd) ** 2).sum()
            return torch.autograd.grad(loss, (ur, xr, yr, zr))

        ms_d = timed(fwd_bwd, max(3, args.steps // 4), 1)
        result["differentiation"] = {
            "workload": "10^6 jittered-lattice particles (s = 0.01, h = 3 s); loss sum (Lap_h u - g)^2, "
                        "gradients with respect to u and the positions",
            "n": pd.n, "nnz": nbd.nnz, "ms_forward_backward": ms_d, "value": pd.n / (ms_d * 1e-3),
            "unit": "particles/s", "kernels": kernels_of(fwd_bwd, 1)}
        log(f"differentiation: {ms_d:.3f} ms forward+backward")
        del dd, pd, nbd, ud, gd, xs

    # ---- pressure-Poisson solve on the 4.0M projection cylinder
    if "poisson" in records and args.poisson_n > 0:
        dp = W.projection_cylinder(args.poisson_n)
        pp = g.Particles.from_dict(ctx, dp)
        nbp = g.build_neighbours(ctx, pp)
        wp = g.gfdm_weights(ctx, pp, nbp, g.GF_BATCHED, g.GF_F64)
        val = g.poisson_assemble(ctx, pp, nbp, wp, dp["row_type"])
        rpp, colp = nbp.export()
        pstar = torch.as_tensor(dp["pstar"], device=dev)
        # b = A p* on the host (scipy, a fixed summation order): the solves then start
        # from the same right-hand side bit for bit in every run
        import scipy.sparse as sp
        A = sp.csr_matrix((val.cpu().numpy(), colp.cpu().numpy(), rpp.cpu().numpy()), shape=(pp.n, pp.n))
        b = torch.as_tensor(A @ dp["pstar"], device=dev)
        del A, val, rpp, colp
        ps = {}
        for mixed, label in ((0, "plain_f64"), (1, "mixed_f32_matrix"), (2, "mixed_ir_f32_vectors")):
            prm = g.solve_params(mixed=mixed)
            g.poisson_solve(ctx, pp, nbp, wp, dp["row_type"], b, params=prm, raise_on_fail=False)   # warm-up
            flush()
            torch.cuda.synchronize()
            x, st = g.poisson_solve(ctx, pp, nbp, wp, dp["row_type"], b, params=prm, raise_on_fail=False)
            err = ((x - pstar).norm() / pstar.norm()).item()
            ctx.profile(True)
            g.poisson_solve(ctx, pp, nbp, wp, dp["row_type"], b, params=prm, raise_on_fail=False)
            prof_p = ctx.profile_read()
            ctx.profile(False)
            rec = dict(err_vs_pstar=err, **st)
            # one Jacobi-BiCGStab iteration: two SpMV on the neighbour tiles (value + 2-byte slot per
            # entry; the vector staged per tile) and the vector passes (26 per iteration)
            for name, vb, xb in (("bicgstab_iter_f64", 8, 8), ("bicgstab_iter_f32val", 4, 8),
                                 ("bicgstab_iter_f32", 4, 4)):
                if name in prof_p:
                    cnt, tot = prof_p[name]
                    it_s = tot / cnt * 1e-3
                    byts = 2.0 * nbp.nnz * (vb + 2) + 26.0 * xb * pp.n
                    rec[name] = {"iterations": cnt, "avg_us": round(it_s * 1e6, 1), "algorithmic_bytes": byts,
                                 "GBs": round(byts / it_s / 1e9, 1),
                                 "hbm_frac": round(byts / it_s / 1e9 / PEAK_HBM_GBS, 4)}
            ps[label] = rec
            log(f"poisson {label}: {st['seconds']:.3f}s, {st['inner_its_total']} iterations, error {err:.2e}")
        result["poisson"] = {
            "workload": "projection cylinder: bulk jet cylinder (r 0.05, height 0.2), uniform h = 3 s, "
                        "Laplacian rows inside, plain Neumann rows on the bottom wall, Dirichlet on the free "
                        "surface; b = A p*, p* = sin(20x+1) cos(20y) (1+5z); Jacobi-BiCGStab to 1e-8",
            "n": pp.n, "nnz": nbp.nnz, **ps,
            "speedup_mixed_vs_f64": ps["plain_f64"]["seconds"] / ps["mixed_f32_matrix"]["seconds"]}
        del dp, pp, nbp, wp, b, pstar, x

    # ---- CPU oracle: baseline and per-output errors (oracle inputs never come from the device)
    if not args.no_cpu_baseline:
        import ctypes

        import oracle
        t0 = time.perf_counter()
        rp_o, col_o = oracle.neighbours(d)
        t_nbr_o = time.perf_counter() - t0
        assert np.array_equal(rp_o, rp) and np.array_equal(col_o, col_np), "neighbour lists differ"
        # the whole cloud's stencils and outputs (the error reference), repeated until ~10 s of wall time
        passes, t_all = 0, 0.0
        while passes < 1 or (t_all < 10.0 and passes < 40):
            t0 = time.perf_counter()
            w_o, st_o, _ = oracle.gfdm_weights(d, rp_o, col_o)
            y_o = oracle.apply(rp_o, col_o, w_o, f)
            t_all += time.perf_counter() - t0
            passes += 1
        t_o = t_all / passes
        try:
            gomp = ctypes.CDLL("libgomp.so.1")
            cores = int(gomp.omp_get_max_threads())
        except OSError:
            gomp, cores = None, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu_model = "unknown"
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        cpu_model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        # one core: a sample of 20,000 rows (every 25th), stencils + application
        one_core = None
        if gomp is not None:
            sample = np.arange(0, N, max(1, N // 20000))
            gomp.omp_set_num_threads(1)
            t0 = time.perf_counter()
            w_s, _, _ = oracle.gfdm_weights(d, rp_o, col_o, rows=sample)
            oracle.apply(rp_o, col_o, w_s, f)
            t1 = time.perf_counter() - t0
            gomp.omp_set_num_threads(cores)
            one_core = {"value": sample.size / t1, "unit": "particles/s", "cores": 1,
                        "sample": f"{sample.size} rows (every {max(1, N // 20000)}th), stencils + application "
                                  f"({t1:.2f} s; the application pass runs over all rows, with zero stencils "
                                  f"outside the sample)"}
        result["cpu_baseline"] = {"value": N / t_o, "unit": "particles/s", "cores": cores, "kind": "oracle",
                                  "cpu_model": cpu_model,
                                  "sample": f"all {N} particles of the workload, stencils + application, mean of "
                                            f"{passes} passes ({t_o:.2f} s each; neighbour search "
                                            f"{t_nbr_o:.2f} s not included)",
                                  "one_core": one_core}
        e32 = oracle.operator_error(w32n, w_o, rp_o)
        e64 = oracle.operator_error(w64n, w_o, rp_o)
        result["operator_error"] = {
            "metric": "per row and stencil |c - c_ref|_2 / |c_ref|_2 against the FP64 oracle (Householder QR)",
            "batched_f32_max": float(e32.max()), "batched_f32_p9999": float(np.quantile(e32, 0.9999)),
            "plain_f64_max": float(e64.max())}
        result["output_error"] = {
            "metric": "max_i |y_i - y_ref_i| / max_i sum_j |c_ref_ij (u_j - u_i)| per output and model",
            "fused_f32_stencils": per_output_errors(yfn, y_o, rp_o, col_o, w_o, f, d["model"]),
            "separate_calls_f32_stencils": per_output_errors(y32n, y_o, rp_o, col_o, w_o, f, d["model"]),
            "plain_f64": per_output_errors(y64n, y_o, rp_o, col_o, w_o, f, d["model"])}
        log(f"oracle {t_o:.2f}s on {cores} cores; f32 err max {e32.max():.2e}, f64 err max {e64.max():.2e}")
        if jet_eval is not None:
            dj, fj, samp, rpj, wjn, yjn, w64jn, y64jn = jet_eval
            rpj_o, colj_o = oracle.neighbours(dj)
            assert np.array_equal(rpj_o, rpj), "jet neighbour lists differ"
            wj_o, stj_o, _ = oracle.gfdm_weights(dj, rpj_o, colj_o, rows=samp)
            yj_o = oracle.apply(rpj_o, colj_o, wj_o, fj)[:, samp]
            sel = np.concatenate([np.arange(rpj_o[i], rpj_o[i + 1]) for i in samp])
            sub = np.concatenate([[0], np.cumsum(np.diff(rpj_o)[samp])])
            wj_o, colj_s = wj_o[sel], colj_o[sel]
            del colj_o
            ej = oracle.operator_error(wjn, wj_o, sub)
            ej64 = oracle.operator_error(w64jn, wj_o, sub)
            result["jet"]["operator_error"] = {"batched_f32_max": float(ej.max()), "plain_f64_max": float(ej64.max()),
                                               "sample": "20,000 random rows"}
            result["jet"]["output_error"] = {
                "fused_f32_stencils": per_output_errors(yjn, yj_o, sub, colj_s, wj_o, fj, dj["model"], rows=samp),
                "plain_f64": per_output_errors(y64jn, yj_o, sub, colj_s, wj_o, fj, dj["model"], rows=samp)}
            log(f"jet operator error f32 {ej.max():.2e}")

    # ---- the convergence study of the advection-diffusion analogue (not part of the default run)
    if args.advdiff:
        from paper_2405_13165_amd.advdiff import AdvectPlate, DiffusionPlate
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
            log(f"advdiff {rec}")
            del plate
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
            log(f"advect {rec}")
        result["advdiff"] = {"kappa": kappa, "t_end": t_end, "study": study,
                             "moving": {"t_end": t_adv, "window": [1.0, 2.0], "study": moving}}

    result["bench_wall_s"] = round(time.time() - t_start, 1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
