"""gf_gfdm_weights_apply_noalloc (the fused stencil call that allocates nothing)
against gf_gfdm_weights_apply on the same inputs, through the C ABI.

Two calls in a row on one device, the second on a smaller cloud: the fixed
workspace keeps the first call's contents, so the second must not depend on
them.  The two entry points run the same kernels, so stencils, applied values
and statuses must agree bit for bit (stricter than the FP32 / FP64
tolerances).  The calls must not change the device's free memory."""
import numpy as np
import pytest
import torch

from paper_2405_13165_amd import gfdm as g
from paper_2405_13165_amd import workloads as W

pytestmark = pytest.mark.gpu


def _outputs(ctx, d, noalloc, kappa_max=None, wtype=g.GF_F32):
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    f = W.test_field(d["x"], d["y"], d["z"])[0]
    u = torch.as_tensor(f, device=ctx.device)
    dt = torch.float32 if wtype == g.GF_F32 else torch.float64
    w = torch.full((nb.nnz, 4), np.nan, dtype=dt, device=ctx.device)
    out = torch.full((4, p.n), np.nan, dtype=torch.float64, device=ctx.device)
    status = torch.full((p.n,), -1, dtype=torch.int8, device=ctx.device)
    prm = g.ls_params(kappa_max=kappa_max)
    return p, nb, u, w, out, status, prm


def _run(ctx, args, noalloc):
    p, nb, u, w, out, status, prm = args
    if noalloc:
        g.gfdm_weights_apply_noalloc(ctx, p, nb, u, w, out, 0xF, params=prm, status=status)
    else:
        g.gfdm_weights_apply(ctx, p, nb, u, 0xF, g.GF_F32 if w.dtype == torch.float32 else g.GF_F64,
                             params=prm, status=status, w_out=w, out=out)
    torch.cuda.synchronize()
    return w.clone(), out.clone(), status.clone()


def test_noalloc_matches_the_allocating_call():
    big = W.mixed_block_film(factor=3)                      # tiled rows only, 56,000 particles
    small = W.jet_impact(n_bulk=12_000, n_film=12_000)      # rows above 128 entries: packed positions
    assert small["x"].size < big["x"].size
    print(f"[noalloc] big n={big['x'].size} small n={small['x'].size}", flush=True)
    ref_ctx = g.Context(0)
    na_ctx = g.Context(0)
    cases = []
    # the small cloud with a low kappa_max, so that part of it goes through the QR fallback queue
    for d, kmax in ((big, None), (small, 2e3)):
        r_args = _outputs(ref_ctx, d, False, kmax)
        ref = _run(ref_ctx, r_args, False)
        cases.append((_outputs(na_ctx, d, True, kmax), ref))
    assert int((cases[1][1][2] == 1).sum()) > 0, "the second cloud should send rows to the QR fallback"
    _run(na_ctx, cases[1][0], True)  # warm-up (kernels resident)
    free0 = torch.cuda.mem_get_info(0)[0]
    got = [_run(na_ctx, args, True) for args, _ in cases]   # big, then small
    free1 = torch.cuda.mem_get_info(0)[0]
    assert abs(free0 - free1) <= (2 << 20), f"device free memory changed by {free0 - free1} bytes"
    for k, ((w, out, st), (w_r, out_r, st_r)) in enumerate(zip(got, [c[1] for c in cases])):
        print(f"[noalloc] call {k}: n={out.shape[1]} nnz={w.shape[0]} fallback rows={int((st == 1).sum())}",
              flush=True)
        assert torch.equal(st, st_r), f"call {k}: statuses differ"
        assert torch.equal(w, w_r), f"call {k}: stencils differ"
        assert torch.equal(out, out_r), f"call {k}: applied values differ"


def test_noalloc_fp64_stencils_and_discarded_stencils():
    d = W.mixed_block_film(factor=10)
    ref_ctx = g.Context(0)
    na_ctx = g.Context(0)
    a_ref = _outputs(ref_ctx, d, False, None, g.GF_F64)
    a_na = _outputs(na_ctx, d, True, None, g.GF_F64)
    w_r, out_r, st_r = _run(ref_ctx, a_ref, False)
    w, out, st = _run(na_ctx, a_na, True)
    assert torch.equal(w, w_r) and torch.equal(out, out_r) and torch.equal(st, st_r)
    # stencils not stored (w_out = NULL): FP32 stencils applied and discarded, both entry points
    p, nb, u, _, out2, status2, prm = a_na
    out2.fill_(np.nan)
    g.gfdm_weights_apply_noalloc(na_ctx, p, nb, u, None, out2, 0xF, params=prm, status=status2, wtype=g.GF_F32)
    pr, nbr_, ur, _, _, _, _ = a_ref
    _, out3 = g.gfdm_weights_apply(ref_ctx, pr, nbr_, ur, 0xF, g.GF_F32, store_weights=False)
    torch.cuda.synchronize()
    assert torch.equal(out2, out3)
