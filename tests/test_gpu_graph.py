"""The fused weights+apply step captured in a HIP graph (through torch's
graph capture) gives, on every replay, exactly what the same call gives
eagerly: new field values between the replays, eager work and
synchronisation between them, outputs cleared before each replay."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("wtype", ["f32", "f64"])
def test_graph_replay_matches_eager(ctx, g, wtype):
    print(f"\n[graph] mixed factor 4, {wtype}", flush=True)
    d = W.mixed_block_film(factor=4)
    p = g.Particles.from_dict(ctx, d)
    nb = g.build_neighbours(ctx, p)
    wt = g.GF_F32 if wtype == "f32" else g.GF_F64
    u = torch.as_tensor(W.test_field(d["x"], d["y"], d["z"])[0], device=ctx.device).clone()
    w = torch.empty((nb.nnz, 4), dtype=torch.float32 if wtype == "f32" else torch.float64, device=ctx.device)
    y = torch.empty((4, p.n), dtype=torch.float64, device=ctx.device)

    def step():
        g.gfdm_weights_apply(ctx, p, nb, u, 0xF, wt, w_out=w, out=y)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up: the library sizes its scratch outside the capture
        step()
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for rep in range(4):
        u.copy_(torch.as_tensor(rng.standard_normal(p.n), device=ctx.device))
        step()
        torch.cuda.synchronize()
        w_ref, y_ref = w.clone(), y.clone()
        w.zero_()
        y.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(w, w_ref), f"stencils differ on replay {rep}"
        assert torch.equal(y, y_ref), f"applied values differ on replay {rep}"
