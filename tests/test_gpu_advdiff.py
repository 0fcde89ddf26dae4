"""The diffusion analogue of the advection-diffusion test (Sec. 7.3) on the
GPU library against the oracle's time loop (same cloud, same ghosts, same
implicit steps; the oracle solves each step exactly by sparse LU), and its
accuracy against the exact heat-kernel solution."""
import numpy as np
import pytest

import oracle
from paper_2405_13165_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KAPPA, T_END = 5e-3, 0.5


@pytest.fixture(scope="module")
def ctx():
    from paper_2405_13165_amd import gfdm
    gfdm.load_library()
    c = gfdm.Context(0)
    yield c
    c.close()


def _steps(h):
    return int(np.ceil(T_END / (0.25 * 0.05 * h * h / KAPPA)))


def test_advdiff_time_loop_matches_oracle(ctx):
    from paper_2405_13165_amd.advdiff import DiffusionPlate
    h = 0.12
    d = W.advdiff_plate(h)
    rows = W.advdiff_rows(d, h)
    steps = _steps(h)
    plate = DiffusionPlate(ctx, d, rows, KAPPA, T_END / steps)
    T, info = plate.run(steps)
    T_o = oracle.advdiff_run(d, rows, KAPPA, T_END, steps)
    err = np.abs(T.cpu().numpy() - T_o).max()
    print(f"\n[advdiff] h={h} n={d['x'].size} ghosts={plate.n_ghosts} steps={steps} {info} max diff {err:.2e}")
    assert err <= 1e-9


def test_advdiff_accuracy_against_exact_solution(ctx):
    from paper_2405_13165_amd.advdiff import DiffusionPlate
    h = 0.06
    d = W.advdiff_plate(h)
    steps = _steps(h)
    plate = DiffusionPlate(ctx, d, W.advdiff_rows(d, h), KAPPA, T_END / steps)
    T, info = plate.run(steps)
    T = T.cpu().numpy()
    ex = W.advdiff_exact(d["x"], d["y"], T_END, KAPPA)
    e2 = np.sqrt(((T - ex) ** 2).sum() / (ex ** 2).sum())
    print(f"\n[advdiff] h={h} e2={e2:.3e} {info}")
    assert e2 < 1e-2
