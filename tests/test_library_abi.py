"""The HIP library loads on a CPU-only host and exports every entry point
declared in include/gfdm.h (no kernel is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfdm.h")
LIB = os.path.join(ROOT, "paper_2405_13165_amd", "libgfdm.so")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(gf_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2405_13165_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_2405_13165_amd import gfdm
    assert sorted(gfdm.EXPORTED) == declared_symbols()


def test_parameter_defaults_follow_the_paper(lib):
    from paper_2405_13165_amd import gfdm
    gfdm.load_library()
    p = gfdm.pca_params()
    assert p.eps_lambda_max == 0.15                      # Sec. 4.1.2
    assert abs(p.theta_star - 3.141592653589793 / 6) < 1e-15  # Sec. 4.1.3
    assert p.literal_rule == 0
    s = gfdm.solve_params()
    assert s.zeta == 0.3 and s.rtol == 1e-8             # Sec. 7.2; tolerance of the solve
    l = gfdm.ls_params()
    assert l.alpha_w == 8.0 and l.kappa_max > 0
    assert gfdm.load_library().gf_version().startswith(b"gfdm")


def test_null_arguments_are_rejected_without_a_device(lib):
    # calls with a NULL context are rejected before touching the device
    from paper_2405_13165_amd import gfdm
    L = gfdm.load_library()
    assert L.gf_build_neighbours(None, None, 0, None) == gfdm.GF_EINVAL
    assert L.gf_apply_stencil(None, None, 0, None, 15, 0, None, None) == gfdm.GF_EINVAL
    assert L.gf_poisson_solve(None, None, None, None, None, None, None, None, None) == gfdm.GF_EINVAL
    assert L.gf_last_error(None) == b"no context"
