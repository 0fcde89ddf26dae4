"""FP64 CPU oracle for the GFDM hot path (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path never calls it, and it shares no
code with the GPU library: the C source in this directory is compiled with gcc
on its own, and this wrapper only marshals numpy arrays through ctypes.

Every function states the part of the paper it follows; the C file holds the
arithmetic.  The pressure solve uses a sparse direct solver (scipy's SuperLU):
the oracle of a linear solve is the solution of the linear system itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gfdm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Parameters the paper fixes (Sec. 4.1.2, 4.1.3, 7.2) and the readings used
# where it is silent (support weight sharpness).
EPS_LAMBDA_MAX = 0.15
THETA_STAR = np.pi / 6.0
ZETA = 0.3
ALPHA_W = 8.0

OP_DX, OP_DY, OP_DZ, OP_LAP = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def _declare(L):
    L.orc_nbr_brute.restype = _I64
    L.orc_nbr_brute.argtypes = [_I64, _P, _P, _P, _P, _P, ctypes.c_int, _P, _P]
    L.orc_nbr_grid.restype = _I64
    L.orc_nbr_grid.argtypes = [_I64, _P, _P, _P, _P, _P, ctypes.c_int, _P, _P]
    L.orc_pca.restype = None
    L.orc_pca.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_classify.restype = None
    L.orc_classify.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                               _P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P]
    L.orc_gfdm_weights.restype = None
    L.orc_gfdm_weights.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                   ctypes.c_double, _P, _I64, _P, _P, _P]
    L.orc_gram_kappa.restype = None
    L.orc_gram_kappa.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_double, _P]
    L.orc_gfdm_weights_normal_ld.restype = None
    L.orc_gfdm_weights_normal_ld.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                             ctypes.c_double, _P]
    L.orc_apply.restype = None
    L.orc_apply.argtypes = [_I64, _P, _P, _P, ctypes.c_uint, _P, _P]
    L.orc_apply_adjoint.restype = None
    L.orc_apply_adjoint.argtypes = [_I64, _P, _P, _P, ctypes.c_uint, _P, _P]
    L.orc_poisson_assemble.restype = None
    L.orc_poisson_assemble.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_double, _P]
    L.orc_transition_3d_to_2d.restype = None
    L.orc_transition_3d_to_2d.argtypes = [_I64] + [_P] * 21
    L.orc_film_height.restype = None
    L.orc_film_height.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_double, _P]
    L.orc_transition_2d_to_3d.restype = _I64
    L.orc_transition_2d_to_3d.argtypes = ([_I64] + [_P] * 9 + [ctypes.c_double, ctypes.c_double]
                                          + [_P] * 3 + [ctypes.c_int, _I64, _I64] + [_P] * 13
                                          + [_I64, _P])
    L.orc_buffer_flags.restype = None
    L.orc_buffer_flags.argtypes = [_I64, _P, _P, _P, _P]
    L.orc_weights_adjoint_x.restype = None
    L.orc_weights_adjoint_x.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                        ctypes.c_double, ctypes.c_uint, _P, _P, _P]


def _p(a):
    """Pointer to a numpy array's data.  The pointer object holds a reference
    to the array, so a temporary (a contiguous copy of a strided view) lives
    as long as the argument list that carries it."""
    if a is None:
        return None
    ptr = ctypes.c_void_p(a.ctypes.data)
    ptr._array = a
    return ptr


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int8)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def _pos(p):
    return (_f64(p["x"]), _f64(p["y"]), _f64(p["z"]), _f64(p["h"]), _i8(p["model"]))


def neighbours(p, cross: bool = False, method: str = "grid"):
    """S_i of Eq. (Nbd) (same-model sets unless cross=True), as CSR with rows
    sorted ascending.  method 'brute' is the O(N^2) definition."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    row_ptr = np.zeros(n + 1, np.int64)
    fn = lib().orc_nbr_brute if method == "brute" else lib().orc_nbr_grid
    nnz = fn(n, _p(x), _p(y), _p(z), _p(h), _p(model), int(cross), _p(row_ptr), None)
    col = np.zeros(max(nnz, 1), np.int32)[:nnz]
    col = np.ascontiguousarray(col)
    fn(n, _p(x), _p(y), _p(z), _p(h), _p(model), int(cross), _p(row_ptr), _p(col))
    return row_ptr, col


def pca(p, row_ptr, col):
    """Eigenvalues (descending), smallest-eigenvalue direction w3 and
    eps_lambda = 2 l3 / (l1 + l2) of the local covariance (Sec. 4.1.2)."""
    x, y, z, _, _ = _pos(p)
    n = x.shape[0]
    lam = np.zeros((n, 3)); w3 = np.zeros((n, 3)); eps = np.zeros(n)
    lib().orc_pca(n, _p(x), _p(y), _p(z), _p(row_ptr), _p(col), _p(lam), _p(w3), _p(eps))
    return lam, w3, eps


def classify(p, row_ptr, col, eps, w3, cross=None, film_height=None, h3d=None, prev=None,
             user=None, eps_max=EPS_LAMBDA_MAX, theta_star=THETA_STAR, literal_rule=False):
    """Transition flags (0 none, 1 bulk->film, 2 film->bulk): Alg. 2,
    Eq. (2Dto3Dcond) and the smoothing rules of Sec. 4.3."""
    n = p["x"].shape[0]
    flag = np.zeros(n, np.uint8)
    xr, xc = (None, None) if cross is None else cross
    L = lib()
    L.orc_classify(n, _p(_i8(p["model"])), _p(_i8(p["kind"])), _p(_f64(p["nx"])),
                   _p(_f64(p["ny"])), _p(_f64(p["nz"])), _p(row_ptr), _p(col), _p(xr), _p(xc),
                   _p(_f64(eps)), _p(_f64(w3.reshape(-1))), _p(_f64(film_height)), _p(_f64(h3d)),
                   _p(_u8(prev)), _p(_u8(user)), eps_max, theta_star, int(literal_rule),
                   _p(flag))
    return flag


def gfdm_weights(p, row_ptr, col, alpha_w=ALPHA_W, rows=None):
    """Second-order GFDM stencils (Eq. GFDM_Definition) by Householder QR.
    Returns w [nnz, 4] (d/dx, d/dy, d/dz, Laplacian), status [n], kappa [n].
    If rows is given, only those rows are computed (others stay zero)."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    nnz = int(row_ptr[-1])
    w = np.zeros((nnz, 4))
    status = np.zeros(n, np.int8)
    kappa = np.zeros(n)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    lib().orc_gfdm_weights(n, _p(x), _p(y), _p(z), _p(h), _p(model), _p(_f64(p["nx"])),
                           _p(_f64(p["ny"])), _p(_f64(p["nz"])), _p(row_ptr), _p(col), alpha_w,
                           _p(r), 0 if r is None else r.shape[0], _p(w), _p(status), _p(kappa))
    return w, status, kappa


def gram_kappa(p, row_ptr, col, alpha_w=ALPHA_W):
    """Per particle kappa_1(G) = ||G||_1 ||G^-1||_1 of the Gram matrix
    G = M^T W M = R^T R of the stencil's least-squares problem (scaled local
    coordinates): the condition estimate behind the FP64 fallback.  0 where
    n_i < m, inf where the QR test finds the problem rank deficient."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    k = np.zeros(n)
    lib().orc_gram_kappa(n, _p(x), _p(y), _p(z), _p(h), _p(model), _p(_f64(p["nx"])), _p(_f64(p["ny"])),
                         _p(_f64(p["nz"])), _p(row_ptr), _p(col), alpha_w, _p(k))
    return k


def gfdm_weights_normal_ld(p, row_ptr, col, alpha_w=ALPHA_W):
    """Same stencils from the normal equations in long double (cross-check)."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    w = np.zeros((int(row_ptr[-1]), 4))
    lib().orc_gfdm_weights_normal_ld(n, _p(x), _p(y), _p(z), _p(h), _p(model),
                                     _p(_f64(p["nx"])), _p(_f64(p["ny"])), _p(_f64(p["nz"])),
                                     _p(row_ptr), _p(col), alpha_w, _p(w))
    return w


def mask_ops(op_mask):
    return [s for s in range(4) if op_mask & (1 << s)]


def apply(row_ptr, col, w, u, op_mask=0xF):
    """y_i^s = sum_{j != i} c_ij^s (u_j - u_i), stacked [K, n]."""
    n = row_ptr.shape[0] - 1
    K = len(mask_ops(op_mask))
    out = np.zeros((K, n))
    lib().orc_apply(n, _p(row_ptr), _p(col), _p(_f64(w)), op_mask, _p(_f64(u)), _p(out))
    return out


def apply_adjoint(row_ptr, col, w, ybar, op_mask=0xF):
    n = row_ptr.shape[0] - 1
    ub = np.zeros(n)
    lib().orc_apply_adjoint(n, _p(row_ptr), _p(col), _p(_f64(w)), op_mask,
                            _p(_f64(np.ascontiguousarray(ybar))), _p(ub))
    return ub


def weights_adjoint_x(p, row_ptr, col, u, ybar, op_mask=0xF, alpha_w=ALPHA_W):
    """Gradient of L with respect to particle positions through the stencil
    weights, for ybar = dL/dy of the differenced application.  [n, 3]."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    xb = np.zeros((n, 3))
    lib().orc_weights_adjoint_x(n, _p(x), _p(y), _p(z), _p(h), _p(model), _p(_f64(p["nx"])),
                                _p(_f64(p["ny"])), _p(_f64(p["nz"])), _p(row_ptr), _p(col),
                                alpha_w, op_mask, _p(_f64(u)),
                                _p(_f64(np.ascontiguousarray(ybar))), _p(xb))
    return xb


def poisson_matrix(p, row_ptr, col, w, row_type, zeta=ZETA):
    """CSR values of the pressure system (interior Laplacian rows, Dirichlet
    identity rows, PDE + zeta*BC Neumann rows)."""
    n = row_ptr.shape[0] - 1
    val = np.zeros(int(row_ptr[-1]))
    lib().orc_poisson_assemble(n, _p(_f64(p["h"])), _p(_f64(p["nx"])), _p(_f64(p["ny"])),
                               _p(_f64(p["nz"])), _p(_i8(row_type)), _p(row_ptr), _p(col),
                               _p(_f64(w)), zeta, _p(val))
    return val


def poisson_solve(row_ptr, col, val, rhs):
    """Exact solution of A p = rhs by sparse LU (the definition of the solve)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = row_ptr.shape[0] - 1
    A = sp.csr_matrix((val, col, row_ptr), shape=(n, n))
    return spla.spsolve(A.tocsc(), rhs)


def csr_matvec(row_ptr, col, val, v):
    import scipy.sparse as sp
    n = row_ptr.shape[0] - 1
    return sp.csr_matrix((val, col, row_ptr), shape=(n, n)) @ v


def transition_3d_to_2d(p, row_ptr, col, flag, mass, rho, phi):
    """Sec. 5.1 / Alg. 3: deletion sets, averaging, mass lumping, film height
    and droplet diameter.  Returns a dict of arrays."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    out = {k: np.zeros(n) for k in ("mass", "rho", "phi", "height", "diam")}
    keep = np.zeros(n, np.uint8)
    owner = np.zeros(n, np.int32)
    lib().orc_transition_3d_to_2d(n, _p(x), _p(y), _p(z), _p(model), _p(_i8(p["kind"])),
                                  _p(_f64(p["nx"])), _p(_f64(p["ny"])), _p(_f64(p["nz"])),
                                  _p(row_ptr), _p(col), _p(_u8(flag)), _p(_f64(mass)),
                                  _p(_f64(rho)), _p(_f64(phi)), _p(out["mass"]), _p(out["rho"]),
                                  _p(out["phi"]), _p(out["height"]), _p(out["diam"]), _p(keep),
                                  _p(owner))
    out["keep"] = keep
    out["owner"] = owner
    return out


# Sharpness of the droplet kernel of Eq. (Height) and the spacing factors of
# Sec. 2.3: the paper leaves them to the models it cites, so they are
# parameters here (readings: alpha = 8; r_min = 0.2, r_max = 0.4, which keeps
# the spacing h/3 of the synthetic clouds inside [r_min h, r_max h]).
ALPHA_FILM = 8.0
R_MIN = 0.2
R_MAX = 0.4
MAX_GAMMA = 1 << 16


def film_height(p, row_ptr, col, diam, alpha=ALPHA_FILM):
    """Eq. (Height): H_i = sum_{j in S_i} alpha/(pi h_j^2) exp(-alpha r_ij^2/h_j^2)
    pi d_j^3/6 for film particles (S_i same-model), 0 for bulk particles."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    H = np.zeros(n)
    lib().orc_film_height(n, _p(x), _p(y), _p(z), _p(h), _p(model), _p(row_ptr), _p(col),
                          _p(_f64(diam)), float(alpha), _p(H))
    return H


def _phi2(phi, n):
    if phi is None:
        return np.zeros((0, n))
    a = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1, n))
    return a


def transition_2d_to_3d(p, sel, height, h3d, mass, rho, phi=None, r_min=R_MIN, r_max=R_MAX,
                        max_gamma=MAX_GAMMA):
    """Sec. 5.2 / Alg. 4 for the film particles `sel` (ascending): each turns
    into a 3D wall particle followed by gamma_i = ceil(H_i / psi~_i) added
    particles at x_i + k psi_i n_i (Eq. psi~, Eq. gamma), mass split evenly,
    density and fields copied.  Returns a dict of the new particle arrays
    (rows of a source consecutive, k = 0..gamma) and `off`."""
    x, y, z, h, model = _pos(p)
    n = x.shape[0]
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    ns = sel.shape[0]
    ph = _phi2(phi, n)
    nphi = ph.shape[0]
    off = np.zeros(ns + 1, np.int64)
    args = [ns, _p(sel), _p(x), _p(y), _p(z), _p(_f64(p["nx"])), _p(_f64(p["ny"])),
            _p(_f64(p["nz"])), _p(_f64(height)), _p(_f64(h3d)), float(r_min), float(r_max),
            _p(_f64(mass)), _p(_f64(rho)), _p(ph if nphi else None), nphi, n, int(max_gamma),
            _p(off)]
    L = lib()
    total = L.orc_transition_2d_to_3d(*args, *([None] * 12), 0, None)
    if total < 0:
        raise ValueError("a particle needs more than max_gamma added particles")
    o = {k: np.zeros(total) for k in ("x", "y", "z", "h", "nx", "ny", "nz", "mass", "rho")}
    o["model"] = np.zeros(total, np.int8)
    o["kind"] = np.zeros(total, np.int8)
    o["phi"] = np.zeros((nphi, total))
    o["src"] = np.zeros(total, np.int32)
    L.orc_transition_2d_to_3d(*args, _p(o["x"]), _p(o["y"]), _p(o["z"]), _p(o["h"]),
                              _p(o["model"]), _p(o["kind"]), _p(o["nx"]), _p(o["ny"]),
                              _p(o["nz"]), _p(o["mass"]), _p(o["rho"]),
                              _p(o["phi"] if nphi else None), total, _p(o["src"]))
    o["height"] = np.zeros(total)
    o["diam"] = np.zeros(total)
    o["off"] = off
    return o


def buffer_flags(p, cross_row_ptr, cross_col):
    """First loop of Alg. 5 (Sec. 6.1): particles with a particle of the other
    model within their support, and those particles themselves."""
    n = p["x"].shape[0]
    flag = np.zeros(n, np.uint8)
    lib().orc_buffer_flags(n, _p(_i8(p["model"])), _p(cross_row_ptr), _p(cross_col), _p(flag))
    return flag


_GHOST_KEYS = ("x", "y", "z", "h", "nx", "ny", "nz", "mass", "rho", "height", "diam")


def buffer_zone(p, cross_row_ptr, cross_col, film_h, h_other, mass, rho, phi=None,
                r_min=R_MIN, r_max=R_MAX, max_gamma=MAX_GAMMA):
    """Ghost particles of Sec. 6.1 / Alg. 5, in the paper's order:
    (1) flag particles near the other model; (2) put an intermediate ghost of
    the same model on every flagged particle; (3) transition the ghosts: the
    3D ghosts as in Sec. 5.1 with every wall ghost flagged (neighbourhoods of
    Eq. (Nbd) among the 3D ghosts themselves; interior and free-surface ghosts
    are mapped onto their nearest wall ghost and deleted), the 2D ghosts as
    in Sec. 5.2.  h_other[i] is the resolution of the other model at particle
    i: the h of the ghosts made from i, and the 3D resolution of psi~.
    Ghosts come out ordered by source index (k = 0..gamma within a 2D source).
    Returns (flag, dict of ghost arrays with 'src')."""
    n = p["x"].shape[0]
    flag = buffer_flags(p, cross_row_ptr, cross_col)
    src = np.nonzero(flag)[0]
    model = np.asarray(p["model"])
    ph = _phi2(phi, n)
    parts = []
    # 3D intermediate ghosts -> 2D ghosts
    g3 = src[model[src] == 0]
    if g3.size:
        sub = {k: np.ascontiguousarray(np.asarray(p[k])[g3]) for k in
               ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz")}
        rp, col = neighbours(sub)
        wall = (sub["kind"] == 2).astype(np.uint8)
        fields = ph[:, g3] if ph.shape[0] else np.zeros((1, g3.size))
        trs = [transition_3d_to_2d(sub, rp, col, wall, np.asarray(mass)[g3],
                                   np.asarray(rho)[g3], f) for f in fields]
        keep = np.nonzero(wall)[0]
        tr = trs[0]
        g = {k: sub[k][keep].astype(np.float64) for k in ("x", "y", "z", "nx", "ny", "nz")}
        g["h"] = np.asarray(h_other, dtype=np.float64)[g3][keep]
        g["model"] = np.ones(keep.size, np.int8)
        g["kind"] = np.full(keep.size, 2, np.int8)
        g["mass"] = tr["mass"][keep]
        g["rho"] = tr["rho"][keep]
        g["height"] = tr["height"][keep]
        g["diam"] = tr["diam"][keep]
        g["phi"] = (np.stack([t["phi"][keep] for t in trs]) if ph.shape[0]
                    else np.zeros((0, keep.size)))
        g["src"] = g3[keep].astype(np.int32)
        parts.append(g)
    # 2D intermediate ghosts -> 3D ghosts
    g2 = src[model[src] == 1]
    if g2.size:
        o = transition_2d_to_3d(p, g2, film_h, h_other, mass, rho, ph if ph.shape[0] else None,
                                r_min, r_max, max_gamma)
        o.pop("off")
        parts.append(o)
    if not parts:
        out = {k: np.zeros(0) for k in _GHOST_KEYS}
        out.update(model=np.zeros(0, np.int8), kind=np.zeros(0, np.int8),
                   phi=np.zeros((ph.shape[0], 0)), src=np.zeros(0, np.int32))
        return flag, out
    out = {k: np.concatenate([q[k] for q in parts]) for k in _GHOST_KEYS + ("model", "kind", "src")}
    out["phi"] = np.concatenate([q["phi"] for q in parts], axis=1)
    order = np.argsort(out["src"], kind="stable")
    out = {k: (v[:, order] if k == "phi" else v[order]) for k, v in out.items()}
    return flag, out


def extend_cloud(p, ghosts):
    """Regular particles followed by ghost particles (one cloud)."""
    keys = ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz")
    return {k: np.concatenate([np.asarray(p[k]), np.asarray(ghosts[k]).astype(np.asarray(p[k]).dtype)])
            for k in keys}


def neighbours_rows(p, n_rows, cross=False):
    """Extended neighbourhoods of Sec. 6.2: rows of particles [0, n_rows) hold
    S_i of Eq. (Nbd) over the whole cloud (regular and ghost particles); the
    particles beyond n_rows (ghosts) get no derivatives, their rows hold only
    themselves."""
    rp, col = neighbours(p, cross=cross)
    n = rp.shape[0] - 1
    lens = np.diff(rp).copy()
    lens[n_rows:] = 1
    rp2 = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp2[1:])
    keep = np.repeat(np.arange(n) < n_rows, np.diff(rp))
    col2 = np.empty(int(rp2[-1]), np.int32)
    reg = np.zeros(n, bool); reg[:n_rows] = True
    pos = np.repeat(reg, lens)
    col2[pos] = col[keep]
    col2[~pos] = np.arange(n_rows, n, dtype=np.int32)
    return rp2, col2


def poisson_split_solve(p, row_ptr, col, w, row_type, n_regular, rhs, p_ghost, zeta=ZETA):
    """Implicit step with ghost neighbours (Sec. 6.2): only regular particles
    are unknowns; the ghost terms of each regular row use the known ghost
    values and move to the right-hand side:
        A_rr p_r = rhs_r - A_rg p_g."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = row_ptr.shape[0] - 1
    val = poisson_matrix(p, row_ptr, col, w, row_type, zeta)
    A = sp.csr_matrix((val, col, row_ptr), shape=(n, n))
    Arr = A[:n_regular, :n_regular]
    Arg = A[:n_regular, n_regular:]
    b = np.asarray(rhs, dtype=np.float64)[:n_regular] - Arg @ np.asarray(p_ghost, dtype=np.float64)
    return spla.spsolve(Arr.tocsc(), b)


def transition_3d_to_2d_cloud(p, row_ptr, col, flag, mass, rho, phi=None, film_height=None, diam=None,
                              h_film=None):
    """Sec. 5.1, Alg. 3 carried to the end: the particles mapped onto a
    transitioning wall particle are deleted and the flagged particles become
    film particles ("remove from the 3D structure, add to the 2D one").  The
    data mapping of every field is the one of transition_3d_to_2d.  Returns a
    dict describing the new cloud in the caller's order without the deleted
    particles: positions and normals copied; h = h_film (or h) for
    transitioned particles; model 1 and kind wall for transitioned particles;
    mass, rho, phi lumped / averaged for them and copied otherwise; height =
    H for transitioned particles, the given film height for film particles,
    0 for bulk; diam likewise; src = original index."""
    n = p["x"].shape[0]
    ph = _phi2(phi, n)
    fields = ph if ph.shape[0] else np.zeros((1, n))
    trs = [transition_3d_to_2d(p, row_ptr, col, flag, mass, rho, f) for f in fields]
    tr = trs[0]
    keep = np.nonzero(tr["keep"] == 1)[0]
    moved = np.asarray(flag)[keep] == 1
    model = np.asarray(p["model"])[keep].astype(np.int8)
    out = {k: np.asarray(p[k], dtype=np.float64)[keep].copy() for k in ("x", "y", "z", "nx", "ny", "nz")}
    h = np.asarray(p["h"], dtype=np.float64)[keep].copy()
    if h_film is not None:
        h[moved] = np.asarray(h_film, dtype=np.float64)[keep][moved]
    out["h"] = h
    out["model"] = np.where(moved, 1, model).astype(np.int8)
    out["kind"] = np.where(moved, 2, np.asarray(p["kind"])[keep]).astype(np.int8)
    out["mass"] = tr["mass"][keep]
    out["rho"] = tr["rho"][keep]
    out["phi"] = (np.stack([t["phi"][keep] for t in trs]) if ph.shape[0] else np.zeros((0, keep.size)))
    film = model == 1
    hgt = np.where(film, 0.0 if film_height is None else np.asarray(film_height)[keep], 0.0)
    dia = np.where(film, 0.0 if diam is None else np.asarray(diam)[keep], 0.0)
    out["height"] = np.where(moved, tr["height"][keep], hgt)
    out["diam"] = np.where(moved, tr["diam"][keep], dia)
    out["src"] = keep.astype(np.int32)
    return out


def advdiff_run(d, rows, kappa, t_end, steps, r_min=R_MIN, r_max=R_MAX, ghost_scale=1.0):
    """Diffusion of T (Eq. AdvDiff with the Lagrangian motion left out: the
    cloud is static, so the interfaces are fixed and, as Sec. 6.2 prescribes
    for that case, the ghosts keep their places and only their data is
    recomputed every step).  Each step: ghost values from the buffer-zone
    data mapping (Alg. 5) of the current T; then one implicit Euler step
    (I - dt kappa Lap) T^{n+1} = T^n over the extended neighbourhoods, with
    regular rows of the given roles (4: implicit diffusion row, 3: zero
    normal flux, 1: held at zero; ghost rows hold their values), solved
    exactly (sparse LU).  Returns T at t_end.  ghost_scale multiplies the
    ghost values (1: the method; 0: a control without coupling)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = d["x"].shape[0]
    rpc, colc = neighbours(d, cross=True)
    T = np.asarray(d["T0"], dtype=np.float64).copy()
    _, g = buffer_zone(d, rpc, colc, d["film_height"], d["h_other"], d["mass"], d["rho"], T[None, :],
                       r_min, r_max)
    e = extend_cloud(d, g)
    ne = e["x"].shape[0]
    rp, col = neighbours_rows(e, n)
    w, _, _ = gfdm_weights(e, rp, col)
    rt = np.concatenate([np.asarray(rows, dtype=np.int8), np.ones(ne - n, np.int8)])
    dt = t_end / steps
    lap = poisson_matrix(e, rp, col, w, np.zeros(ne, np.int8))
    bc = poisson_matrix(e, rp, col, w, np.where(rt == 4, 0, rt).astype(np.int8))
    rid = np.repeat(np.arange(ne), np.diff(rp))
    val = np.where(rt[rid] == 4, (col == rid).astype(np.float64) - dt * kappa * lap, bc)
    lu = spla.splu(sp.csr_matrix((val, col, rp), shape=(ne, ne)).tocsc())
    for _ in range(steps):
        _, g = buffer_zone(d, rpc, colc, d["film_height"], d["h_other"], d["mass"], d["rho"], T[None, :],
                           r_min, r_max)
        rhs = np.concatenate([T, ghost_scale * g["phi"][0]])
        rhs[:n][rt[:n] != 4] = 0.0
        T = lu.solve(rhs)[:n]
    return T


_CLOUD_KEYS = ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz", "mass", "rho", "T", "H", "edge")


def _rows_of(c, h):
    """Row roles: zero normal flux on 3D walls and free surfaces, zero on the
    plate's edge, implicit diffusion rows elsewhere (as W.advdiff_rows)."""
    rt = np.full(c["x"].shape[0], 4, np.int8)
    rt[(c["model"] == 0) & (c["kind"] != 0)] = 3
    rt[c["edge"] > 0.5] = 1
    return rt


def advect_step(c, h, kappa, dt, x0=1.0, x1=2.0, r_min=R_MIN, r_max=R_MAX):
    """One model-adaptive step of the advection-diffusion case (Sec. 7.2):
    Lagrangian move with v = (1, 0, 0); film particles inside [x0, x1]
    transition to 3D (Sec. 5.2), 3D wall particles beyond x1 transition to
    2D with their columns (Sec. 5.1); then ghosts (Alg. 5), extended
    neighbourhoods (Sec. 6.2) and one implicit Euler diffusion step, solved
    exactly.  c: dict of particle arrays (_CLOUD_KEYS); returns the new one.
    The film thickness H and the edge marker travel as fields.  With
    kappa = 0 (pure advection) the step ends after the transitions."""
    c = {k: np.asarray(v).copy() for k, v in c.items()}
    c["x"] = c["x"] + dt * 1.0
    # 2D -> 3D
    flag2 = ((c["model"] == 1) & (c["x"] >= x0) & (c["x"] <= x1))
    if flag2.any():
        sel = np.nonzero(flag2)[0]
        o = transition_2d_to_3d(c, sel, c["H"], c["h"], c["mass"], c["rho"], np.stack([c["T"], c["edge"]]),
                                r_min, r_max)
        keep = np.nonzero(~flag2)[0]
        new = {k: o[k] for k in ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz", "mass", "rho")}
        new["T"] = o["phi"][0]
        new["edge"] = o["phi"][1]
        new["H"] = np.zeros(o["x"].size)
        c = {k: np.concatenate([c[k][keep], new[k].astype(c[k].dtype)]) for k in _CLOUD_KEYS}
    # 3D -> 2D
    flag1 = ((c["model"] == 0) & (c["kind"] == 2) & (c["x"] > x1)).astype(np.uint8)
    if flag1.any():
        rp, col = neighbours(c)
        o = transition_3d_to_2d_cloud(c, rp, col, flag1, c["mass"], c["rho"], np.stack([c["T"], c["edge"]]),
                                      film_height=c["H"], h_film=c["h"])
        c = {k: o[k] for k in ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz", "mass", "rho")}
        c["T"] = o["phi"][0]
        c["edge"] = o["phi"][1]
        c["H"] = o["height"]
    if kappa == 0.0:
        return c
    # ghosts, extended neighbourhoods, one implicit diffusion step
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = c["x"].size
    rpc, colc = neighbours(c, cross=True)
    _, g = buffer_zone(c, rpc, colc, c["H"], c["h"], c["mass"], c["rho"], c["T"][None, :], r_min, r_max)
    e = extend_cloud(c, g)
    ne = e["x"].size
    rp, col = neighbours_rows(e, n)
    w, _, _ = gfdm_weights(e, rp, col)
    rt = np.concatenate([_rows_of(c, h), np.ones(ne - n, np.int8)])
    lap = poisson_matrix(e, rp, col, w, np.zeros(ne, np.int8))
    bc = poisson_matrix(e, rp, col, w, np.where(rt == 4, 0, rt).astype(np.int8))
    rid = np.repeat(np.arange(ne), np.diff(rp))
    val = np.where(rt[rid] == 4, (col == rid).astype(np.float64) - dt * kappa * lap, bc)
    rhs = np.concatenate([c["T"], g["phi"][0]])
    rhs[:n][rt[:n] != 4] = 0.0
    c["T"] = spla.spsolve(sp.csr_matrix((val, col, rp), shape=(ne, ne)).tocsc(), rhs)[:n]
    return c


def operator_error(w, w_ref, row_ptr):
    """Per row and stencil: |c - c_ref|_2 / |c_ref|_2 over the row's entries.
    Rows/stencils whose reference is identically zero are reported as the
    absolute norm of c instead.  Returns an [n, 4] array."""
    n = row_ptr.shape[0] - 1
    rid = np.repeat(np.arange(n), np.diff(row_ptr))
    d2 = np.stack([np.bincount(rid, (w[:, s] - w_ref[:, s]) ** 2, minlength=n) for s in range(4)], 1)
    r2 = np.stack([np.bincount(rid, w_ref[:, s] ** 2, minlength=n) for s in range(4)], 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(r2 > 0, np.sqrt(d2 / np.where(r2 > 0, r2, 1)), np.sqrt(d2))
    return e
