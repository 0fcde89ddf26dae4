"""Python binding of libgfdm (ctypes).  Argument marshalling only: every
step runs in the HIP kernels of the library.  Tensors must live on the
context's device; calls enqueue on torch's current stream.

The names follow the C ABI in include/gfdm.h (gf_build_neighbours ->
build_neighbours, ...).  If the library is missing this module raises on
import of the library: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfdm.so")

GF_OK, GF_EINVAL, GF_ENOMEM, GF_EHIP, GF_ECAPACITY, GF_ENOTCONV, GF_EBREAKDOWN = 0, -1, -2, -3, -4, -5, -6
GF_F64, GF_F32 = 0, 1
GF_PLAIN_F64, GF_BATCHED = 0, 1
GF_F32_QR_FALLBACK64 = GF_BATCHED
OP_DX, OP_DY, OP_DZ, OP_LAP = 1, 2, 4, 8
ROW_INTERIOR, ROW_DIRICHLET, ROW_NEUMANN_COMBINED, ROW_NEUMANN, ROW_IMPLICIT = 0, 1, 2, 3, 4

_STATUS_NAMES = {0: "GF_OK", -1: "GF_EINVAL", -2: "GF_ENOMEM", -3: "GF_EHIP", -4: "GF_ECAPACITY",
                 -5: "GF_ENOTCONV", -6: "GF_EBREAKDOWN"}


class GfdmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("h", ctypes.c_void_p), ("model", ctypes.c_void_p),
                ("kind", ctypes.c_void_p), ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p),
                ("nz", ctypes.c_void_p)]


class PcaParams(ctypes.Structure):
    _fields_ = [("eps_lambda_max", ctypes.c_double), ("theta_star", ctypes.c_double),
                ("literal_rule", ctypes.c_int)]


class LsParams(ctypes.Structure):
    _fields_ = [("alpha_w", ctypes.c_double), ("kappa_max", ctypes.c_double)]


class LsStats(ctypes.Structure):
    _fields_ = [("n_ok", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("n_rank_deficient", ctypes.c_int64), ("n_too_few", ctypes.c_int64),
                ("kappa_max_seen", ctypes.c_double)]


class SolveParams(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int), ("mixed", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("zeta", ctypes.c_double), ("check_every", ctypes.c_int), ("implicit_a", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_its", ctypes.c_int), ("inner_its_total", ctypes.c_int),
                ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("final_rel_res", ctypes.c_double), ("seconds", ctypes.c_double)]


class NewParticles(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in (
        "x", "y", "z", "h", "model", "kind", "nx", "ny", "nz", "mass", "rho", "phi", "height", "diam", "src")]


EXPORTED = [
    "gf_version", "gf_create", "gf_set_stream", "gf_destroy", "gf_last_error",
    "gf_build_neighbours", "gf_nbr_info", "gf_nbr_view", "gf_nbr_export", "gf_nbr_free",
    "gf_pca_params_default", "gf_classify_pca", "gf_ls_params_default", "gf_gfdm_weights",
    "gf_apply_stencil", "gf_gfdm_weights_apply", "gf_poisson_assemble", "gf_solve_params_default",
    "gf_poisson_solve", "gf_transition_3d_to_2d", "gf_apply_stencil_adjoint",
    "gf_gfdm_weights_adjoint", "gf_profile_enable", "gf_profile_read", "gf_autotune", "gf_set_team_sizes", "gf_set_tile_capacity",
    "gf_build_neighbours_rows", "gf_film_height", "gf_transition_2d_to_3d", "gf_buffer_flags", "gf_buffer_zone",
    "gf_transition_3d_to_2d_cloud", "gf_gfdm_weights_apply_noalloc", "gf_noalloc_workspace_bytes",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgfdm.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2405_13165_amd/build.py "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(path)
    P, I64, I32, U, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint, ctypes.c_double
    PP = ctypes.POINTER(_Particles)
    L.gf_version.restype = ctypes.c_char_p
    L.gf_create.argtypes = [I32, P, ctypes.POINTER(P)]
    L.gf_set_stream.argtypes = [P, P]
    L.gf_destroy.argtypes = [P]
    L.gf_destroy.restype = None
    L.gf_last_error.argtypes = [P]
    L.gf_last_error.restype = ctypes.c_char_p
    L.gf_build_neighbours.argtypes = [P, PP, I32, ctypes.POINTER(P)]
    L.gf_nbr_info.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_int32)]
    L.gf_nbr_export.argtypes = [P, P, P, P]
    L.gf_nbr_view.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(P), ctypes.POINTER(P)]
    L.gf_nbr_free.argtypes = [P]
    L.gf_nbr_free.restype = None
    L.gf_pca_params_default.argtypes = [ctypes.POINTER(PcaParams)]
    L.gf_pca_params_default.restype = None
    L.gf_classify_pca.argtypes = [P, PP, P, P, P, P, P, P, ctypes.POINTER(PcaParams), P, P, P, P]
    L.gf_ls_params_default.argtypes = [ctypes.POINTER(LsParams)]
    L.gf_ls_params_default.restype = None
    L.gf_gfdm_weights.argtypes = [P, PP, P, I32, ctypes.POINTER(LsParams), I32, P, P, P,
                                  ctypes.POINTER(LsStats)]
    L.gf_apply_stencil.argtypes = [P, P, I32, P, U, I32, P, P]
    L.gf_gfdm_weights_apply.argtypes = [P, PP, P, ctypes.POINTER(LsParams), I32, P, U, P, P, P]
    L.gf_gfdm_weights_apply_noalloc.argtypes = [P, PP, P, ctypes.POINTER(LsParams), I32, P, U, P, P, P]
    L.gf_noalloc_workspace_bytes.argtypes = []
    L.gf_noalloc_workspace_bytes.restype = ctypes.c_size_t
    L.gf_poisson_assemble.argtypes = [P, PP, P, P, P, D, P]
    L.gf_solve_params_default.argtypes = [ctypes.POINTER(SolveParams)]
    L.gf_solve_params_default.restype = None
    L.gf_poisson_solve.argtypes = [P, PP, P, P, P, P, P, ctypes.POINTER(SolveParams),
                                   ctypes.POINTER(SolveStats)]
    L.gf_transition_3d_to_2d.argtypes = [P, PP, P] + [P] * 11
    L.gf_apply_stencil_adjoint.argtypes = [P, P, I32, P, U, P, P]
    L.gf_gfdm_weights_adjoint.argtypes = [P, PP, P, ctypes.POINTER(LsParams), U, P, P, P, P]
    L.gf_autotune.argtypes = [P, PP, P, I32, P]
    L.gf_set_team_sizes.argtypes = [P, P, P]
    L.gf_profile_enable.argtypes = [P, I32]
    L.gf_set_tile_capacity.argtypes = [P, I32]
    L.gf_profile_read.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
    L.gf_build_neighbours_rows.argtypes = [P, PP, I32, I64, ctypes.POINTER(P)]
    L.gf_film_height.argtypes = [P, PP, P, P, D, P]
    NP = ctypes.POINTER(NewParticles)
    L.gf_transition_2d_to_3d.argtypes = [P, PP, P, P, P, D, D, P, P, P, I32, NP, ctypes.POINTER(I64)]
    L.gf_buffer_flags.argtypes = [P, PP, P, P, P]
    L.gf_buffer_zone.argtypes = [P, PP, P, P, P, P, D, D, P, P, P, I32, NP, ctypes.POINTER(I64), P]
    L.gf_transition_3d_to_2d_cloud.argtypes = [P, PP, P, P, P, P, P, I32, P, P, P, NP, ctypes.POINTER(I64)]
    for name in EXPORTED:
        getattr(L, name)  # every declared entry point must resolve
    _lib = L
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class _DevArray:
    """__cuda_array_interface__ of device memory the library owns (no copy)."""

    def __init__(self, ptr, count, typestr):
        self.__cuda_array_interface__ = {"shape": (int(count),), "typestr": typestr, "data": (int(ptr or 0), False),
                                         "version": 2}


def _alias(ptr, count, dtype, ctx):
    typestr = {torch.int64: "<i8", torch.int32: "<i4"}[dtype]
    if count == 0 or not ptr:
        return torch.empty(0, dtype=dtype, device=ctx.device)
    return torch.as_tensor(_DevArray(ptr, count, typestr), device=ctx.device)


def _dev_tensor(t, dtype, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


class Context:
    """A library context on one device, enqueuing on torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self.lib.gf_create(device, None, ctypes.byref(h))
        if st != GF_OK:
            raise GfdmError(st, "gf_create failed")
        self.handle = h

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.check(self.lib.gf_set_stream(self.handle, ctypes.c_void_p(s)))

    def check(self, st):
        if st != GF_OK:
            raise GfdmError(st, self.lib.gf_last_error(self.handle).decode())

    def profile(self, on: bool = True):
        """Bracket every library kernel with HIP events (gf_profile_enable)."""
        self.check(self.lib.gf_profile_enable(self.handle, int(on)))

    def set_tile_capacity(self, entries: int = 0):
        """LDS staging limit of the tile kernels (gf_set_tile_capacity); 0 restores the defaults."""
        self.check(self.lib.gf_set_tile_capacity(self.handle, int(entries)))

    def profile_read(self):
        """{kernel name: (launches, total ms)} since the last read; synchronises."""
        buf = ctypes.create_string_buffer(1 << 16)
        self.check(self.lib.gf_profile_read(self.handle, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms = line.split()
            out[name] = (int(cnt), float(ms))
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Particles:
    """Device copies of a particle cloud (structure of arrays)."""

    def __init__(self, ctx: Context, x, y, z, h, model, kind=None, nx=None, ny=None, nz=None):
        dev = ctx.device
        self.x = _dev_tensor(x, torch.float64, dev)
        self.y = _dev_tensor(y, torch.float64, dev)
        self.z = _dev_tensor(z, torch.float64, dev)
        self.h = _dev_tensor(h, torch.float64, dev)
        self.model = _dev_tensor(model, torch.int8, dev)
        self.kind = _dev_tensor(kind, torch.int8, dev)
        self.nx = _dev_tensor(nx, torch.float64, dev)
        self.ny = _dev_tensor(ny, torch.float64, dev)
        self.nz = _dev_tensor(nz, torch.float64, dev)
        self.n = int(self.x.shape[0])
        self.refresh()

    @classmethod
    def from_dict(cls, ctx, d):
        return cls(ctx, d["x"], d["y"], d["z"], d["h"], d["model"], d.get("kind"), d.get("nx"),
                   d.get("ny"), d.get("nz"))

    def refresh(self):
        self.s = _Particles(self.n, _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.h),
                            _ptr(self.model), _ptr(self.kind), _ptr(self.nx), _ptr(self.ny),
                            _ptr(self.nz))
        return self

    def with_positions(self, x, y, z):
        q = object.__new__(Particles)
        q.__dict__.update(self.__dict__)
        q.x, q.y, q.z = x.contiguous(), y.contiguous(), z.contiguous()
        return q.refresh()


class Neighbours:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        n, nnz, mr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        ctx.check(ctx.lib.gf_nbr_info(handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(mr)))
        self.n, self.nnz, self.max_row = n.value, nnz.value, mr.value

    def export(self):
        """(row_ptr int64 [n+1], col int32 [nnz]) device tensors."""
        row_ptr = torch.empty(self.n + 1, dtype=torch.int64, device=self.ctx.device)
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.ctx.device)[: self.nnz]
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.gf_nbr_export(self.ctx.handle, self.handle, _ptr(row_ptr),
                                                  _ptr(col) if self.nnz else None))
        return row_ptr, col

    def view(self):
        """(row_ptr int64 [n+1], col int32 [nnz]) device tensors that alias the
        handle's own lists (gf_nbr_view, no copy); valid while the handle lives."""
        nnz, rp, cp = ctypes.c_int64(), ctypes.c_void_p(), ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.gf_nbr_view(self.handle, ctypes.byref(nnz), ctypes.byref(rp), ctypes.byref(cp)))
        return _alias(rp.value, self.n + 1, torch.int64, self.ctx), _alias(cp.value, nnz.value, torch.int32, self.ctx)

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.gf_nbr_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_neighbours(ctx: Context, p: Particles, cross_model: bool = False, n_rows=None) -> Neighbours:
    """gf_build_neighbours, or gf_build_neighbours_rows when n_rows is given
    (particles from n_rows on are ghosts: neighbours of others, rows of their own)."""
    h = ctypes.c_void_p()
    ctx._sync_stream()
    if n_rows is None:
        ctx.check(ctx.lib.gf_build_neighbours(ctx.handle, ctypes.byref(p.s), int(cross_model), ctypes.byref(h)))
    else:
        ctx.check(ctx.lib.gf_build_neighbours_rows(ctx.handle, ctypes.byref(p.s), int(cross_model), int(n_rows),
                                                   ctypes.byref(h)))
    return Neighbours(ctx, h)


def pca_params(eps_lambda_max=0.15, theta_star=None, literal_rule=False):
    prm = PcaParams()
    load_library().gf_pca_params_default(ctypes.byref(prm))
    prm.eps_lambda_max = eps_lambda_max
    if theta_star is not None:
        prm.theta_star = theta_star
    prm.literal_rule = int(literal_rule)
    return prm


def classify_pca(ctx, p, same, cross=None, film_height=None, h3d=None, prev=None, user=None,
                 params=None, want_flags=True):
    """Returns (lam [n,3], w3 [n,3], eps [n], flag [n] uint8 or None)."""
    dev = ctx.device
    lam = torch.empty((p.n, 3), dtype=torch.float64, device=dev)
    w3 = torch.empty((p.n, 3), dtype=torch.float64, device=dev)
    eps = torch.empty(p.n, dtype=torch.float64, device=dev)
    flag = torch.empty(p.n, dtype=torch.uint8, device=dev) if want_flags else None
    fh = _dev_tensor(film_height, torch.float64, dev)
    h3 = _dev_tensor(h3d, torch.float64, dev)
    pv = _dev_tensor(prev, torch.uint8, dev)
    us = _dev_tensor(user, torch.uint8, dev)
    prm = params if params is not None else pca_params()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_classify_pca(ctx.handle, ctypes.byref(p.s), same.handle,
                                      cross.handle if cross is not None else None, _ptr(fh), _ptr(h3),
                                      _ptr(pv), _ptr(us), ctypes.byref(prm), _ptr(lam), _ptr(w3),
                                      _ptr(eps), _ptr(flag)))
    return lam, w3, eps, flag


def ls_params(alpha_w=8.0, kappa_max=None):
    prm = LsParams()
    load_library().gf_ls_params_default(ctypes.byref(prm))
    prm.alpha_w = alpha_w
    if kappa_max is not None:
        prm.kappa_max = kappa_max
    return prm


def gfdm_weights(ctx, p, nbr, prec=GF_BATCHED, wtype=GF_F32, params=None, out=None,
                 status=None, kappa=None, stats=False):
    """Stencil weights [nnz, 4] (dx, dy, dz, Laplacian) of dtype wtype."""
    dt = torch.float32 if wtype == GF_F32 else torch.float64
    w = out if out is not None else torch.empty((max(nbr.nnz, 1), 4), dtype=dt, device=ctx.device)[: nbr.nnz]
    prm = params if params is not None else ls_params()
    st = LsStats() if stats else None
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_gfdm_weights(ctx.handle, ctypes.byref(p.s), nbr.handle, prec, ctypes.byref(prm),
                                      wtype, _ptr(w), _ptr(status), _ptr(kappa),
                                      ctypes.byref(st) if st is not None else None))
    if stats:
        return w, {k: getattr(st, k) for k, _ in LsStats._fields_}
    return w


def autotune(ctx, p, nbr, wtype=GF_F32):
    """Pick team sizes per group for the stencil, application and fused kernels.
    Returns {'weights', 'apply', 'fused': [8 ints]} (bulk bands 0-3, film bands 0-3)."""
    out = (ctypes.c_int * 24)()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_autotune(ctx.handle, ctypes.byref(p.s), nbr.handle, wtype, out))
    return {"weights": list(out[:8]), "apply": list(out[8:16]), "fused": list(out[16:24])}


def set_team_sizes(ctx, weights=None, apply=None, fused=None):
    """Set the team sizes of the stencil, application and fused kernels (each a
    list of 8 ints in gf_autotune's layout, 0 = keep; None keeps all 8).
    Returns the previous sizes as {'weights', 'apply', 'fused'}."""
    teams = (ctypes.c_int * 24)()
    for k, v in enumerate((weights, apply, fused)):
        if v is not None:
            if len(v) != 8:
                raise ValueError("8 team sizes per kernel")
            for q in range(8):
                teams[8 * k + q] = int(v[q])
    prev = (ctypes.c_int * 24)()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_set_team_sizes(ctx.handle, teams, prev))
    return {"weights": list(prev[:8]), "apply": list(prev[8:16]), "fused": list(prev[16:24])}


def _nops(mask):
    return bin(mask & 0xF).count("1")


def apply_stencil(ctx, nbr, w, u, op_mask=0xF, out=None):
    wtype = GF_F32 if w.dtype == torch.float32 else GF_F64
    io = GF_F32 if u.dtype == torch.float32 else GF_F64
    o = out if out is not None else torch.empty((_nops(op_mask), nbr.n), dtype=u.dtype, device=ctx.device)
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_apply_stencil(ctx.handle, nbr.handle, wtype, _ptr(w), op_mask, io, _ptr(u), _ptr(o)))
    return o


def gfdm_weights_apply(ctx, p, nbr, u, op_mask=0xF, wtype=GF_F32, params=None, store_weights=True,
                       status=None, w_out=None, out=None):
    dt = torch.float32 if wtype == GF_F32 else torch.float64
    w = None
    if store_weights:
        w = w_out if w_out is not None else torch.empty((max(nbr.nnz, 1), 4), dtype=dt, device=ctx.device)[: nbr.nnz]
    o = out if out is not None else torch.empty((_nops(op_mask), p.n), dtype=torch.float64, device=ctx.device)
    prm = params if params is not None else ls_params()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_gfdm_weights_apply(ctx.handle, ctypes.byref(p.s), nbr.handle, ctypes.byref(prm), wtype,
                                            _ptr(w), op_mask, _ptr(u), _ptr(o), _ptr(status)))
    return w, o


def gfdm_weights_apply_noalloc(ctx, p, nbr, u, w_out, out, op_mask=0xF, params=None, status=None, wtype=None):
    """gf_gfdm_weights_apply_noalloc: as gfdm_weights_apply with caller-given
    outputs (w_out may be None: stencils of type wtype, default FP32, are
    applied and discarded) and no allocation inside the library."""
    if wtype is None:
        wtype = GF_F32 if (w_out is None or w_out.dtype == torch.float32) else GF_F64
    prm = params if params is not None else ls_params()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_gfdm_weights_apply_noalloc(ctx.handle, ctypes.byref(p.s), nbr.handle, ctypes.byref(prm),
                                                    wtype, _ptr(w_out), op_mask, _ptr(u), _ptr(out), _ptr(status)))
    return w_out, out


def poisson_assemble(ctx, p, nbr, w64, row_type, zeta=0.3):
    val = torch.empty(max(nbr.nnz, 1), dtype=torch.float64, device=ctx.device)[: nbr.nnz]
    rt = _dev_tensor(row_type, torch.int8, ctx.device)
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_poisson_assemble(ctx.handle, ctypes.byref(p.s), nbr.handle, _ptr(w64), _ptr(rt), zeta,
                                          _ptr(val)))
    return val


def solve_params(**kw):
    prm = SolveParams()
    load_library().gf_solve_params_default(ctypes.byref(prm))
    for k, v in kw.items():
        setattr(prm, k, v)
    return prm


def poisson_solve(ctx, p, nbr, w64, row_type, rhs, x0=None, params=None, raise_on_fail=True):
    """Returns (solution, stats dict)."""
    rt = _dev_tensor(row_type, torch.int8, ctx.device)
    x = torch.zeros(p.n, dtype=torch.float64, device=ctx.device) if x0 is None else x0.clone()
    prm = params if params is not None else solve_params()
    st = SolveStats()
    ctx._sync_stream()
    status = ctx.lib.gf_poisson_solve(ctx.handle, ctypes.byref(p.s), nbr.handle, _ptr(w64), _ptr(rt), _ptr(rhs),
                                      _ptr(x), ctypes.byref(prm), ctypes.byref(st))
    stats = {k: getattr(st, k) for k, _ in SolveStats._fields_}
    stats["status"] = status
    if raise_on_fail:
        ctx.check(status)
    return x, stats


def transition_3d_to_2d(ctx, p, nbr, flag, mass, rho, phi):
    dev = ctx.device
    f64 = lambda: torch.empty(p.n, dtype=torch.float64, device=dev)
    out = {k: f64() for k in ("mass", "rho", "phi", "height", "diam")}
    out["keep"] = torch.empty(p.n, dtype=torch.uint8, device=dev)
    out["owner"] = torch.empty(p.n, dtype=torch.int32, device=dev)
    fl = _dev_tensor(flag, torch.uint8, dev)
    m = _dev_tensor(mass, torch.float64, dev)
    r = _dev_tensor(rho, torch.float64, dev)
    ph = _dev_tensor(phi, torch.float64, dev)
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_transition_3d_to_2d(ctx.handle, ctypes.byref(p.s), nbr.handle, _ptr(fl), _ptr(m), _ptr(r),
                                             _ptr(ph), _ptr(out["mass"]), _ptr(out["rho"]), _ptr(out["phi"]),
                                             _ptr(out["height"]), _ptr(out["diam"]), _ptr(out["keep"]),
                                             _ptr(out["owner"])))
    return out


R_MIN, R_MAX, ALPHA_FILM = 0.2, 0.4, 8.0
_NEW_F64 = ("x", "y", "z", "h", "nx", "ny", "nz", "mass", "rho", "height", "diam")


def film_height(ctx, p, same, diam, alpha=ALPHA_FILM, out=None):
    """gf_film_height: Eq. (Height) at film particles, 0 at bulk particles."""
    dev = ctx.device
    d = _dev_tensor(diam, torch.float64, dev)
    out = torch.empty(p.n, dtype=torch.float64, device=dev) if out is None else out
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_film_height(ctx.handle, ctypes.byref(p.s), same.handle, _ptr(d), float(alpha), _ptr(out)))
    return out


def _new_buffers(dev, cap, nphi):
    c = max(int(cap), 1)
    o = {k: torch.empty(c, dtype=torch.float64, device=dev) for k in _NEW_F64}
    o["model"] = torch.empty(c, dtype=torch.int8, device=dev)
    o["kind"] = torch.empty(c, dtype=torch.int8, device=dev)
    o["src"] = torch.empty(c, dtype=torch.int32, device=dev)
    o["phi"] = torch.empty((max(nphi, 1), c), dtype=torch.float64, device=dev)
    st = NewParticles(int(cap), *[_ptr(o[k]) for k in ("x", "y", "z", "h", "model", "kind", "nx", "ny", "nz",
                                                      "mass", "rho", "phi", "height", "diam", "src")])
    return o, st


def _phi_rows(phi, n, dev):
    if phi is None:
        return None, 0
    t = _dev_tensor(phi, torch.float64, dev).reshape(-1, n).contiguous()
    return t, int(t.shape[0])


def _grow_call(ctx, call, nphi, guess_attr):
    """Runs a call that writes new particles, growing the buffers once if the
    first guess of the count was too small (the call reports the count)."""
    dev = ctx.device
    cap = getattr(ctx, guess_attr, 1024)
    for _ in range(2):
        o, st = _new_buffers(dev, cap, nphi)
        cnt = ctypes.c_int64(0)
        ctx._sync_stream()
        status = call(ctypes.byref(st), ctypes.byref(cnt))
        if status == GF_ECAPACITY and cnt.value > cap:
            cap = cnt.value + cnt.value // 4 + 64
            setattr(ctx, guess_attr, cap)
            continue
        ctx.check(status)
        k = cnt.value
        out = {key: (v[:nphi, :k] if key == "phi" else v[:k]) for key, v in o.items()}
        return out
    raise GfdmError(GF_ECAPACITY, "particle count changed between calls")


def transition_2d_to_3d(ctx, p, flag, height, h3d, mass, rho, phi=None, r_min=R_MIN, r_max=R_MAX):
    """gf_transition_2d_to_3d: dict of the new 3D particles (flag == 2 film particles)."""
    dev = ctx.device
    fl = _dev_tensor(flag, torch.uint8, dev)
    H = _dev_tensor(height, torch.float64, dev)
    h3 = _dev_tensor(h3d, torch.float64, dev)
    m = _dev_tensor(mass, torch.float64, dev)
    r = _dev_tensor(rho, torch.float64, dev)
    ph, nphi = _phi_rows(phi, p.n, dev)
    return _grow_call(ctx, lambda st, cnt: ctx.lib.gf_transition_2d_to_3d(
        ctx.handle, ctypes.byref(p.s), _ptr(fl), _ptr(H), _ptr(h3), float(r_min), float(r_max), _ptr(m), _ptr(r),
        _ptr(ph), nphi, st, cnt), nphi, "_cap_2d3d")


def buffer_flags(ctx, p, same, cross, out=None):
    """gf_buffer_flags: uint8 [n], 1 near a particle of the other model."""
    out = torch.empty(p.n, dtype=torch.uint8, device=ctx.device) if out is None else out
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_buffer_flags(ctx.handle, ctypes.byref(p.s), same.handle, cross.handle, _ptr(out)))
    return out


def buffer_zone(ctx, p, same, cross, film_h, h_other, mass, rho, phi=None, r_min=R_MIN, r_max=R_MAX):
    """gf_buffer_zone: (buffer flags, dict of ghost particle arrays)."""
    dev = ctx.device
    H = _dev_tensor(film_h, torch.float64, dev)
    ho = _dev_tensor(h_other, torch.float64, dev)
    m = _dev_tensor(mass, torch.float64, dev)
    r = _dev_tensor(rho, torch.float64, dev)
    ph, nphi = _phi_rows(phi, p.n, dev)
    flag = torch.empty(p.n, dtype=torch.uint8, device=dev)
    g = _grow_call(ctx, lambda st, cnt: ctx.lib.gf_buffer_zone(
        ctx.handle, ctypes.byref(p.s), same.handle, cross.handle, _ptr(H), _ptr(ho), float(r_min), float(r_max),
        _ptr(m), _ptr(r), _ptr(ph), nphi, st, cnt, _ptr(flag)), nphi, "_cap_ghosts")
    return flag, g


def transition_3d_to_2d_cloud(ctx, p, nbr, flag, mass, rho, phi=None, film_height=None, diam=None, h_film=None):
    """gf_transition_3d_to_2d_cloud: dict of the new cloud (deleted particles
    left out, flagged ones turned into film particles, fields mapped)."""
    dev = ctx.device
    fl = _dev_tensor(flag, torch.uint8, dev)
    m = _dev_tensor(mass, torch.float64, dev)
    r = _dev_tensor(rho, torch.float64, dev)
    fh = _dev_tensor(film_height, torch.float64, dev)
    dm = _dev_tensor(diam, torch.float64, dev)
    hf = _dev_tensor(h_film, torch.float64, dev)
    ph, nphi = _phi_rows(phi, p.n, dev)
    ctx._cap_cloud = max(getattr(ctx, "_cap_cloud", 0), p.n)   # never more particles than before
    return _grow_call(ctx, lambda st, cnt: ctx.lib.gf_transition_3d_to_2d_cloud(
        ctx.handle, ctypes.byref(p.s), nbr.handle, _ptr(fl), _ptr(m), _ptr(r), _ptr(ph), nphi, _ptr(fh), _ptr(dm),
        _ptr(hf), st, cnt), nphi, "_cap_cloud")


def extend_particles(ctx, p, ghosts):
    """Regular particles followed by the ghosts (Sec. 6.2), as one cloud."""
    cat = lambda a, b: torch.cat([a, b.to(a.dtype)])
    return Particles(ctx, cat(p.x, ghosts["x"]), cat(p.y, ghosts["y"]), cat(p.z, ghosts["z"]),
                     cat(p.h, ghosts["h"]), cat(p.model, ghosts["model"]), cat(p.kind, ghosts["kind"]),
                     cat(p.nx, ghosts["nx"]), cat(p.ny, ghosts["ny"]), cat(p.nz, ghosts["nz"]))


def apply_stencil_adjoint(ctx, nbr, w, ybar, op_mask=0xF):
    wtype = GF_F32 if w.dtype == torch.float32 else GF_F64
    ub = torch.empty(nbr.n, dtype=torch.float64, device=ctx.device)
    yb = ybar.to(torch.float64).contiguous()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_apply_stencil_adjoint(ctx.handle, nbr.handle, wtype, _ptr(w), op_mask, _ptr(yb), _ptr(ub)))
    return ub


def gfdm_weights_adjoint(ctx, p, nbr, u, ybar, op_mask=0xF, params=None, xbar=None, status=None):
    """Accumulates dL/dx into xbar [n, 3] (created as zeros if None) and returns it.
    status: the int8 statuses of the forward stencil call (rows 2 and 3 contribute nothing)."""
    xb = torch.zeros((p.n, 3), dtype=torch.float64, device=ctx.device) if xbar is None else xbar
    prm = params if params is not None else ls_params()
    uu = u.to(torch.float64).contiguous()
    yb = ybar.to(torch.float64).contiguous()
    ctx._sync_stream()
    ctx.check(ctx.lib.gf_gfdm_weights_adjoint(ctx.handle, ctypes.byref(p.s), nbr.handle, ctypes.byref(prm), op_mask,
                                              _ptr(uu), _ptr(yb), _ptr(status), _ptr(xb)))
    return xb


class StencilOp(torch.autograd.Function):
    """out = apply(weights(x, y, z), u) with the hand-written adjoints.

    forward(u, x, y, z, ctx_, p, nbr, op_mask, wtype) -> out [K, n] FP64.
    Gradients flow to u (transpose application) and to the positions
    (adjoint through the local least-squares problems, weights recomputed).
    The neighbour sets are held fixed (they change only on a set of measure
    zero, where the support weight vanishes continuously)."""

    @staticmethod
    def forward(fctx, u, x, y, z, lib_ctx, p, nbr, op_mask, wtype):
        q = p.with_positions(x.detach().to(torch.float64), y.detach().to(torch.float64),
                             z.detach().to(torch.float64))
        status = torch.empty(p.n, dtype=torch.int8, device=lib_ctx.device)
        w = gfdm_weights(lib_ctx, q, nbr, GF_BATCHED, wtype, status=status)
        uu = u.detach().to(torch.float64).contiguous()
        out = apply_stencil(lib_ctx, nbr, w, uu, op_mask)
        fctx.save_for_backward(uu, x, y, z)
        fctx.extra = (lib_ctx, p, nbr, op_mask, w, status)
        return out

    @staticmethod
    def backward(fctx, gout):
        uu, x, y, z = fctx.saved_tensors
        lib_ctx, p, nbr, op_mask, w, status = fctx.extra
        gout = gout.contiguous().to(torch.float64)
        gu = apply_stencil_adjoint(lib_ctx, nbr, w, gout, op_mask) if fctx.needs_input_grad[0] else None
        gx = gy = gz = None
        if any(fctx.needs_input_grad[1:4]):
            q = p.with_positions(x.detach().to(torch.float64), y.detach().to(torch.float64),
                                 z.detach().to(torch.float64))
            xb = gfdm_weights_adjoint(lib_ctx, q, nbr, uu, gout, op_mask, status=status)
            gx, gy, gz = xb[:, 0].contiguous(), xb[:, 1].contiguous(), xb[:, 2].contiguous()
        return gu, gx, gy, gz, None, None, None, None, None


def stencil_op(lib_ctx, p, nbr, u, x, y, z, op_mask=OP_LAP, wtype=GF_F32):
    return StencilOp.apply(u, x, y, z, lib_ctx, p, nbr, op_mask, wtype)
