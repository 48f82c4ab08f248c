"""ctypes binding of librsolve.so (C-ABI in include/rsolve.h).

Argument marshalling only: device buffers are torch tensors on the current
HIP device, streams are torch streams, and every computation runs in the
library's HIP kernels.  If the shared library is missing this module raises
at load time; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsolve.so")

RS_OK, RS_NOT_CONVERGED = 0, 1
ABF, QIMPES, FRS, FRS_ABF = 0, 1, 2, 3
SM_BJ, SM_DILU, SM_RAS, SM_RAS1 = 0, 1, 2, 3


class RsError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class CprOpts(C.Structure):
    _fields_ = [("smoother", C.c_int), ("theta", C.c_double), ("max_row_sum", C.c_double),
                ("coarse_n", C.c_int), ("max_levels", C.c_int), ("lu_max", C.c_int),
                ("coarse_sweeps", C.c_int), ("stages", C.c_int), ("smooth", C.c_int), ("trunc", C.c_double)]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("rtol", C.c_double), ("maxit", C.c_int), ("zero_guess", C.c_int)]


class BicgstabOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int), ("zero_guess", C.c_int)]


class ThermalParams(C.Structure):
    """rs_thermal_params (rsolve.h)."""
    _fields_ = [(nm, C.c_double) for nm in
                ("dx", "dy", "dz", "dt", "ctrans", "p_ref", "t_ref", "rhow_ref", "cpw", "ct1w", "ct2w", "cptw",
                 "rhoo_ref", "cpo", "ct1o", "ct2o", "cpto", "avisc_o", "bvisc_o", "cpl_o")] + \
               [("cpg", C.c_double * 5)] + \
               [(nm, C.c_double) for nm in
                ("hvr_w", "ev_w", "tcrit_w", "por_ref", "cpor", "cp_rock", "kw", "ko", "kr", "pv_btu",
                 "jmol_btu", "p_bh", "t_inj", "bbl_ft3")]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("status", C.c_int),
                ("relres", C.c_double), ("est_relres", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp, _i, _i64, _d = C.c_void_p, C.c_int, C.c_int64, C.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(or python paper_1812_03952_amd/build.py) first")
        L = C.CDLL(LIB_PATH)
        sig = {
            "rs_cpr_opts_default": (None, [C.POINTER(CprOpts)]),
            "rs_gmres_opts_default": (None, [C.POINTER(GmresOpts)]),
            "rs_bicgstab_opts_default": (None, [C.POINTER(BicgstabOpts)]),
            "rs_status_string": (C.c_char_p, [_i]),
            "rs_bsr_create": (_i, [_i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
            "rs_bsr_update": (_i, [_vp, _vp, _vp]),
            "rs_decouple": (_i, [_vp, _i, _i, _vp, C.POINTER(_vp)]),
            "rs_bsr_update_decouple": (_i, [_vp, _vp, _i, _i, _vp, C.POINTER(_vp)]),
            "rs_bsr_attach_decouple": (_i, [_vp, _vp, _i, _i, _vp, C.POINTER(_vp)]),
            "rs_cpr_setup": (_i, [_vp, _vp, C.POINTER(CprOpts), _vp, C.POINTER(_vp)]),
            "rs_gmres_solve": (_i, [_vp, _vp, _vp, _vp, C.POINTER(GmresOpts), C.POINTER(SolveInfo), _vp]),
            "rs_bicgstab_solve": (_i, [_vp, _vp, _vp, _vp, C.POINTER(BicgstabOpts), C.POINTER(SolveInfo), _vp]),
            "rs_adjoint_solve": (_i, [_vp, _i, _i, C.POINTER(CprOpts), _vp, _vp, C.POINTER(GmresOpts),
                                      C.POINTER(SolveInfo), _vp]),
            "rs_bsr_destroy": (None, [_vp]),
            "rs_dcpl_destroy": (None, [_vp]),
            "rs_cpr_destroy": (None, [_vp]),
            "rs_spmv": (_i, [_vp, _vp, _vp, _vp]),
            "rs_cpr_apply": (_i, [_vp, _vp, _vp, _vp]),
            "rs_assemble": (_i, [_i, _i, _i, _vp, _d, _d, _vp, _vp, _vp, _d, _i, _vp, _vp, _vp, _vp, _vp]),
            "rs_pattern": (_i, [_i, _i, _i, _vp, _vp, C.POINTER(_i64), _vp]),
            "rs_grad_vals": (_i, [_vp, _vp, _vp, _vp, _vp]),
            "rs_grad_logk": (_i, [_i, _i, _i, _vp, _d, _d, _vp, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
            "rs_dcpl_get": (_i, [_vp, _vp, _vp]),
            "rs_cpr_nlevels": (_i, [_vp]),
            "rs_cpr_level": (_i, [_vp, _i, C.POINTER(_i), C.POINTER(_i64), _vp, _vp, _vp, _vp, _vp]),
            "rs_cpr_level_p": (_i, [_vp, _i, C.POINTER(_i64), _vp, _vp, _vp]),
            "rs_cpr_smoother_get": (_i, [_vp, _vp]),
            "rs_cpr_vcycle": (_i, [_vp, _vp, _vp, _vp]),
            "rs_dense_inverse": (_i, [_i, _vp, _vp, _vp]),
            "rs_dense_inverse_noalloc": (_i, [_i, _vp, _vp, _vp]),
            "rs_thermal_params_default": (None, [C.POINTER(ThermalParams)]),
            "rs_thermal_assemble": (_i, [_i, _i, _i, C.POINTER(ThermalParams), _vp, _vp, _vp, _vp, _vp, _i, _vp,
                                         _vp, _vp, _vp, _vp, _vp]),
            "rs_thermal_state": (_i, [_i64, C.POINTER(ThermalParams), _vp, _vp, _vp, _vp, _vp, _vp]),
            "rs_pool_trim": (None, []),
            "rs_pool_usage": (None, [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def pool_trim():
    """Return the library's cached device blocks to the HIP runtime."""
    lib().rs_pool_trim()


def pool_usage() -> tuple[int, int]:
    """(bytes held by live handles, bytes cached for reuse)."""
    live, cached = C.c_size_t(0), C.c_size_t(0)
    lib().rs_pool_usage(C.byref(live), C.byref(cached))
    return live.value, cached.value


def status_string(st: int) -> str:
    return lib().rs_status_string(st).decode()


def _check(st, what, ok=(RS_OK,)):
    if st not in ok:
        raise RsError(st, what)
    return st


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor, dtype, n=None):
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"contiguous {dtype} tensor expected, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _set_fields(o, kw):
    # a misspelt option would otherwise become a plain Python attribute that
    # the library never sees
    names = {f for f, _ in type(o)._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"{type(o).__name__} has no option {k!r} (options: {', '.join(sorted(names))})")
        setattr(o, k, v)
    return o


def cpr_opts(**kw) -> CprOpts:
    o = CprOpts()
    lib().rs_cpr_opts_default(C.byref(o))
    return _set_fields(o, kw)


def gmres_opts(**kw) -> GmresOpts:
    o = GmresOpts()
    lib().rs_gmres_opts_default(C.byref(o))
    return _set_fields(o, kw)


def bicgstab_opts(**kw) -> BicgstabOpts:
    o = BicgstabOpts()
    lib().rs_bicgstab_opts_default(C.byref(o))
    return _set_fields(o, kw)


# ---------------------------------------------------------------------------
class Bsr:
    """Handle of a block matrix held by the library (rs_bsr)."""

    def __init__(self, h, nx, ny, nz, nnzb):
        self.h, self.nx, self.ny, self.nz, self.nnzb = h, nx, ny, nz, nnzb
        self.n = nx * ny * nz
        self.attached = []          # value tensors A may refer to, kept alive here

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rs_bsr_destroy(self.h)
            self.h = None


class Dcpl:
    def __init__(self, h, A, method, prec):
        self.h, self.A, self.method, self.prec = h, A, method, prec

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rs_dcpl_destroy(self.h)
            self.h = None


class Cpr:
    def __init__(self, h, A, D):
        self.h, self.A, self.D = h, A, D

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rs_cpr_destroy(self.h)
            self.h = None


def pattern(nx, ny, nz, device=None, stream=None):
    """7-point block pattern (row_ptr, col_idx) as int32 device tensors."""
    n = nx * ny * nz
    faces = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    nnzb = n + 2 * faces
    rp = torch.empty(n + 1, dtype=torch.int32, device=device or "cuda")
    ci = torch.empty(nnzb, dtype=torch.int32, device=device or "cuda")
    out = C.c_int64(0)
    _check(lib().rs_pattern(nx, ny, nz, _ptr(rp, torch.int32), _ptr(ci, torch.int32), C.byref(out),
                            _stream(stream)), "rs_pattern")
    return rp, ci


def bsr_create(nx, ny, nz, row_ptr, col_idx, vals, stream=None) -> Bsr:
    h = C.c_void_p()
    nnzb = col_idx.numel()
    _check(lib().rs_bsr_create(nx, ny, nz, 4, nnzb, _ptr(row_ptr, torch.int32),
                               _ptr(col_idx, torch.int32), _ptr(vals, torch.float64, 16 * nnzb),
                               _stream(stream), C.byref(h)), "rs_bsr_create")
    return Bsr(h, nx, ny, nz, nnzb)


# Statuses after which the library has taken the new values (A holds or
# refers to them); after any other error A may still refer to older ones.
_TAKEN = (0, -4, -5)


def bsr_update(A: Bsr, vals, stream=None):
    st = lib().rs_bsr_update(A.h, _ptr(vals, torch.float64, 16 * A.nnzb), _stream(stream))
    if st in _TAKEN:
        A.attached = []
    _check(st, "rs_bsr_update")


def bsr_update_decouple(A: Bsr, vals, method=ABF, prec=64, stream=None) -> Dcpl:
    """bsr_update(A, vals) and decouple(A, method, prec) in one pass."""
    h = C.c_void_p()
    st = lib().rs_bsr_update_decouple(A.h, _ptr(vals, torch.float64, 16 * A.nnzb), method, prec,
                                      _stream(stream), C.byref(h))
    if st in _TAKEN:
        A.attached = []
    _check(st, "rs_bsr_update_decouple")
    return Dcpl(h, A, method, prec)


def bsr_attach_decouple(A: Bsr, vals, method=ABF, prec=64, stream=None) -> Dcpl:
    """As bsr_update_decouple, but A refers to `vals` in place (no copy).
    A keeps the tensor alive until its next update or attach; the caller
    must not change it meanwhile."""
    h = C.c_void_p()
    st = lib().rs_bsr_attach_decouple(A.h, _ptr(vals, torch.float64, 16 * A.nnzb), method, prec,
                                      _stream(stream), C.byref(h))
    A.attached = [vals] if st in _TAKEN else A.attached + [vals]
    _check(st, "rs_bsr_attach_decouple")
    return Dcpl(h, A, method, prec)


def decouple(A: Bsr, method=ABF, prec=64, stream=None) -> Dcpl:
    h = C.c_void_p()
    _check(lib().rs_decouple(A.h, method, prec, _stream(stream), C.byref(h)), "rs_decouple")
    return Dcpl(h, A, method, prec)


def cpr_setup(A: Bsr, D: Dcpl, opts: CprOpts | None = None, stream=None) -> Cpr:
    h = C.c_void_p()
    _check(lib().rs_cpr_setup(A.h, D.h, None if opts is None else C.byref(opts), _stream(stream),
                              C.byref(h)), "rs_cpr_setup")
    return Cpr(h, A, D)


def gmres_solve(A: Bsr, M: Cpr, b, x, opts: GmresOpts | None = None, stream=None, check=True) -> dict:
    info = SolveInfo()
    N = 4 * A.n
    st = lib().rs_gmres_solve(A.h, M.h, _ptr(b, torch.float64, N), _ptr(x, torch.float64, N),
                              None if opts is None else C.byref(opts), C.byref(info), _stream(stream))
    if check:
        _check(st, "rs_gmres_solve", ok=(RS_OK, RS_NOT_CONVERGED))
    d = info.as_dict()
    d["return"] = st
    return d


def bicgstab_solve(A: Bsr, M: Cpr, b, x, opts: BicgstabOpts | None = None, stream=None, check=True) -> dict:
    info = SolveInfo()
    N = 4 * A.n
    st = lib().rs_bicgstab_solve(A.h, M.h, _ptr(b, torch.float64, N), _ptr(x, torch.float64, N),
                                 None if opts is None else C.byref(opts), C.byref(info), _stream(stream))
    if check:
        _check(st, "rs_bicgstab_solve", ok=(RS_OK, RS_NOT_CONVERGED))
    d = info.as_dict()
    d["return"] = st
    return d


def adjoint_solve(A: Bsr, w, lam, method=ABF, prec=64, cpr: CprOpts | None = None,
                  opts: GmresOpts | None = None, stream=None) -> dict:
    info = SolveInfo()
    N = 4 * A.n
    st = lib().rs_adjoint_solve(A.h, method, prec, None if cpr is None else C.byref(cpr),
                                _ptr(w, torch.float64, N), _ptr(lam, torch.float64, N),
                                None if opts is None else C.byref(opts), C.byref(info), _stream(stream))
    _check(st, "rs_adjoint_solve", ok=(RS_OK, RS_NOT_CONVERGED))
    d = info.as_dict()
    d["return"] = st
    return d


def spmv(A: Bsr, x, y, stream=None):
    N = 4 * A.n
    _check(lib().rs_spmv(A.h, _ptr(x, torch.float64, N), _ptr(y, torch.float64, N), _stream(stream)), "rs_spmv")


def cpr_apply(M: Cpr, r, z, stream=None):
    N = 4 * M.A.n
    _check(lib().rs_cpr_apply(M.h, _ptr(r, torch.float64, N), _ptr(z, torch.float64, N), _stream(stream)),
           "rs_cpr_apply")


def cpr_vcycle(M: Cpr, b, x, stream=None):
    _check(lib().rs_cpr_vcycle(M.h, _ptr(b, torch.float64, M.A.n), _ptr(x, torch.float64, M.A.n),
                               _stream(stream)), "rs_cpr_vcycle")


def dense_inverse(a, inv, stream=None):
    """inv = a^{-1} for a dense n x n FP64 device matrix (row-major), by the
    AMG coarsest-level kernels."""
    n = a.shape[0]
    _check(lib().rs_dense_inverse(n, _ptr(a, torch.float64, n * n), _ptr(inv, torch.float64, n * n),
                                  _stream(stream)), "rs_dense_inverse")


DENSE_NOALLOC_MAX = 1024


def dense_inverse_noalloc(a, inv, stream=None):
    """dense_inverse without device allocation: the library's static scratch
    array (n <= DENSE_NOALLOC_MAX; calls overlapping on one GPU race)."""
    n = a.shape[0]
    _check(lib().rs_dense_inverse_noalloc(n, _ptr(a, torch.float64, n * n), _ptr(inv, torch.float64, n * n),
                                          _stream(stream)), "rs_dense_inverse_noalloc")


def assemble(nx, ny, nz, logk, kvkh, tscale, Mf, Mb, B, dt, wcell, wu, row_ptr, vals, stream=None):
    n = nx * ny * nz
    nw = wcell.numel()
    _check(lib().rs_assemble(nx, ny, nz, _ptr(logk, torch.float64, n), float(kvkh), float(tscale),
                             _ptr(Mf, torch.float64, 48 * n), _ptr(Mb, torch.float64, 48 * n),
                             _ptr(B, torch.float64, 16 * n), float(dt), nw,
                             _ptr(wcell, torch.int32) if nw else None, _ptr(wu, torch.float64) if nw else None,
                             _ptr(row_ptr, torch.int32, n + 1), _ptr(vals, torch.float64), _stream(stream)),
           "rs_assemble")


def grad_vals(A: Bsr, lam, x, G, stream=None):
    N = 4 * A.n
    _check(lib().rs_grad_vals(A.h, _ptr(lam, torch.float64, N), _ptr(x, torch.float64, N),
                              _ptr(G, torch.float64, 16 * A.nnzb), _stream(stream)), "rs_grad_vals")


def grad_logk(nx, ny, nz, logk, kvkh, tscale, Mf, Mb, wcell, wu, row_ptr, G, g, stream=None):
    n = nx * ny * nz
    nw = wcell.numel()
    _check(lib().rs_grad_logk(nx, ny, nz, _ptr(logk, torch.float64, n), float(kvkh), float(tscale),
                              _ptr(Mf, torch.float64, 48 * n), _ptr(Mb, torch.float64, 48 * n), nw,
                              _ptr(wcell, torch.int32) if nw else None, _ptr(wu, torch.float64) if nw else None,
                              _ptr(row_ptr, torch.int32, n + 1), _ptr(G, torch.float64),
                              _ptr(g, torch.float64, n), _stream(stream)), "rs_grad_logk")


# ---- the system of one Newton step of the thermal model subset -----------------
def thermal_params(**kw) -> ThermalParams:
    q = ThermalParams()
    lib().rs_thermal_params_default(C.byref(q))
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def thermal_assemble(nx, ny, nz, q: ThermalParams, kx, ky, kz, u, uold, wcell, wkind, wval, vals=None, res=None,
                     stream=None):
    """Jacobian values (caller layout, 16*nnzb) into `vals` and residual (4n)
    into `res` (either may be None, not both)."""
    n = nx * ny * nz
    nw = wcell.numel()
    _check(lib().rs_thermal_assemble(nx, ny, nz, C.byref(q), _ptr(kx, torch.float64, n), _ptr(ky, torch.float64, n),
                                     _ptr(kz, torch.float64, n), _ptr(u, torch.float64, 4 * n),
                                     _ptr(uold, torch.float64, 4 * n), nw,
                                     _ptr(wcell, torch.int32) if nw else None, _ptr(wkind, torch.int32) if nw else None,
                                     _ptr(wval, torch.float64) if nw else None,
                                     None if vals is None else _ptr(vals, torch.float64),
                                     None if res is None else _ptr(res, torch.float64, 4 * n), _stream(stream)),
           "rs_thermal_assemble")


def thermal_state(q: ThermalParams, p, sw, so, t, u, stream=None):
    n = p.numel()
    _check(lib().rs_thermal_state(n, C.byref(q), _ptr(p, torch.float64, n), _ptr(sw, torch.float64, n),
                                  _ptr(so, torch.float64, n), _ptr(t, torch.float64, n),
                                  _ptr(u, torch.float64, 4 * n), _stream(stream)), "rs_thermal_state")


# ---- inspection ---------------------------------------------------------------
def dcpl_get(D: Dcpl):
    A = D.A
    vals = np.zeros(16 * A.nnzb)
    dinv = np.zeros(16 * A.n)
    _check(lib().rs_dcpl_get(D.h, vals.ctypes.data, dinv.ctypes.data), "rs_dcpl_get")
    return vals.reshape(-1, 4, 4), dinv.reshape(-1, 4, 4)


def cpr_nlevels(M: Cpr) -> int:
    return lib().rs_cpr_nlevels(M.h)


def cpr_level(M: Cpr, l: int) -> dict:
    n, nnz = C.c_int(0), C.c_int64(0)
    L = lib()
    _check(L.rs_cpr_level(M.h, l, C.byref(n), C.byref(nnz), None, None, None, None, None), "rs_cpr_level")
    n, nnz = n.value, nnz.value
    rp = np.zeros(n + 1, np.int32); ci = np.zeros(max(nnz, 1), np.int32)
    a = np.zeros(max(nnz, 1)); d = np.zeros(max(n, 1)); agg = np.zeros(max(n, 1), np.int32)
    _check(L.rs_cpr_level(M.h, l, None, None, rp.ctypes.data, ci.ctypes.data, a.ctypes.data,
                          d.ctypes.data, agg.ctypes.data), "rs_cpr_level")
    return dict(n=n, nnz=nnz, rp=rp, ci=ci[:nnz], a=a[:nnz], dl1=d[:n], agg=agg[:n])


def cpr_level_p(M: Cpr, l: int):
    """Smoothed prolongator of level l as (rp, ci, v) host arrays."""
    L = lib()
    nnz = C.c_int64(0)
    _check(L.rs_cpr_level_p(M.h, l, C.byref(nnz), None, None, None), "rs_cpr_level_p")
    n = cpr_level(M, l)["n"]
    rp = np.zeros(n + 1, np.int32); ci = np.zeros(max(nnz.value, 1), np.int32); v = np.zeros(max(nnz.value, 1))
    _check(L.rs_cpr_level_p(M.h, l, C.byref(nnz), rp.ctypes.data, ci.ctypes.data, v.ctypes.data), "rs_cpr_level_p")
    return rp, ci[:nnz.value], v[:nnz.value]


def cpr_smoother_get(M: Cpr):
    d = np.zeros(16 * M.A.n)
    _check(lib().rs_cpr_smoother_get(M.h, d.ctypes.data), "rs_cpr_smoother_get")
    return d.reshape(-1, 4, 4)


# ---- convenience: a synthetic problem resident on the device ------------------
class DeviceProblem:
    """Seeded draws of a synthetic problem copied to the device, with its
    pattern and the Jacobian assembled by the library (rs_assemble)."""

    def __init__(self, prob, device="cuda", stream=None):
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.nx, self.ny, self.nz = prob.nx, prob.ny, prob.nz
        self.n = prob.n
        self.kvkh, self.tscale, self.dt = prob.kvkh, prob.tscale, prob.dt
        self.logk = torch.as_tensor(prob.logk, **f64)
        self.Mf = torch.as_tensor(prob.Mf.reshape(-1), **f64)
        self.Mb = torch.as_tensor(prob.Mb.reshape(-1), **f64)
        self.B = torch.as_tensor(prob.B.reshape(-1), **f64)
        self.wcell = torch.as_tensor(prob.well_cell, dtype=torch.int32, device=dev)
        self.wu = torch.as_tensor(prob.well_u, **f64)
        self.b = torch.as_tensor(prob.b, **f64)
        self.w = torch.as_tensor(prob.w, **f64)
        self.row_ptr, self.col_idx = pattern(self.nx, self.ny, self.nz, device=dev, stream=stream)
        self.vals = torch.empty(16 * self.col_idx.numel(), **f64)
        self.assemble(self.logk, self.vals, stream)

    def assemble(self, logk, vals, stream=None):
        assemble(self.nx, self.ny, self.nz, logk, self.kvkh, self.tscale, self.Mf, self.Mb, self.B,
                 self.dt, self.wcell, self.wu, self.row_ptr, vals, stream)
        return vals

    def bsr(self, stream=None) -> Bsr:
        return bsr_create(self.nx, self.ny, self.nz, self.row_ptr, self.col_idx, self.vals, stream)
