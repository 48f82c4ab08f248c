"""FP64 CPU reference (oracle) for the CPR-GMRES solve.

TEST INFRASTRUCTURE ONLY: imported by `tests/`, by `__graft_entry__.smoke()`
and by the CPU-baseline leg of `bench.py`, and by nothing else.  The HIP
library never imports, links or calls anything here, and nothing here uses
the HIP library.

The arithmetic lives in plain C (`oracle/*.c`, built with gcc, no FMA
contraction); this module only marshals numpy arrays through ctypes.
Every function follows a passage of Liu & Chen, arXiv 1812.03952, cited at
its C definition.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = ["bsr.c", "decouple.c", "amg.c", "cpr.c", "ras.c", "thermal.c"]

ABF, QIMPES, FRS, FRS_ABF = 0, 1, 2, 3
SM_BJ, SM_DILU, SM_RAS, SM_RAS1 = 0, 1, 2, 3


def build() -> str:
    """Compile liboracle.so with gcc (always rebuilds)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", _SO + ".tmp"] + [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class AmgOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_row_sum", C.c_double), ("coarse_n", C.c_int),
                ("max_levels", C.c_int), ("lu_max", C.c_int), ("coarse_sweeps", C.c_int),
                ("smooth", C.c_int), ("trunc", C.c_double)]


class ThermalParams(C.Structure):
    _fields_ = [(nm, C.c_double) for nm in
                ("dx", "dy", "dz", "dt", "ctrans", "p_ref", "t_ref", "rhow_ref", "cpw", "ct1w", "ct2w", "cptw",
                 "rhoo_ref", "cpo", "ct1o", "ct2o", "cpto", "avisc_o", "bvisc_o", "cpl_o")] + \
               [("cpg", C.c_double * 5)] + \
               [(nm, C.c_double) for nm in
                ("hvr_w", "ev_w", "tcrit_w", "por_ref", "cpor", "cp_rock", "kw", "ko", "kr", "pv_btu",
                 "jmol_btu", "p_bh", "t_inj", "bbl_ft3")]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("status", C.c_int),
                ("relres", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.or_nnzb.restype = C.c_int64
        L.or_nnzb.argtypes = [C.c_int] * 3
        L.or_pattern.argtypes = [C.c_int] * 3 + [_i32p, _i32p]
        L.or_assemble.argtypes = [C.c_int] * 3 + [_f64p, C.c_double, C.c_double, _f64p, _f64p, _f64p,
                                                  C.c_double, C.c_int, _i32p, _f64p,
                                                  _i32p, _i32p, _f64p]
        L.or_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_spmv.restype = None
        L.or_transpose.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p]
        L.or_decouple.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, _f64p]
        L.or_extract_pressure.argtypes = [C.c_int64, _f64p, _f64p]
        L.or_extract_pressure.restype = None
        L.or_bj_setup.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p]
        L.or_dilu_setup.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p]
        L.or_bj_apply.argtypes = [C.c_int, _f64p, _f64p, _f64p]
        L.or_bj_apply.restype = None
        L.or_dilu_apply.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
        L.or_dilu_apply.restype = None
        L.or_amg_defaults.argtypes = [C.POINTER(AmgOpts)]
        L.or_amg_defaults.restype = None
        L.or_amg_setup.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.POINTER(AmgOpts),
                                   C.POINTER(C.c_int)]
        L.or_amg_setup.restype = C.c_void_p
        L.or_amg_nlevels.argtypes = [C.c_void_p]
        L.or_amg_level_n.argtypes = [C.c_void_p, C.c_int]
        L.or_amg_level_nnz.argtypes = [C.c_void_p, C.c_int]
        L.or_amg_level_nnz.restype = C.c_int64
        L.or_amg_coarsest_is_lu.argtypes = [C.c_void_p]
        L.or_amg_level_get.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 6
        L.or_amg_level_get.restype = None
        L.or_amg_level_p.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 3
        L.or_amg_level_p.restype = C.c_int64
        L.or_amg_vcycle.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_amg_vcycle.restype = None
        L.or_amg_free.argtypes = [C.c_void_p]
        L.or_amg_free.restype = None
        L.or_cpr_setup.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, C.c_int, C.c_int64, C.c_int,
                                   C.POINTER(AmgOpts), C.POINTER(C.c_int)]
        L.or_ras_restrict.argtypes = [C.c_int, C.c_int64, _i32p, _i32p, _f64p] + [C.c_void_p] * 3
        L.or_free.argtypes = [C.c_void_p]
        L.or_free.restype = None
        L.or_cpr_setup.restype = C.c_void_p
        L.or_cpr_apply.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_cpr_apply.restype = None
        for nm in ("or_cpr_decoupled", "or_cpr_dinv", "or_cpr_dinv2", "or_cpr_pressure"):
            getattr(L, nm).argtypes = [C.c_void_p]
            getattr(L, nm).restype = C.POINTER(C.c_double)
        L.or_cpr_amg.argtypes = [C.c_void_p]
        L.or_cpr_amg.restype = C.c_void_p
        L.or_cpr_free.argtypes = [C.c_void_p]
        L.or_cpr_free.restype = None
        L.or_gmres.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _f64p, _f64p,
                               C.c_int, C.c_double, C.c_int, C.POINTER(Info), C.c_void_p,
                               C.c_int]
        L.or_bicgstab.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _f64p, _f64p,
                                  C.c_double, C.c_int, C.POINTER(Info), C.c_void_p, C.c_int]
        L.or_rasov_setup.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int64, C.c_int, C.POINTER(C.c_int)]
        L.or_rasov_setup.restype = C.c_void_p
        L.or_rasov_apply.argtypes = [C.c_void_p, _f64p, _f64p, _f64p]
        L.or_rasov_apply.restype = None
        L.or_rasov_owned_dinv.argtypes = [C.c_void_p, _f64p]
        L.or_rasov_owned_dinv.restype = None
        L.or_rasov_ext.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_rasov_ext_dinv.argtypes = [C.c_void_p, C.c_int, _f64p]
        L.or_rasov_ext_dinv.restype = None
        L.or_rasov_free.argtypes = [C.c_void_p]
        L.or_rasov_free.restype = None
        L.or_thermal_defaults.argtypes = [C.POINTER(ThermalParams)]
        L.or_thermal_defaults.restype = None
        L.or_thermal_assemble.argtypes = [C.c_int] * 3 + [C.POINTER(ThermalParams), _f64p, _f64p, _f64p,
                                                         _f64p, _f64p, C.c_int, _i32p, _i32p, _f64p,
                                                         _i32p, _i32p, C.c_void_p, C.c_void_p]
        L.or_thermal_props.argtypes = [C.POINTER(ThermalParams), _f64p, _f64p]
        L.or_thermal_props.restype = None
        L.or_relperm.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.or_relperm.restype = C.c_double
        L.or_stone2.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_stone2.restype = C.c_double
        L.or_water_visc.argtypes = [C.c_double, C.POINTER(C.c_double)]
        L.or_water_visc.restype = C.c_double
        L.or_water_enthalpy.argtypes = [C.POINTER(ThermalParams), C.c_double, C.POINTER(C.c_double)]
        L.or_water_enthalpy.restype = C.c_double
        L.or_thermal_state.argtypes = [C.POINTER(ThermalParams), C.c_int, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.or_thermal_state.restype = None
        L.or_grad_logk.argtypes = [C.c_int] * 3 + [_f64p, C.c_double, C.c_double, _f64p, _f64p, C.c_int,
                                                   _i32p, _f64p, _f64p, _f64p, _f64p]
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    pass


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


# ---------------------------------------------------------------------------
class BSR:
    """Host block-sparse matrix: rp (n+1,), ci (nnzb,), v (nnzb, 4, 4)."""

    def __init__(self, nx, ny, nz, rp, ci, v):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n = nx * ny * nz
        self.rp = _c(rp, np.int32)
        self.ci = _c(ci, np.int32)
        self.v = _c(v, np.float64).reshape(-1, 4, 4)

    @property
    def nnzb(self):
        return self.ci.shape[0]

    def with_values(self, v):
        return BSR(self.nx, self.ny, self.nz, self.rp, self.ci, v)

    def dense(self):
        n = self.n
        D = np.zeros((4 * n, 4 * n))
        rows = np.repeat(np.arange(n), np.diff(self.rp))
        for p in range(self.nnzb):
            i, j = rows[p], self.ci[p]
            D[4 * i:4 * i + 4, 4 * j:4 * j + 4] = self.v[p]
        return D


def pattern(nx, ny, nz):
    L = lib()
    n = nx * ny * nz
    nnzb = L.or_nnzb(nx, ny, nz)
    rp = np.zeros(n + 1, np.int32)
    ci = np.zeros(nnzb, np.int32)
    _check(L.or_pattern(nx, ny, nz, rp, ci), "or_pattern")
    return rp, ci


def assemble(prob, logk=None) -> BSR:
    """Jacobian of a `synth.Problem` (optionally with another log-permeability)."""
    L = lib()
    rp, ci = pattern(prob.nx, prob.ny, prob.nz)
    v = np.zeros(ci.shape[0] * 16)
    lk = prob.logk if logk is None else logk
    _check(L.or_assemble(prob.nx, prob.ny, prob.nz, _c(lk, np.float64), prob.kvkh, prob.tscale,
                         _c(prob.Mf, np.float64).reshape(-1), _c(prob.Mb, np.float64).reshape(-1),
                         _c(prob.B, np.float64).reshape(-1), prob.dt,
                         int(prob.well_cell.shape[0]), _c(prob.well_cell, np.int32),
                         _c(prob.well_u, np.float64), rp, ci, v), "or_assemble")
    return BSR(prob.nx, prob.ny, prob.nz, rp, ci, v)


def spmv(A: BSR, x):
    y = np.zeros(4 * A.n)
    lib().or_spmv(A.n, A.rp, A.ci, A.v.reshape(-1), _c(x, np.float64), y)
    return y


def transpose(A: BSR) -> BSR:
    vt = np.zeros(A.nnzb * 16)
    _check(lib().or_transpose(A.n, A.rp, A.ci, A.v.reshape(-1), vt), "or_transpose")
    return A.with_values(vt)


def decouple(A: BSR, method=ABF):
    vt = np.zeros(A.nnzb * 16)
    dinv = np.zeros(A.n * 16)
    _check(lib().or_decouple(A.n, A.rp, A.ci, A.v.reshape(-1), method, vt, dinv), "or_decouple")
    return A.with_values(vt), dinv.reshape(-1, 4, 4)


def extract_pressure(At: BSR):
    ap = np.zeros(At.nnzb)
    lib().or_extract_pressure(At.nnzb, At.v.reshape(-1), ap)
    return ap


def bj_setup(At: BSR):
    d = np.zeros(At.n * 16)
    _check(lib().or_bj_setup(At.n, At.rp, At.ci, At.v.reshape(-1), d), "or_bj_setup")
    return d.reshape(-1, 4, 4)


def dilu_setup(At: BSR):
    d = np.zeros(At.n * 16)
    _check(lib().or_dilu_setup(At.n, At.rp, At.ci, At.v.reshape(-1), d), "or_dilu_setup")
    return d.reshape(-1, 4, 4)


def ras_restrict(At: BSR, sub=None) -> BSR:
    """The block-diagonal restriction of At to subdomains of `sub` consecutive
    cells (default nx*ny: the xy-layers); zero-overlap RAS is DILU of it."""
    L = lib()
    sub = At.nx * At.ny if sub is None else int(sub)
    prp, pci, pv = C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(L.or_ras_restrict(At.n, sub, At.rp, At.ci, At.v.reshape(-1), C.byref(prp), C.byref(pci),
                             C.byref(pv)), "or_ras_restrict")
    try:
        rp = np.ctypeslib.as_array(C.cast(prp, C.POINTER(C.c_int)), shape=(At.n + 1,)).copy()
        nk = int(rp[-1])
        ci = np.ctypeslib.as_array(C.cast(pci, C.POINTER(C.c_int)), shape=(max(nk, 1),))[:nk].copy()
        v = np.ctypeslib.as_array(C.cast(pv, C.POINTER(C.c_double)), shape=(max(nk, 1) * 16,))[:16 * nk].copy()
    finally:
        for q in (prp, pci, pv):
            L.or_free(q)
    return BSR(At.nx, At.ny, At.nz, rp, ci, v)


def bj_apply(dinv2, r):
    z = np.zeros_like(r, dtype=np.float64)
    lib().or_bj_apply(dinv2.shape[0], _c(dinv2, np.float64).reshape(-1), _c(r, np.float64), z)
    return z


def dilu_apply(At: BSR, dinv2, r):
    z = np.zeros(4 * At.n)
    lib().or_dilu_apply(At.n, At.rp, At.ci, At.v.reshape(-1), _c(dinv2, np.float64).reshape(-1),
                        _c(r, np.float64), z)
    return z


def amg_opts(**kw) -> AmgOpts:
    o = AmgOpts()
    lib().or_amg_defaults(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class AMG:
    """Aggregation AMG hierarchy on a scalar CSR matrix."""

    def __init__(self, rp, ci, a, **opts):
        L = lib()
        self._o = amg_opts(**opts)
        st = C.c_int(0)
        n = rp.shape[0] - 1
        self._h = L.or_amg_setup(n, _c(rp, np.int32), _c(ci, np.int32), _c(a, np.float64),
                                 C.byref(self._o), C.byref(st))
        self._own = True
        _check(st.value, "or_amg_setup")

    @classmethod
    def _borrow(cls, h):
        self = cls.__new__(cls)
        self._h = h
        self._own = False
        return self

    @property
    def nlevels(self):
        return lib().or_amg_nlevels(self._h)

    @property
    def coarsest_is_lu(self):
        return bool(lib().or_amg_coarsest_is_lu(self._h))

    def level(self, l):
        L = lib()
        n = L.or_amg_level_n(self._h, l)
        nnz = L.or_amg_level_nnz(self._h, l)
        rp = np.zeros(n + 1, np.int32); ci = np.zeros(max(nnz, 1), np.int32)
        a = np.zeros(max(nnz, 1)); d = np.zeros(max(n, 1)); agg = np.zeros(max(n, 1), np.int32)
        st = np.zeros(max(nnz, 1), np.int32)
        L.or_amg_level_get(self._h, l, rp.ctypes.data, ci.ctypes.data, a.ctypes.data,
                           d.ctypes.data, agg.ctypes.data, st.ctypes.data)
        return dict(n=n, nnz=nnz, rp=rp, ci=ci[:nnz], a=a[:nnz], dl1=d[:n], agg=agg[:n],
                    strong=st[:nnz])

    def prolongator(self, l):
        """The smoothed prolongator of level l as (rp, ci, v), or None when
        level l uses the piecewise-constant one (its agg array)."""
        L = lib()
        nnz = L.or_amg_level_p(self._h, l, None, None, None)
        if nnz < 0:
            return None
        n = L.or_amg_level_n(self._h, l)
        rp = np.zeros(n + 1, np.int32); ci = np.zeros(max(nnz, 1), np.int32); v = np.zeros(max(nnz, 1))
        L.or_amg_level_p(self._h, l, rp.ctypes.data, ci.ctypes.data, v.ctypes.data)
        return rp, ci[:nnz], v[:nnz]

    def vcycle(self, b):
        b = _c(b, np.float64)
        x = np.zeros_like(b)
        lib().or_amg_vcycle(self._h, b, x)
        return x

    def __del__(self):
        if getattr(self, "_own", False) and getattr(self, "_h", None):
            lib().or_amg_free(self._h)
            self._h = None


class RasOv:
    """Restricted additive Schwarz with overlap ov on a decoupled block matrix
    (subdomains of sub consecutive cells, DILU on each extension)."""

    def __init__(self, At: BSR, sub=None, ov=1):
        L = lib()
        self.A = At
        sub = At.nx * At.ny if sub is None else int(sub)
        self.sub = sub
        st = C.c_int(0)
        self._h = L.or_rasov_setup(At.n, At.rp, At.ci, At.v.reshape(-1), sub, int(ov), C.byref(st))
        if st.value != 0:
            L.or_rasov_free(self._h)
            self._h = None
            _check(st.value, "or_rasov_setup")
        self.nsub = (At.n + sub - 1) // sub

    def apply(self, r):
        z = np.zeros(4 * self.A.n)
        lib().or_rasov_apply(self._h, _c(self.A.v.reshape(-1), np.float64), _c(r, np.float64), z)
        return z

    def owned_dinv(self):
        d = np.zeros(16 * self.A.n)
        lib().or_rasov_owned_dinv(self._h, d)
        return d.reshape(-1, 4, 4)

    def ext(self, m):
        ne = lib().or_rasov_ext(self._h, m, None)
        e = np.zeros(ne, np.int32)
        lib().or_rasov_ext(self._h, m, e.ctypes.data)
        return e

    def ext_dinv(self, m):
        ne = lib().or_rasov_ext(self._h, m, None)
        d = np.zeros(16 * ne)
        lib().or_rasov_ext_dinv(self._h, m, d)
        return d.reshape(-1, 4, 4)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_rasov_free(self._h)
            self._h = None


class CPR:
    """CPR preconditioner on a block matrix: pressure then full (stages=2)
    or the three-stage CPR-FPF (stages=3)."""

    def __init__(self, A: BSR, method=ABF, smoother=SM_DILU, sub=None, stages=2, **amg_kw):
        """sub: cells per RAS subdomain (SM_RAS only); default nx*ny, the xy-layers."""
        L = lib()
        self.A = A
        self._o = amg_opts(**amg_kw)
        st = C.c_int(0)
        sub = A.nx * A.ny if sub is None else int(sub)
        self._h = L.or_cpr_setup(A.n, A.rp, A.ci, A.v.reshape(-1), method, smoother, sub, int(stages),
                                 C.byref(self._o), C.byref(st))
        if st.value != 0:
            L.or_cpr_free(self._h)
            self._h = None
            _check(st.value, "or_cpr_setup")

    def _arr(self, fn, count):
        p = getattr(lib(), fn)(self._h)
        return np.ctypeslib.as_array(p, shape=(count,)).copy()

    def decoupled(self) -> BSR:
        return self.A.with_values(self._arr("or_cpr_decoupled", 16 * self.A.nnzb))

    def dinv(self):
        return self._arr("or_cpr_dinv", 16 * self.A.n).reshape(-1, 4, 4)

    def dinv2(self):
        return self._arr("or_cpr_dinv2", 16 * self.A.n).reshape(-1, 4, 4)

    def pressure(self):
        return self._arr("or_cpr_pressure", self.A.nnzb)

    def amg(self) -> AMG:
        a = AMG._borrow(lib().or_cpr_amg(self._h))
        a._keep = self
        return a

    def apply(self, r):
        z = np.zeros(4 * self.A.n)
        lib().or_cpr_apply(self._h, _c(r, np.float64), z)
        return z

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_cpr_free(self._h)
            self._h = None


def gmres(A: BSR, b, M: CPR | None = None, x0=None, restart=30, rtol=1e-8, maxit=300,
          hist=False):
    """Flexible GMRES(restart); returns (x, info dict)."""
    x = np.zeros(4 * A.n) if x0 is None else np.array(x0, dtype=np.float64)
    info = Info()
    h = np.zeros(maxit + 1) if hist else None
    st = lib().or_gmres(A.n, A.rp, A.ci, A.v.reshape(-1), None if M is None else M._h,
                        _c(b, np.float64), x, restart, rtol, maxit, C.byref(info),
                        None if h is None else h.ctypes.data, 0 if h is None else h.shape[0])
    if st < 0:
        _check(st, "or_gmres")
    d = dict(iters=info.iters, cycles=info.cycles, status=info.status, relres=info.relres)
    if hist:
        d["hist"] = h[:info.iters]
    return x, d


def bicgstab(A: BSR, b, M: CPR | None = None, x0=None, rtol=1e-8, maxit=300, hist=False):
    """Right-preconditioned BiCGSTAB; returns (x, info dict)."""
    x = np.zeros(4 * A.n) if x0 is None else np.array(x0, dtype=np.float64)
    info = Info()
    h = np.zeros(maxit + 1) if hist else None
    st = lib().or_bicgstab(A.n, A.rp, A.ci, A.v.reshape(-1), None if M is None else M._h,
                           _c(b, np.float64), x, rtol, maxit, C.byref(info),
                           None if h is None else h.ctypes.data, 0 if h is None else h.shape[0])
    if st < 0:
        _check(st, "or_bicgstab")
    d = dict(iters=info.iters, cycles=info.cycles, status=info.status, relres=info.relres)
    if hist:
        d["hist"] = h[:info.iters]
    return x, d


def grad_logk(prob, lam, x, logk=None):
    g = np.zeros(prob.n)
    lk = prob.logk if logk is None else logk
    _check(lib().or_grad_logk(prob.nx, prob.ny, prob.nz, _c(lk, np.float64), prob.kvkh, prob.tscale,
                              _c(prob.Mf, np.float64).reshape(-1),
                              _c(prob.Mb, np.float64).reshape(-1),
                              int(prob.well_cell.shape[0]), _c(prob.well_cell, np.int32),
                              _c(prob.well_u, np.float64), _c(lam, np.float64),
                              _c(x, np.float64), g), "or_grad_logk")
    return g


# ---------------------------------------------------------------------------
# thermal model subset (thermal.c)

def thermal_params(**kw) -> ThermalParams:
    q = ThermalParams()
    lib().or_thermal_defaults(C.byref(q))
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def thermal_state(q: ThermalParams, p, sw, so, t):
    """Unknowns (p, N_w, N_o, T) per cell from p, S_w, S_o, T."""
    n = len(p)
    u = np.zeros(4 * n)
    lib().or_thermal_state(C.byref(q), n, _c(p, np.float64), _c(sw, np.float64), _c(so, np.float64),
                           _c(t, np.float64), u)
    return u


def thermal_assemble(tp, q: ThermalParams, u, uold, jacobian=True):
    """Residual (4n) and, if asked, the Jacobian as a BSR on the 7-point
    pattern, for the thermal problem tp (synth.ThermalProblem)."""
    n = tp.nx * tp.ny * tp.nz
    rp, ci = pattern(tp.nx, tp.ny, tp.nz)
    res = np.zeros(4 * n)
    vals = np.zeros(16 * int(rp[-1])) if jacobian else None
    st = lib().or_thermal_assemble(tp.nx, tp.ny, tp.nz, C.byref(q), _c(tp.kx, np.float64), _c(tp.ky, np.float64),
                                   _c(tp.kz, np.float64), _c(u, np.float64), _c(uold, np.float64),
                                   int(tp.wcell.shape[0]), _c(tp.wcell, np.int32), _c(tp.wkind, np.int32),
                                   _c(tp.wval, np.float64), rp, ci,
                                   None if vals is None else vals.ctypes.data, res.ctypes.data)
    _check(st, "or_thermal_assemble")
    J = None if vals is None else BSR(tp.nx, tp.ny, tp.nz, rp, ci, vals.reshape(-1, 4, 4))
    return res, J


def thermal_props(q: ThermalParams, u4):
    out = np.zeros(9)
    lib().or_thermal_props(C.byref(q), _c(u4, np.float64), out)
    return dict(zip(("sw", "so", "lw", "lo", "hw", "ho", "e", "kt", "vol"), out))


def relperm(which, s):
    d = C.c_double(0.0)
    v = lib().or_relperm(which, float(s), C.byref(d))
    return v, d.value


def stone2(sw, sg):
    a, b = C.c_double(0.0), C.c_double(0.0)
    v = lib().or_stone2(float(sw), float(sg), C.byref(a), C.byref(b))
    return v, a.value, b.value


def water_visc(t):
    d = C.c_double(0.0)
    return lib().or_water_visc(float(t), C.byref(d)), d.value


def water_enthalpy(q, t):
    d = C.c_double(0.0)
    return lib().or_water_enthalpy(C.byref(q), float(t), C.byref(d)), d.value
