"""The C-ABI library loads and exports every function include/rsolve.h declares
(no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "rsolve.h")
SO = os.path.join(ROOT, "paper_1812_03952_amd", "librsolve.so")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = _declared()
    for f in ("rs_bsr_create", "rs_decouple", "rs_cpr_setup", "rs_gmres_solve", "rs_adjoint_solve"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(SO), reason="librsolve.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(SO)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(SO), reason="librsolve.so not built")
def test_host_only_calls():
    lib = ctypes.CDLL(SO)
    lib.rs_status_string.restype = ctypes.c_char_p
    assert lib.rs_status_string(0) == b"ok"
    assert b"singular" in lib.rs_status_string(-4)


@pytest.mark.skipif(not os.path.exists(SO), reason="librsolve.so not built")
def test_option_names_are_checked():
    """The binding's option structs take only the fields the header declares
    (a misspelt name is an error, not a silently ignored attribute)."""
    from paper_1812_03952_amd import rsolve as rs
    assert rs.cpr_opts(smoother=rs.SM_RAS, theta=0.25).theta == 0.25
    assert rs.gmres_opts(restart=5).restart == 5
    for make, bad in ((rs.cpr_opts, "smooter"), (rs.gmres_opts, "restrat"), (rs.bicgstab_opts, "rtl")):
        with pytest.raises(TypeError):
            make(**{bad: 1})


@pytest.mark.skipif(not os.path.exists(SO), reason="librsolve.so not built")
@pytest.mark.parametrize("dims", [(1 << 21, 1 << 21, 1 << 21), (1 << 16, 1 << 16, 1), (1024, 1024, 1024),
                                  (0, 4, 4), (4, -1, 4)])
def test_grid_extents_rejected_before_any_device_call(dims):
    """Grids over 2^30 cells (whose cell count would overflow int64 or the
    int32 indices) or with an empty extent are refused on the host, before
    any pointer is used or any kernel launched (dummy pointers here)."""
    lib = ctypes.CDLL(SO)
    nx, ny, nz = dims
    dummy = ctypes.c_void_p(256)
    out = ctypes.c_void_p()
    lib.rs_bsr_create.argtypes = [ctypes.c_int] * 4 + [ctypes.c_int64] + [ctypes.c_void_p] * 5
    assert lib.rs_bsr_create(nx, ny, nz, 4, 7, dummy, dummy, dummy, None, ctypes.byref(out)) == -1
    lib.rs_pattern.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 4
    assert lib.rs_pattern(nx, ny, nz, dummy, dummy, None, None) == -1
