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
