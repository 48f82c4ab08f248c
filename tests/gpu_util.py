"""Helpers for the GPU parity tests: move an oracle-assembled problem to the
device and build the library's handles on it."""
import numpy as np
import torch

import oracle
from paper_1812_03952_amd import rsolve as rs


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def upload(A: "oracle.BSR"):
    rp = dev(A.rp, torch.int32)
    ci = dev(A.ci, torch.int32)
    v = dev(A.v.reshape(-1))
    return rs.bsr_create(A.nx, A.ny, A.nz, rp, ci, v)


def relerr(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def maxrel(a, b):
    """Largest entry error relative to the largest reference entry: catches a
    local error that the 2-norm of the whole vector would average away."""
    a = np.asarray(a); b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def assert_close(got, ref, tol):
    """2-norm relative error within tol and every entry within 10 tol of the
    reference's largest entry."""
    e2, emax = relerr(got, ref), maxrel(got, ref)
    assert e2 <= tol and emax <= 10 * tol, (e2, emax, tol)
