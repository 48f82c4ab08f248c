"""GPU parity of rs_bicgstab_solve (right-preconditioned BiCGSTAB with CPR)
against the oracle's BiCGSTAB: iterates after k iterations, iteration
counts, converged solutions, the half-iteration case A = 4 I, status paths
and bitwise repeatability."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, relerr, upload
from paper_1812_03952_amd import rsolve as rs

pytestmark = pytest.mark.gpu


def _setup(A, prec=64, smoother=rs.SM_RAS, **kw):
    B = upload(A)
    return B, rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=smoother, **kw))


@pytest.mark.parametrize("smoother", [rs.SM_BJ, rs.SM_DILU, rs.SM_RAS])
def test_iterates_match_oracle(smoother):
    """x after k = 1..3 iterations (rtol 0) against the oracle's BiCGSTAB
    with the oracle's CPR, FP64 throughout."""
    dims = (12, 10, 6)
    p = synth.make(*dims, seed=53, sigma=2.0, shale=0.1,
                   wells=synth.wells_vertical_pair(*dims, (0, 0), (dims[0] - 1, dims[1] - 1)))
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=smoother, coarse_n=20)
    B, M = _setup(A, 64, smoother, coarse_n=20)
    for k in range(1, 4):
        xo, io = oracle.bicgstab(A, p.b, Mo, rtol=0.0, maxit=k)
        x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
        info = rs.bicgstab_solve(B, M, dev(p.b), x, rs.bicgstab_opts(rtol=0.0, maxit=k))
        assert info["return"] == 1 and info["iters"] == k == io["iters"]
        assert relerr(x.cpu().numpy(), xo) <= 1e-10, k


@pytest.mark.parametrize("cfg", [0])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("smoother", [rs.SM_DILU, rs.SM_RAS])
def test_bicgstab_solution(cfg, prec, smoother):
    """Converged solves against the oracle solved to 1e-13; in FP64 the
    iteration count equals the oracle's at the same rtol."""
    p = synth.config(cfg)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=smoother)
    xo, _ = oracle.bicgstab(A, p.b, Mo, rtol=1e-13, maxit=300)
    B, M = _setup(A, prec, smoother)
    x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    info = rs.bicgstab_solve(B, M, dev(p.b), x, rs.bicgstab_opts(rtol=1e-8))
    xg = x.cpu().numpy()
    true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / np.linalg.norm(p.b)
    assert info["return"] == 0 and true <= 1e-8 and abs(true - info["relres"]) <= 1e-12
    assert relerr(xg, xo) <= 1e-5
    if prec == 64:
        _, io8 = oracle.bicgstab(A, p.b, Mo, rtol=1e-8)
        assert info["iters"] == io8["iters"]


def test_multiple_of_identity_one_half_iteration():
    p = synth.small(3, 2, 2, seed=5)
    A = oracle.assemble(p)
    v = np.zeros_like(A.v)
    for i in range(A.n):
        for q in range(A.rp[i], A.rp[i + 1]):
            if A.ci[q] == i:
                v[q] = 4.0 * np.eye(4)
    A4 = A.with_values(v)
    B, M = _setup(A4, 64, rs.SM_BJ)
    x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    info = rs.bicgstab_solve(B, M, dev(p.b), x, rs.bicgstab_opts(rtol=1e-14))
    assert info["return"] == 0 and info["iters"] == 1 and info["cycles"] == 1
    assert np.array_equal(x.cpu().numpy(), p.b / 4.0)


def test_bicgstab_status_and_repeatability():
    p = synth.config(0)
    A = oracle.assemble(p)
    B, M = _setup(A, 32)
    b = dev(p.b)
    xs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        rs.bicgstab_solve(B, M, b, x)
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
    x = torch.zeros_like(b)
    info = rs.bicgstab_solve(B, M, b, x, rs.bicgstab_opts(maxit=1, rtol=1e-15))
    assert info["return"] == 1 and info["iters"] == 1
    bb = b.clone(); bb[5] = float("nan")
    info = rs.bicgstab_solve(B, M, bb, torch.zeros_like(b), check=False)
    assert info["return"] == -5
    x = torch.ones_like(b)
    info = rs.bicgstab_solve(B, M, torch.zeros_like(b), x)
    assert info["return"] == 0 and info["iters"] == 0 and not x.any()
    # a start at the converged solution needs no iteration
    x = torch.tensor(xs[0], device="cuda")
    info = rs.bicgstab_solve(B, M, b, x)
    assert info["return"] == 0 and info["iters"] == 0
    # GMRES and BiCGSTAB reach the same solution
    xg = torch.zeros_like(b)
    rs.gmres_solve(B, M, b, xg, rs.gmres_opts(rtol=1e-10))
    xb = torch.zeros_like(b)
    rs.bicgstab_solve(B, M, b, xb, rs.bicgstab_opts(rtol=1e-10))
    assert relerr(xb.cpu().numpy(), xg.cpu().numpy()) <= 1e-6
