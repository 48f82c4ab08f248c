"""Second stage as RAS with overlap 1 (each xy-layer extended by its two
neighbour layers, block ILU(0) of the extension, restricted prolongation)
against the oracle's overlapping RAS, through the C-ABI.

The owned cells' factors are compared bitwise in FP64 (the device forms the
Schur term of the layer below with the oracle's operations in its order);
the CPR apply is compared in norm and element by element (FP64 1e-10 and
1e-9 of the largest entry, FP32 1e-4 and 2e-4); solves compare iteration
counts (FP64) and solutions."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1812_03952_amd import rsolve as rs
from gpu_util import dev, relerr, upload

pytestmark = pytest.mark.gpu


def _prob(dims, seed=3, **kw):
    nx, ny, nz = dims
    w = synth.wells_vertical_pair(nx, ny, nz, (0, 0), (nx - 1, ny - 1)) if nx * ny > 1 else None
    return synth.make(nx, ny, nz, seed=seed, wells=w, **kw)


@pytest.mark.parametrize("method", [rs.ABF, rs.QIMPES, rs.FRS])
@pytest.mark.parametrize("dims", [(20, 20, 10), (5, 3, 4), (1, 1, 7), (7, 1, 5), (6, 5, 1), (4, 4, 2)])
def test_ras1_owned_factors_bitwise(dims, method):
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, method=method, smoother=oracle.SM_RAS1)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, method, 64), rs.cpr_opts(smoother=rs.SM_RAS1))
    assert np.array_equal(rs.cpr_smoother_get(Mg), Mo.dinv2())


def _check_apply(z, ref, prec):
    e = np.abs(z - ref).max() / np.abs(ref).max()
    if prec == 64:
        assert relerr(z, ref) <= 1e-10 and e <= 1e-9, (relerr(z, ref), e)
    else:
        assert relerr(z, ref) <= 1e-4 and e <= 2e-4, (relerr(z, ref), e)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("stages", [2, 3])
@pytest.mark.parametrize("dims", [(20, 20, 10), (7, 1, 5), (1, 1, 1), (6, 5, 1), (4, 4, 2), (33, 17, 9)])
def test_ras1_cpr_apply(dims, stages, prec):
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=oracle.SM_RAS1, stages=stages)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS1, stages=stages))
    r = np.random.default_rng(7).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.cpr_apply(Mg, dev(r), z)
    _check_apply(z.cpu().numpy(), Mo.apply(r), prec)


@pytest.mark.parametrize("dims,prec", [((5, 300, 2), 64), ((3, 480, 2), 64), ((3, 520, 3), 32),
                                       ((2, 960, 2), 32), ((37, 19, 3), 32), ((1, 241, 4), 32)])
def test_ras1_wide_layers(dims, prec):
    """Layers with more lines than one pass covers, and in FP32 layers split
    into several strips (five sweeps per apply, each with its own tickets)."""
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=oracle.SM_RAS1)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS1))
    if prec == 64:
        assert np.array_equal(rs.cpr_smoother_get(Mg), Mo.dinv2())
    r = np.random.default_rng(9).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    for _ in range(2):                    # the second apply reuses tags and words
        rs.cpr_apply(Mg, dev(r), z)
        _check_apply(z.cpu().numpy(), Mo.apply(r), prec)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", ["gmres", "bicgstab"])
def test_ras1_solves(solver, prec):
    p = synth.config(0)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=oracle.SM_RAS1)
    xt, it = oracle.gmres(A, p.b, Mo, rtol=1e-13)
    assert it["status"] == 0
    if solver == "gmres":
        xo, io = oracle.gmres(A, p.b, Mo, rtol=1e-8)
    else:
        xo, io = oracle.bicgstab(A, p.b, Mo, rtol=1e-8)
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS1))
    x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    if solver == "gmres":
        info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(rtol=1e-8, zero_guess=1))
    else:
        info = rs.bicgstab_solve(B, M, dev(p.b), x, rs.bicgstab_opts(rtol=1e-8, zero_guess=1))
    xg = x.cpu().numpy()
    true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / np.linalg.norm(p.b)
    assert info["return"] == 0 and true <= 1e-8 and relerr(xg, xt) <= 1e-6
    if prec == 64:
        assert info["iters"] == io["iters"] and relerr(xg, xo) <= 1e-12


def test_ras1_full_size_100x100x50():
    """The 100x100x50 workload with the overlap-1 second stage, in the
    benchmark's configuration (values attached in place, x0 = 0)."""
    p = synth.config(1)
    dp = rs.DeviceProblem(p)
    Ao = oracle.assemble(p).with_values(dp.vals.cpu().numpy().reshape(-1, 4, 4))
    Mo = oracle.CPR(Ao, smoother=oracle.SM_RAS1)
    xo, io = oracle.gmres(Ao, p.b, Mo, rtol=1e-8)
    xt, it = oracle.gmres(Ao, p.b, Mo, rtol=1e-13)
    assert io["status"] == 0 and it["status"] == 0
    nb = np.linalg.norm(p.b)
    A = dp.bsr()
    for prec in (64, 32):
        D = rs.bsr_attach_decouple(A, dp.vals, rs.ABF, prec)
        M = rs.cpr_setup(A, D, rs.cpr_opts(smoother=rs.SM_RAS1))
        x = torch.zeros_like(dp.b)
        info = rs.gmres_solve(A, M, dp.b, x, rs.gmres_opts(rtol=1e-8, zero_guess=1))
        xg = x.cpu().numpy()
        true = np.linalg.norm(p.b - oracle.spmv(Ao, xg)) / nb
        print(f"RAS(1) prec {prec}: iters {info['iters']} (oracle {io['iters']}), true {true:.2e}, "
              f"|x - x_oracle| {relerr(xg, xo):.2e}, |x - x_tight| {relerr(xg, xt):.2e}")
        assert info["return"] == 0 and true <= 1e-8 and relerr(xg, xt) <= 1e-6
        if prec == 64:
            assert info["iters"] == io["iters"] and relerr(xg, xo) <= 1e-12
        del M, D
