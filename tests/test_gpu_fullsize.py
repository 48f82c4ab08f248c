"""Parity at the full workload sizes, in the configuration bench.py times
(bsr_attach_decouple -> cpr_setup -> gmres_solve from x0 = 0, RAS second
stage):
the 100x100x50 and 200x200x100 systems solved by the library and by the FP64
oracle, the true residual recomputed by the oracle, every solution compared
with a tight oracle reference (rtol 1e-13) to 1e-6 relative, and
sampled SpMV rows computed one by one on the host."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, relerr
from paper_1812_03952_amd import rsolve as rs

pytestmark = pytest.mark.gpu


_TIGHT = {}


def _tight(cfg, Ao, p, Mo=None):
    """The oracle's solution of the device-assembled system at rtol 1e-13."""
    if cfg not in _TIGHT:
        Mo = Mo if Mo is not None else oracle.CPR(Ao, smoother=oracle.SM_RAS)
        xt, it = oracle.gmres(Ao, p.b, Mo, rtol=1e-13)
        assert it["status"] == 0 and it["relres"] <= 1e-13
        _TIGHT[cfg] = xt
    return _TIGHT[cfg]


def _solve(dp, prec, rtol=1e-8, smoother=rs.SM_RAS):
    A = dp.bsr()
    D = rs.bsr_attach_decouple(A, dp.vals, rs.ABF, prec)
    M = rs.cpr_setup(A, D, rs.cpr_opts(smoother=smoother))
    x = torch.zeros_like(dp.b)
    info = rs.gmres_solve(A, M, dp.b, x, rs.gmres_opts(rtol=rtol, zero_guess=1))
    return A, x, info


@pytest.mark.parametrize("cfg", [1, 2])
def test_full_size_solve_against_oracle(cfg):
    p = synth.config(cfg)
    dp = rs.DeviceProblem(p)
    Ao = oracle.assemble(p)
    # the device assembly equals the oracle's up to exp() rounding ...
    got = dp.vals.cpu().numpy().reshape(-1, 4, 4)
    assert np.all(np.abs(got - Ao.v) <= 4e-16 * 8 * np.abs(Ao.v).max(axis=(1, 2), keepdims=True))
    # ... and the oracle solves the same matrix as the library
    Ao = Ao.with_values(got)
    Mo = oracle.CPR(Ao, smoother=oracle.SM_RAS)
    xo, io = oracle.gmres(Ao, p.b, Mo, rtol=1e-8)
    assert io["status"] == 0
    xt = _tight(cfg, Ao, p, Mo)
    nb = np.linalg.norm(p.b)
    for prec in (64, 32):
        _, x, info = _solve(dp, prec)
        xg = x.cpu().numpy()
        true = np.linalg.norm(p.b - oracle.spmv(Ao, xg)) / nb
        assert info["return"] == 0 and true <= 1e-8 and abs(true - info["relres"]) <= 1e-10
        err = relerr(xg, xo)
        errt = relerr(xg, xt)
        print(f"cfg {cfg} prec {prec}: iters {info['iters']} (oracle {io['iters']}), true relres {true:.2e}, "
              f"|x - x_oracle|/|x_oracle| {err:.2e}, against the 1e-13 reference {errt:.2e}")
        assert errt <= 1e-6
        assert info["iters"] == io["iters"]
        if prec == 64:
            # the same iteration in another summation order (measured 2e-16 and 5e-16)
            assert err <= 1e-12
        else:
            # FP32-stored preconditioner: the Krylov iterates move by rounding of
            # M only (measured 3e-13 and 9e-14)
            assert err <= 1e-8


@pytest.mark.parametrize("attach", [False, True])
@pytest.mark.parametrize("cfg", [2])
def test_full_size_spmv_sampled_rows(cfg, attach):
    p = synth.config(cfg)
    dp = rs.DeviceProblem(p)
    A = dp.bsr()
    if attach:
        rs.bsr_attach_decouple(A, dp.vals, rs.ABF, 32)   # the SpMV reads dp.vals in place
    N = 4 * p.n
    x = torch.randn(N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    y = torch.empty_like(x)
    rs.spmv(A, x, y)
    xh, yh = x.cpu().numpy(), y.cpu().numpy()
    rp, ci = oracle.pattern(p.nx, p.ny, p.nz)
    vals = dp.vals.cpu().numpy().reshape(-1, 4, 4)
    rows = np.random.default_rng(5).choice(p.n, size=2000, replace=False)
    rows = np.concatenate([rows, [0, p.n - 1, p.nx * p.ny - 1, p.n - p.nx * p.ny]])
    for c in rows:
        acc = np.zeros(4)
        for q in range(rp[c], rp[c + 1]):
            acc += vals[q] @ xh[4 * ci[q]:4 * ci[q] + 4]
        assert np.allclose(yh[4 * c:4 * c + 4], acc, rtol=1e-13, atol=1e-13 * np.abs(acc).max())


@pytest.mark.parametrize("cfg", [1, 2])
def test_full_size_bicgstab_against_oracle(cfg):
    """The same path with BiCGSTAB as the outer solver."""
    p = synth.config(cfg)
    dp = rs.DeviceProblem(p)
    Ao = oracle.assemble(p).with_values(dp.vals.cpu().numpy().reshape(-1, 4, 4))
    Mo = oracle.CPR(Ao, smoother=oracle.SM_RAS)
    xo, io = oracle.bicgstab(Ao, p.b, Mo, rtol=1e-8)
    assert io["status"] == 0
    xt = _tight(cfg, Ao, p, Mo)
    nb = np.linalg.norm(p.b)
    A = dp.bsr()
    for prec in (64, 32):
        rs.bsr_update(A, dp.vals)
        M = rs.cpr_setup(A, rs.decouple(A, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS))
        x = torch.zeros_like(dp.b)
        info = rs.bicgstab_solve(A, M, dp.b, x, rs.bicgstab_opts(rtol=1e-8))
        xg = x.cpu().numpy()
        true = np.linalg.norm(p.b - oracle.spmv(Ao, xg)) / nb
        err = relerr(xg, xo)
        print(f"cfg {cfg} prec {prec}: iters {info['iters']} (oracle {io['iters']}), true relres {true:.2e}, "
              f"|x - x_oracle|/|x_oracle| {err:.2e}")
        assert info["return"] == 0 and true <= 1e-8 and abs(true - info["relres"]) <= 1e-10
        assert relerr(xg, xt) <= 1e-6
        if prec == 64:
            assert info["iters"] == io["iters"] and err <= 1e-9
        else:
            assert err <= 1e-6


def test_full_size_fpf_frs_against_oracle():
    """100x100x50 with FRS decoupling and CPR-FPF (RAS full-system stages),
    GMRES, FP64 and FP32 preconditioner, against the oracle."""
    p = synth.config(1)
    dp = rs.DeviceProblem(p)
    Ao = oracle.assemble(p).with_values(dp.vals.cpu().numpy().reshape(-1, 4, 4))
    xo, io = oracle.gmres(Ao, p.b, oracle.CPR(Ao, method=oracle.FRS, smoother=oracle.SM_RAS, stages=3), rtol=1e-8)
    assert io["status"] == 0
    xt = _tight(1, Ao, p)
    nb = np.linalg.norm(p.b)
    A = dp.bsr()
    for prec in (64, 32):
        M = rs.cpr_setup(A, rs.decouple(A, rs.FRS, prec), rs.cpr_opts(smoother=rs.SM_RAS, stages=3))
        x = torch.zeros_like(dp.b)
        info = rs.gmres_solve(A, M, dp.b, x, rs.gmres_opts(rtol=1e-8))
        xg = x.cpu().numpy()
        true = np.linalg.norm(p.b - oracle.spmv(Ao, xg)) / nb
        err = relerr(xg, xo)
        print(f"FRS + CPR-FPF prec {prec}: iters {info['iters']} (oracle {io['iters']}), true relres {true:.2e}, "
              f"|x - x_oracle|/|x_oracle| {err:.2e}")
        assert info["return"] == 0 and true <= 1e-8 and relerr(xg, xt) <= 1e-6
        if prec == 64:
            assert info["iters"] == io["iters"] and err <= 1e-9
        else:
            assert err <= 1e-6
