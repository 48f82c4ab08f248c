"""Restarted GMRES on the device against the oracle, through the C-ABI.

Covers what a solve that converges inside its first cycle never reaches:
  - cycles after the first: the true residual b - A x of the last update,
    V_0 scaled in place, the cycle's first preconditioner pass run directly
    rather than fused into the previous step;
  - x0 != 0 (zero_guess = 0 with a non-zero d_x) and x0 = 0 implied
    (zero_guess = 1, d_x full of NaN);
  - maxit reached inside the second cycle;
  - the happy breakdown (h_{j+1,j} ~ 0) that ends a cycle early;
  - the coarsest AMG level relaxed by l1-Jacobi sweeps instead of inverted.
FP64: iteration and cycle counts equal the oracle's with the same restart,
and x agrees to 1e-12 (the same iteration in another summation order).
FP32 preconditioner: the true FP64 residual meets rtol and x agrees with a
tightly converged oracle solution to 1e-6."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1812_03952_amd import rsolve as rs
from gpu_util import assert_close, dev, relerr, upload

pytestmark = pytest.mark.gpu


def _problem(name):
    if name == "cfg0":
        return synth.config(0)
    # 12x10x6, sigma 2 with 10 % shale: more steps than the 20x20x10 workload
    return synth.make(12, 10, 6, seed=5, sigma=2.0, shale=0.1,
                      wells=synth.wells_vertical_pair(12, 10, 6, (0, 0), (11, 9)))


def _x0(n, zero_guess):
    if zero_guess:
        return np.zeros(4 * n)
    return 0.1 * np.random.default_rng(11).standard_normal(4 * n)


def _x_dev(x0, zero_guess):
    x = dev(x0)
    if zero_guess:
        x.fill_(float("nan"))       # zero_guess = 1 must not read d_x
    return x


# (problem, smoother, restart): each needs at least two cycles at rtol 1e-12
CASES = [("cfg0", rs.SM_BJ, 2), ("cfg0", rs.SM_BJ, 3), ("cfg0", rs.SM_RAS, 2),
         ("p12", rs.SM_BJ, 3), ("p12", rs.SM_BJ, 4), ("p12", rs.SM_RAS, 3), ("p12", rs.SM_DILU, 4)]


@pytest.mark.parametrize("zero_guess", [1, 0])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-sm{c[1]}-m{c[2]}")
def test_restart_fp64_matches_oracle(case, zero_guess):
    name, sm, m = case
    p = _problem(name)
    A = oracle.assemble(p)
    x0 = _x0(A.n, zero_guess)
    xo, io = oracle.gmres(A, p.b, oracle.CPR(A, smoother=sm), x0=x0, restart=m, rtol=1e-12, maxit=300)
    assert io["status"] == 0 and io["cycles"] >= 2
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 64), rs.cpr_opts(smoother=sm))
    x = _x_dev(x0, zero_guess)
    print(f"{name} smoother {sm} restart {m} zero_guess {zero_guess}", flush=True)
    info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(restart=m, rtol=1e-12, zero_guess=zero_guess))
    xg = x.cpu().numpy()
    true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / np.linalg.norm(p.b)
    print(f"  iters {info['iters']} cycles {info['cycles']} (oracle {io['iters']}, {io['cycles']}), "
          f"true {true:.2e}, |x - x_oracle| {relerr(xg, xo):.2e}")
    assert info["return"] == 0 and true <= 1e-12 * 1.0001
    assert abs(true - info["relres"]) <= 1e-14
    assert info["iters"] == io["iters"] and info["cycles"] == io["cycles"]
    assert relerr(xg, xo) <= 1e-12


@pytest.mark.parametrize("zero_guess", [1, 0])
@pytest.mark.parametrize("case", CASES[:4], ids=lambda c: f"{c[0]}-sm{c[1]}-m{c[2]}")
def test_restart_fp32_preconditioner(case, zero_guess):
    name, sm, m = case
    p = _problem(name)
    A = oracle.assemble(p)
    x0 = _x0(A.n, zero_guess)
    xt, it = oracle.gmres(A, p.b, oracle.CPR(A, smoother=sm), rtol=1e-13, maxit=300)
    assert it["status"] == 0
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32), rs.cpr_opts(smoother=sm))
    x = _x_dev(x0, zero_guess)
    print(f"{name} smoother {sm} restart {m} zero_guess {zero_guess} FP32", flush=True)
    info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(restart=m, rtol=1e-8, zero_guess=zero_guess))
    xg = x.cpu().numpy()
    true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / np.linalg.norm(p.b)
    print(f"  iters {info['iters']} cycles {info['cycles']}, true {true:.2e}, "
          f"|x - x_tight| {relerr(xg, xt):.2e}")
    assert info["return"] == 0 and info["cycles"] >= 2
    assert true <= 1e-8 and abs(true - info["relres"]) <= 1e-14
    assert relerr(xg, xt) <= 1e-6


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("zero_guess", [1, 0])
def test_maxit_inside_second_cycle(zero_guess, prec):
    """restart 4, maxit 6: the solve stops after step 2 of cycle 2, not
    converged, with x = x0 + the two cycles' updates."""
    p = _problem("p12")
    A = oracle.assemble(p)
    x0 = _x0(A.n, zero_guess)
    xo, io = oracle.gmres(A, p.b, oracle.CPR(A, smoother=oracle.SM_BJ), x0=x0, restart=4, rtol=1e-14, maxit=6)
    assert io["status"] == 1 and io["iters"] == 6 and io["cycles"] == 2
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_BJ))
    x = _x_dev(x0, zero_guess)
    info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(restart=4, rtol=1e-14, maxit=6,
                                                           zero_guess=zero_guess))
    xg = x.cpu().numpy()
    true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / np.linalg.norm(p.b)
    assert info["return"] == rs.RS_NOT_CONVERGED and info["iters"] == 6 and info["cycles"] == 2
    assert abs(true - info["relres"]) <= 1e-14 + 1e-12 * true
    if prec == 64:
        # |true - relres_oracle| <= ||A|| ||x - x_oracle|| / ||b||: absolute, since
        # the relative difference of a 1e-8 residual under rounding is ~1e-10
        assert relerr(xg, xo) <= 1e-12 and abs(true - io["relres"]) <= 1e-14
    else:
        assert relerr(xg, xo) <= 1e-5


def _scaled_identity(dims):
    """A = 4 I: block-diagonal, every diagonal block 4 I_4 (no flux
    couplings, no wells).  ABF gives A~ = I and the CPR preconditioner is
    then A^{-1} exactly, so A M^{-1} = I and every Krylov space is invariant
    after one step."""
    p = synth.make(*dims, seed=53, sigma=1.0, storage=0.0)
    p.Mf[:] = 0.0
    p.Mb[:] = 0.0
    p.B[:] = 4.0 * np.eye(4)
    return p, oracle.assemble(p)


@pytest.mark.parametrize("smoother", [rs.SM_BJ, rs.SM_DILU, rs.SM_RAS])
@pytest.mark.parametrize("dims", [(4, 3, 2), (20, 20, 10)])
def test_happy_breakdown(dims, smoother):
    """The pressure matrix of A = 4 I is the identity: every row is weak, no
    aggregate forms, and the fine level is the only one (on 20x20x10 after
    the structured fine-level set-up, above coarse_n and lu_max, so its
    l1-Jacobi coarsest solve reads the CSR arrays built for it then)."""
    p, A = _scaled_identity(dims)
    xe = p.b / 4.0
    Mo = oracle.CPR(A, smoother=smoother)
    _, io = oracle.gmres(A, p.b, Mo, rtol=1e-12, maxit=30)
    assert io["iters"] == 1 and io["cycles"] == 1 and Mo.amg().nlevels == 1
    B = upload(A)
    r = np.random.default_rng(3).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    M32 = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32), rs.cpr_opts(smoother=smoother))
    assert rs.cpr_nlevels(M32) == 1
    rs.cpr_apply(M32, dev(r), z)
    assert relerr(z.cpu().numpy(), r / 4.0) <= 1e-7          # FP32 rounding of r only
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 64), rs.cpr_opts(smoother=smoother))
    assert rs.cpr_nlevels(M) == 1
    L0 = rs.cpr_level(M, 0)
    assert np.array_equal(L0["dl1"], Mo.amg().level(0)["dl1"]) and np.all(L0["agg"] == -1)
    rs.cpr_apply(M, dev(r), z)
    assert np.array_equal(z.cpu().numpy(), r / 4.0)
    x = torch.full((4 * A.n,), float("nan"), dtype=torch.float64, device="cuda")
    info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(rtol=1e-12, zero_guess=1))
    xg = x.cpu().numpy()
    assert info["return"] == 0 and info["iters"] == 1 and info["cycles"] == 1
    assert relerr(xg, xe) <= 1e-14
    # rtol = 0: the estimate never meets it, so only the breakdown test ends
    # a cycle; every cycle is one step and nothing divides by h_{1,0} ~ 0
    _, io = oracle.gmres(A, p.b, oracle.CPR(A, smoother=smoother), rtol=0.0, maxit=3)
    assert io["iters"] == io["cycles"]
    x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(rtol=0.0, maxit=3, zero_guess=1))
    xg = x.cpu().numpy()
    assert info["return"] in (rs.RS_OK, rs.RS_NOT_CONVERGED)
    assert info["iters"] == info["cycles"] >= 1 and np.all(np.isfinite(xg))
    assert relerr(xg, xe) <= 1e-14 and info["relres"] <= 1e-14


@pytest.mark.parametrize("coarse_n,lu_max,sweeps", [(200, 10, 4), (5000, 10, 3), (50, 1, 6)])
def test_coarsest_l1_jacobi(coarse_n, lu_max, sweeps):
    """A coarsest level above lu_max is relaxed by coarse_sweeps l1-Jacobi
    sweeps from zero (the oracle's branch, pinned by the Jacobi polynomial):
    the V-cycle and a whole FP64 solve against the oracle."""
    p = _prob33()
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, coarse_n=coarse_n, lu_max=lu_max, coarse_sweeps=sweeps)
    assert not Mo.amg().coarsest_is_lu
    opts = rs.cpr_opts(coarse_n=coarse_n, lu_max=lu_max, coarse_sweeps=sweeps)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 64), opts)
    assert rs.cpr_nlevels(Mg) == Mo.amg().nlevels
    b = np.random.default_rng(5).standard_normal(A.n)
    x = torch.empty(A.n, dtype=torch.float64, device="cuda")
    rs.cpr_vcycle(Mg, dev(b), x)
    ref = Mo.amg().vcycle(b)
    assert_close(x.cpu().numpy(), ref, 1e-11)
    r = np.random.default_rng(7).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.cpr_apply(Mg, dev(r), z)
    assert_close(z.cpu().numpy(), Mo.apply(r), 1e-10)
    xo, io = oracle.gmres(A, p.b, Mo, rtol=1e-10)
    xs = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    info = rs.gmres_solve(B, Mg, dev(p.b), xs, rs.gmres_opts(rtol=1e-10, zero_guess=1))
    assert info["return"] == 0 and info["iters"] == io["iters"]
    assert relerr(xs.cpu().numpy(), xo) <= 1e-12
    # the FP32 hierarchy takes the same branch
    M32 = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32), opts)
    info = rs.gmres_solve(B, M32, dev(p.b), xs, rs.gmres_opts(rtol=1e-8, zero_guess=1))
    true = np.linalg.norm(p.b - oracle.spmv(A, xs.cpu().numpy())) / np.linalg.norm(p.b)
    assert info["return"] == 0 and true <= 1e-8


def _prob33():
    return synth.make(33, 17, 9, seed=3, sigma=2.0, shale=0.1,
                      wells=synth.wells_vertical_pair(33, 17, 9, (0, 0), (32, 16)))
