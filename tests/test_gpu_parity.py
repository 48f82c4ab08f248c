"""HIP path against the FP64 oracle, element by element, through the C-ABI.

Inputs are seeded synthetic problems; both sides get the same assembled
matrix (from the oracle), so every difference is the kernels'.  Where the
library keeps the oracle's operation order (pattern, decoupling, AMG
setup) the results are compared bitwise; elsewhere FMA contraction and
reduction order differ and the tolerance is stated per test."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1812_03952_amd import rsolve as rs
from gpu_util import assert_close, dev, relerr, upload

pytestmark = pytest.mark.gpu

GRIDS = [(1, 1, 1), (1, 1, 7), (6, 1, 1), (1, 5, 1), (5, 3, 4), (20, 20, 10), (33, 17, 9)]


def _prob(dims, seed=3, **kw):
    nx, ny, nz = dims
    w = synth.wells_vertical_pair(nx, ny, nz, (0, 0), (nx - 1, ny - 1)) if nx * ny > 1 else None
    return synth.make(nx, ny, nz, seed=seed, wells=w, **kw)


@pytest.mark.parametrize("dims", GRIDS)
def test_pattern_and_assembly(dims):
    p = _prob(dims, sigma=1.5)
    rp, ci = oracle.pattern(*dims)
    drp, dci = rs.pattern(*dims)
    assert np.array_equal(drp.cpu().numpy(), rp) and np.array_equal(dci.cpu().numpy(), ci)
    A = oracle.assemble(p)
    dp = rs.DeviceProblem(p)
    torch.cuda.synchronize()
    got = dp.vals.cpu().numpy().reshape(-1, 4, 4)
    scale = np.abs(A.v).max(axis=(1, 2), keepdims=True)
    assert np.all(np.abs(got - A.v) <= 4e-16 * 8 * scale)     # exp() may differ by an ulp


@pytest.mark.parametrize("dims", GRIDS)
def test_spmv(dims):
    p = _prob(dims, sigma=2.0, shale=0.1)
    A = oracle.assemble(p)
    M = upload(A)
    x = np.random.default_rng(1).standard_normal(4 * A.n)
    y = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.spmv(M, dev(x), y)
    ref = oracle.spmv(A, x)
    bound = 1e-15 * 8 * np.abs(A.v).sum(axis=2).max() * np.abs(x).max() * 7
    assert np.abs(y.cpu().numpy() - ref).max() <= bound


@pytest.mark.parametrize("method", [rs.ABF, rs.QIMPES, rs.FRS, rs.FRS_ABF])
@pytest.mark.parametrize("dims", [(5, 3, 4), (20, 20, 10), (1, 1, 7)])
def test_decouple_fp64_bitwise(method, dims):
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    At, dinv = oracle.decouple(A, method)
    D = rs.decouple(upload(A), method, 64)
    vals, dd = rs.dcpl_get(D)
    assert np.array_equal(vals, At.v)
    assert np.array_equal(dd, dinv)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("method", [rs.ABF, rs.QIMPES, rs.FRS, rs.FRS_ABF])
def test_update_decouple_fused(method, prec):
    """rs_bsr_update_decouple equals rs_bsr_update then rs_decouple, bitwise:
    the stored values (through the SpMV) and every decoupled array."""
    p = _prob((20, 20, 10), sigma=1.5)
    A = oracle.assemble(p)
    v2 = A.v * 1.0
    v2[:, 0, :] *= 1.25                             # new values on the same pattern
    vals = dev(v2.reshape(-1))
    B1, B2 = upload(A), upload(A)
    rs.bsr_update(B1, vals)
    D1 = rs.decouple(B1, method, prec)
    D2 = rs.bsr_update_decouple(B2, vals, method, prec)
    for a, b in zip(rs.dcpl_get(D1), rs.dcpl_get(D2)):
        assert np.array_equal(a, b)
    x = dev(np.random.default_rng(3).standard_normal(4 * A.n))
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    rs.spmv(B1, x, y1)
    rs.spmv(B2, x, y2)
    assert torch.equal(y1, y2)
    # errors: non-finite values, misaligned values
    bad = vals.clone(); bad[17] = float("inf")
    with pytest.raises(rs.RsError) as e:
        rs.bsr_update_decouple(B2, bad, method, prec)
    assert e.value.status == -5
    buf = torch.zeros(vals.numel() + 1, dtype=torch.float64, device="cuda")
    buf[1:] = vals
    with pytest.raises(rs.RsError):
        rs.bsr_update_decouple(B2, buf[1:], method, prec)


def test_decouple_fp32():
    p = _prob((20, 20, 10), sigma=1.5)
    A = oracle.assemble(p)
    At, dinv = oracle.decouple(A)
    D = rs.decouple(upload(A), rs.ABF, 32)
    vals, dd = rs.dcpl_get(D)
    assert np.array_equal(vals, At.v.astype(np.float32).astype(np.float64))
    assert np.array_equal(dd, dinv.astype(np.float32).astype(np.float64))


def test_decouple_errors():
    p = _prob((2, 2, 1))
    A = oracle.assemble(p)
    v = A.v.copy()
    v[A.rp[1] + 1] = 0.0
    with pytest.raises(rs.RsError) as e:
        rs.decouple(upload(A.with_values(v)), rs.ABF, 64)
    assert e.value.status == -4
    rp = dev(A.rp, torch.int32); ci = dev(A.ci, torch.int32)
    bad = ci.clone(); bad[0] = 3
    with pytest.raises(rs.RsError) as e:
        rs.bsr_create(2, 2, 1, rp, bad, dev(A.v.reshape(-1)))
    assert e.value.status == -1
    v = A.v.copy(); v[0, 0, 0] = np.nan
    with pytest.raises(rs.RsError) as e:
        rs.bsr_create(2, 2, 1, rp, ci, dev(v.reshape(-1)))
    assert e.value.status == -5
    # row starts out of range (negative, past nnzb, decreasing): refused
    # before any column index is read through them
    for r, val in ((1, -5), (2, -(1 << 30)), (1, 10 ** 6), (3, 1)):
        badrp = rp.clone(); badrp[r] = val
        with pytest.raises(rs.RsError) as e:
            rs.bsr_create(2, 2, 1, badrp, ci, dev(A.v.reshape(-1)))
        assert e.value.status == -1, (r, val)


def test_options_rejected():
    """Out-of-range options of the set-up and the solvers give RS_E_ARG."""
    p = _prob((4, 4, 2))
    A = oracle.assemble(p)
    B = upload(A)
    D = rs.decouple(B, rs.ABF, 64)
    nan = float("nan")
    for kw in (dict(smoother=7), dict(coarse_n=0), dict(max_levels=0), dict(lu_max=0), dict(lu_max=8193),
               dict(coarse_sweeps=0), dict(stages=1), dict(stages=4), dict(theta=nan), dict(max_row_sum=nan)):
        with pytest.raises(rs.RsError) as e:
            rs.cpr_setup(B, D, rs.cpr_opts(**kw))
        assert e.value.status == -1, kw
    M = rs.cpr_setup(B, D, rs.cpr_opts(smoother=rs.SM_RAS))
    b = dev(np.ones(4 * A.n))
    x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    for kw in (dict(restart=0), dict(restart=33), dict(maxit=-1), dict(rtol=-1.0), dict(rtol=nan)):
        with pytest.raises(rs.RsError) as e:
            rs.gmres_solve(B, M, b, x, rs.gmres_opts(**kw))
        assert e.value.status == -1, kw
    for kw in (dict(maxit=-1), dict(rtol=nan)):
        with pytest.raises(rs.RsError) as e:
            rs.bicgstab_solve(B, M, b, x, rs.bicgstab_opts(**kw))
        assert e.value.status == -1, kw
    info = rs.gmres_solve(B, M, b, x, rs.gmres_opts(zero_guess=1))       # the handles still work
    assert info["return"] == 0


@pytest.mark.parametrize("dims,sigma", [((20, 20, 10), 1.0), ((33, 17, 9), 2.0), ((40, 40, 20), 2.0)])
def test_amg_hierarchy_bitwise(dims, sigma):
    p = _prob(dims, sigma=sigma, shale=0.1 if sigma > 1.5 else 0.0)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, coarse_n=50)
    B = upload(A)
    D = rs.decouple(B, rs.ABF, 64)
    Mg = rs.cpr_setup(B, D, rs.cpr_opts(coarse_n=50))
    ho = Mo.amg()
    assert rs.cpr_nlevels(Mg) == ho.nlevels
    for l in range(ho.nlevels):
        Lo, Lg = ho.level(l), rs.cpr_level(Mg, l)
        assert Lo["n"] == Lg["n"] and Lo["nnz"] == Lg["nnz"]
        assert np.array_equal(Lo["rp"], Lg["rp"]) and np.array_equal(Lo["ci"], Lg["ci"])
        assert np.array_equal(Lo["a"], Lg["a"])
        assert np.array_equal(Lo["dl1"], Lg["dl1"])
        if l < ho.nlevels - 1:
            assert np.array_equal(Lo["agg"], Lg["agg"])


@pytest.mark.parametrize("smoother", [rs.SM_BJ, rs.SM_DILU, rs.SM_RAS])
@pytest.mark.parametrize("method", [rs.ABF, rs.QIMPES])
def test_smoother_factors(method, smoother):
    p = _prob((20, 20, 10), sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, method=method, smoother=smoother)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, method, 64), rs.cpr_opts(smoother=smoother))
    assert np.array_equal(rs.cpr_smoother_get(Mg), Mo.dinv2())


@pytest.mark.parametrize("coarse_n,max_levels", [(50, 20), (200, 20), (5000, 2)])
def test_vcycle(coarse_n, max_levels):
    """The coarsest inverse: one-workgroup elimination (<= 256 rows) and the
    launch-per-column one (larger coarsest level)."""
    p = _prob((33, 17, 9), sigma=2.0, shale=0.1)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, coarse_n=coarse_n, max_levels=max_levels, lu_max=8192)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 64),
                      rs.cpr_opts(coarse_n=coarse_n, max_levels=max_levels, lu_max=8192))
    nc = rs.cpr_level(Mg, rs.cpr_nlevels(Mg) - 1)["n"]
    assert (nc > 256) == (coarse_n == 5000)
    b = np.random.default_rng(5).standard_normal(A.n)
    x = torch.empty(A.n, dtype=torch.float64, device="cuda")
    rs.cpr_vcycle(Mg, dev(b), x)
    ref = Mo.amg().vcycle(b)
    assert_close(x.cpu().numpy(), ref, 1e-11)


@pytest.mark.parametrize("smoother", [rs.SM_BJ, rs.SM_DILU, rs.SM_RAS])
@pytest.mark.parametrize("method", [rs.ABF, rs.QIMPES, rs.FRS])
@pytest.mark.parametrize("dims", [(20, 20, 10), (7, 1, 5), (1, 1, 1)])
def test_cpr_apply(method, smoother, dims):
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, method=method, smoother=smoother)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, method, 64), rs.cpr_opts(smoother=smoother))
    r = np.random.default_rng(7).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.cpr_apply(Mg, dev(r), z)
    assert_close(z.cpu().numpy(), Mo.apply(r), 1e-10)


@pytest.mark.parametrize("dims,prec", [((5, 300, 2), 64), ((3, 480, 2), 64), ((3, 520, 2), 32),
                                       ((2, 960, 1), 32), ((37, 19, 3), 64), ((1, 241, 2), 32)])
def test_ras_wide_layers(dims, prec):
    """Layers with more lines than one pass of the sweep covers (several lines
    per thread group) and odd extents: factors bitwise (FP64) and the apply."""
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=oracle.SM_RAS)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS))
    if prec == 64:
        assert np.array_equal(rs.cpr_smoother_get(Mg), Mo.dinv2())
    r = np.random.default_rng(9).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.cpr_apply(Mg, dev(r), z)
    assert_close(z.cpu().numpy(), Mo.apply(r), 1e-10 if prec == 64 else 1e-4)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("dims", [(3, 448, 128), (3, 450, 128), (6, 256, 128), (5, 75, 100), (4, 40, 300),
                                  (7, 112, 64), (3, 16, 20)])
def test_ras_strip_shapes(dims, prec):
    """The sweeps at the edges of their launch shapes: strips of 224 lines
    (the largest the quad-per-cell strip sweeps take), 225 (one lane per line
    in FP32, one workgroup per layer in FP64), 128, uneven strips (38 + 37
    lines), more layers than CUs (one strip each), four strips, one 16-line
    strip.  The FP64 factors (one workgroup per layer) are compared bit for
    bit.  Both sweeps are compared through the CPR apply, twice in a row (the
    tickets and tags of a second launch)."""
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, smoother=oracle.SM_RAS)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS))
    if prec == 64:
        assert np.array_equal(rs.cpr_smoother_get(Mg), Mo.dinv2())
    for seed in (9, 10):
        r = np.random.default_rng(seed).standard_normal(4 * A.n)
        z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
        rs.cpr_apply(Mg, dev(r), z)
        assert_close(z.cpu().numpy(), Mo.apply(r), 1e-4 if prec == 32 else 1e-10)


def test_ras_layer_limit():
    """Layers wider than the sweep kernels take (ny > 480 in FP64, > 960 in FP32) are refused."""
    for ny, prec in ((481, 64), (961, 32)):
        p = _prob((2, ny, 1), sigma=1.0)
        A = oracle.assemble(p)
        B = upload(A)
        with pytest.raises(rs.RsError):
            rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=rs.SM_RAS))


@pytest.mark.parametrize("smoother", [rs.SM_BJ, rs.SM_DILU, rs.SM_RAS])
@pytest.mark.parametrize("method", [rs.ABF, rs.FRS, rs.FRS_ABF])
@pytest.mark.parametrize("dims", [(20, 20, 10), (7, 1, 5), (1, 1, 1)])
def test_cpr_apply_fpf(method, smoother, dims):
    """Three-stage CPR-FPF against the oracle's five steps (the device
    updates the step-4 residual through column 0 of A~ instead of
    recomputing it: equal in exact arithmetic)."""
    p = _prob(dims, sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, method=method, smoother=smoother, stages=3)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, method, 64), rs.cpr_opts(smoother=smoother, stages=3))
    r = np.random.default_rng(7).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.cpr_apply(Mg, dev(r), z)
    assert_close(z.cpu().numpy(), Mo.apply(r), 1e-10)
    Mg32 = rs.cpr_setup(B, rs.decouple(B, method, 32), rs.cpr_opts(smoother=smoother, stages=3))
    rs.cpr_apply(Mg32, dev(r), z)
    assert_close(z.cpu().numpy(), Mo.apply(r), 1e-4)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("method,smoother", [(rs.FRS, rs.SM_RAS), (rs.FRS_ABF, rs.SM_DILU), (rs.ABF, rs.SM_BJ)])
def test_fpf_solves(method, smoother, prec):
    """GMRES and BiCGSTAB with CPR-FPF on the 20x20x10 workload: true residual
    1e-8, solution within 1e-6 of the oracle's solve at the same rtol and of
    a tight (1e-13) oracle solution, iteration counts equal in FP64."""
    p = synth.config(0)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A, method=method, smoother=smoother, stages=3)
    xt, it = oracle.gmres(A, p.b, Mo, rtol=1e-13)
    assert it["status"] == 0
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, method, prec), rs.cpr_opts(smoother=smoother, stages=3))
    nb = np.linalg.norm(p.b)
    for solver in ("gmres", "bicgstab"):
        if solver == "gmres":
            xo, io = oracle.gmres(A, p.b, Mo, rtol=1e-8)
            x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
            info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(rtol=1e-8))
        else:
            xo, io = oracle.bicgstab(A, p.b, Mo, rtol=1e-8)
            x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
            info = rs.bicgstab_solve(B, M, dev(p.b), x, rs.bicgstab_opts(rtol=1e-8))
        xg = x.cpu().numpy()
        true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / nb
        assert info["return"] == 0 and true <= 1e-8, solver
        assert relerr(xg, xo) <= 1e-6 and relerr(xg, xt) <= 1e-6, solver
        if prec == 64:
            assert info["iters"] == io["iters"], solver


def test_cpr_apply_fp32_close_to_fp64():
    p = _prob((20, 20, 10), sigma=1.5)
    A = oracle.assemble(p)
    Mo = oracle.CPR(A)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32))
    r = np.random.default_rng(7).standard_normal(4 * A.n)
    z = torch.empty(4 * A.n, dtype=torch.float64, device="cuda")
    rs.cpr_apply(Mg, dev(r), z)
    assert_close(z.cpu().numpy(), Mo.apply(r), 1e-4)


@pytest.mark.parametrize("smoother", [rs.SM_DILU, rs.SM_RAS])
@pytest.mark.parametrize("cfg", [0])
@pytest.mark.parametrize("prec", [64, 32])
def test_gmres_solution(cfg, prec, smoother):
    p = synth.config(cfg)
    A = oracle.assemble(p)
    xo, io = oracle.gmres(A, p.b, oracle.CPR(A, smoother=smoother), rtol=1e-13, maxit=300)
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec), rs.cpr_opts(smoother=smoother))
    x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
    info = rs.gmres_solve(B, M, dev(p.b), x, rs.gmres_opts(rtol=1e-8))
    xg = x.cpu().numpy()
    true = np.linalg.norm(p.b - oracle.spmv(A, xg)) / np.linalg.norm(p.b)
    assert info["return"] == 0 and true <= 1e-8 and abs(true - info["relres"]) <= 1e-12
    # against the oracle's solution at rtol 1e-13: 1e-6 relative
    # (measured under 1e-10 on this workload)
    assert relerr(xg, xo) <= 1e-6
    if prec == 64:
        xo8, io8 = oracle.gmres(A, p.b, oracle.CPR(A, smoother=smoother), rtol=1e-8)
        assert info["iters"] == io8["iters"]


@pytest.mark.parametrize("solver", ["gmres", "bicgstab"])
def test_zero_guess_ignores_x(solver):
    """zero_guess = 1 starts from x0 = 0 without a product with A, whatever
    d_x holds: bitwise the solve from a zero d_x with zero_guess = 0."""
    p = synth.config(0)
    A = oracle.assemble(p)
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32), rs.cpr_opts(smoother=rs.SM_RAS))
    b = dev(p.b)
    solve = rs.gmres_solve if solver == "gmres" else rs.bicgstab_solve
    opts = rs.gmres_opts if solver == "gmres" else rs.bicgstab_opts
    x0 = torch.zeros_like(b)
    i0 = solve(B, M, b, x0, opts(zero_guess=0))
    x1 = torch.full_like(b, float("nan"))
    i1 = solve(B, M, b, x1, opts(zero_guess=1))
    assert i0["return"] == 0 and i1["return"] == 0 and i0["iters"] == i1["iters"]
    assert torch.equal(x0, x1) and i0["relres"] == i1["relres"]


def test_vectors_must_be_16_byte_aligned():
    p = synth.config(0)
    A = oracle.assemble(p)
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32))
    N = 4 * A.n
    buf = torch.zeros(N + 1, dtype=torch.float64, device="cuda")
    ok = torch.zeros(N, dtype=torch.float64, device="cuda")
    for call in (lambda: rs.gmres_solve(B, M, buf[1:], ok),
                 lambda: rs.gmres_solve(B, M, ok, buf[1:]),
                 lambda: rs.bicgstab_solve(B, M, buf[1:], ok),
                 lambda: rs.spmv(B, buf[1:], ok)):
        with pytest.raises(rs.RsError) as e:
            call()
        assert e.value.status == -1


def test_gmres_deterministic_and_status():
    p = synth.config(0)
    A = oracle.assemble(p)
    B = upload(A)
    M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 64))
    b = dev(p.b)
    xs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        rs.gmres_solve(B, M, b, x)
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
    x = torch.zeros_like(b)
    info = rs.gmres_solve(B, M, b, x, rs.gmres_opts(maxit=1, rtol=1e-14))
    assert info["return"] == 1 and info["iters"] == 1
    bb = b.clone(); bb[5] = float("nan")
    info = rs.gmres_solve(B, M, bb, torch.zeros_like(b), check=False)
    assert info["return"] == -5
    info = rs.gmres_solve(B, M, torch.zeros_like(b), x)
    assert info["return"] == 0 and info["iters"] == 0 and not x.any()


@pytest.mark.parametrize("prec", [64, 32])
def test_dilu_pipeline_repeatable(prec):
    """The pipelined DILU sweeps exchange brick faces between workgroups:
    repeated applications must agree bitwise, and with the oracle."""
    p = _prob((100, 100, 50), seed=11, sigma=1.5)
    A = oracle.assemble(p)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, prec))
    r = dev(np.random.default_rng(3).standard_normal(4 * A.n))
    z0 = torch.empty_like(r)
    rs.cpr_apply(Mg, r, z0)
    for _ in range(20):
        z = torch.empty_like(r)
        rs.cpr_apply(Mg, r, z)
        assert torch.equal(z, z0)
    if prec == 64:
        Mo = oracle.CPR(A)
        assert np.array_equal(rs.cpr_smoother_get(Mg), Mo.dinv2())
        assert_close(z0.cpu().numpy(), Mo.apply(r.cpu().numpy()), 1e-10)


def test_pool_reuse_is_transparent():
    """Handles destroyed and rebuilt reuse pooled (dirty) device memory: the
    solve is bitwise the same, before and after returning the cache."""
    p = synth.config(0)
    A = oracle.assemble(p)
    xs = []
    for trim in (False, False, True):
        if trim:
            rs.pool_trim()
            assert rs.pool_usage()[1] == 0
        B = upload(A)
        M = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 32), rs.cpr_opts(smoother=rs.SM_RAS))
        x = torch.zeros(4 * A.n, dtype=torch.float64, device="cuda")
        info = rs.gmres_solve(B, M, dev(p.b), x)
        assert info["return"] == 0
        xs.append(x.cpu().numpy())
        del M, B
        torch.cuda.synchronize()
        assert rs.pool_usage()[1] > 0
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])


def test_bsr_values_must_be_16_byte_aligned():
    p = synth.small(3, 3, 2, seed=4)
    A = oracle.assemble(p)
    rp, ci = dev(A.rp, torch.int32), dev(A.ci, torch.int32)
    buf = torch.zeros(16 * A.nnzb + 1, dtype=torch.float64, device="cuda")
    buf[1:] = dev(A.v.reshape(-1))
    with pytest.raises(rs.RsError):
        rs.bsr_create(A.nx, A.ny, A.nz, rp, ci, buf[1:])
    B = rs.bsr_create(A.nx, A.ny, A.nz, rp, ci, buf[1:].clone())
    with pytest.raises(rs.RsError):
        rs.bsr_update(B, buf[1:])


INV_SIZES = [1, 2, 3, 45, 64, 65, 107, 108, 109, 150, 156, 157, 200, 256, 257, 300]


def _inverse(a):
    inv = torch.empty_like(a)
    rs.dense_inverse(a, inv)
    return inv.cpu().numpy()


@pytest.mark.parametrize("n", INV_SIZES)
def test_dense_inverse_needs_pivoting(n):
    """Coarsest-level inverse on matrices that need row pivoting: a random
    row permutation of a diagonally dominant matrix (zero diagonal wherever
    the permutation moves a row) and a Gaussian matrix.  Checked by the
    definition A X = I and against LAPACK's inverse."""
    rng = np.random.default_rng(1000 + n)
    D = rng.standard_normal((n, n)) + np.diag(n + rng.random(n))
    for A in (D[rng.permutation(n)], rng.standard_normal((n, n))):
        X = _inverse(dev(np.ascontiguousarray(A)))
        cond = np.linalg.cond(A)
        assert np.abs(A @ X - np.eye(n)).max() <= 1e-14 * n * cond
        assert relerr(X, np.linalg.inv(A)) <= 1e-14 * n * cond


@pytest.mark.parametrize("n", [64, 128])
def test_dense_inverse_ties(n):
    """Sylvester-Hadamard matrices: every pivot search is a tie between
    entries of equal magnitude, and H^{-1} = H / n exactly."""
    H = np.ones((1, 1))
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    X = _inverse(dev(H))
    assert np.abs(X - H / n).max() <= 1e-15


@pytest.mark.parametrize("n", [1, 60, 130, 200, 300])
def test_dense_inverse_singular(n):
    """A zero row leaves no nonzero pivot for the last column it could hold."""
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A[rng.integers(n)] = 0.0
    with pytest.raises(rs.RsError):
        _inverse(dev(A))


@pytest.mark.parametrize("dims,lo,hi", [((7, 7, 7), 1, 108), ((11, 11, 6), 89, 108), ((11, 11, 7), 109, 156),
                                        ((13, 13, 7), 109, 156), ((13, 13, 8), 157, 256), ((20, 20, 10), 257, 2048)])
def test_coarsest_inverse_paths(dims, lo, hi):
    """Two-level hierarchies whose coarsest level falls in each range of the
    coarsest-inverse kernels (register tiles 2 x 6 up to 108 rows and 4 x 6
    up to 156, one workgroup in global memory up to 256, one launch pair per
    column beyond): the V-cycle against the oracle's, which inverts by dense
    LU."""
    p = _prob(dims, sigma=2.0, shale=0.1)
    A = oracle.assemble(p)
    opts = dict(coarse_n=A.n - 1, max_levels=2, lu_max=2048)
    Mo = oracle.CPR(A, **opts)
    B = upload(A)
    Mg = rs.cpr_setup(B, rs.decouple(B, rs.ABF, 64), rs.cpr_opts(**opts))
    nc = rs.cpr_level(Mg, 1)["n"]
    assert lo <= nc <= hi or (lo == 1 and nc <= hi), nc
    b = np.random.default_rng(11).standard_normal(A.n)
    x = torch.empty(A.n, dtype=torch.float64, device="cuda")
    rs.cpr_vcycle(Mg, dev(b), x)
    assert_close(x.cpu().numpy(), Mo.amg().vcycle(b), 1e-11)
