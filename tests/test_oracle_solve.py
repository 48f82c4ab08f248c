"""Oracle CPR preconditioner, flexible GMRES and adjoint gradient, pinned by
dense algebra, a closed-form (DCT) solution, finite differences and
duality."""
import numpy as np
import pytest
import scipy.fft

import oracle
import synth


def _blockdiag(blocks):
    n = blocks.shape[0]
    D = np.zeros((4 * n, 4 * n))
    for i in range(n):
        D[4 * i:4 * i + 4, 4 * i:4 * i + 4] = blocks[i]
    return D


@pytest.mark.parametrize("stages", [2, 3])
@pytest.mark.parametrize("smoother", [oracle.SM_BJ, oracle.SM_DILU, oracle.SM_RAS])
@pytest.mark.parametrize("method", [oracle.ABF, oracle.QIMPES, oracle.FRS])
def test_cpr_dense_composition(method, smoother, stages):
    """With a single-level (exact) pressure solve, S = M2^{-1} and
    C = Pi_p A_p^{-1} Pi_r:
       two-stage    M^{-1} = [C + S(I - A~ C)] D^{-1}
       three-stage  M^{-1} = [S + (C + S(I - A~ C))(I - A~ S)] D^{-1}
    and for the three-stage form its error propagation
       I - A~ M^{-1} D = (I - A~ S)(I - A~ C)(I - A~ S)."""
    p = synth.small(4, 3, 2, seed=29)
    A = oracle.assemble(p)
    M = oracle.CPR(A, method=method, smoother=smoother, stages=stages)
    assert M.amg().nlevels == 1
    n = A.n; N = 4 * n
    At = M.decoupled()
    Dt = At.dense()
    Dinv = _blockdiag(M.dinv())
    Ap = Dt[0::4, 0::4]
    Pi_p = np.zeros((N, n)); Pi_p[np.arange(0, N, 4), np.arange(n)] = 1.0
    Cm = Pi_p @ np.linalg.solve(Ap, Pi_p.T)
    if smoother == oracle.SM_BJ:
        M2 = _blockdiag(np.linalg.inv(M.dinv2()))
        M2inv = np.linalg.inv(M2)
    else:
        d2 = M.dinv2()
        lower = np.tril(Dt, -1) * 0; upper = lower.copy()
        nxy = p.nx * p.ny
        for i in range(n):
            for j in range(n):
                if smoother == oracle.SM_RAS and i // nxy != j // nxy:
                    continue        # zero-overlap RAS: no coupling between layers
                if j < i: lower[4*i:4*i+4, 4*j:4*j+4] = Dt[4*i:4*i+4, 4*j:4*j+4]
                if j > i: upper[4*i:4*i+4, 4*j:4*j+4] = Dt[4*i:4*i+4, 4*j:4*j+4]
        Dblk = _blockdiag(np.linalg.inv(d2))
        M2inv = np.linalg.inv((Dblk + lower) @ _blockdiag(d2) @ (Dblk + upper))
    I = np.eye(N)
    if stages == 2:
        ref = (Cm + M2inv @ (I - Dt @ Cm)) @ Dinv
    else:
        ref = (M2inv + (Cm + M2inv @ (I - Dt @ Cm)) @ (I - Dt @ M2inv)) @ Dinv
    got = np.stack([M.apply(e) for e in np.eye(N)], 1)
    assert np.allclose(got, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    if stages == 3:
        E = I - Dt @ got @ np.linalg.inv(Dinv)
        Ef = (I - Dt @ M2inv) @ (I - Dt @ Cm) @ (I - Dt @ M2inv)
        assert np.allclose(E, Ef, rtol=1e-7, atol=1e-8 * max(1.0, np.abs(Ef).max()))


def test_gmres_exact_in_n_steps():
    """GMRES with restart >= N terminates in at most N steps (2x2x1: N = 16)."""
    p = synth.small(2, 2, 1, seed=31)
    A = oracle.assemble(p)
    x, info = oracle.gmres(A, p.b, None, restart=30, rtol=1e-12, maxit=40)
    assert info["status"] == 0 and info["iters"] <= 16 and info["cycles"] == 1
    assert np.allclose(x, np.linalg.solve(A.dense(), p.b), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("dims,sigma", [((4, 3, 2), 1.0), ((10, 10, 5), 1.5), ((10, 10, 5), 2.0)])
def test_cpr_gmres_vs_dense_lu(dims, sigma):
    p = synth.make(*dims, seed=37, sigma=sigma, shale=0.1 if sigma == 2.0 else 0.0,
                   wells=synth.wells_vertical_pair(*dims, (0, 0), (dims[0] - 1, dims[1] - 1)))
    A = oracle.assemble(p)
    xref = np.linalg.solve(A.dense(), p.b)
    for method, smoother, stages in ((oracle.ABF, oracle.SM_DILU, 2), (oracle.QIMPES, oracle.SM_DILU, 2),
                                     (oracle.ABF, oracle.SM_RAS, 2), (oracle.FRS, oracle.SM_RAS, 3),
                                     (oracle.FRS_ABF, oracle.SM_BJ, 3)):
        M = oracle.CPR(A, method=method, smoother=smoother, stages=stages, coarse_n=20)
        x, info = oracle.gmres(A, p.b, M, rtol=1e-12, maxit=200)
        assert info["status"] == 0 and info["relres"] <= 1e-12
        r = p.b - A.dense() @ x
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(p.b) * 1.0001
        cond = np.linalg.cond(A.dense())
        assert np.linalg.norm(x - xref) <= max(1e-12 * cond, 1e-10) * np.linalg.norm(xref)


def test_cpr_gmres_dct_closed_form():
    """Homogeneous k, M = I (all faces), B = a*I, no wells: A = (a I + T L_N) (x) I_4
    with L_N the Neumann 7-point graph Laplacian, diagonalised by the DCT-II."""
    nx, ny, nz = 16, 12, 10
    a, kk = 2.0, 100.0
    p = synth.make(nx, ny, nz, seed=41, sigma=0.0, kvkh=1.0, tscale=1.0)
    p.logk[:] = np.log(kk)
    p.Mf[:] = np.eye(4); p.Mb[:] = np.eye(4); p.B[:] = a * np.eye(4)
    A = oracle.assemble(p)
    M = oracle.CPR(A)
    x, info = oracle.gmres(A, p.b, M, rtol=1e-12, maxit=300)
    assert info["status"] == 0
    lam = lambda m: 2.0 - 2.0 * np.cos(np.pi * np.arange(m) / m)
    ev = a + kk * (lam(nz)[:, None, None] + lam(ny)[None, :, None] + lam(nx)[None, None, :])
    B = p.b.reshape(nz, ny, nx, 4)
    X = np.empty_like(B)
    for u in range(4):
        bh = scipy.fft.dctn(B[..., u], type=2, norm="ortho")
        X[..., u] = scipy.fft.idctn(bh / ev, type=2, norm="ortho")
    xd = X.reshape(-1)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_gmres_status_paths():
    p = synth.small(5, 4, 3, seed=43)
    A = oracle.assemble(p)
    M = oracle.CPR(A)
    _, info = oracle.gmres(A, p.b, M, rtol=1e-14, maxit=1)
    assert info["status"] == 1 and info["iters"] == 1
    x, info = oracle.gmres(A, np.zeros(4 * A.n), M)
    assert info["status"] == 0 and info["iters"] == 0 and not x.any()
    b = p.b.copy(); b[3] = np.nan
    with pytest.raises(oracle.OracleError, match="-5"):
        oracle.gmres(A, b, M)


def test_gmres_estimate_tracks_true_residual():
    p = synth.config(0)
    A = oracle.assemble(p)
    M = oracle.CPR(A)
    x, info = oracle.gmres(A, p.b, M, rtol=1e-8, hist=True)
    assert info["status"] == 0
    true = np.linalg.norm(p.b - oracle.spmv(A, x)) / np.linalg.norm(p.b)
    assert abs(true - info["relres"]) <= 1e-12
    assert abs(info["hist"][-1] - true) <= 1e-10


def _J(p, logk):
    A = oracle.assemble(p, logk)
    x = np.linalg.solve(A.dense(), p.b)
    return p.w @ x


def test_adjoint_duality_fd_and_dense():
    p = synth.make(4, 3, 3, seed=47, sigma=1.5,
                   wells=synth.wells_vertical_pair(4, 3, 3, (0, 0), (3, 2)))
    A = oracle.assemble(p)
    At = oracle.transpose(A)
    x, ix = oracle.gmres(A, p.b, oracle.CPR(A), rtol=1e-14, maxit=200)
    lam, il = oracle.gmres(At, p.w, oracle.CPR(At), rtol=1e-14, maxit=200)
    assert ix["status"] == 0 and il["status"] == 0
    # duality: lambda^T b = w^T x
    assert abs(lam @ p.b - p.w @ x) <= 1e-12 * abs(p.w @ x) + 1e-14
    # dense adjoint
    assert np.allclose(lam, np.linalg.solve(A.dense().T, p.w), rtol=1e-10, atol=1e-12)
    g = oracle.grad_logk(p, lam, x)
    h = 1e-5
    fd = np.array([(_J(p, p.logk + h * e) - _J(p, p.logk - h * e)) / (2 * h)
                   for e in np.eye(p.n)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def _scaled_identity_problem(dims, diag):
    """A block-diagonal system whose every diagonal block is diag(d): no flux
    couplings (M = 0), no wells, accumulation B = diag(d), dt = 1."""
    p = synth.make(*dims, seed=53, sigma=1.0, storage=0.0)
    p.Mf[:] = 0.0
    p.Mb[:] = 0.0
    p.B[:] = np.diag(diag)
    return p, oracle.assemble(p)


def test_gmres_happy_breakdown():
    """Happy breakdown: when the Krylov space of b under A M^{-1} is invariant
    after k steps, h_{k,k-1} vanishes, the cycle ends there and x is exact.
    A = c I (no preconditioner): one step, x = b / c.  A = blockdiag of
    diag(c1, c2, c1, c2): the minimal polynomial has degree 2, two steps.
    With rtol = 0 the estimate never meets the bound, so only the breakdown
    test can end a cycle: every cycle is one step long, and x stays finite
    (v_1 = w / h_{1,0} would divide by ~0)."""
    p, A = _scaled_identity_problem((4, 3, 2), [4.0, 4.0, 4.0, 4.0])
    x, info = oracle.gmres(A, p.b, None, restart=30, rtol=1e-12, maxit=30)
    assert info["status"] == 0 and info["iters"] == 1 and info["cycles"] == 1
    assert np.linalg.norm(x - p.b / 4.0) <= 1e-15 * np.linalg.norm(p.b / 4.0)
    x, info = oracle.gmres(A, p.b, None, restart=30, rtol=0.0, maxit=3)
    assert np.all(np.isfinite(x)) and info["iters"] == info["cycles"] >= 1
    assert np.linalg.norm(x - p.b / 4.0) <= 1e-15 * np.linalg.norm(p.b / 4.0)
    p, A = _scaled_identity_problem((4, 3, 2), [2.0, 8.0, 2.0, 8.0])
    x, info = oracle.gmres(A, p.b, None, restart=30, rtol=1e-12, maxit=30)
    assert info["status"] == 0 and info["iters"] == 2 and info["cycles"] == 1
    xe = p.b / np.tile([2.0, 8.0, 2.0, 8.0], A.n)
    assert np.linalg.norm(x - xe) <= 1e-14 * np.linalg.norm(xe)
    # with CPR on A = 4 I, M^{-1} = A^{-1} exactly: breakdown at the first step
    p, A = _scaled_identity_problem((4, 3, 2), [4.0, 4.0, 4.0, 4.0])
    x, info = oracle.gmres(A, p.b, oracle.CPR(A), restart=30, rtol=0.0, maxit=3)
    assert info["iters"] == info["cycles"] >= 1 and np.all(np.isfinite(x))
    assert np.linalg.norm(x - p.b / 4.0) <= 1e-15 * np.linalg.norm(p.b / 4.0)


@pytest.mark.parametrize("restart", [2, 3, 4])
def test_gmres_restart_cycles(restart):
    """Restarted GMRES(m) with m small on a 12x10x6 sigma-2 draw: several
    cycles, each starting from the true residual of the last update.  Pinned
    by the dense-LU solution and by the minimal-residual property of a cycle:
    after one cycle from x0 no x0 + K_m(A M^{-1}, r0) M^{-1}-combination has a
    smaller residual, checked against the least-squares solution over the
    explicitly built (unorthogonalised, then QR-orthogonalised) basis."""
    p = synth.make(12, 10, 6, seed=5, sigma=2.0, shale=0.1,
                   wells=synth.wells_vertical_pair(12, 10, 6, (0, 0), (11, 9)))
    A = oracle.assemble(p)
    M = oracle.CPR(A, smoother=oracle.SM_BJ)
    x, info = oracle.gmres(A, p.b, M, restart=restart, rtol=1e-12, maxit=300)
    assert info["status"] == 0 and info["cycles"] >= 2
    assert info["iters"] <= restart * info["cycles"] and info["iters"] > restart * (info["cycles"] - 1)
    Ad = A.dense()
    xref = np.linalg.solve(Ad, p.b)
    assert np.linalg.norm(p.b - Ad @ x) <= 1e-12 * np.linalg.norm(p.b) * 1.0001
    assert np.linalg.norm(x - xref) <= 1e-9 * np.linalg.norm(xref)
    # one cycle from x0 = 0 minimises ||b - A x|| over x in M^{-1} K_m(A M^{-1}, b)
    x1, i1 = oracle.gmres(A, p.b, M, restart=restart, rtol=1e-12, maxit=restart)
    assert i1["iters"] == restart and i1["cycles"] == 1 and i1["status"] == 1
    Zs, v = [], p.b / np.linalg.norm(p.b)
    Kv = [v]
    for _ in range(restart):
        z = M.apply(Kv[-1])
        Zs.append(z)
        w = Ad @ z
        for u in Kv:                                  # orthogonalise for conditioning only
            w = w - (u @ w) * u
        Kv.append(w / np.linalg.norm(w))
    Z = np.stack(Zs, 1)
    y, *_ = np.linalg.lstsq(Ad @ Z, p.b, rcond=None)
    best = np.linalg.norm(p.b - Ad @ (Z @ y))
    got = np.linalg.norm(p.b - Ad @ x1)
    assert got <= best * (1 + 1e-8) + 1e-14 * np.linalg.norm(p.b)
    assert np.linalg.norm(x1 - Z @ y) <= 1e-8 * np.linalg.norm(Z @ y)


def test_workload_without_unit_scaling_and_storage_stalls():
    """The synthetic recipe's two readings (field-unit Darcy constant on the
    transmissibilities, storage on the non-pressure diagonal) are what make
    the Jacobian a CPR target.  Without them (tscale 1, storage 0) random
    positive 4x4 flux blocks put about a third of the spectrum in the left
    half-plane, and CPR-GMRES(30) stalls near a relative residual of 1 after
    300 steps; with them the spectrum is in the right half-plane and the
    same solves converge in a few steps."""
    w = synth.wells_vertical_pair(10, 10, 5, (0, 0), (9, 9))
    ps = synth.make(10, 10, 5, seed=37, sigma=1.0, wells=w, storage=0.0, tscale=1.0)
    pc = synth.make(10, 10, 5, seed=37, sigma=1.0, wells=w)
    evs = np.linalg.eigvals(oracle.assemble(ps).dense())
    evc = np.linalg.eigvals(oracle.assemble(pc).dense())
    assert np.mean(evs.real < 0) > 0.2 and np.all(evc.real > 0)
    nx, ny, nz = 20, 20, 10
    w = synth.wells_vertical_pair(nx, ny, nz, (5, 5), (15, 15))
    ps = synth.make(nx, ny, nz, seed=synth.SEED_BASE, sigma=1.0, kvkh=0.1, wells=w, storage=0.0, tscale=1.0)
    As, Ac = oracle.assemble(ps), oracle.assemble(synth.config(0))
    for method, smoother in ((oracle.ABF, oracle.SM_DILU), (oracle.QIMPES, oracle.SM_RAS)):
        _, i = oracle.gmres(As, ps.b, oracle.CPR(As, method=method, smoother=smoother), rtol=1e-8, maxit=300)
        assert i["status"] == 1 and i["iters"] == 300 and i["relres"] > 0.99
        _, i = oracle.gmres(Ac, synth.config(0).b, oracle.CPR(Ac, method=method, smoother=smoother), rtol=1e-8)
        assert i["status"] == 0 and i["iters"] <= 10
