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
