"""Oracle BiCGSTAB (right-preconditioned), pinned by an independent
implementation of the same recurrence (SciPy's), the one-half-iteration case
A = c I, the agreement of the updated and the recomputed residual, the dense
LU solution, and the closed-form (DCT) solution of the separable problem."""
import numpy as np
import pytest
import scipy.fft
import scipy.sparse.linalg as sla

import oracle
import synth


def _prob(dims, seed=53, sigma=1.5):
    return synth.make(*dims, seed=seed, sigma=sigma,
                      wells=synth.wells_vertical_pair(*dims, (0, 0), (dims[0] - 1, dims[1] - 1)))


@pytest.mark.parametrize("precond", [False, True])
def test_iterates_match_independent_implementation(precond):
    """x after k iterations equals SciPy's BiCGSTAB after k iterations (same
    recurrence; right preconditioner M^{-1} = the oracle's CPR apply, with
    block Jacobi and a multi-level AMG so that it is not exact).  Without a
    preconditioner the two drift apart by rounding as k grows (about 3e-10 at
    k = 5 on this system), far below the O(1) of a wrong term."""
    dims = (12, 10, 6) if precond else (8, 6, 4)
    p = synth.make(*dims, seed=53, sigma=2.0 if precond else 1.5, shale=0.1 if precond else 0.0,
                   wells=synth.wells_vertical_pair(*dims, (0, 0), (dims[0] - 1, dims[1] - 1)))
    A = oracle.assemble(p)
    Ad = A.dense()
    N = Ad.shape[0]
    M = oracle.CPR(A, smoother=oracle.SM_BJ, coarse_n=20) if precond else None
    Mop = sla.LinearOperator((N, N), matvec=M.apply) if precond else None
    for k in range(1, 5 if precond else 6):
        x, info = oracle.bicgstab(A, p.b, M, rtol=0.0, maxit=k)
        assert info["iters"] == k
        xs, code = sla.bicgstab(Ad, p.b, rtol=0.0, atol=0.0, maxiter=k, M=Mop)
        assert code == k
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs), k
        assert np.linalg.norm(p.b - Ad @ x) > 1e-12 * np.linalg.norm(p.b)    # not yet converged


def test_multiple_of_identity_one_half_iteration():
    """A = 4 I: v = 4 r, alpha = 1/4, s = 0 exactly, so x = b / 4 after one
    iteration that stops at s."""
    p = synth.small(3, 2, 2, seed=5)
    A = oracle.assemble(p)
    v = np.zeros_like(A.v)
    for i in range(A.n):
        for q in range(A.rp[i], A.rp[i + 1]):
            if A.ci[q] == i:
                v[q] = 4.0 * np.eye(4)
    A4 = A.with_values(v)
    x, info = oracle.bicgstab(A4, p.b, None, rtol=1e-14, maxit=5)
    assert info["status"] == 0 and info["iters"] == 1 and info["cycles"] == 1
    assert np.array_equal(x, p.b / 4.0)


def test_updated_residual_tracks_true_residual():
    """||r_k|| from the recurrence equals ||b - A x_k|| to rounding, for every
    k (x_k from a run stopped after k iterations)."""
    p = _prob((4, 3, 2), seed=59)
    A = oracle.assemble(p)
    M = oracle.CPR(A)
    _, info = oracle.bicgstab(A, p.b, M, rtol=0.0, maxit=8, hist=True)
    bn = np.linalg.norm(p.b)
    for k in range(1, 9):
        xk, _ = oracle.bicgstab(A, p.b, M, rtol=0.0, maxit=k)
        true = np.linalg.norm(p.b - oracle.spmv(A, xk)) / bn
        assert abs(info["hist"][k - 1] - true) <= 1e-10 + 1e-8 * true, k


@pytest.mark.parametrize("dims,sigma", [((4, 3, 2), 1.0), ((10, 10, 5), 1.5), ((10, 10, 5), 2.0)])
def test_cpr_bicgstab_vs_dense_lu(dims, sigma):
    p = synth.make(*dims, seed=61, sigma=sigma, shale=0.1 if sigma == 2.0 else 0.0,
                   wells=synth.wells_vertical_pair(*dims, (0, 0), (dims[0] - 1, dims[1] - 1)))
    A = oracle.assemble(p)
    Ad = A.dense()
    xref = np.linalg.solve(Ad, p.b)
    cond = np.linalg.cond(Ad)
    for method, smoother in ((oracle.ABF, oracle.SM_DILU), (oracle.QIMPES, oracle.SM_BJ),
                             (oracle.ABF, oracle.SM_RAS)):
        M = oracle.CPR(A, method=method, smoother=smoother, coarse_n=20)
        x, info = oracle.bicgstab(A, p.b, M, rtol=1e-12, maxit=200)
        assert info["status"] == 0 and info["relres"] <= 1e-12
        assert np.linalg.norm(p.b - Ad @ x) <= 1.0001e-12 * np.linalg.norm(p.b)
        assert np.linalg.norm(x - xref) <= max(1e-12 * cond, 1e-10) * np.linalg.norm(xref)


def test_bicgstab_dct_closed_form():
    """The separable problem of the GMRES closed-form test, solved by
    CPR-BiCGSTAB, against its DCT-II solution."""
    nx, ny, nz = 16, 12, 10
    a, kk = 2.0, 100.0
    p = synth.make(nx, ny, nz, seed=41, sigma=0.0, kvkh=1.0, tscale=1.0)
    p.logk[:] = np.log(kk)
    p.Mf[:] = np.eye(4); p.Mb[:] = np.eye(4); p.B[:] = a * np.eye(4)
    A = oracle.assemble(p)
    x, info = oracle.bicgstab(A, p.b, oracle.CPR(A), rtol=1e-12, maxit=300)
    assert info["status"] == 0
    lam = lambda m: 2.0 - 2.0 * np.cos(np.pi * np.arange(m) / m)
    ev = a + kk * (lam(nz)[:, None, None] + lam(ny)[None, :, None] + lam(nx)[None, None, :])
    B = p.b.reshape(nz, ny, nx, 4)
    X = np.empty_like(B)
    for u in range(4):
        X[..., u] = scipy.fft.idctn(scipy.fft.dctn(B[..., u], type=2, norm="ortho") / ev, type=2, norm="ortho")
    assert np.linalg.norm(x - X.reshape(-1)) <= 1e-10 * np.linalg.norm(X)


def test_bicgstab_status_paths():
    p = synth.small(5, 4, 3, seed=43)
    A = oracle.assemble(p)
    M = oracle.CPR(A)
    _, info = oracle.bicgstab(A, p.b, M, rtol=1e-15, maxit=1)
    assert info["status"] == 1 and info["iters"] == 1
    x, info = oracle.bicgstab(A, np.zeros(4 * A.n), M)
    assert info["status"] == 0 and info["iters"] == 0 and not x.any()
    b = p.b.copy(); b[3] = np.nan
    with pytest.raises(oracle.OracleError, match="-5"):
        oracle.bicgstab(A, b, M)
    # a start from the exact solution needs no iteration
    xe = np.linalg.solve(A.dense(), p.b)
    x, info = oracle.bicgstab(A, p.b, M, x0=xe, rtol=1e-8)
    assert info["status"] == 0 and info["iters"] == 0
