"""Oracle block linear algebra pinned by dense computations.

SpMV (Fig. fig-mv), block transpose, decoupling (Eqs. decoupled-eq,
decoupled-abf; GJE with row pivoting), pressure extraction, block-Jacobi and
block ILU(0).
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def prob():
    p = synth.small(4, 3, 3, seed=5, sigma=1.5)
    return p, oracle.assemble(p)


def _blockdiag(blocks):
    n = blocks.shape[0]
    D = np.zeros((4 * n, 4 * n))
    for i in range(n):
        D[4 * i:4 * i + 4, 4 * i:4 * i + 4] = blocks[i]
    return D


def _diag_blocks(A):
    out = np.zeros((A.n, 4, 4))
    for i in range(A.n):
        for p in range(A.rp[i], A.rp[i + 1]):
            if A.ci[p] == i:
                out[i] = A.v[p]
    return out


def test_spmv_dense(prob):
    p, A = prob
    x = np.random.default_rng(0).standard_normal(4 * A.n)
    D = A.dense()
    y = oracle.spmv(A, x)
    assert np.allclose(y, D @ x, rtol=1e-13, atol=1e-13 * np.abs(D).sum(1).max())


def test_transpose_dense(prob):
    _, A = prob
    assert np.array_equal(oracle.transpose(A).dense(), A.dense().T)


@pytest.mark.parametrize("method", [oracle.ABF, oracle.QIMPES, oracle.FRS, oracle.FRS_ABF])
def test_decouple_dense_and_solution_invariant(prob, method):
    p, A = prob
    At, dinv = oracle.decouple(A, method)
    D = A.dense()
    Dinv = _blockdiag(dinv)
    assert np.allclose(At.dense(), Dinv @ D, rtol=1e-10, atol=1e-10)
    x = np.linalg.solve(D, p.b)
    assert np.allclose(np.linalg.solve(At.dense(), Dinv @ p.b), x, rtol=1e-9, atol=1e-9 * np.abs(x).max())
    if method == oracle.ABF:
        # D_abf = diag(A_11..A_nn): D^{-1} is the inverse of each diagonal block, A~_ii = I
        assert np.allclose(dinv, np.linalg.inv(_diag_blocks(A)), rtol=1e-10, atol=1e-12)
        assert np.array_equal(_diag_blocks(At), np.broadcast_to(np.eye(4), (A.n, 4, 4)))


def test_frs_is_row_sum(prob):
    """FRS (Eq. decoupled-frs): D^{-1} = F, ones in row 0 and on the diagonal;
    row 0 of every block becomes the column sums, rows 1-3 are unchanged."""
    _, A = prob
    At, d = oracle.decouple(A, oracle.FRS)
    F = np.eye(4); F[0, :] = 1.0
    assert np.array_equal(d, np.broadcast_to(F, (A.n, 4, 4)))
    assert np.allclose(At.v[:, 0, :], A.v.sum(axis=1), rtol=1e-15, atol=1e-15 * np.abs(A.v).max())
    assert np.array_equal(At.v[:, 1:, :], A.v[:, 1:, :])
    # the pressure matrix of FRS holds the column-0 sums of each block
    assert np.allclose(oracle.extract_pressure(At), A.v[:, :, 0].sum(axis=1), rtol=1e-15,
                       atol=1e-15 * np.abs(A.v).max())


def test_frs_then_abf_equals_abf(prob):
    """Two-stage FRS+ABF: (F A_ii)^{-1} F A_ij = A_ii^{-1} A_ij in exact
    arithmetic, so it matches ABF to rounding, with A~_ii = I."""
    _, A = prob
    Aa, da = oracle.decouple(A, oracle.ABF)
    Af, df = oracle.decouple(A, oracle.FRS_ABF)
    scale = np.abs(Aa.v).max()
    assert np.allclose(Af.v, Aa.v, rtol=1e-11, atol=1e-12 * scale)
    assert np.allclose(df, da, rtol=1e-11, atol=1e-12 * np.abs(da).max())
    assert np.array_equal(_diag_blocks(Af), np.broadcast_to(np.eye(4), (A.n, 4, 4)))
    F = np.eye(4); F[0, :] = 1.0
    assert np.allclose(df, np.linalg.inv(_diag_blocks(A) * 0 + F @ _diag_blocks(A)) @ F, rtol=1e-10,
                       atol=1e-12 * np.abs(df).max())


def test_quasi_impes_row_equals_abf_row(prob):
    _, A = prob
    Aa, _ = oracle.decouple(A, oracle.ABF)
    Aq, dq = oracle.decouple(A, oracle.QIMPES)
    assert np.allclose(Aq.v[:, 0, :], Aa.v[:, 0, :], rtol=1e-9, atol=1e-12)
    assert np.array_equal(Aq.v[:, 1:, :], A.v[:, 1:, :])
    assert np.allclose(_diag_blocks(Aq)[:, 0, :], np.broadcast_to([1.0, 0, 0, 0], (A.n, 4)), atol=1e-12)
    assert np.array_equal(dq[:, 1:, :], np.broadcast_to(np.eye(4)[1:], (A.n, 3, 4)))


def test_gje_pivoting_on_permuted_block():
    """A diagonal block needing row exchanges (zero leading entry) is handled."""
    p = synth.make(2, 1, 1, seed=3, tscale=1.0)
    A = oracle.assemble(p)
    P = np.array([[0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0]], float)
    v = A.v.copy()
    for q in range(A.nnzb):
        v[q] = P @ v[q]
    A2 = A.with_values(v)
    At, dinv = oracle.decouple(A2)
    assert np.allclose(At.dense(), _blockdiag(dinv) @ A2.dense(), atol=1e-11)


def test_singular_block_reported():
    p = synth.small(2, 2, 1, seed=2)
    A = oracle.assemble(p)
    v = A.v.copy()
    v[A.rp[1] + 1] = 0.0          # the diagonal block of cell 1 (columns 0, 1, 3 -> slot 1)
    assert A.ci[A.rp[1] + 1] == 1
    with pytest.raises(oracle.OracleError, match="-4"):
        oracle.decouple(A.with_values(v))


def test_pressure_extraction(prob):
    _, A = prob
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    Dt = At.dense()
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    assert np.array_equal(ap, Dt[4 * rows, 4 * A.ci])


def test_block_jacobi(prob):
    _, A = prob
    Aq, _ = oracle.decouple(A, oracle.QIMPES)
    d2 = oracle.bj_setup(Aq)
    r = np.random.default_rng(1).standard_normal(4 * A.n)
    z = oracle.bj_apply(d2, r)
    assert np.allclose(_blockdiag(_diag_blocks(Aq)) @ z, r, atol=1e-10)
    Aa, _ = oracle.decouple(A, oracle.ABF)
    assert np.allclose(oracle.bj_apply(oracle.bj_setup(Aa), r), r, atol=1e-14)


@pytest.mark.parametrize("dims", [(4, 3, 3), (1, 1, 6), (5, 1, 1), (2, 3, 1)])
def test_dilu_is_block_ilu0(dims):
    """(L U)_ij = A~_ij on the block pattern with L = (D + A~_lower) D^{-1},
    U = D + A~_upper, and DILU apply = the two dense triangular solves."""
    p = synth.small(*dims, seed=8, sigma=1.0)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    d2 = oracle.dilu_setup(At)
    Dt = At.dense()
    n = A.n
    Dblk = _blockdiag(np.linalg.inv(d2))
    lower = np.zeros_like(Dt); upper = np.zeros_like(Dt)
    for i in range(n):
        for j in range(n):
            if j < i: lower[4*i:4*i+4, 4*j:4*j+4] = Dt[4*i:4*i+4, 4*j:4*j+4]
            if j > i: upper[4*i:4*i+4, 4*j:4*j+4] = Dt[4*i:4*i+4, 4*j:4*j+4]
    L = (Dblk + lower) @ _blockdiag(d2)
    U = Dblk + upper
    LU = L @ U
    mask = np.zeros_like(Dt, bool)
    rows = np.repeat(np.arange(n), np.diff(A.rp))
    for i, j in zip(rows, A.ci):
        mask[4*i:4*i+4, 4*j:4*j+4] = True
    scale = np.abs(Dt).max()
    assert np.allclose(LU[mask], Dt[mask], atol=1e-11 * scale)
    r = np.random.default_rng(2).standard_normal(4 * n)
    z = oracle.dilu_apply(At, d2, r)
    assert np.allclose(LU @ z, r, atol=1e-9 * np.abs(r).max())
