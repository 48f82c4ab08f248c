"""Zero-overlap restricted additive Schwarz with block ILU(0) (DILU) in each
xy-layer subdomain: pinned by the block-Jacobi structure (each layer solved on
its own extracted matrix), the ILU(0) identity on the restricted pattern,
the global DILU when one subdomain holds every cell, and the CPR composition
(parametrised in test_oracle_solve)."""
import numpy as np
import pytest

import oracle
import synth


def _blockdiag(blocks):
    n = blocks.shape[0]
    D = np.zeros((4 * n, 4 * n))
    for i in range(n):
        D[4 * i:4 * i + 4, 4 * i:4 * i + 4] = blocks[i]
    return D


def _decoupled(dims, seed=3):
    p = synth.small(*dims, seed=seed, sigma=1.5)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    return p, A, At


def test_restriction_drops_exactly_the_z_couplings():
    p, A, At = _decoupled((5, 4, 3))
    R = oracle.ras_restrict(At)
    nxy = p.nx * p.ny
    assert R.nnzb == A.nnzb - 2 * nxy * (p.nz - 1)
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    dropped = np.abs(A.ci - rows) == nxy
    kept_rows = np.repeat(np.arange(A.n), np.diff(R.rp))
    assert np.array_equal(R.ci, A.ci[~dropped]) and np.array_equal(kept_rows, rows[~dropped])
    assert np.array_equal(R.v, At.v[~dropped])


def test_each_layer_is_its_own_dilu():
    """Block Jacobi over layers: the factors and the solve of each layer equal
    the DILU of that layer's matrix taken alone as an nx x ny x 1 system."""
    p, A, At = _decoupled((4, 3, 3))
    nxy = p.nx * p.ny
    R = oracle.ras_restrict(At)
    d2 = oracle.dilu_setup(R)
    r = np.random.default_rng(5).standard_normal(4 * A.n)
    z = oracle.dilu_apply(R, d2, r)
    Dt = At.dense()
    rp2, ci2 = oracle.pattern(p.nx, p.ny, 1)
    rows2 = np.repeat(np.arange(nxy), np.diff(rp2))
    for k in range(p.nz):
        sl = slice(4 * nxy * k, 4 * nxy * (k + 1))
        Dk = Dt[sl, sl]
        v = np.stack([Dk[4 * i:4 * i + 4, 4 * j:4 * j + 4] for i, j in zip(rows2, ci2)])
        Ak = oracle.BSR(p.nx, p.ny, 1, rp2, ci2, v)
        dk = oracle.dilu_setup(Ak)
        assert np.array_equal(dk, d2[nxy * k:nxy * (k + 1)])
        zk = oracle.dilu_apply(Ak, dk, r[sl])
        assert np.array_equal(zk, z[sl])


def test_layer_local_response():
    """A right-hand side supported in one layer gives a solution in that layer only."""
    p, A, At = _decoupled((3, 3, 4))
    nxy = p.nx * p.ny
    R = oracle.ras_restrict(At)
    d2 = oracle.dilu_setup(R)
    r = np.zeros(4 * A.n)
    r[4 * nxy * 2:4 * nxy * 3] = np.random.default_rng(6).standard_normal(4 * nxy)
    z = oracle.dilu_apply(R, d2, r)
    assert np.all(z[:4 * nxy * 2] == 0) and np.all(z[4 * nxy * 3:] == 0)
    assert np.any(z[4 * nxy * 2:4 * nxy * 3] != 0)


@pytest.mark.parametrize("dims", [(4, 3, 3), (5, 1, 2), (1, 1, 4)])
def test_ras_ilu0_identity(dims):
    """(D+L) D^{-1} (D+U) agrees with the restricted matrix on its pattern and
    has no block between different layers."""
    p, A, At = _decoupled(dims, seed=11)
    R = oracle.ras_restrict(At)
    d2 = oracle.dilu_setup(R)
    n = A.n
    Rd = R.dense()
    lower = np.zeros_like(Rd); upper = np.zeros_like(Rd)
    for i in range(n):
        for j in range(n):
            if j < i: lower[4*i:4*i+4, 4*j:4*j+4] = Rd[4*i:4*i+4, 4*j:4*j+4]
            if j > i: upper[4*i:4*i+4, 4*j:4*j+4] = Rd[4*i:4*i+4, 4*j:4*j+4]
    Dblk = _blockdiag(np.linalg.inv(d2))
    LU = (Dblk + lower) @ _blockdiag(d2) @ (Dblk + upper)
    rows = np.repeat(np.arange(n), np.diff(R.rp))
    mask = np.zeros_like(Rd, bool)
    for i, j in zip(rows, R.ci):
        mask[4*i:4*i+4, 4*j:4*j+4] = True
    assert np.allclose(LU[mask], Rd[mask], atol=1e-11 * np.abs(Rd).max())
    nxy = p.nx * p.ny
    layer = np.repeat(np.arange(n) // nxy, 4)
    assert np.all(LU[layer[:, None] != layer[None, :]] == 0)


def test_one_subdomain_is_global_dilu():
    p, A, At = _decoupled((4, 3, 3))
    Mr = oracle.CPR(A, smoother=oracle.SM_RAS, sub=A.n)
    Md = oracle.CPR(A, smoother=oracle.SM_DILU)
    assert np.array_equal(Mr.dinv2(), Md.dinv2())
    r = np.random.default_rng(7).standard_normal(4 * A.n)
    assert np.array_equal(Mr.apply(r), Md.apply(r))


def test_single_layer_grid_equals_dilu():
    p, A, At = _decoupled((5, 4, 1))
    Mr = oracle.CPR(A, smoother=oracle.SM_RAS)
    Md = oracle.CPR(A, smoother=oracle.SM_DILU)
    r = np.random.default_rng(8).standard_normal(4 * A.n)
    assert np.array_equal(Mr.apply(r), Md.apply(r))
