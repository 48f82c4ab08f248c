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


# ---- overlapping RAS (overlap 1 is the paper's default) ---------------------

def _grid_ext(p, sub, m, ov):
    """Cells within grid (Manhattan) distance ov of the cells m*sub .. (m+1)*sub-1:
    on the 7-point stencil the graph distance is the Manhattan distance."""
    n = p.n
    own = np.arange(m * sub, min(n, (m + 1) * sub))
    c = np.arange(n)
    i, j, k = c % p.nx, (c // p.nx) % p.ny, c // (p.nx * p.ny)
    oi, oj, ok = own % p.nx, (own // p.nx) % p.ny, own // (p.nx * p.ny)
    d = (np.abs(i[:, None] - oi[None, :]) + np.abs(j[:, None] - oj[None, :])
         + np.abs(k[:, None] - ok[None, :])).min(axis=1)
    return np.flatnonzero(d <= ov)


def _dense_block_ilu0(Ad, nb):
    """Block ILU(0) of a dense block matrix on its own nonzero block pattern,
    written from the factorisation L U with L unit-lower (block), U upper,
    (L U)_ij = A_ij on the pattern: returns L U as a dense matrix."""
    blk = lambda a, i, j: a[4 * i:4 * i + 4, 4 * j:4 * j + 4]
    nz = np.array([[np.any(blk(Ad, i, j) != 0) for j in range(nb)] for i in range(nb)])
    L = np.eye(4 * nb)
    U = np.zeros_like(Ad)
    for i in range(nb):
        for j in range(nb):
            if not nz[i, j] and i != j:
                continue
            s = blk(Ad, i, j).copy()
            for k in range(min(i, j)):
                s -= blk(L, i, k) @ blk(U, k, j)
            if j < i:
                L[4 * i:4 * i + 4, 4 * j:4 * j + 4] = s @ np.linalg.inv(blk(U, j, j))
            else:
                U[4 * i:4 * i + 4, 4 * j:4 * j + 4] = s
    return L @ U


def _dense_ras(p, At, sub, ov):
    """sum_m R0_m^T (ILU0 of A~[E_m, E_m])^{-1} R_m as a dense operator."""
    Ad = At.dense()
    N = 4 * p.n
    Mop = np.zeros((N, N))
    for m in range((p.n + sub - 1) // sub):
        E = _grid_ext(p, sub, m, ov)
        idx = (4 * E[:, None] + np.arange(4)[None, :]).reshape(-1)
        Aloc = Ad[np.ix_(idx, idx)]
        Sloc = np.linalg.inv(_dense_block_ilu0(Aloc, E.size))
        own = (E >= m * sub) & (E < min(p.n, (m + 1) * sub))
        rows = np.repeat(own, 4)
        Mop[np.ix_(idx[rows], idx)] = Sloc[rows, :]
    return Mop


@pytest.mark.parametrize("dims,subf", [((5, 4, 3), "layer"), ((6, 5, 4), "layer"), ((6, 5, 4), "strip2"),
                                       ((7, 3, 2), "strip1"), ((1, 1, 6), "layer")])
def test_rasov_overlap0_is_zero_overlap_ras(dims, subf):
    p, A, At = _decoupled(dims)
    sub = {"layer": p.nx * p.ny, "strip2": 2 * p.nx, "strip1": p.nx}[subf]
    r = np.random.default_rng(4).standard_normal(4 * A.n)
    R = oracle.ras_restrict(At, sub=sub)
    ref = oracle.dilu_apply(R, oracle.dilu_setup(R), r)
    got = oracle.RasOv(At, sub=sub, ov=0).apply(r)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dims", [(5, 4, 3), (4, 4, 5), (3, 2, 1)])
def test_rasov_covering_overlap_is_global_dilu(dims):
    """One subdomain, or layers with an overlap reaching every layer: each
    local problem is the whole matrix, so RAS is the global DILU."""
    p, A, At = _decoupled(dims)
    r = np.random.default_rng(5).standard_normal(4 * A.n)
    ref = oracle.dilu_apply(At, oracle.dilu_setup(At), r)
    assert np.array_equal(oracle.RasOv(At, sub=A.n, ov=1).apply(r), ref)
    assert np.array_equal(oracle.RasOv(At, sub=p.nx * p.ny, ov=p.nz).apply(r), ref)


@pytest.mark.parametrize("dims,sub_lines,ov", [((5, 4, 3), 4, 1), ((6, 5, 4), 5, 1), ((6, 5, 4), 2, 1),
                                               ((5, 4, 4), 4, 2), ((4, 3, 3), 1, 1)])
def test_rasov_extensions_are_grid_neighbourhoods(dims, sub_lines, ov):
    p, A, At = _decoupled(dims)
    sub = sub_lines * p.nx
    R = oracle.RasOv(At, sub=sub, ov=ov)
    for m in range(R.nsub):
        assert np.array_equal(R.ext(m), _grid_ext(p, sub, m, ov))
    if sub_lines == p.ny and ov == 1:      # layers: the layer and its two neighbours
        nxy = p.nx * p.ny
        for m in range(p.nz):
            assert np.array_equal(R.ext(m), np.arange(max(0, m - 1) * nxy, min(p.nz, m + 2) * nxy))


@pytest.mark.parametrize("dims,sub_lines,ov", [((4, 3, 3), 3, 1), ((3, 3, 4), 3, 1), ((4, 3, 3), 1, 1),
                                               ((3, 2, 4), 2, 2)])
def test_rasov_dense_composition(dims, sub_lines, ov):
    """Against the dense operator sum_m R0_m^T (L_m U_m)^{-1} R_m with L_m U_m
    the block ILU(0) of the restricted matrix, factorised densely."""
    p, A, At = _decoupled(dims, seed=11)
    sub = sub_lines * p.nx
    R = oracle.RasOv(At, sub=sub, ov=ov)
    Mop = _dense_ras(p, At, sub, ov)
    got = np.stack([R.apply(e) for e in np.eye(4 * A.n)], 1)
    assert np.allclose(got, Mop, rtol=1e-10, atol=1e-12 * np.abs(Mop).max())


def test_rasov_owned_pivots():
    """The pivots kept for an owned cell are those of its own subdomain's
    extension: for layer subdomains with overlap 1, the middle layer of the
    three-layer DILU (the first layer of the extension for the bottom one)."""
    p, A, At = _decoupled((5, 4, 4))
    nxy = p.nx * p.ny
    R = oracle.RasOv(At, ov=1)
    own = R.owned_dinv()
    for m in range(p.nz):
        lo, hi = max(0, m - 1), min(p.nz, m + 2)
        cells = np.arange(lo * nxy, hi * nxy)
        sel = np.zeros(A.n, bool); sel[cells] = True
        keep = sel[A.ci] & np.repeat(sel, np.diff(A.rp))
        rows = np.repeat(np.arange(A.n), np.diff(A.rp))[keep]
        rp = np.concatenate([[0], np.cumsum(np.bincount(rows - lo * nxy, minlength=cells.size))]).astype(np.int32)
        sub_m = oracle.BSR(p.nx, p.ny, hi - lo, rp, (A.ci[keep] - lo * nxy).astype(np.int32), At.v[keep])
        d = oracle.dilu_setup(sub_m)
        off = (m - lo) * nxy
        assert np.array_equal(own[m * nxy:(m + 1) * nxy], d[off:off + nxy])
        assert np.array_equal(R.ext_dinv(m), d)


@pytest.mark.parametrize("stages", [2, 3])
def test_cpr_with_overlap1_ras_dense_composition(stages):
    """CPR whose full-system stage is RAS with overlap 1 over the layers, with
    a single exact pressure level: the composition of the CPR oracle's
    docstring with S the dense overlapping RAS operator."""
    p = synth.small(4, 3, 3, seed=29)
    A = oracle.assemble(p)
    M = oracle.CPR(A, smoother=oracle.SM_RAS1, stages=stages)
    assert M.amg().nlevels == 1
    n = A.n; N = 4 * n
    At = M.decoupled()
    Dt = At.dense()
    Dinv = _blockdiag(M.dinv())
    Pi_p = np.zeros((N, n)); Pi_p[np.arange(0, N, 4), np.arange(n)] = 1.0
    Cm = Pi_p @ np.linalg.solve(Dt[0::4, 0::4], Pi_p.T)
    S = _dense_ras(p, At, p.nx * p.ny, 1)
    I = np.eye(N)
    if stages == 2:
        ref = (Cm + S @ (I - Dt @ Cm)) @ Dinv
    else:
        ref = (S + (Cm + S @ (I - Dt @ Cm)) @ (I - Dt @ S)) @ Dinv
    got = np.stack([M.apply(e) for e in I], 1)
    assert np.allclose(got, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    # the pivots reported for the second stage are the owned ones
    assert np.array_equal(M.dinv2(), oracle.RasOv(At, ov=1).owned_dinv())
