"""Attached values (rs_bsr_attach_decouple): the library reads the caller's
CSR blocks in place.  Every result must be bitwise equal to the copying
path (rs_bsr_update_decouple), which the other parity tests pin to the
oracle: the decoupled arrays, the SpMV, a whole CPR-GMRES solve and the
adjoint solve, on grids with every kind of boundary row."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, upload
from paper_1812_03952_amd import rsolve as rs

pytestmark = pytest.mark.gpu

GRIDS = [(1, 1, 1), (1, 1, 7), (6, 1, 1), (1, 5, 1), (5, 3, 4), (20, 20, 10), (33, 17, 9)]


def _prob(dims, seed=3, **kw):
    nx, ny, nz = dims
    w = synth.wells_vertical_pair(nx, ny, nz, (0, 0), (nx - 1, ny - 1)) if nx * ny > 1 else None
    return synth.make(nx, ny, nz, seed=seed, wells=w, **kw)


def _new_values(A):
    v2 = A.v * 1.0
    v2[:, 0, :] *= 1.25                             # new values on the same pattern
    return v2.reshape(-1)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("method", [rs.ABF, rs.QIMPES, rs.FRS, rs.FRS_ABF])
@pytest.mark.parametrize("dims", GRIDS)
def test_attach_equals_copy(dims, method, prec):
    A = oracle.assemble(_prob(dims, sigma=1.5))
    v2 = _new_values(A)
    B1, B2 = upload(A), upload(A)
    D1 = rs.bsr_update_decouple(B1, dev(v2), method, prec)
    D2 = rs.bsr_attach_decouple(B2, dev(v2), method, prec)
    for a, b in zip(rs.dcpl_get(D1), rs.dcpl_get(D2)):
        assert np.array_equal(a, b)
    # rs_decouple on the attached values
    for a, b in zip(rs.dcpl_get(D1), rs.dcpl_get(rs.decouple(B2, method, prec))):
        assert np.array_equal(a, b)
    x = dev(np.random.default_rng(3).standard_normal(4 * A.n))
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    rs.spmv(B1, x, y1)
    rs.spmv(B2, x, y2)
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("solver", ["gmres", "bicgstab"])
@pytest.mark.parametrize("dims", [(20, 20, 10), (33, 17, 9)])
def test_attach_solve_bitwise(dims, solver):
    """A whole solve (FP32 RAS preconditioner, x0 = 0) on attached values
    equals the one on copied values, bit for bit, with the same count."""
    p = _prob(dims, sigma=2.0, shale=0.1)
    A = oracle.assemble(p)
    v2 = _new_values(A)
    b = dev(p.b)
    out = []
    for attach in (False, True):
        B = upload(A)
        f = rs.bsr_attach_decouple if attach else rs.bsr_update_decouple
        D = f(B, dev(v2), rs.ABF, 32)
        M = rs.cpr_setup(B, D, rs.cpr_opts(smoother=rs.SM_RAS))
        x = torch.zeros_like(b)
        if solver == "gmres":
            info = rs.gmres_solve(B, M, b, x, rs.gmres_opts(rtol=1e-10, zero_guess=1))
        else:
            info = rs.bicgstab_solve(B, M, b, x, rs.bicgstab_opts(rtol=1e-10, zero_guess=1))
        assert info["return"] == 0
        out.append((x, info["iters"], info["relres"]))
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]


def test_attach_adjoint_bitwise():
    """The transpose behind rs_adjoint_solve reads attached values in place."""
    p = _prob((12, 10, 6), sigma=1.5)
    A = oracle.assemble(p)
    v2 = _new_values(A)
    w = dev(p.w)
    o = rs.gmres_opts(rtol=1e-12, maxit=600)
    lams = []
    for attach in (False, True):
        B = upload(A)
        (rs.bsr_attach_decouple if attach else rs.bsr_update_decouple)(B, dev(v2), rs.ABF, 64)
        lam = torch.zeros_like(w)
        info = rs.adjoint_solve(B, w, lam, opts=o)
        assert info["return"] == 0
        lams.append(lam)
    assert torch.equal(lams[0], lams[1])


def test_attach_reads_in_place_until_update():
    """While attached, A reads the caller's buffer (a change to it shows in
    the SpMV); rs_bsr_update brings A back to its own copy."""
    A = oracle.assemble(_prob((9, 7, 5), sigma=1.5))
    v2 = _new_values(A)
    B = upload(A)
    vals = dev(v2)
    rs.bsr_attach_decouple(B, vals, rs.ABF, 64)
    assert B.attached and B.attached[0] is vals
    x = dev(np.random.default_rng(4).standard_normal(4 * A.n))
    y = torch.empty_like(x)
    vals.mul_(2.0)                                  # exact: every product doubles
    rs.spmv(B, x, y)
    assert np.array_equal(y.cpu().numpy(), 2.0 * _spmv_copied(B, A, v2, x))
    # back to a copy: later changes to the buffer no longer show
    rs.bsr_update(B, vals)
    assert B.attached == []
    rs.spmv(B, x, y)
    y_before = y.clone()
    vals.zero_()
    rs.spmv(B, x, y)
    assert torch.equal(y, y_before)


def _spmv_copied(B, A, v, x):
    """A x for values v through a copying handle (the reference for the
    in-place test)."""
    C = upload(A)
    rs.bsr_update(C, dev(v))
    y = torch.empty_like(x)
    rs.spmv(C, x, y)
    return y.cpu().numpy()


def test_attach_errors():
    A = oracle.assemble(_prob((5, 3, 4), sigma=1.5))
    v2 = _new_values(A)
    B = upload(A)
    good = dev(v2)
    rs.bsr_attach_decouple(B, good, rs.ABF, 64)
    x = dev(np.random.default_rng(5).standard_normal(4 * A.n))
    y0, y = torch.empty_like(x), torch.empty_like(x)
    rs.spmv(B, x, y0)
    # misaligned values: RS_E_ARG, and A still reads the buffer attached before
    buf = torch.zeros(good.numel() + 1, dtype=torch.float64, device="cuda")
    buf[1:] = good
    with pytest.raises(rs.RsError) as e:
        rs.bsr_attach_decouple(B, buf[1:], rs.ABF, 64)
    assert e.value.status == -1
    rs.spmv(B, x, y)
    assert torch.equal(y, y0)
    # non-finite values: RS_E_NONFINITE, and A refers to them
    bad = good.clone()
    bad[17] = float("inf")
    with pytest.raises(rs.RsError) as e:
        rs.bsr_attach_decouple(B, bad, rs.ABF, 64)
    assert e.value.status == -5
    assert B.attached[-1] is bad
    # a singular diagonal block: RS_E_SINGULAR
    sing = v2.reshape(-1, 4, 4).copy()
    sing[0] = 0.0                                   # cell 0's first block is its diagonal
    with pytest.raises(rs.RsError) as e:
        rs.bsr_attach_decouple(B, dev(sing.reshape(-1)), rs.ABF, 64)
    assert e.value.status == -4
