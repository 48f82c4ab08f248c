"""The 400x400x200 workload (32M cells, 128M unknowns, 223M stored blocks,
28.6 GB of FP64 values): too large for the oracle's preconditioner on the
host, so it is checked by what holds at any size.

  - the Jacobian assembled on the device, solved in the configuration the
    benchmark times (values attached in place, ABF, FP32 preconditioner with
    the RAS second stage, GMRES from x0 = 0 to 1e-8);
  - the true FP64 relative residual recomputed on the host by the oracle's
    SpMV, row chunk by row chunk, from the device's values;
  - sampled rows of the library's SpMV computed one by one on the host, among
    them the rows whose value offsets (16 doubles per block) pass 2^31 and
    the last layer (offsets up to 3.57e9), from the 7-plane copy (whose
    upper slot planes also start past 2^31) and from attached values.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1812_03952_amd import rsolve as rs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def cfg3():
    p = synth.config(3)
    dp = rs.DeviceProblem(p)
    torch.cuda.synchronize()
    # the draws are not needed once the values are assembled
    dp.Mf = dp.Mb = dp.B = None
    p.Mf = p.Mb = p.B = None
    torch.cuda.empty_cache()
    rp, ci = oracle.pattern(p.nx, p.ny, p.nz)
    yield p, dp, rp, ci
    del dp
    rs.pool_trim()
    torch.cuda.empty_cache()


def _host_residual(p, dp, rp, ci, x, chunk=2_000_000):
    """||b - A x|| / ||b|| with A's values copied from the device chunk by
    chunk and multiplied by the oracle's SpMV (the full x, the chunk's rows)."""
    L = oracle.lib()
    ss = 0.0
    for c0 in range(0, p.n, chunk):
        c1 = min(p.n, c0 + chunk)
        q0, q1 = int(rp[c0]), int(rp[c1])
        v = dp.vals[16 * q0:16 * q1].cpu().numpy()
        rpc = np.ascontiguousarray(rp[c0:c1 + 1] - q0, dtype=np.int32)
        cic = np.ascontiguousarray(ci[q0:q1])
        y = np.empty(4 * (c1 - c0))
        L.or_spmv(c1 - c0, rpc, cic, v, x, y)
        r = p.b[4 * c0:4 * c1] - y
        ss += float(r @ r)
    return np.sqrt(ss) / np.linalg.norm(p.b)


def test_config3_solve_true_residual(cfg3):
    p, dp, rp, ci = cfg3
    assert p.n == 32_000_000 and rp[-1] == 223_360_000
    A = dp.bsr()
    D = rs.bsr_attach_decouple(A, dp.vals, rs.ABF, 32)
    M = rs.cpr_setup(A, D, rs.cpr_opts(smoother=rs.SM_RAS))
    x = torch.zeros_like(dp.b)
    info = rs.gmres_solve(A, M, dp.b, x, rs.gmres_opts(rtol=1e-8, zero_guess=1))
    xh = x.cpu().numpy()
    del M, D, A
    torch.cuda.empty_cache()
    true = _host_residual(p, dp, rp, ci, xh)
    print(f"400x400x200 FP32 preconditioner: iters {info['iters']}, library relres {info['relres']:.3e}, "
          f"host relres {true:.3e}")
    assert info["return"] == 0 and info["relres"] <= 1e-8
    assert true <= 1e-8 and abs(true - info["relres"]) <= 1e-10


@pytest.mark.parametrize("attach", [False, True])
def test_config3_spmv_sampled_rows(cfg3, attach):
    p, dp, rp, ci = cfg3
    A = dp.bsr()
    if attach:
        rs.bsr_attach_decouple(A, dp.vals, rs.ABF, 32)
    x = torch.randn(4 * p.n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    y = torch.empty_like(x)
    rs.spmv(A, x, y)
    torch.cuda.synchronize()
    del A
    nxy = p.nx * p.ny
    rows = list(np.random.default_rng(5).choice(p.n, size=1500, replace=False))
    c = int(np.searchsorted(16 * rp.astype(np.int64), 2 ** 31))   # first row past 2^31
    assert 0 < c < p.n and 16 * int(rp[c - 1]) < 2 ** 31 <= 16 * int(rp[c])
    rows += [c - 2, c - 1, c, c + 1]
    rows += [0, nxy - 1, p.n - nxy, p.n - 1] + list(range(p.n - 300, p.n))
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    xh = x.cpu().numpy()
    for c in rows:
        q0, q1 = int(rp[c]), int(rp[c + 1])
        blk = dp.vals[16 * q0:16 * q1].cpu().numpy().reshape(-1, 4, 4)
        acc = np.zeros(4)
        for t, q in enumerate(range(q0, q1)):
            acc += blk[t] @ xh[4 * ci[q]:4 * ci[q] + 4]
        got = y[4 * c:4 * c + 4].cpu().numpy()
        assert np.allclose(got, acc, rtol=1e-13, atol=1e-13 * np.abs(acc).max()), c
