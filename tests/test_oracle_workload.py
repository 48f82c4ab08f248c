"""The reading of the synthetic workload, pinned on the oracle.

The paper's thermal Jacobians are not available, so the inputs are seeded
draws.  Two constants of the recipe are readings of their own: the
field-unit transmissibility constant (1.127e-3) and a storage term of 1000 on
the non-pressure unknowns.  These tests record why: without them (unit
transmissibility, no storage term) random positive 4x4 flux blocks make the
system indefinite enough that CPR-GMRES(30) makes no progress in 300
iterations, while with them it converges in a few, and the matrices are
well conditioned (so a 1e-8 residual fixes the solution far below 1e-6)."""
import numpy as np
import pytest

import oracle
import synth


def _cfg0(**kw):
    nx, ny, nz = 20, 20, 10
    return synth.make(nx, ny, nz, seed=synth.SEED_BASE, sigma=1.0, kvkh=0.1,
                      wells=synth.wells_vertical_pair(nx, ny, nz, (5, 5), (15, 15)), **kw)


@pytest.mark.parametrize("smoother", [oracle.SM_DILU, oracle.SM_RAS])
def test_unit_recipe_stalls(smoother):
    """tscale 1, storage 0: GMRES(30) with ABF + CPR stays at a relative
    residual above 0.99 after 300 iterations."""
    p = _cfg0(storage=0.0, tscale=1.0)
    A = oracle.assemble(p)
    M = oracle.CPR(A, method=oracle.ABF, smoother=smoother)
    _, info = oracle.gmres(A, p.b, M, rtol=1e-8, maxit=300)
    assert info["status"] != 0 and info["iters"] == 300
    assert info["relres"] > 0.99


@pytest.mark.parametrize("smoother", [oracle.SM_DILU, oracle.SM_RAS])
def test_committed_recipe_converges(smoother):
    """The committed recipe (config 0 exactly): converged to 1e-8 within one
    restart cycle, and the true residual agrees."""
    p = synth.config(0)
    A = oracle.assemble(p)
    M = oracle.CPR(A, method=oracle.ABF, smoother=smoother)
    x, info = oracle.gmres(A, p.b, M, rtol=1e-8, maxit=300)
    assert info["status"] == 0 and info["cycles"] == 1 and info["iters"] <= 10
    res = np.linalg.norm(p.b - oracle.spmv(A, x)) / np.linalg.norm(p.b)
    assert res <= 1e-8


def _small(sigma, shale, **kw):
    return synth.make(10, 10, 5, seed=synth.SEED_BASE, sigma=sigma, kvkh=0.1, shale=shale,
                      wells=synth.wells_vertical_pair(10, 10, 5, (2, 2), (7, 7)), **kw)


@pytest.mark.parametrize("sigma,shale", [(1.0, 0.0), (2.0, 0.1)])
def test_condition_numbers(sigma, shale):
    """2-norm condition numbers at 10x10x5: about 8e2 with the committed
    constants, above 1e5 with the unit recipe.  With kappa below 1e4 a
    relative residual of 1e-8 bounds the relative error by 1e-4 at worst, and
    the measured error of a 1e-8 solve is far below the 1e-6 target."""
    A = oracle.assemble(_small(sigma, shale))
    kappa = np.linalg.cond(A.dense())
    assert 1e2 < kappa < 1e4, kappa
    A_unit = oracle.assemble(_small(sigma, shale, storage=0.0, tscale=1.0))
    assert np.linalg.cond(A_unit.dense()) > 1e5


def test_residual_1e8_fixes_solution():
    """On config 0, the rtol-1e-8 solve is within 1e-9 (relative) of the
    rtol-1e-13 solve."""
    p = synth.config(0)
    A = oracle.assemble(p)
    M = oracle.CPR(A, method=oracle.ABF, smoother=oracle.SM_DILU)
    x8, _ = oracle.gmres(A, p.b, M, rtol=1e-8)
    x13, _ = oracle.gmres(A, p.b, M, rtol=1e-13)
    err = np.linalg.norm(x8 - x13) / np.linalg.norm(x13)
    assert err <= 1e-9, err
