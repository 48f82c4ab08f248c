"""Oracle Jacobian assembly pinned by invariants and a hand-computed case.

Section "Numerical Methods" (transmissibility): harmonic mean of the
geometric part, one value shared by the two cells of a face, zero on
boundary faces; Eq. mat-ja: cell-by-cell block numbering.
"""
import numpy as np
import pytest

import oracle
import synth


def _faces(nx, ny, nz):
    n = nx * ny * nz
    for c in range(n):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        if i < nx - 1: yield c, c + 1, 0
        if j < ny - 1: yield c, c + nx, 1
        if k < nz - 1: yield c, c + nx * ny, 2


def _block(A, i, j):
    for p in range(A.rp[i], A.rp[i + 1]):
        if A.ci[p] == j:
            return A.v[p]
    return None


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 1, 1), (1, 4, 1), (1, 1, 5), (3, 4, 2), (5, 3, 4)])
def test_pattern_is_grid_adjacency(dims):
    nx, ny, nz = dims
    rp, ci = oracle.pattern(nx, ny, nz)
    n = nx * ny * nz
    assert rp[-1] == synth.grid_nnzb(nx, ny, nz)
    coords = np.stack(np.unravel_index(np.arange(n), (nz, ny, nx)), 1)
    for c in range(n):
        cols = ci[rp[c]:rp[c + 1]]
        assert np.all(np.diff(cols) > 0)
        expect = [d for d in range(n) if np.abs(coords[d] - coords[c]).sum() <= 1]
        assert list(cols) == expect


def test_transmissibility_symmetric_and_rowsum():
    p = synth.small(5, 4, 3, seed=21, sigma=1.5)
    A = oracle.assemble(p)
    n = p.n
    T = {}
    for a, b, d in _faces(p.nx, p.ny, p.nz):
        Tab = -_block(A, a, b) / p.Mf[d, a]
        Tba = -_block(A, b, a) / p.Mb[d, a]
        # one T per face, recovered identically from both rows
        assert np.allclose(Tab, Tab[0, 0], rtol=1e-14)
        assert np.allclose(Tba, Tab[0, 0], rtol=1e-14)
        T[(a, b)] = Tab[0, 0]
    # diagonal block = accumulation + wells - sum of off-diagonal blocks
    W = np.zeros(n); W[p.well_cell] = p.well_u * np.exp(p.logk[p.well_cell])
    for c in range(n):
        s = sum(A.v[q] for q in range(A.rp[c], A.rp[c + 1]))
        assert np.allclose(s, p.B[c] / p.dt + W[c] * np.eye(4), rtol=1e-12, atol=1e-12 * np.abs(A.v[A.rp[c]:A.rp[c + 1]]).max())
    # every face of the grid has a T, and only those
    assert len(T) == (A.nnzb - n) // 2


def test_two_cell_hand_example():
    """Two cells along x, k = (1, 3) (tscale 1): T = 2*1*3/(1+3) = 1.5."""
    p = synth.make(2, 1, 1, seed=1, sigma=0.0, tscale=1.0)
    p.logk[:] = np.log([1.0, 3.0])
    p.Mf[:] = 0.0; p.Mb[:] = 0.0
    p.Mf[0, 0] = np.full((4, 4), 0.5)
    p.Mb[0, 0] = np.arange(16).reshape(4, 4) / 16.0
    p.B[:] = 2.0 * np.eye(4)
    p.dt = 4.0
    A = oracle.assemble(p)
    T = 1.5
    assert np.allclose(_block(A, 0, 1), -T * 0.5)
    assert np.allclose(_block(A, 1, 0), -T * np.arange(16).reshape(4, 4) / 16.0)
    assert np.allclose(_block(A, 0, 0), 0.5 * np.eye(4) + T * 0.5)
    assert np.allclose(_block(A, 1, 1), 0.5 * np.eye(4) + T * np.arange(16).reshape(4, 4) / 16.0)


def test_vertical_anisotropy_and_wells():
    p = synth.make(1, 1, 2, seed=2, sigma=0.0, kvkh=0.25, tscale=1.0,
                   wells=(np.array([1], np.int32), np.array([-1], np.int8)))
    p.logk[:] = np.log(8.0)
    A = oracle.assemble(p)
    Tz = 0.25 * 8.0            # harmonic mean of equal vertical permeabilities
    assert np.allclose(_block(A, 0, 1), -Tz * p.Mf[2, 0], rtol=1e-14)
    W = p.well_u[0] * 8.0
    assert np.allclose(_block(A, 1, 1), p.B[1] + Tz * p.Mb[2, 0] + W * np.eye(4), rtol=1e-13)
