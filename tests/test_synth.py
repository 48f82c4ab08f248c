"""Synthetic input generator: reproducibility and recipe properties."""
import numpy as np

import synth


def test_reproducible_and_seeded():
    a = synth.small(5, 4, 3, seed=11)
    b = synth.small(5, 4, 3, seed=11)
    c = synth.small(5, 4, 3, seed=12)
    for f in ("logk", "Mf", "Mb", "B", "b", "w", "well_u"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert not np.array_equal(a.Mf, c.Mf)


def test_recipe_ranges():
    p = synth.small(6, 5, 4, seed=3)
    assert p.Mf.shape == (3, p.n, 4, 4) and p.Mb.shape == (3, p.n, 4, 4)
    assert p.Mf.min() >= 0.1 and p.Mf.max() <= 1.0
    assert p.Mb.min() >= 0.1 and p.Mb.max() <= 1.0
    # accumulation: row diagonally dominant, storage on the non-pressure diagonal
    off = p.B.copy()
    for q in range(4):
        off[:, q, q] = 0.0
    diag = np.einsum("nii->ni", p.B)
    assert np.all(diag > off.sum(axis=2))
    assert np.all(diag[:, 1:] > synth.STORAGE)
    assert np.all(diag[:, 0] < 4.0)
    assert p.tscale == synth.DARCY


def test_shale_fraction_and_value():
    p = synth.make(10, 10, 10, seed=4, sigma=2.0, shale=0.1)
    shale = np.isclose(p.logk, np.log(1e-3))
    assert shale.sum() == 100


def test_config_well_layouts():
    p0 = synth.config(0)
    assert p0.n == 4000 and p0.nnzb == 26400
    assert p0.well_cell.shape[0] == 20 and (p0.well_kind < 0).sum() == 10
    # objective weights only on producer cells
    w = p0.w.reshape(-1, 4)
    prod = p0.well_cell[p0.well_kind < 0]
    assert np.all(w[prod] > 0.0)
    mask = np.ones(p0.n, bool); mask[prod] = False
    assert np.all(w[mask] == 0.0)


def test_threaded_uniform_fill_is_the_sequential_stream():
    """The slice-wise threaded fill gives exactly Generator.uniform's draws,
    for slices that divide the array and for a ragged last slice."""
    for shape, sl in (((3, 50, 4, 4), 64), ((7, 4, 4), 12), ((1000,), 4), ((10,), 1 << 24)):
        ref = synth._rng(99, 3).uniform(0.1, 1.0, size=shape)
        got = synth._uniform(99, 3, 0.1, 1.0, shape, slice_len=sl)
        assert np.array_equal(got, ref), (shape, sl)
    ref = synth._rng(5, 4).uniform(0.0, 1.0, size=(9, 4, 4))
    assert np.array_equal(synth._uniform(5, 4, 0.0, 1.0, (9, 4, 4), slice_len=8), ref)


def test_draws_unchanged():
    """The bench workloads' draws are those of the sequential generator (the
    first entries of the 20x20x10 workload, written from Generator.uniform)."""
    p = synth.config(0)
    s = synth.SEED_BASE
    assert np.array_equal(p.Mf, synth._rng(s, 2).uniform(0.1, 1.0, size=(3, p.n, 4, 4)))
    assert np.array_equal(p.Mb, synth._rng(s, 3).uniform(0.1, 1.0, size=(3, p.n, 4, 4)))
