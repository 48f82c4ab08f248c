"""Seeded synthetic inputs for the CPR-GMRES solve.

This module only draws random numbers and lays them out.  It holds none of
the solver's arithmetic: transmissibilities, the Jacobian, its decoupling and
everything after are computed separately by the FP64 reference in `oracle/`
and by the HIP library in `paper_1812_03952_amd/`, which both take these
draws as input.

The draws stand in for the Jacobian of the paper's thermal model (four
unknowns per grid block: p, N_w, N_o, T), which needs model files that are
not available.  The recipe follows the paper's description of the linear
system (Section "Linear Solver", Eq. mat-ja: block rows numbered cell by
cell) and of transmissibility (Section "Numerical Methods": harmonic mean of
the geometric part, zero on no-flow boundary faces):

* log-permeability  theta_c = ln(100) + sigma * N(0,1), i.i.d. per cell;
  a shale fraction of cells (chosen without replacement) is set to
  k = 1e-3.  Vertical permeability is kv/kh times the horizontal one.
* For every cell c and axis d in (x, y, z), two independent 4x4 blocks
  Mf[d, c], Mb[d, c] with entries U[0.1, 1]: Mf couples row c to its +d
  neighbour, Mb couples the +d neighbour's row back to c.  Entries for
  cells on the +d boundary are drawn but unused.
* Face transmissibility is the harmonic mean of the two cells' directional
  permeabilities times DARCY = 1.127e-3, the field-unit constant taking
  mD * ft to bbl/(day psi cp), with unit geometry (A/dd = 1 ft); the
  paper's examples are in field units.  The constant is passed to the
  assembly as `tscale`.
* Accumulation block B_c: off-diagonal entries U[0, 1), diagonal entries
  1 + (sum of the row's off-diagonal entries), i.e. row diagonally dominant,
  plus a storage term STORAGE = 1000 on the diagonal of the three
  non-pressure unknowns (N_w, N_o, T): mass and heat storage per day
  dominate their flux derivatives, while the pressure column only carries
  the O(1) compressibility-like part.  (Without this split, random positive
  4x4 flux blocks make a quarter or more of the spectrum indefinite and no
  CPR variant converges; the measurements are recorded with the design.)
* Wells: perforated cells get a source coefficient u_c = DARCY * U[1, 10]
  (multiplied by the cell's own permeability when assembled).
* Right-hand side b ~ N(0, 1) per unknown; objective weights w ~ U[0, 1]
  on all four unknowns of producer cells, zero elsewhere.

Cell numbering is c = i + nx*(j + ny*k), 0-based, i fastest.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os

import numpy as np

SEED_BASE = 1812039520
DARCY = 1.127e-3      # field-unit transmissibility constant, mD*ft -> bbl/(day psi cp)
STORAGE = 1000.0      # storage coefficient of N_w, N_o, T per unit time

# purpose ids: each kind of draw has its own stream so that changing one
# size never shifts another draw
_P_LOGK, _P_SHALE, _P_MF, _P_MB, _P_B, _P_WELL, _P_RHS, _P_OBJ = range(8)


def _rng(seed: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed & 0xFFFFFFFFFFFFFFFF, purpose]))


_SLICE = 1 << 24          # doubles per slice of a threaded uniform fill (multiple of 4)


def _uniform(seed: int, purpose: int, low: float, high: float, shape, slice_len: int = _SLICE) -> np.ndarray:
    """The draws of _rng(seed, purpose).uniform(low, high, shape), bitwise,
    filled slice by slice on a thread pool (numpy fills without the GIL).
    Slice k starts at draw k * slice_len: a fresh Philox advanced by
    slice_len / 4 counter blocks per slice, since one block gives four 64-bit
    words and a double takes one.  uniform() is low + (high - low) * u, which
    the slice computes as u * (high - low) + low, the same two roundings."""
    assert slice_len % 4 == 0
    out = np.empty(shape)
    flat = out.reshape(-1)
    width = high - low

    def fill(off):
        bg = np.random.Philox(key=[seed & 0xFFFFFFFFFFFFFFFF, purpose])
        bg.advance(off // 4)
        seg = flat[off:off + slice_len]
        np.random.Generator(bg).random(out=seg)
        seg *= width
        seg += low

    offs = list(range(0, flat.size, slice_len))
    if len(offs) <= 1:
        for off in offs:
            fill(off)
    else:
        with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(fill, offs))
    return out


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    logk: np.ndarray          # (n,) float64, log of horizontal permeability
    kvkh: float               # vertical / horizontal permeability ratio
    tscale: float             # transmissibility constant multiplying the harmonic mean
    Mf: np.ndarray            # (3, n, 4, 4) float64
    Mb: np.ndarray            # (3, n, 4, 4) float64
    B: np.ndarray             # (n, 4, 4) float64 accumulation block
    dt: float
    well_cell: np.ndarray     # (nw,) int32, sorted ascending
    well_u: np.ndarray        # (nw,) float64
    well_kind: np.ndarray     # (nw,) int8: +1 injector, -1 producer
    b: np.ndarray             # (4n,) float64 right-hand side
    w: np.ndarray             # (4n,) float64 objective weights
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nnzb(self) -> int:
        return grid_nnzb(self.nx, self.ny, self.nz)


def grid_nnzb(nx: int, ny: int, nz: int) -> int:
    """Stored 4x4 blocks of the 7-point pattern: diagonal plus two per interior face."""
    n = nx * ny * nz
    faces = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    return n + 2 * faces


def cell_index(nx, ny, i, j, k):
    return i + nx * (j + ny * k)


def _wells_pairs(nx, ny, nz, pairs):
    """pairs: list of (injector cells, producer cells) as lists of (i,j,k)."""
    cells, kinds = [], []
    for inj, prod in pairs:
        for (i, j, k) in inj:
            cells.append(cell_index(nx, ny, i, j, k)); kinds.append(1)
        for (i, j, k) in prod:
            cells.append(cell_index(nx, ny, i, j, k)); kinds.append(-1)
    cells = np.asarray(cells, dtype=np.int64)
    kinds = np.asarray(kinds, dtype=np.int8)
    cells, first = np.unique(cells, return_index=True)   # a cell perforated twice counts once
    return cells.astype(np.int32), kinds[first]


def wells_vertical_pair(nx, ny, nz, inj_ij, prod_ij):
    inj = [(inj_ij[0], inj_ij[1], k) for k in range(nz)]
    prod = [(prod_ij[0], prod_ij[1], k) for k in range(nz)]
    return _wells_pairs(nx, ny, nz, [(inj, prod)])


def wells_vertical_grid(nx, ny, nz, na, nb, dx=6):
    """na x nb vertical pairs on a regular areal grid; injector dx cells
    before the pattern centre along x, producer dx cells after it."""
    pairs = []
    sa, sb = nx // na, ny // nb
    for a in range(na):
        for b_ in range(nb):
            ci = sa // 2 + sa * a
            cj = sb // 2 + sb * b_
            ii = max(0, min(nx - 1, ci - dx)); ip = max(0, min(nx - 1, ci + dx))
            pairs.append(([(ii, cj, k) for k in range(nz)], [(ip, cj, k) for k in range(nz)]))
    return _wells_pairs(nx, ny, nz, pairs)


def wells_horizontal(nx, ny, nz, js, ks_inj, dk):
    """Horizontal pairs along x (all i): injector at (j, k_inj), producer dk
    cells further along z, as in the SAGD layouts of the paper's examples."""
    pairs = []
    for j in js:
        for ki in ks_inj:
            kp = ki + dk
            if not (0 <= j < ny and 0 <= ki < nz and 0 <= kp < nz):
                continue
            pairs.append(([(i, j, ki) for i in range(nx)], [(i, j, kp) for i in range(nx)]))
    return _wells_pairs(nx, ny, nz, pairs)


def make(nx, ny, nz, *, seed, sigma=1.0, kvkh=0.1, shale=0.0, wells=None, dt=1.0,
         storage=STORAGE, tscale=DARCY, name="") -> Problem:
    """Draw one synthetic problem.  `wells` is (cells, kinds) or None."""
    n = nx * ny * nz
    logk = math.log(100.0) + sigma * _rng(seed, _P_LOGK).standard_normal(n)
    if shale > 0.0:
        ns = int(round(shale * n))
        idx = _rng(seed, _P_SHALE).choice(n, size=ns, replace=False)
        logk[idx] = math.log(1e-3)
    Mf = _uniform(seed, _P_MF, 0.1, 1.0, (3, n, 4, 4))
    Mb = _uniform(seed, _P_MB, 0.1, 1.0, (3, n, 4, 4))
    B = _uniform(seed, _P_B, 0.0, 1.0, (n, 4, 4))
    eye = np.eye(4, dtype=bool)
    B[:, eye] = 0.0
    B[:, eye] = 1.0 + B.sum(axis=2)
    for q in (1, 2, 3):
        B[:, q, q] += storage
    if wells is None:
        wc = np.zeros(0, np.int32); wk = np.zeros(0, np.int8)
    else:
        wc, wk = wells
    wu = tscale * _rng(seed, _P_WELL).uniform(1.0, 10.0, size=wc.shape[0])
    b = _rng(seed, _P_RHS).standard_normal(4 * n)
    wobj = np.zeros((n, 4))
    prod = wc[wk < 0]
    wobj[prod, :] = _rng(seed, _P_OBJ).uniform(0.0, 1.0, size=(prod.shape[0], 4))
    return Problem(nx, ny, nz, logk, float(kvkh), float(tscale), Mf, Mb, B, float(dt),
                   np.ascontiguousarray(wc, np.int32), wu, wk, b, wobj.reshape(-1), name)


# ---------------------------------------------------------------------------
# the five benchmark workloads (seed_i = SEED_BASE + i)

def config(i: int) -> Problem:
    s = SEED_BASE + i
    if i == 0:      # 20x20x10, one vertical pair
        nx, ny, nz = 20, 20, 10
        return make(nx, ny, nz, seed=s, sigma=1.0, kvkh=0.1,
                    wells=wells_vertical_pair(nx, ny, nz, (5, 5), (15, 15)), name="cfg0-20x20x10")
    if i in (1, 4):  # 100x100x50, 8 vertical pairs
        nx, ny, nz = 100, 100, 50
        return make(nx, ny, nz, seed=s, sigma=1.5, kvkh=0.1,
                    wells=wells_vertical_grid(nx, ny, nz, 4, 2), name=f"cfg{i}-100x100x50")
    if i == 2:      # 200x200x100, 10% shale, 50 horizontal pairs
        nx, ny, nz = 200, 200, 100
        return make(nx, ny, nz, seed=s, sigma=2.0, kvkh=0.1, shale=0.10,
                    wells=wells_horizontal(nx, ny, nz, [2 + 4 * m for m in range(50)], [47], 5),
                    name="cfg2-200x200x100")
    if i == 3:      # 400x400x200, 400 horizontal pairs
        nx, ny, nz = 400, 400, 200
        return make(nx, ny, nz, seed=s, sigma=2.0, kvkh=0.05,
                    wells=wells_horizontal(nx, ny, nz, [10 + 20 * a for a in range(20)],
                                           [2 + 10 * b for b in range(20)], 5),
                    name="cfg3-400x400x200")
    raise ValueError(i)


def small(nx, ny, nz, seed=7, sigma=1.0, kvkh=0.1, shale=0.0, wells=True) -> Problem:
    """Small test problem with one vertical pair (if the grid allows)."""
    w = None
    if wells and nx * ny > 1:
        w = wells_vertical_pair(nx, ny, nz, (0, 0), (nx - 1, ny - 1))
    return make(nx, ny, nz, seed=seed, sigma=sigma, kvkh=kvkh, shale=shale, wells=w,
                name=f"small-{nx}x{ny}x{nz}")


# ---------------------------------------------------------------------------
# inputs of the thermal model subset: a grid, permeabilities, wells and two
# states (this Newton iterate and the previous time step) as raw draws

@dataclasses.dataclass
class ThermalProblem:
    nx: int
    ny: int
    nz: int
    kx: np.ndarray            # (n,) md
    ky: np.ndarray
    kz: np.ndarray
    wcell: np.ndarray         # (nw,) int32, ascending
    wkind: np.ndarray         # (nw,) int32: +1 injector, -1 producer
    wval: np.ndarray          # (nw,) injector: water rate bbl/day; producer: well index md ft
    p: np.ndarray             # this iterate: pressure (psi), S_w, S_o, T (deg F)
    sw: np.ndarray
    so: np.ndarray
    t: np.ndarray
    p0: np.ndarray            # previous time step
    sw0: np.ndarray
    so0: np.ndarray
    t0: np.ndarray


_P_TSTATE, _P_TOLD = 8, 9


def thermal_problem(nx, ny, nz, *, seed, sigma=1.0, kvkh=0.1, wells=None, wi=1.0e4, inj_bbl=None):
    """Draws for one Newton step of the thermal subset, around the heavy-oil
    example of the paper's validation section (initial p 75 psi, T 125 F,
    S_w 0.45; injection at 450 F, producers' well index 1e4 md ft, injector
    100 bbl/day per well): p ~ 75 + U[0,25], T ~ 125 + 325 U^2, S_w ~
    U[0.46, 0.84] (inside the relative-permeability tables), S_o = 1 - S_w;
    the previous step a little cooler and lower in pressure and S_w.  Each
    injector perforation takes inj_bbl (default 100 / nz, a vertical well's
    share)."""
    base = make(nx, ny, nz, seed=seed, sigma=sigma, kvkh=kvkh, wells=wells)
    n = nx * ny * nz
    k = np.exp(base.logk)
    r = _rng(seed, _P_TSTATE)
    p = 75.0 + 25.0 * r.random(n)
    t = 125.0 + 325.0 * r.random(n) ** 2
    sw = 0.46 + 0.38 * r.random(n)
    r0 = _rng(seed, _P_TOLD)
    p0 = p - 5.0 * r0.random(n)
    t0 = t - 10.0 * r0.random(n)
    sw0 = sw - 0.01 * r0.random(n)
    inj = 100.0 / nz if inj_bbl is None else inj_bbl
    wk = base.well_kind.astype(np.int32)
    wval = np.where(wk > 0, inj, wi).astype(np.float64)
    return ThermalProblem(nx, ny, nz, k, k.copy(), kvkh * k, base.well_cell.astype(np.int32), wk, wval,
                          p, sw, 1.0 - sw, t, p0, sw0, 1.0 - sw0, t0)
