"""Oracle residual and Jacobian of the thermal model subset (water, one oil
component, energy; unknowns p, N_w, N_o, T), pinned by the paper's printed
tables and constants, closed forms, conservation and central finite
differences of the residual."""
import os

import numpy as np
import pytest
import scipy.integrate

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "thermal_tables.txt")


def _tables():
    out, cur = {}, None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("table "):
            cur = line.split()[1]
            out[cur] = []
        else:
            out[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def test_tables_at_nodes():
    T = _tables()
    for row in T["swt"]:
        assert oracle.relperm(0, row[0])[0] == row[1] and oracle.relperm(1, row[0])[0] == row[2]
    for row in T["slt"]:
        assert oracle.relperm(2, row[0])[0] == row[1] and oracle.relperm(3, row[0])[0] == row[2]
    for row in T["wvis"]:
        mu, _ = oracle.water_visc(row[0] * 1.8 + 32.0)
        assert abs(mu - row[1]) <= 1e-14 * row[1]
    q = oracle.thermal_params()
    c = T["water_cpg"][0]
    assert list(q.cpg) == list(c[:5]) and q.hvr_w == c[5] and q.ev_w == c[6]
    lo = T["lo"][0]
    assert (q.rhoo_ref, q.cpo, q.ct1o, q.avisc_o, q.bvisc_o) == tuple(lo)
    # between nodes: the chord, constant beyond the ends
    assert oracle.relperm(0, 0.525)[0] == pytest.approx(0.5 * (0.000552 + 0.00312), rel=1e-14)
    assert oracle.relperm(1, 0.9) == (0.0, 0.0) and oracle.relperm(1, 0.2) == (0.4, 0.0)


@pytest.mark.parametrize("sw", [0.45, 0.5, 0.612, 0.7, 0.84])
def test_stone2_reductions(sw):
    """Stone II: with no gas k_ro = k_row(S_w); at connate water k_ro =
    k_rog(S_l); and its derivatives against central differences."""
    kro, dsw, dsg = oracle.stone2(sw, 0.0)
    assert kro == pytest.approx(oracle.relperm(1, sw)[0], rel=1e-14, abs=1e-16)
    for sg in (0.03, 0.113, 0.217):                   # S_l = 1 - S_g away from the table's nodes
        k, _, _ = oracle.stone2(0.45, sg)
        assert k == pytest.approx(oracle.relperm(3, 1.0 - sg)[0], rel=1e-13, abs=1e-16)
        h = 1e-7
        k1, dw, dg = oracle.stone2(sw + 0.003, sg)
        fw = (oracle.stone2(sw + 0.003 + h, sg)[0] - oracle.stone2(sw + 0.003 - h, sg)[0]) / (2 * h)
        fg = (oracle.stone2(sw + 0.003, sg + h)[0] - oracle.stone2(sw + 0.003, sg - h)[0]) / (2 * h)
        if k1 > 0:
            assert dw == pytest.approx(fw, rel=1e-6, abs=1e-9)
            assert dg == pytest.approx(fg, rel=1e-6, abs=1e-9)


def test_water_enthalpy_closed_form():
    """H_w = integral of the printed heat-capacity polynomial from T_ref minus
    hvr (T_crit - T)^ev, in J/gmol with t in deg C, then in Btu/lbmole."""
    q = oracle.thermal_params()
    c = list(q.cpg)
    trc = (q.t_ref - 32.0) / 1.8
    for tf in (60.0, 125.0, 300.0, 450.0, 700.0):
        tc = (tf - 32.0) / 1.8
        hg, _ = scipy.integrate.quad(lambda t: sum(ck * t ** k for k, ck in enumerate(c)), trc, tc, epsabs=1e-12)
        hv = q.hvr_w * (q.tcrit_w - tc) ** q.ev_w if tc < q.tcrit_w else 0.0
        h, dh = oracle.water_enthalpy(q, tf)
        assert h == pytest.approx((hg - hv) * 453.59237 / 1055.05585, rel=1e-12)
        fd = (oracle.water_enthalpy(q, tf + 1e-4)[0] - oracle.water_enthalpy(q, tf - 1e-4)[0]) / 2e-4
        assert dh == pytest.approx(fd, rel=1e-7)


def _states(tp, q):
    u = oracle.thermal_state(q, tp.p, tp.sw, tp.so, tp.t)
    u0 = oracle.thermal_state(q, tp.p0, tp.sw0, tp.so0, tp.t0)
    return u, u0


def _tp(dims, seed=71):
    nx, ny, nz = dims
    w = synth.wells_vertical_pair(nx, ny, nz, (0, 0), (nx - 1, ny - 1)) if nx * ny > 1 else None
    return synth.thermal_problem(nx, ny, nz, seed=seed, sigma=1.0, wells=w)


def test_constraint_vanishes_on_consistent_states():
    """States built with S_w + S_o = 1 satisfy the saturation constraint."""
    tp = _tp((4, 3, 2))
    q = oracle.thermal_params()
    u, _ = _states(tp, q)
    for c in range(tp.nx * tp.ny * tp.nz):
        pr = oracle.thermal_props(q, u[4 * c:4 * c + 4])
        assert abs(pr["vol"]) <= 1e-15 and abs(pr["sw"] + pr["so"] - 1.0) <= 1e-14
        assert pr["sw"] == pytest.approx(tp.sw[c], rel=1e-14)


@pytest.mark.parametrize("dims,seed", [((3, 3, 2), 71), ((4, 3, 2), 72), ((2, 2, 3), 73), ((5, 1, 1), 74)])
def test_jacobian_central_differences(dims, seed):
    """Every Jacobian entry against (R(u + h e) - R(u - h e)) / 2h, h = 1e-6 |u_j|."""
    tp = _tp(dims, seed)
    q = oracle.thermal_params()
    u, u0 = _states(tp, q)
    r, J = oracle.thermal_assemble(tp, q, u, u0)
    Jd = J.dense()
    N = u.size
    fd = np.zeros((N, N))
    for j in range(N):
        h = 1e-6 * abs(u[j])
        up, um = u.copy(), u.copy()
        up[j] += h; um[j] -= h
        fd[:, j] = (oracle.thermal_assemble(tp, q, up, u0, jacobian=False)[0]
                    - oracle.thermal_assemble(tp, q, um, u0, jacobian=False)[0]) / (2 * h)
    scale = np.abs(Jd).max(axis=1, keepdims=True)
    err = np.abs(fd - Jd) / scale
    assert err.max() <= 2e-6, err.max()
    # the stored pattern holds every nonzero of the finite-difference Jacobian
    assert np.all(np.abs(fd)[Jd == 0] <= 1e-6 * scale.repeat(N, 1)[Jd == 0])


def test_flows_conserve():
    """With the accumulation and the wells removed, what leaves one cell
    enters its neighbour: the residuals of each conserved quantity sum to
    zero, and so does every column of the flow Jacobian."""
    tp = _tp((4, 3, 3), 75)
    tp.wcell = tp.wcell[:0]; tp.wkind = tp.wkind[:0]; tp.wval = tp.wval[:0]
    q = oracle.thermal_params(dt=float("inf"))         # no accumulation: V/dt = 0 exactly
    u, u0 = _states(tp, q)
    r, J = oracle.thermal_assemble(tp, q, u, u0)
    R = r.reshape(-1, 4)
    for e in range(3):
        assert abs(R[:, e].sum()) <= 1e-12 * np.abs(R[:, e]).sum()
    Jd = J.dense()
    for e in range(3):
        cols = Jd[e::4, :].sum(axis=0)
        assert np.all(np.abs(cols) <= 1e-12 * np.abs(Jd[e::4, :]).sum(axis=0) + 1e-300)


def test_wells_and_accumulation_terms():
    """A single cell (no faces): the residual is the accumulation minus the
    well terms; a producer removes water and oil in proportion to their
    mobilities, with their enthalpies."""
    tp = synth.thermal_problem(1, 1, 1, seed=5)
    q = oracle.thermal_params()
    u, u0 = _states(tp, q)
    acc = q.dx * q.dy * q.dz / q.dt
    r, _ = oracle.thermal_assemble(tp, q, u, u0)
    pr, p0 = oracle.thermal_props(q, u), oracle.thermal_props(q, u0)
    # rows: water, oil, energy, volume; unknowns: p, N_w, N_o, T
    assert r[0] == pytest.approx(acc * (u[1] - u0[1]), rel=1e-14)
    assert r[1] == pytest.approx(acc * (u[2] - u0[2]), rel=1e-14)
    assert r[2] == pytest.approx(acc * (pr["e"] - p0["e"]), rel=1e-14)
    assert r[3] == pytest.approx(acc * pr["vol"], abs=1e-12 * acc)
    tp.wcell = np.array([0], np.int32); tp.wkind = np.array([-1], np.int32); tp.wval = np.array([1e4])
    rw, _ = oracle.thermal_assemble(tp, q, u, u0)
    qw, qo = rw[0] - r[0], rw[1] - r[1]              # produced (the residual gains -Q)
    wi = q.ctrans * 1e4 * (u[0] - q.p_bh)
    assert qw == pytest.approx(wi * pr["lw"], rel=1e-12) and qo == pytest.approx(wi * pr["lo"], rel=1e-12)
    assert rw[2] - r[2] == pytest.approx(qw * pr["hw"] + qo * pr["ho"], rel=1e-12)
