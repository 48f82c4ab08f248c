"""Oracle aggregation AMG pinned by hand cases, graph properties and dense
algebra.  Parameters follow the paper's AMG defaults (Section
"Preconditioners", Fig. fig-ds-amg-par)."""
import os
from collections import deque

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "amg_defaults.txt")


def _golden():
    d = {}
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            d[k] = float(v)
    return d


def test_defaults_match_paper_figure():
    g = _golden()
    o = oracle.amg_opts()
    assert o.theta == g["strength"]
    assert o.max_row_sum == g["max_row_sum"]
    assert g["maxit"] == 1 and g["itr_relax"] == 2   # one V-cycle; 1 pre + 1 post sweep


def _csr(rows):
    """rows: list of dicts col->val (must be structurally symmetric)."""
    rp = [0]; ci = []; a = []
    for r in rows:
        for c in sorted(r):
            ci.append(c); a.append(r[c])
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(a)


def test_strength_hand_case():
    # row 0: off-diagonals -1, -0.6, -0.4, +0.5 -> strong to 1 and 2 only (theta 0.5)
    # row 1: |row sum| = 1.8, not above 0.9*2 -> its two -0.1 entries are strong
    # row 5: |row sum| = 0.95 > 0.9*|1| -> all weak
    rows = [
        {0: 3.0, 1: -1.0, 2: -0.6, 3: -0.4, 4: 0.5},
        {0: -0.1, 1: 2.0, 5: -0.1},
        {0: -1.0, 2: 1.5},
        {0: -1.0, 3: 1.5},
        {0: -1.0, 4: 1.5},
        {1: -0.05, 5: 1.0},
    ]
    rp, ci, a = _csr(rows)
    h = oracle.AMG(rp, ci, a, coarse_n=1)
    L = h.level(0)
    strong = {(i, int(ci[p])) for i in range(6) for p in range(rp[i], rp[i + 1]) if L["strong"][p]}
    # directional strength: 0->1, 0->2, and rows 1..4 are strong to 0;
    # symmetrised: an edge counts in both rows if either direction is strong
    assert (0, 1) in strong and (0, 2) in strong and (1, 0) in strong and (2, 0) in strong
    assert (0, 3) in strong and (3, 0) in strong          # strong from row 3's side
    assert (0, 4) in strong and (4, 0) in strong          # strong from row 4's side
    assert (1, 5) in strong and (5, 1) in strong          # row 1 strong to 5; row 5 itself all weak
    assert all(i != j for i, j in strong)


def _fmix32(h):
    h = np.uint64(h) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16); h = (h * np.uint64(0x85EBCA6B)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(13); h = (h * np.uint64(0xC2B2AE35)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    return int(h)


def _key(i, level):
    return (_fmix32((i + 0x9E3779B9 * (level + 1)) & 0xFFFFFFFF) << 32) | i


def _adj(L):
    n = L["n"]
    adj = [[] for _ in range(n)]
    for i in range(n):
        for p in range(L["rp"][i], L["rp"][i + 1]):
            if L["strong"][p]:
                adj[i].append(int(L["ci"][p]))
    return adj


def _within2(adj, v):
    seen = {v: 0}
    q = deque([v])
    while q:
        u = q.popleft()
        if seen[u] == 2:
            continue
        for w in adj[u]:
            if w not in seen:
                seen[w] = seen[u] + 1
                q.append(w)
    return seen


@pytest.mark.parametrize("dims,sigma", [((8, 7, 5), 1.0), ((12, 10, 4), 2.0)])
def test_mis2_aggregation_properties(dims, sigma):
    p = synth.make(*dims, seed=13, sigma=sigma, shale=0.1 if sigma > 1.5 else 0.0)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=10)
    assert h.nlevels >= 2
    for l in range(h.nlevels - 1):
        L = h.level(l)
        adj = _adj(L)
        n = L["n"]
        agg = L["agg"]
        iso = [len(adj[v]) == 0 for v in range(n)]
        # strength graph is symmetric
        for v in range(n):
            for u in adj[v]:
                assert v in adj[u]
        nc = agg.max() + 1
        for I in range(nc):
            assert np.any(agg == I)
        keys = {v: _key(v, l) for v in range(n)}
        # build a distance-2 independent set by brute force over the priority order
        order = sorted((v for v in range(n) if not iso[v]), key=lambda v: -keys[v])
        taken = set(); blocked = set()
        for v in order:
            if v in blocked or v in taken:
                continue
            taken.add(v)
            blocked.update(_within2(adj, v).keys())
        mis = sorted(taken)
        # (1) pairwise distance >= 3, (2) every other non-isolated vertex has a root within 2
        for v in mis:
            d = _within2(adj, v)
            assert not any(u in taken for u in d if u != v)
        for v in range(n):
            if iso[v] or v in taken:
                continue
            d = _within2(adj, v)
            assert any(u in taken and keys[u] > keys[v] for u in d)
        # aggregates numbered by increasing root index; the root is in its own aggregate
        assert nc == len(mis)
        for I, r in enumerate(mis):
            assert agg[r] == I
            for u in adj[r]:
                assert agg[u] == I                       # phase 1: strength neighbours
        # isolated vertices stay unaggregated; everyone else is aggregated
        for v in range(n):
            assert (agg[v] < 0) == iso[v]
        # phase 2: a vertex with no root neighbour joins the largest-|a| phase-1 neighbour
        phase1 = {r for r in mis} | {u for r in mis for u in adj[r]}
        for v in range(n):
            if iso[v] or v in phase1:
                continue
            best = None
            for q in range(L["rp"][v], L["rp"][v + 1]):
                u = int(L["ci"][q])
                if L["strong"][q] and u in phase1:
                    cand = (abs(L["a"][q]), -agg[u])
                    best = cand if best is None or cand > best else best
            assert agg[v] == -best[1]


def test_galerkin_identity():
    p = synth.make(9, 8, 4, seed=17, sigma=1.5)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=5)
    for l in range(h.nlevels - 1):
        F = h.level(l); Cl = h.level(l + 1)
        n, nc = F["n"], Cl["n"]
        Af = np.zeros((n, n)); Af[np.repeat(np.arange(n), np.diff(F["rp"])), F["ci"]] = F["a"]
        Ac = np.zeros((nc, nc)); Ac[np.repeat(np.arange(nc), np.diff(Cl["rp"])), Cl["ci"]] = Cl["a"]
        P = np.zeros((n, nc))
        for i, I in enumerate(F["agg"]):
            if I >= 0:
                P[i, I] = 1.0
        assert np.allclose(Ac, P.T @ Af @ P, rtol=1e-12, atol=1e-13 * np.abs(Af).max())
        # l1 diagonal
        s = np.abs(Af).sum(1)
        assert np.allclose(np.abs(F["dl1"]), s)
        assert np.all(np.sign(F["dl1"]) == np.where(np.diag(Af) < 0, -1, 1))


def test_vcycle_is_two_level_operator():
    """With two levels and a dense coarsest solve, one V-cycle is the linear
    operator  B = S + (I - S A) P A_c^{-1} P^T (I - A S) ...  written out:
      x1 = S b;  x2 = x1 + P Ac^{-1} P^T (b - A x1);  x3 = x2 + S (b - A x2)
    with S = diag(1/d)."""
    p = synth.make(6, 5, 3, seed=19, sigma=1.0)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=40)
    assert h.nlevels == 2 and h.coarsest_is_lu
    F = h.level(0); Cl = h.level(1)
    n, nc = F["n"], Cl["n"]
    Af = np.zeros((n, n)); Af[np.repeat(np.arange(n), np.diff(F["rp"])), F["ci"]] = F["a"]
    P = np.zeros((n, nc))
    for i, I in enumerate(F["agg"]):
        if I >= 0:
            P[i, I] = 1.0
    Ac = P.T @ Af @ P
    S = np.diag(1.0 / F["dl1"])
    I = np.eye(n)
    CG = P @ np.linalg.solve(Ac, P.T)
    Bop = S + CG @ (I - Af @ S)
    Bop = Bop + S @ (I - Af @ Bop)
    Vd = np.stack([h.vcycle(e) for e in I], 1)
    assert np.allclose(Vd, Bop, rtol=1e-10, atol=1e-12 * np.abs(Bop).max())


def test_single_level_is_exact_solve():
    p = synth.make(4, 3, 2, seed=23, sigma=1.0)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    h = oracle.AMG(A.rp, A.ci, ap)      # n = 24 <= coarse_n: dense LU only
    assert h.nlevels == 1
    n = A.n
    Af = np.zeros((n, n)); Af[np.repeat(np.arange(n), np.diff(A.rp)), A.ci] = ap
    b = np.random.default_rng(3).standard_normal(n)
    assert np.allclose(h.vcycle(b), np.linalg.solve(Af, b), rtol=1e-11)


def _dense(L):
    n = L["n"]
    Ad = np.zeros((n, n))
    Ad[np.repeat(np.arange(n), np.diff(L["rp"])), L["ci"]] = L["a"]
    return Ad


def _jacobi_poly(Ad, d, k):
    """k l1-Jacobi sweeps from x = 0 as a matrix: sum_{i<k} (I - S A)^i S,
    S = diag(1/d) (the Neumann partial sum, not the sweep recurrence)."""
    n = Ad.shape[0]
    S = np.diag(1.0 / d)
    E = np.eye(n) - S @ Ad
    Q, T = np.zeros((n, n)), np.eye(n)
    for _ in range(k):
        Q = Q + T @ S
        T = E @ T
    return Q


@pytest.mark.parametrize("sweeps", [1, 2, 4, 7])
def test_coarsest_l1_jacobi_fallback(sweeps):
    """A coarsest level larger than lu_max is not inverted but relaxed by
    coarse_sweeps l1-Jacobi sweeps from zero.  Single level: the V-cycle is
    the Jacobi polynomial of A.  Two levels: the two-level operator with that
    polynomial in place of A_c^{-1}."""
    p = synth.make(6, 5, 3, seed=19, sigma=1.0)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=1000, lu_max=10, coarse_sweeps=sweeps)
    assert h.nlevels == 1 and not h.coarsest_is_lu
    F = h.level(0)
    Ad = _dense(F)
    Vd = np.stack([h.vcycle(e) for e in np.eye(F["n"])], 1)
    ref = _jacobi_poly(Ad, F["dl1"], sweeps)
    assert np.allclose(Vd, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=40, lu_max=1, coarse_sweeps=sweeps)
    assert h.nlevels == 2 and not h.coarsest_is_lu
    F, Cl = h.level(0), h.level(1)
    n, nc = F["n"], Cl["n"]
    Af = _dense(F)
    P = np.zeros((n, nc))
    for i, I in enumerate(F["agg"]):
        if I >= 0:
            P[i, I] = 1.0
    Ac = P.T @ Af @ P
    S = np.diag(1.0 / F["dl1"])
    I = np.eye(n)
    CG = P @ _jacobi_poly(Ac, Cl["dl1"], sweeps) @ P.T
    Bop = S + CG @ (I - Af @ S)
    Bop = Bop + S @ (I - Af @ Bop)
    Vd = np.stack([h.vcycle(e) for e in I], 1)
    assert np.allclose(Vd, Bop, rtol=1e-10, atol=1e-12 * np.abs(Bop).max())
    # many sweeps on a diagonally dominant coarsest level approach A_c^{-1}
    if sweeps == 7:
        h = oracle.AMG(A.rp, A.ci, ap, coarse_n=1000, lu_max=10, coarse_sweeps=400)
        b = np.random.default_rng(2).standard_normal(F["n"])
        rho = np.abs(np.linalg.eigvals(np.eye(F["n"]) - np.diag(1 / F["dl1"]) @ Af)).max()
        if rho < 0.95:
            assert np.allclose(h.vcycle(b), np.linalg.solve(Af, b), rtol=1e-6)


# ---- smoothed aggregation (option smooth=1, the figure's trunc error) ----------

def _chain(n):
    """1-D Laplacian, tridiagonal (-1, 2, -1), Dirichlet ends."""
    rows = []
    for i in range(n):
        r = {i: 2.0}
        if i > 0:
            r[i - 1] = -1.0
        if i < n - 1:
            r[i + 1] = -1.0
        rows.append(r)
    return _csr(rows)


def _dense_p(h, l, n, nc):
    rp, ci, v = h.prolongator(l)
    P = np.zeros((n, nc))
    P[np.repeat(np.arange(n), np.diff(rp)), ci] = v
    return P


def test_smoothed_prolongator_1d_hat():
    """The textbook smoothed-aggregation prolongator of the 1-D Laplacian
    (Vanek, Mandel, Brezina 1996): rho = max_i sum_j |a_ij| / a_ii = 2, so
    omega = 2/3 and P = P_t - A P_t / 3, the piecewise-linear hat: weight 1
    inside an aggregate, 2/3 on its end nodes, 1/3 on the nodes just outside
    it.  No weight is below 1e-2 of its row's largest, so none is dropped."""
    n = 31
    rp, ci, a = _chain(n)
    h = oracle.AMG(rp, ci, a, coarse_n=3, smooth=1)
    F = h.level(0)
    agg = F["agg"]
    assert (agg >= 0).all()
    nc = int(agg.max()) + 1
    P = _dense_p(h, 0, n, nc)
    for J in range(nc):
        mem = np.flatnonzero(agg == J)
        assert np.array_equal(mem, np.arange(mem[0], mem[-1] + 1))   # consecutive runs in 1-D
        s, e = mem[0], mem[-1]
        exp = np.zeros(n)
        exp[s:e + 1] = 1.0
        if e > s:
            exp[s] = exp[e] = 2.0 / 3.0
        else:
            exp[s] = 1.0 / 3.0                      # a one-node aggregate: 1 - 2/3
        if s > 0:
            exp[s - 1] = 1.0 / 3.0
        if e < n - 1:
            exp[e + 1] = 1.0 / 3.0
        # the Dirichlet end nodes have one neighbour only: 1 - (2 - 1)/3 = 2/3
        # as own weight whatever their position in the aggregate
        if s == 0 and e > 0:
            exp[0] = 2.0 / 3.0
        if e == n - 1 and s < n - 1:
            exp[n - 1] = 2.0 / 3.0
        assert np.allclose(P[:, J], exp, rtol=0, atol=1e-15), (J, P[:, J], exp)


def test_truncation_recovers_tentative_on_1d():
    """trunc = 0.6 on the 1-D Laplacian: every 1/3 weight is below 0.6 times
    its row's largest (1 or 2/3), so it is dropped and the row's kept weight
    is scaled to the former row sum: P becomes the piecewise-constant P_t
    (rows with a single 2/3 at a Dirichlet end excepted, whose row sum was
    2/3 and stays 2/3)."""
    n = 31
    rp, ci, a = _chain(n)
    h = oracle.AMG(rp, ci, a, coarse_n=3, smooth=1, trunc=0.6)
    agg = h.level(0)["agg"]
    nc = int(agg.max()) + 1
    P = _dense_p(h, 0, n, nc)
    Pt = np.zeros((n, nc)); Pt[np.arange(n), agg] = 1.0
    inner = np.ones(n, bool); inner[[0, n - 1]] = False
    assert np.allclose(P[inner], Pt[inner], rtol=0, atol=1e-15)
    assert np.count_nonzero(P[0]) == 1 and np.count_nonzero(P[n - 1]) == 1


def test_smoothed_prolongator_preserves_constants():
    """With A 1 = 0 (a periodic 2-D Laplacian: every row sums to zero) the
    smoothing step maps 1 to 1 - omega D^{-1} A 1 = 1 and the truncation
    keeps each row sum, so P 1 = 1 for every row at the default trunc."""
    m = 9
    rows = []
    for j in range(m):
        for i in range(m):
            c = i + m * j
            r = {c: 4.0}
            for q in (((i + 1) % m) + m * j, ((i - 1) % m) + m * j, i + m * ((j + 1) % m), i + m * ((j - 1) % m)):
                r[q] = r.get(q, 0.0) - 1.0
            rows.append(r)
    rp, ci, a = _csr(rows)
    h = oracle.AMG(rp, ci, a, coarse_n=3, smooth=1, max_row_sum=1e30)
    agg = h.level(0)["agg"]
    assert (agg >= 0).all()
    rp_, ci_, v = h.prolongator(0)
    sums = np.add.reduceat(v, rp_[:-1])
    assert np.allclose(sums, 1.0, rtol=0, atol=1e-14)


def _sa_problem():
    p = synth.make(9, 8, 4, seed=17, sigma=1.5)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    return A, oracle.extract_pressure(At)


def test_smoothed_galerkin_identity():
    """A_c = P^T A P with the returned smoothed P, level by level."""
    A, ap = _sa_problem()
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=5, smooth=1, max_row_sum=1e30)
    assert h.nlevels >= 3
    for l in range(h.nlevels - 1):
        F = h.level(l); Cl = h.level(l + 1)
        n, nc = F["n"], Cl["n"]
        Af = np.zeros((n, n)); Af[np.repeat(np.arange(n), np.diff(F["rp"])), F["ci"]] = F["a"]
        Ac = np.zeros((nc, nc)); Ac[np.repeat(np.arange(nc), np.diff(Cl["rp"])), Cl["ci"]] = Cl["a"]
        P = _dense_p(h, l, n, nc)
        assert np.allclose(Ac, P.T @ Af @ P, rtol=1e-12, atol=1e-13 * np.abs(Af).max())


def test_smoothed_vcycle_is_two_level_operator():
    """As the piecewise-constant case, with the smoothed P:
      x1 = S b;  x2 = x1 + P Ac^{-1} P^T (b - A x1);  x3 = x2 + S (b - A x2)."""
    p = synth.make(6, 5, 3, seed=19, sigma=1.0)
    A = oracle.assemble(p)
    At, _ = oracle.decouple(A)
    ap = oracle.extract_pressure(At)
    h = oracle.AMG(A.rp, A.ci, ap, coarse_n=40, smooth=1)
    assert h.nlevels == 2 and h.coarsest_is_lu
    F = h.level(0); Cl = h.level(1)
    n, nc = F["n"], Cl["n"]
    Af = np.zeros((n, n)); Af[np.repeat(np.arange(n), np.diff(F["rp"])), F["ci"]] = F["a"]
    P = _dense_p(h, 0, n, nc)
    Ac = P.T @ Af @ P
    S = np.diag(1.0 / F["dl1"])
    I = np.eye(n)
    CG = P @ np.linalg.solve(Ac, P.T)
    Bop = S + CG @ (I - Af @ S)
    Bop = Bop + S @ (I - Af @ Bop)
    Vd = np.stack([h.vcycle(e) for e in I], 1)
    assert np.allclose(Vd, Bop, rtol=1e-10, atol=1e-12 * np.abs(Bop).max())


def test_smoothed_cpr_gmres_converges():
    """CPR-GMRES with the smoothed-aggregation pressure stage on config 0."""
    p = synth.config(0)
    A = oracle.assemble(p)
    M = oracle.CPR(A, method=oracle.ABF, smoother=oracle.SM_RAS, smooth=1)
    x, info = oracle.gmres(A, p.b, M, rtol=1e-8)
    assert info["status"] == 0
    assert np.linalg.norm(p.b - oracle.spmv(A, x)) / np.linalg.norm(p.b) <= 1e-8
