/* amg.c -- aggregation AMG for the pressure stage of CPR.  FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper uses Hypre's AMG with the defaults of Fig. fig-ds-amg-par
 * (one V-cycle, strength 0.5, max row sum 0.9, two relaxation sweeps, ...).
 * Here the pressure solve is an aggregation AMG whose parameters are taken
 * from that figure:
 *   strength   j strongly influences i if -a_ij >= theta * max_{k!=i}(-a_ik);
 *              a row with |sum_j a_ij| > max_row_sum*|a_ii| has no strong
 *              connections; the strength graph is symmetrised (edge if
 *              either direction is strong).
 *   roots      a distance-2 maximal independent set of the strength graph,
 *              defined as the greedy one: visit vertices by decreasing
 *              priority key (fmix32 hash of the index, index in the low
 *              word) and take every vertex with no taken vertex within two
 *              strength edges.  Vertices with no strength edge are left out.
 *   aggregates each root with its strength neighbours; then every vertex
 *              still unassigned joins the aggregate of the neighbour (one
 *              assigned in the first pass) with the largest |a_ij|, ties to
 *              the lowest aggregate id.  Aggregates are numbered in
 *              increasing root index.  Isolated vertices stay unaggregated
 *              (zero row of P) and are handled by the smoother alone.
 *   P, A_c     piecewise-constant P, R = P^T, A_c = P^T A P; each coarse
 *              entry summed over members in increasing fine index, each
 *              member's row in increasing column order.
 *   smoothed   (option) the tentative P_t above smoothed by one damped
 *              Jacobi step, P = (I - omega D^{-1} A) P_t, D = diag(A),
 *              omega = 4 / (3 rho), rho = max_i sum_j |a_ij| / |a_ii| (a
 *              bound of the spectral radius of D^{-1} A); then the
 *              figure's interpolation truncation: in each row of P the
 *              weights below trunc times the row's largest |weight| are
 *              dropped and the kept ones scaled to the row's former sum.
 *              A_c = P^T (A P), R = P^T.
 *   smoother   l1-Jacobi x += (b - A x) / d,  d_i = sgn(a_ii) sum_j |a_ij|;
 *              one sweep before and one after the coarse correction.
 *   coarsest   dense LU with partial pivoting in FP64 up to lu_max rows;
 *              a larger coarsest level (one that no aggregate forms on,
 *              since all its rows are weak) is relaxed by coarse_sweeps
 *              l1-Jacobi sweeps from zero, as the figure relaxes there.
 * Pinned by: strength and aggregation brute force on small graphs, the
 * Galerkin identity against dense P^T A P, and the V-cycle as a linear
 * operator against its dense two-level formula; the smoothed prolongator by
 * its dense definition, by P 1 = 1 when A 1 = 0, and by the truncation rule
 * entry by entry.  The convergence rate of the
 * cycle is parity unpinned (the paper reports none).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define MAXL 32

typedef struct {
  int n, nc;
  int64_t nnz;
  int *rp, *ci;
  double *a;
  double *dl1;
  int *strong;   /* per stored entry: symmetric strength edge (off-diagonal) */
  int *agg;      /* per row: aggregate (coarse row) or -1 */
  /* smoothed prolongator (n x nc CSR, columns ascending); NULL when P is
   * the piecewise-constant one given by agg */
  int *prp, *pci;
  double *pv;
} level_t;

struct or_amg {
  int nl;
  level_t L[MAXL];
  int lu;              /* coarsest solved by dense LU */
  double *lu_a;        /* n x n LU factors, row-major */
  int *lu_piv;
  int coarse_sweeps;
};

void or_amg_defaults(or_amg_opts *o) {
  o->theta = 0.5;          /* Fig. fig-ds-amg-par: strength    */
  o->max_row_sum = 0.9;    /* Fig. fig-ds-amg-par: max_row_sum */
  /* the figure relaxes on the coarsest level (coarsest_relax_type); here a
   * coarsest level of at most lu_max rows is solved exactly and a larger one
   * (a level whose rows are all weak, so no aggregate forms) is relaxed */
  o->coarse_n = 256;
  o->max_levels = 20;
  o->lu_max = 256;
  o->coarse_sweeps = 4;
  o->smooth = 0;
  o->trunc = 1e-2;         /* Fig. fig-ds-amg-par: trunc error */
}

/* MurmurHash3 32-bit finaliser (Appleby), used as a fixed vertex priority. */
static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

static uint64_t prio_key(int i, int level) {
  uint32_t h = fmix32((uint32_t)i + 0x9e3779b9u * (uint32_t)(level + 1));
  return ((uint64_t)h << 32) | (uint32_t)i;
}

static int cmp_key_desc(const void *x, const void *y) {
  uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
  return a < b ? 1 : (a > b ? -1 : 0);
}

static void strength(level_t *L, const or_amg_opts *o) {
  int *dir = (int *)calloc((size_t)L->nnz, sizeof(int));
  for (int64_t i = 0; i < L->n; ++i) {
    double aii = 0.0, nm = 0.0, s = 0.0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
      double a = L->a[p];
      s = s + a;
      if (L->ci[p] == i) aii = a;
      else if (-a > nm) nm = -a;
    }
    if (fabs(s) > o->max_row_sum * fabs(aii)) continue;
    if (!(nm > 0.0)) continue;
    double thr = o->theta * nm;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p)
      if (L->ci[p] != i && -L->a[p] >= thr) dir[p] = 1;
  }
  for (int64_t i = 0; i < L->n; ++i)
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
      int64_t j = L->ci[p];
      int t = 0;
      if (j != i)
        for (int64_t q = L->rp[j]; q < L->rp[j + 1]; ++q)
          if (L->ci[q] == i) { t = dir[q]; break; }
      L->strong[p] = (j != i) && (dir[p] || t);
    }
  free(dir);
}

/* Greedy distance-2 MIS and aggregation; returns the number of aggregates. */
static int aggregate(level_t *L, int level) {
  int n = L->n;
  int *state = (int *)calloc((size_t)n, sizeof(int));   /* 0 free 1 root 2 blocked 3 isolated */
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  int nk = 0;
  for (int i = 0; i < n; ++i) {
    int deg = 0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) deg += L->strong[p];
    if (deg == 0) state[i] = 3;
    else keys[nk++] = prio_key(i, level);
  }
  qsort(keys, (size_t)nk, sizeof(uint64_t), cmp_key_desc);
  for (int t = 0; t < nk; ++t) {
    int v = (int)(keys[t] & 0xffffffffu);
    if (state[v] != 0) continue;
    state[v] = 1;
    for (int64_t p = L->rp[v]; p < L->rp[v + 1]; ++p) {
      if (!L->strong[p]) continue;
      int u = L->ci[p];
      if (state[u] == 0) state[u] = 2;
      for (int64_t q = L->rp[u]; q < L->rp[u + 1]; ++q)
        if (L->strong[q] && state[L->ci[q]] == 0) state[L->ci[q]] = 2;
    }
  }
  int nc = 0;
  int *id = (int *)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) id[i] = (state[i] == 1) ? nc++ : -1;
  int *agg1 = (int *)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    agg1[i] = -1;
    if (state[i] == 1) { agg1[i] = id[i]; continue; }
    if (state[i] == 3) continue;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p)
      if (L->strong[p] && state[L->ci[p]] == 1) { agg1[i] = id[L->ci[p]]; break; }
  }
  for (int i = 0; i < n; ++i) {
    L->agg[i] = agg1[i];
    if (agg1[i] >= 0 || state[i] == 3) continue;
    double bw = -1.0;
    int ba = -1;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
      if (!L->strong[p]) continue;
      int ag = agg1[L->ci[p]];
      if (ag < 0) continue;
      double wgt = fabs(L->a[p]);
      if (wgt > bw || (wgt == bw && ag < ba)) { bw = wgt; ba = ag; }
    }
    L->agg[i] = ba;
  }
  free(state); free(keys); free(id); free(agg1);
  return nc;
}

static int cmp_int(const void *x, const void *y) {
  int a = *(const int *)x, b = *(const int *)y;
  return (a > b) - (a < b);
}

/* A_c = P^T A P for piecewise-constant P. */
static void galerkin(const level_t *F, level_t *C) {
  int n = F->n, nc = F->nc;
  int *cnt = (int *)calloc((size_t)nc + 1, sizeof(int));
  for (int i = 0; i < n; ++i) if (F->agg[i] >= 0) cnt[F->agg[i] + 1]++;
  for (int I = 0; I < nc; ++I) cnt[I + 1] += cnt[I];
  int *mem = (int *)malloc(sizeof(int) * (size_t)(cnt[nc] > 0 ? cnt[nc] : 1));
  int *fill = (int *)calloc((size_t)nc, sizeof(int));
  for (int i = 0; i < n; ++i)
    if (F->agg[i] >= 0) { int I = F->agg[i]; mem[cnt[I] + fill[I]++] = i; }
  int *mark = (int *)malloc(sizeof(int) * (size_t)nc);
  int *slot = (int *)malloc(sizeof(int) * (size_t)nc);
  for (int I = 0; I < nc; ++I) mark[I] = -1;
  /* pass 1: count */
  C->n = nc;
  C->rp = (int *)malloc(sizeof(int) * ((size_t)nc + 1));
  C->rp[0] = 0;
  for (int I = 0; I < nc; ++I) {
    int m = 0;
    for (int t = cnt[I]; t < cnt[I + 1]; ++t) {
      int i = mem[t];
      for (int64_t p = F->rp[i]; p < F->rp[i + 1]; ++p) {
        int J = F->agg[F->ci[p]];
        if (J < 0 || mark[J] == I) continue;
        mark[J] = I; ++m;
      }
    }
    C->rp[I + 1] = C->rp[I] + m;
  }
  C->nnz = C->rp[nc];
  C->ci = (int *)malloc(sizeof(int) * (size_t)(C->nnz > 0 ? C->nnz : 1));
  C->a = (double *)malloc(sizeof(double) * (size_t)(C->nnz > 0 ? C->nnz : 1));
  for (int I = 0; I < nc; ++I) mark[I] = -1;
  /* pass 2: accumulate in member order, then sort the row by column */
  int *pidx = (int *)malloc(sizeof(int) * (size_t)nc);
  double *tv = (double *)malloc(sizeof(double) * (size_t)nc);
  for (int I = 0; I < nc; ++I) {
    int m = 0;
    int64_t base = C->rp[I];
    for (int t = cnt[I]; t < cnt[I + 1]; ++t) {
      int i = mem[t];
      for (int64_t p = F->rp[i]; p < F->rp[i + 1]; ++p) {
        int J = F->agg[F->ci[p]];
        if (J < 0) continue;
        if (mark[J] != I) { mark[J] = I; slot[J] = m; C->ci[base + m] = J; C->a[base + m] = 0.0; ++m; }
        C->a[base + slot[J]] = C->a[base + slot[J]] + F->a[p];
      }
    }
    for (int s = 0; s < m; ++s) { pidx[s] = C->ci[base + s]; tv[s] = C->a[base + s]; }
    qsort(&C->ci[base], (size_t)m, sizeof(int), cmp_int);
    for (int s = 0; s < m; ++s) C->a[base + s] = tv[slot[C->ci[base + s]]];
    (void)pidx;
  }
  free(cnt); free(mem); free(fill); free(mark); free(slot); free(pidx); free(tv);
}

/* Sort the m entries (cols, vals) of one sparse row by column. */
static void sort_row(int m, int *cols, double *vals) {
  for (int a = 1; a < m; ++a) {
    int c = cols[a];
    double v = vals[a];
    int b = a - 1;
    while (b >= 0 && cols[b] > c) { cols[b + 1] = cols[b]; vals[b + 1] = vals[b]; --b; }
    cols[b + 1] = c; vals[b + 1] = v;
  }
}

/* Smoothed prolongator of level L (aggregates in L->agg, L->nc of them):
 *   row i of A P_t:  acc_J = sum of a_ij over the stored j (ascending) with
 *                    agg[j] = J;
 *   P_s[i][J] = [J == agg[i]] - omega * (acc_J / a_ii)   (P_t's row when
 *                    a_ii = 0);
 *   truncation:      with m_i = max_J |P_s[i][J]|, entries with
 *                    |P_s[i][J]| < trunc * m_i are dropped; if any was, the
 *                    kept ones are multiplied by s_all / s_kept (row sums
 *                    over ascending J, s_kept != 0).
 * Returns OR_OK. */
static int smooth_prolongator(level_t *L, double trunc) {
  const int n = L->n, nc = L->nc;
  double rho = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0, d = 0.0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
      s = s + fabs(L->a[p]);
      if (L->ci[p] == i) d = L->a[p];
    }
    if (d != 0.0) { double q = s / fabs(d); if (q > rho) rho = q; }
  }
  const double omega = rho > 0.0 ? 4.0 / (3.0 * rho) : 0.0;
  L->prp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
  /* at most one entry per stored column (the own aggregate comes through
   * the diagonal) plus the own aggregate when the row has no diagonal */
  int64_t cap = L->rp[n] + n;
  L->pci = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
  L->pv = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
  int *mark = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
  int *slot = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
  for (int J = 0; J < nc; ++J) mark[J] = -1;
  int64_t w = 0;
  L->prp[0] = 0;
  for (int i = 0; i < n; ++i) {
    int *cols = L->pci + w;
    double *vals = L->pv + w;
    int m = 0;
    double d = 0.0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
      const int j = L->ci[p];
      if (j == i) d = L->a[p];
      const int J = L->agg[j];
      if (J < 0) continue;
      if (mark[J] != i) { mark[J] = i; slot[J] = m; cols[m] = J; vals[m] = 0.0; ++m; }
      vals[slot[J]] = vals[slot[J]] + L->a[p];
    }
    const int own = L->agg[i];
    if (own >= 0 && mark[own] != i) { mark[own] = i; slot[own] = m; cols[m] = own; vals[m] = 0.0; ++m; }
    for (int t = 0; t < m; ++t) {
      const double delta = cols[t] == own ? 1.0 : 0.0;
      vals[t] = d != 0.0 ? delta - omega * (vals[t] / d) : delta;
    }
    sort_row(m, cols, vals);
    if (trunc > 0.0 && m > 0) {
      double mx = 0.0, sall = 0.0, skeep = 0.0;
      for (int t = 0; t < m; ++t) { if (fabs(vals[t]) > mx) mx = fabs(vals[t]); sall = sall + vals[t]; }
      const double thr = trunc * mx;
      int k = 0;
      for (int t = 0; t < m; ++t)
        if (fabs(vals[t]) >= thr) { cols[k] = cols[t]; vals[k] = vals[t]; skeep = skeep + vals[k]; ++k; }
      if (k < m && skeep != 0.0) {
        const double scale = sall / skeep;
        for (int t = 0; t < k; ++t) vals[t] = vals[t] * scale;
      }
      m = k;
    }
    w += m;
    L->prp[i + 1] = (int)w;
  }
  free(mark); free(slot);
  return OR_OK;
}

/* A_c = P^T (A P) for a general P (the smoothed one):
 *   row i of AP:   (AP)_iJ = sum over A's row i (ascending j) and P's row j
 *                  of a_ij * p_jJ;
 *   coarse row I:  (A_c)_IJ = sum over the fine rows i with p_iI != 0, in
 *                  ascending i, of p_iI * (AP)_iJ;
 * each row's entries in ascending column order. */
static void galerkin_general(const level_t *F, level_t *C) {
  const int n = F->n, nc = F->nc;
  int *mark = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
  int *slot = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
  for (int J = 0; J < nc; ++J) mark[J] = -1;
  /* AP, row by row (entries bounded by the sum of the P rows it touches) */
  int64_t cap = 0;
  for (int i = 0; i < n; ++i)
    for (int64_t p = F->rp[i]; p < F->rp[i + 1]; ++p) cap += F->prp[F->ci[p] + 1] - F->prp[F->ci[p]];
  int64_t *aprp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int *apci = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
  double *apv = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
  int64_t w = 0;
  aprp[0] = 0;
  for (int i = 0; i < n; ++i) {
    int *cols = apci + w;
    double *vals = apv + w;
    int m = 0;
    for (int64_t p = F->rp[i]; p < F->rp[i + 1]; ++p) {
      const int j = F->ci[p];
      for (int64_t q = F->prp[j]; q < F->prp[j + 1]; ++q) {
        const int J = F->pci[q];
        if (mark[J] != i) { mark[J] = i; slot[J] = m; cols[m] = J; vals[m] = 0.0; ++m; }
        vals[slot[J]] = vals[slot[J]] + F->a[p] * F->pv[q];
      }
    }
    sort_row(m, cols, vals);
    w += m;
    aprp[i + 1] = w;
  }
  /* P^T by columns: fine rows of each coarse row I in ascending i */
  int64_t *trp = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
  for (int64_t q = 0; q < F->prp[n]; ++q) trp[F->pci[q] + 1]++;
  for (int I = 0; I < nc; ++I) trp[I + 1] += trp[I];
  int *tri = (int *)malloc(sizeof(int) * (size_t)(F->prp[n] > 0 ? F->prp[n] : 1));
  double *trv = (double *)malloc(sizeof(double) * (size_t)(F->prp[n] > 0 ? F->prp[n] : 1));
  int64_t *fill = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
  for (int i = 0; i < n; ++i)
    for (int64_t q = F->prp[i]; q < F->prp[i + 1]; ++q) {
      const int I = F->pci[q];
      tri[trp[I] + fill[I]] = i; trv[trp[I] + fill[I]] = F->pv[q]; fill[I]++;
    }
  /* coarse rows: accumulate into scratch rows, then pack */
  for (int J = 0; J < nc; ++J) mark[J] = -1;
  int *rcols = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
  double *rvals = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
  C->n = nc;
  C->rp = (int *)malloc(sizeof(int) * ((size_t)nc + 1));
  int64_t ccap = 16 * (int64_t)(nc > 0 ? nc : 1);
  C->ci = (int *)malloc(sizeof(int) * (size_t)ccap);
  C->a = (double *)malloc(sizeof(double) * (size_t)ccap);
  int64_t cw = 0;
  C->rp[0] = 0;
  for (int I = 0; I < nc; ++I) {
    int m = 0;
    for (int64_t t = trp[I]; t < trp[I + 1]; ++t) {
      const int i = tri[t];
      const double pi = trv[t];
      for (int64_t q = aprp[i]; q < aprp[i + 1]; ++q) {
        const int J = apci[q];
        if (mark[J] != I) { mark[J] = I; slot[J] = m; rcols[m] = J; rvals[m] = 0.0; ++m; }
        rvals[slot[J]] = rvals[slot[J]] + pi * apv[q];
      }
    }
    sort_row(m, rcols, rvals);
    if (cw + m > ccap) {
      while (cw + m > ccap) ccap *= 2;
      C->ci = (int *)realloc(C->ci, sizeof(int) * (size_t)ccap);
      C->a = (double *)realloc(C->a, sizeof(double) * (size_t)ccap);
    }
    memcpy(C->ci + cw, rcols, sizeof(int) * (size_t)m);
    memcpy(C->a + cw, rvals, sizeof(double) * (size_t)m);
    cw += m;
    C->rp[I + 1] = (int)cw;
  }
  C->nnz = cw;
  free(mark); free(slot); free(aprp); free(apci); free(apv); free(trp); free(tri); free(trv); free(fill);
  free(rcols); free(rvals);
}

static void l1diag(level_t *L) {
  for (int64_t i = 0; i < L->n; ++i) {
    double s = 0.0, aii = 0.0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) {
      s = s + fabs(L->a[p]);
      if (L->ci[p] == i) aii = L->a[p];
    }
    if (s == 0.0) s = 1.0;
    L->dl1[i] = (aii < 0.0) ? -s : s;
  }
}

static void alloc_level_aux(level_t *L) {
  L->dl1 = (double *)malloc(sizeof(double) * (size_t)(L->n > 0 ? L->n : 1));
  L->strong = (int *)calloc((size_t)(L->nnz > 0 ? L->nnz : 1), sizeof(int));
  L->agg = (int *)malloc(sizeof(int) * (size_t)(L->n > 0 ? L->n : 1));
  for (int i = 0; i < L->n; ++i) L->agg[i] = -1;
  L->nc = 0;
}

/* Dense LU with partial pivoting (first largest |entry|), in place. */
static int dense_lu(int n, double *a, int *piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (fabs(a[(int64_t)r * n + k]) > fabs(a[(int64_t)p * n + k])) p = r;
    piv[k] = p;
    if (a[(int64_t)p * n + k] == 0.0) return OR_E_SINGULAR;
    if (p != k)
      for (int c = 0; c < n; ++c) {
        double t = a[(int64_t)k * n + c]; a[(int64_t)k * n + c] = a[(int64_t)p * n + c]; a[(int64_t)p * n + c] = t;
      }
    for (int r = k + 1; r < n; ++r) {
      double l = a[(int64_t)r * n + k] / a[(int64_t)k * n + k];
      a[(int64_t)r * n + k] = l;
      for (int c = k + 1; c < n; ++c) a[(int64_t)r * n + c] = a[(int64_t)r * n + c] - l * a[(int64_t)k * n + c];
    }
  }
  return OR_OK;
}

static void dense_lu_solve(int n, const double *a, const int *piv, const double *b, double *x) {
  for (int i = 0; i < n; ++i) x[i] = b[i];
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < i; ++c) x[i] = x[i] - a[(int64_t)i * n + c] * x[c];
  for (int i = n - 1; i >= 0; --i) {
    for (int c = i + 1; c < n; ++c) x[i] = x[i] - a[(int64_t)i * n + c] * x[c];
    x[i] = x[i] / a[(int64_t)i * n + i];
  }
}

or_amg *or_amg_setup(int n, const int *rp, const int *ci, const double *a,
                     const or_amg_opts *o, int *status) {
  or_amg *h = (or_amg *)calloc(1, sizeof(or_amg));
  *status = OR_OK;
  level_t *L0 = &h->L[0];
  L0->n = n;
  L0->nnz = rp[n];
  L0->rp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
  L0->ci = (int *)malloc(sizeof(int) * (size_t)(L0->nnz > 0 ? L0->nnz : 1));
  L0->a = (double *)malloc(sizeof(double) * (size_t)(L0->nnz > 0 ? L0->nnz : 1));
  memcpy(L0->rp, rp, sizeof(int) * ((size_t)n + 1));
  memcpy(L0->ci, ci, sizeof(int) * (size_t)L0->nnz);
  memcpy(L0->a, a, sizeof(double) * (size_t)L0->nnz);
  h->nl = 1;
  for (int l = 0;; ++l) {
    level_t *L = &h->L[l];
    alloc_level_aux(L);
    l1diag(L);
    if (L->n <= o->coarse_n || h->nl >= o->max_levels || h->nl >= MAXL) break;
    strength(L, o);
    int nc = aggregate(L, l);
    if (nc == 0 || nc >= L->n) { for (int i = 0; i < L->n; ++i) L->agg[i] = -1; break; }
    L->nc = nc;
    if (o->smooth) {
      smooth_prolongator(L, o->trunc);
      galerkin_general(L, &h->L[l + 1]);
    } else {
      galerkin(L, &h->L[l + 1]);
    }
    h->nl++;
  }
  level_t *C = &h->L[h->nl - 1];
  h->coarse_sweeps = o->coarse_sweeps;
  if (C->n <= o->lu_max) {
    int m = C->n;
    h->lu = 1;
    h->lu_a = (double *)calloc((size_t)m * (size_t)m + 1, sizeof(double));
    h->lu_piv = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int i = 0; i < m; ++i)
      for (int64_t p = C->rp[i]; p < C->rp[i + 1]; ++p) h->lu_a[(int64_t)i * m + C->ci[p]] = C->a[p];
    *status = dense_lu(m, h->lu_a, h->lu_piv);
  }
  return h;
}

int or_amg_nlevels(const or_amg *h) { return h->nl; }
int or_amg_level_n(const or_amg *h, int l) { return h->L[l].n; }
int64_t or_amg_level_nnz(const or_amg *h, int l) { return h->L[l].nnz; }
int or_amg_coarsest_is_lu(const or_amg *h) { return h->lu; }

int64_t or_amg_level_p(const or_amg *h, int l, int *prp, int *pci, double *pv) {
  if (l < 0 || l >= h->nl - 1 || !h->L[l].prp) return -1;
  const level_t *L = &h->L[l];
  const int64_t nnz = L->prp[L->n];
  if (prp) memcpy(prp, L->prp, sizeof(int) * ((size_t)L->n + 1));
  if (pci) memcpy(pci, L->pci, sizeof(int) * (size_t)nnz);
  if (pv) memcpy(pv, L->pv, sizeof(double) * (size_t)nnz);
  return nnz;
}

void or_amg_level_get(const or_amg *h, int l, int *rp, int *ci, double *a,
                      double *dl1, int *agg, int *strong) {
  const level_t *L = &h->L[l];
  if (rp) memcpy(rp, L->rp, sizeof(int) * ((size_t)L->n + 1));
  if (ci) memcpy(ci, L->ci, sizeof(int) * (size_t)L->nnz);
  if (a) memcpy(a, L->a, sizeof(double) * (size_t)L->nnz);
  if (dl1) memcpy(dl1, L->dl1, sizeof(double) * (size_t)L->n);
  if (agg) memcpy(agg, L->agg, sizeof(int) * (size_t)L->n);
  if (strong) memcpy(strong, L->strong, sizeof(int) * (size_t)L->nnz);
}

static void csr_residual(const level_t *L, const double *b, const double *x, double *r) {
  for (int64_t i = 0; i < L->n; ++i) {
    double s = 0.0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) s = s + L->a[p] * x[L->ci[p]];
    r[i] = b[i] - s;
  }
}

static void vcycle(const or_amg *h, int l, const double *b, double *x) {
  const level_t *L = &h->L[l];
  int n = L->n;
  double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (l == h->nl - 1) {
    if (h->lu) {
      dense_lu_solve(n, h->lu_a, h->lu_piv, b, x);
    } else {
      for (int i = 0; i < n; ++i) x[i] = b[i] / L->dl1[i];
      for (int s = 1; s < h->coarse_sweeps; ++s) {
        csr_residual(L, b, x, r);
        for (int i = 0; i < n; ++i) x[i] = x[i] + r[i] / L->dl1[i];
      }
    }
    free(r);
    return;
  }
  int nc = L->nc;
  double *bc = (double *)calloc((size_t)nc, sizeof(double));
  double *xc = (double *)malloc(sizeof(double) * (size_t)nc);
  for (int i = 0; i < n; ++i) x[i] = b[i] / L->dl1[i];            /* pre-smooth from 0 */
  csr_residual(L, b, x, r);
  if (L->prp) {
    for (int i = 0; i < n; ++i)                                      /* restrict: P^T r */
      for (int64_t q = L->prp[i]; q < L->prp[i + 1]; ++q)
        bc[L->pci[q]] = bc[L->pci[q]] + L->pv[q] * r[i];
  } else {
    for (int i = 0; i < n; ++i)                                      /* restrict: P^T r */
      if (L->agg[i] >= 0) bc[L->agg[i]] = bc[L->agg[i]] + r[i];
  }
  vcycle(h, l + 1, bc, xc);
  if (L->prp) {
    for (int i = 0; i < n; ++i) {                                    /* prolong: x += P xc */
      double s = 0.0;
      for (int64_t q = L->prp[i]; q < L->prp[i + 1]; ++q) s = s + L->pv[q] * xc[L->pci[q]];
      x[i] = x[i] + s;
    }
  } else {
    for (int i = 0; i < n; ++i)                                      /* prolong: x += P xc */
      if (L->agg[i] >= 0) x[i] = x[i] + xc[L->agg[i]];
  }
  csr_residual(L, b, x, r);                                          /* post-smooth */
  for (int i = 0; i < n; ++i) x[i] = x[i] + r[i] / L->dl1[i];
  free(r); free(bc); free(xc);
}

void or_amg_vcycle(const or_amg *h, const double *b, double *x) { vcycle(h, 0, b, x); }

void or_amg_free(or_amg *h) {
  if (!h) return;
  for (int l = 0; l < h->nl; ++l) {
    level_t *L = &h->L[l];
    free(L->rp); free(L->ci); free(L->a); free(L->dl1); free(L->strong); free(L->agg);
    free(L->prp); free(L->pci); free(L->pv);
  }
  free(h->lu_a); free(h->lu_piv);
  free(h);
}
