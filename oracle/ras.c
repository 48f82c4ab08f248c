/* ras.c -- restricted additive Schwarz with overlap, the second stage of the
 * CPR preconditioner.  FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Section "Preconditioners": the paper's parallel second stage is RAS, with
 * an overlap of 1 by default, and ILU(k) / block ILU(k) as the solver on each
 * subdomain.  Here
 *   - subdomain m owns the cells [m*sub, min(n, (m+1)*sub)) (with cells
 *     numbered i fastest and sub = nx*ny: the xy-layers of the grid);
 *   - its extension E_m adds every cell reached from an owned cell in at most
 *     ov steps along the stored pattern (for layer subdomains and ov = 1:
 *     the layers just below and above);
 *   - the local problem is A~ restricted to E_m (couplings leaving E_m are
 *     dropped), in natural order, and its solver is the block ILU(0) of that
 *     restricted matrix, which on the 7-point block pattern is its DILU
 *     (or_dilu_setup / or_dilu_apply);
 *   - restricted prolongation: cell c takes the value of the local solution
 *     of the subdomain that owns it,
 *         z = sum_m R0_m^T (DILU of A~[E_m, E_m])^{-1} R_m r.
 * With ov = 0 every extension is the owned range and this is the zero-overlap
 * RAS of or_ras_restrict.
 * Pinned by: ov = 0 against or_ras_restrict + DILU (bitwise); one subdomain
 * (sub >= n) and, for layer subdomains, ov >= nz against the global DILU
 * (bitwise); the dense composition of the local ILU factors on tiny grids. */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

struct or_rasov {
  int n, nsub;
  int64_t sub;
  int *eptr;          /* [nsub+1]: extension m is ext[eptr[m] .. eptr[m+1]) */
  int *ext;           /* extension cells, ascending within each subdomain     */
  int64_t *bptr;      /* [nsub+1]: local blocks of subdomain m                */
  int *rpl;           /* local row pointers, (eptr[m+1]-eptr[m]+1) per m      */
  int64_t *rptr;      /* [nsub+1]: offset of subdomain m's rows in rpl        */
  int *cil;           /* local column of each local block                     */
  int64_t *posl;      /* position of each local block in the global CSR       */
  double *dinv;       /* DILU pivots D^{-1}, 16 per extension cell            */
  int maxext;
  int64_t maxblk;
};

static int cmp_int(const void *x, const void *y) {
  int a = *(const int *)x, b = *(const int *)y;
  return (a > b) - (a < b);
}

/* copy the local blocks of subdomain m into vl (16 doubles each) */
static void gather_blocks(const or_rasov *R, int m, const double *vt, double *vl) {
  for (int64_t q = R->bptr[m]; q < R->bptr[m + 1]; ++q)
    memcpy(&vl[16 * (q - R->bptr[m])], &vt[16 * R->posl[q]], 16 * sizeof(double));
}

or_rasov *or_rasov_setup(int n, const int *rp, const int *ci, const double *vt, int64_t sub, int ov,
                         int *status) {
  *status = OR_OK;
  if (n < 1 || sub < 1 || ov < 0) { *status = OR_E_ARG; return NULL; }
  or_rasov *R = (or_rasov *)calloc(1, sizeof(or_rasov));
  R->n = n;
  R->sub = sub;
  R->nsub = (int)((n + sub - 1) / sub);
  int nsub = R->nsub;
  int *mark = (int *)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) mark[i] = -1;
  int *front = (int *)malloc(sizeof(int) * (size_t)n);
  int *loc = (int *)malloc(sizeof(int) * (size_t)n);
  /* pass 1: extension sizes and block counts */
  R->eptr = (int *)calloc((size_t)nsub + 1, sizeof(int));
  R->bptr = (int64_t *)calloc((size_t)nsub + 1, sizeof(int64_t));
  R->rptr = (int64_t *)calloc((size_t)nsub + 1, sizeof(int64_t));
  int cap = 0;
  int64_t ecap = 0;
  R->ext = NULL;
  for (int m = 0; m < nsub; ++m) {
    int a = (int)((int64_t)m * sub), b = (int)(((int64_t)m + 1) * sub < n ? ((int64_t)m + 1) * sub : n);
    int ne = 0;
    for (int c = a; c < b; ++c) { mark[c] = m; front[ne++] = c; }
    int f0 = 0, f1 = ne;
    for (int step = 0; step < ov; ++step) {
      for (int t = f0; t < f1; ++t) {
        int c = front[t];
        for (int64_t p = rp[c]; p < rp[c + 1]; ++p) {
          int j = ci[p];
          if (mark[j] != m) { mark[j] = m; front[ne++] = j; }
        }
      }
      f0 = f1; f1 = ne;
    }
    qsort(front, (size_t)ne, sizeof(int), cmp_int);
    if (R->eptr[m] + (int64_t)ne > ecap) {
      ecap = 2 * (R->eptr[m] + (int64_t)ne) + 16;
      R->ext = (int *)realloc(R->ext, sizeof(int) * (size_t)ecap);
    }
    memcpy(&R->ext[R->eptr[m]], front, sizeof(int) * (size_t)ne);
    R->eptr[m + 1] = R->eptr[m] + ne;
    int64_t nb = 0;
    for (int t = 0; t < ne; ++t) {
      int c = front[t];
      for (int64_t p = rp[c]; p < rp[c + 1]; ++p) nb += (mark[ci[p]] == m);
    }
    R->bptr[m + 1] = R->bptr[m] + nb;
    R->rptr[m + 1] = R->rptr[m] + ne + 1;
    if (ne > cap) cap = ne;
    if (nb > R->maxblk) R->maxblk = nb;
  }
  R->maxext = cap;
  /* pass 2: local patterns (restricted rows, renumbered columns) */
  int64_t ntot = R->eptr[nsub];
  R->rpl = (int *)malloc(sizeof(int) * (size_t)R->rptr[nsub]);
  R->cil = (int *)malloc(sizeof(int) * (size_t)(R->bptr[nsub] > 0 ? R->bptr[nsub] : 1));
  R->posl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->bptr[nsub] > 0 ? R->bptr[nsub] : 1));
  R->dinv = (double *)malloc(sizeof(double) * 16 * (size_t)(ntot > 0 ? ntot : 1));
  for (int i = 0; i < n; ++i) loc[i] = -1;
  double *vl = (double *)malloc(sizeof(double) * 16 * (size_t)(R->maxblk > 0 ? R->maxblk : 1));
  for (int m = 0; m < nsub && *status == OR_OK; ++m) {
    const int *E = &R->ext[R->eptr[m]];
    int ne = R->eptr[m + 1] - R->eptr[m];
    for (int t = 0; t < ne; ++t) loc[E[t]] = t;
    int *rl = &R->rpl[R->rptr[m]];
    int64_t q = R->bptr[m];
    rl[0] = 0;
    for (int t = 0; t < ne; ++t) {
      int c = E[t];
      for (int64_t p = rp[c]; p < rp[c + 1]; ++p) {
        if (loc[ci[p]] < 0) continue;
        R->cil[q] = loc[ci[p]];
        R->posl[q] = p;
        ++q;
      }
      rl[t + 1] = (int)(q - R->bptr[m]);
    }
    gather_blocks(R, m, vt, vl);
    *status = or_dilu_setup(ne, rl, &R->cil[R->bptr[m]], vl, &R->dinv[16 * (int64_t)R->eptr[m]]);
    for (int t = 0; t < ne; ++t) loc[E[t]] = -1;
  }
  free(vl); free(mark); free(front); free(loc);
  return R;
}

void or_rasov_apply(const or_rasov *R, const double *vt, const double *r, double *z) {
  double *vl = (double *)malloc(sizeof(double) * 16 * (size_t)(R->maxblk > 0 ? R->maxblk : 1));
  double *rl = (double *)malloc(sizeof(double) * 4 * (size_t)(R->maxext > 0 ? R->maxext : 1));
  double *zl = (double *)malloc(sizeof(double) * 4 * (size_t)(R->maxext > 0 ? R->maxext : 1));
  for (int m = 0; m < R->nsub; ++m) {
    const int *E = &R->ext[R->eptr[m]];
    int ne = R->eptr[m + 1] - R->eptr[m];
    for (int t = 0; t < ne; ++t) memcpy(&rl[4 * t], &r[4 * (int64_t)E[t]], 4 * sizeof(double));
    gather_blocks(R, m, vt, vl);
    or_dilu_apply(ne, &R->rpl[R->rptr[m]], &R->cil[R->bptr[m]], vl, &R->dinv[16 * (int64_t)R->eptr[m]], rl, zl);
    int64_t a = (int64_t)m * R->sub, b = a + R->sub < R->n ? a + R->sub : R->n;
    for (int t = 0; t < ne; ++t)
      if (E[t] >= a && E[t] < b) memcpy(&z[4 * (int64_t)E[t]], &zl[4 * t], 4 * sizeof(double));
  }
  free(vl); free(rl); free(zl);
}

/* DILU pivots of the owned cells, each from the subdomain that owns it
 * (16 doubles per cell, into dinv2[16 n]). */
void or_rasov_owned_dinv(const or_rasov *R, double *dinv2) {
  for (int m = 0; m < R->nsub; ++m) {
    const int *E = &R->ext[R->eptr[m]];
    int ne = R->eptr[m + 1] - R->eptr[m];
    int64_t a = (int64_t)m * R->sub, b = a + R->sub < R->n ? a + R->sub : R->n;
    for (int t = 0; t < ne; ++t)
      if (E[t] >= a && E[t] < b)
        memcpy(&dinv2[16 * (int64_t)E[t]], &R->dinv[16 * ((int64_t)R->eptr[m] + t)], 16 * sizeof(double));
  }
}

/* Size of the extension of subdomain m, and its cells (ascending) if ext != NULL. */
int or_rasov_ext(const or_rasov *R, int m, int *ext) {
  int ne = R->eptr[m + 1] - R->eptr[m];
  if (ext) memcpy(ext, &R->ext[R->eptr[m]], sizeof(int) * (size_t)ne);
  return ne;
}

/* DILU pivots of the extension of subdomain m (16 doubles per extension cell). */
void or_rasov_ext_dinv(const or_rasov *R, int m, double *dinv) {
  int ne = R->eptr[m + 1] - R->eptr[m];
  memcpy(dinv, &R->dinv[16 * (int64_t)R->eptr[m]], sizeof(double) * 16 * (size_t)ne);
}

void or_rasov_free(or_rasov *R) {
  if (!R) return;
  free(R->eptr); free(R->ext); free(R->bptr); free(R->rpl); free(R->rptr); free(R->cil);
  free(R->posl); free(R->dinv);
  free(R);
}
