/* bsr.c -- 7-point block pattern, Jacobian assembly from the synthetic draws,
 * block SpMV and block transpose.  FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

int64_t or_nnzb(int nx, int ny, int nz) {
  int64_t n = (int64_t)nx * ny * nz;
  int64_t faces = (int64_t)(nx - 1) * ny * nz + (int64_t)nx * (ny - 1) * nz +
                  (int64_t)nx * ny * (nz - 1);
  return n + 2 * faces;
}

/* Neighbour of cell c in slot s of the sorted 7-point row:
 * s = 0:-z 1:-y 2:-x 3:self 4:+x 5:+y 6:+z.  Returns -1 outside the grid. */
static int64_t nbr(int nx, int ny, int nz, int64_t c, int s) {
  int64_t nxy = (int64_t)nx * ny;
  int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
  switch (s) {
    case 0: return k > 0 ? c - nxy : -1;
    case 1: return j > 0 ? c - nx : -1;
    case 2: return i > 0 ? c - 1 : -1;
    case 3: return c;
    case 4: return i < nx - 1 ? c + 1 : -1;
    case 5: return j < ny - 1 ? c + nx : -1;
    default: return k < nz - 1 ? c + nxy : -1;
  }
}

/* The block pattern of the paper's Jacobian (Eq. mat-ja) for a 7-point
 * finite-difference stencil: row c holds the diagonal block and one block per
 * grid neighbour sharing a face (no-flow boundary faces carry none). */
int or_pattern(int nx, int ny, int nz, int *rp, int *ci) {
  if (nx < 1 || ny < 1 || nz < 1) return OR_E_ARG;
  int64_t n = (int64_t)nx * ny * nz, p = 0;
  rp[0] = 0;
  for (int64_t c = 0; c < n; ++c) {
    for (int s = 0; s < 7; ++s) {
      int64_t q = nbr(nx, ny, nz, c, s);
      if (q >= 0) ci[p++] = (int)q;
    }
    rp[c + 1] = (int)p;
  }
  return OR_OK;
}

/* Harmonic mean of the geometric transmissibility part with unit geometry
 * (A/dd = 1): the paper applies harmonic averaging to K*A/dd at a face
 * (Section "Numerical Methods", transmissibility equation). */
static double harmonic(double p, double q) { return ((2.0 * p) * q) / (p + q); }

/* Assemble the synthetic Jacobian.
 *   T_d(c) = tscale * harmonic mean of the directional permeabilities
 *   off-diagonal block  A[c][c+e_d] = -T_d(c) * Mf[d][c]
 *                       A[c+e_d][c] = -T_d(c) * Mb[d][c]
 *   diagonal block      A[c][c] = B_c/dt + sum over the row's faces of T*M
 *                                 (+ u_c*k_c*I in perforated cells)
 * i.e. the diagonal is the negated sum of the row's off-diagonal blocks plus
 * the accumulation term, and the face transmissibility is shared by both
 * cells (same value in both rows) and zero on boundary faces (Section
 * "Numerical Methods").  Well terms follow the Peaceman form Q = WI*(...)
 * with WI proportional to the cell permeability (Section "Well Modeling").
 * Summation order of the diagonal: B/dt, then faces in column order, then
 * the well term.
 * Pinned by: T_ab = T_ba recovered from both rows, zero blocks across
 * boundaries, exact row-sum identity sum_j A_ij = B_i/dt + W_i, and a
 * two-cell worked example computed by hand. */
int or_assemble(int nx, int ny, int nz, const double *logk, double kvkh, double tscale,
                const double *Mf, const double *Mb, const double *B, double dt,
                int nw, const int *wcell, const double *wu,
                const int *rp, const int *ci, double *v) {
  int64_t n = (int64_t)nx * ny * nz;
  double *k = (double *)malloc(sizeof(double) * (size_t)n);
  double *wsrc = (double *)calloc((size_t)n, sizeof(double));
  if (!k || !wsrc) { free(k); free(wsrc); return OR_E_ARG; }
  for (int64_t c = 0; c < n; ++c) k[c] = exp(logk[c]);
  for (int w = 0; w < nw; ++w) {
    if (wcell[w] < 0 || wcell[w] >= n) { free(k); free(wsrc); return OR_E_ARG; }
    wsrc[wcell[w]] = wu[w] * k[wcell[w]];
  }
  static const int axis[7] = {2, 1, 0, -1, 0, 1, 2};
  for (int64_t c = 0; c < n; ++c) {
    double acc[16];
    for (int e = 0; e < 16; ++e) acc[e] = B[16 * c + e] / dt;
    int64_t p = rp[c], diagpos = -1;
    for (int s = 0; s < 7; ++s) {
      int64_t q = nbr(nx, ny, nz, c, s);
      if (q < 0) continue;
      if (p >= rp[c + 1] || ci[p] != q) { free(k); free(wsrc); return OR_E_ARG; }
      if (s == 3) { diagpos = p++; continue; }
      int d = axis[s];
      int64_t lo = q < c ? q : c, hi = q < c ? c : q;
      double pa = k[lo], pb = k[hi];
      if (d == 2) { pa = kvkh * pa; pb = kvkh * pb; }
      double T = tscale * harmonic(pa, pb);
      const double *M = (q > c) ? &Mf[(d * n + c) * 16] : &Mb[(d * n + q) * 16];
      for (int e = 0; e < 16; ++e) {
        double t = T * M[e];
        v[16 * p + e] = -t;
        acc[e] = acc[e] + t;
      }
      ++p;
    }
    if (p != rp[c + 1] || diagpos < 0) { free(k); free(wsrc); return OR_E_ARG; }
    if (wsrc[c] != 0.0)
      for (int r = 0; r < 4; ++r) acc[5 * r] = acc[5 * r] + wsrc[c];
    memcpy(&v[16 * diagpos], acc, sizeof(acc));
  }
  free(k);
  free(wsrc);
  return OR_OK;
}

/* y = A x with 4x4 blocks (Fig. fig-mv, y = A*x), left to right in column
 * order.  Pinned by the dense product on small grids. */
void or_spmv(int n, const int *rp, const int *ci, const double *v,
             const double *x, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      const double *a = &v[16 * p];
      const double *xx = &x[4 * (int64_t)ci[p]];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) s[r] = s[r] + a[4 * r + c] * xx[c];
    }
    for (int r = 0; r < 4; ++r) y[4 * i + r] = s[r];
  }
}

/* Position of column j in row i, -1 if absent (columns sorted ascending). */
static int64_t find_col(const int *rp, const int *ci, int64_t i, int64_t j) {
  int64_t lo = rp[i], hi = rp[i + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (ci[mid] == j) return mid;
    if (ci[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* A^T on the same (structurally symmetric) pattern: block (j,i) of A^T is the
 * transpose of block (i,j) of A.  Pinned by the dense transpose. */
int or_transpose(int n, const int *rp, const int *ci, const double *v, double *vt) {
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      int64_t q = find_col(rp, ci, ci[p], i);
      if (q < 0) return OR_E_ARG;
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) vt[16 * q + 4 * c + r] = v[16 * p + 4 * r + c];
    }
  return OR_OK;
}
