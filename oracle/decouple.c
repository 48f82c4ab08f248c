/* decouple.c -- ABF / quasi-IMPES decoupling, pressure-matrix extraction,
 * block-Jacobi and block ILU(0) second stage.  FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* Gauss-Jordan elimination on a 4-row augmented system [L | R], L 4x4 and R
 * 4 x w, with partial (row) pivoting only: on exit R holds L^{-1} R.  This is
 * the block-by-block GJE the paper adopts as a decoupling method (Section
 * "Decoupling Methods": [D | A | b] -> [I | A~ | b~], row reordering only).
 * Pivot: the largest |entry| at or below the diagonal, ties to the lowest
 * row.  A pivot of magnitude <= 1e-300 or <= 1e-14 * max|L| is singular.
 * Row p is scaled by the reciprocal of its pivot; every other row q then
 * gets row_q -= L[q][p] * row_p.  Pinned by the dense inverse product. */
static int gje4(double L[4][4], double *R, int w) {
  double amax = 0.0;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) amax = fmax(amax, fabs(L[r][c]));
  if (!(amax == amax) || isinf(amax)) return OR_E_NONFINITE;
  for (int p = 0; p < 4; ++p) {
    int piv = p;
    for (int r = p + 1; r < 4; ++r)
      if (fabs(L[r][p]) > fabs(L[piv][p])) piv = r;
    double pv = L[piv][p];
    if (fabs(pv) <= 1e-300 || fabs(pv) <= 1e-14 * amax) return OR_E_SINGULAR;
    if (piv != p) {
      for (int c = 0; c < 4; ++c) { double t = L[p][c]; L[p][c] = L[piv][c]; L[piv][c] = t; }
      for (int c = 0; c < w; ++c) { double t = R[p * w + c]; R[p * w + c] = R[piv * w + c]; R[piv * w + c] = t; }
    }
    double inv = 1.0 / pv;
    for (int c = p + 1; c < 4; ++c) L[p][c] = L[p][c] * inv;
    for (int c = 0; c < w; ++c) R[p * w + c] = R[p * w + c] * inv;
    L[p][p] = 1.0;
    for (int q = 0; q < 4; ++q) {
      if (q == p) continue;
      double f = L[q][p];
      for (int c = p + 1; c < 4; ++c) L[q][c] = L[q][c] - f * L[p][c];
      for (int c = 0; c < w; ++c) R[q * w + c] = R[q * w + c] - f * R[p * w + c];
      L[q][p] = 0.0;
    }
  }
  return OR_OK;
}

static int64_t diag_pos(const int *rp, const int *ci, int64_t i) {
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
    if (ci[p] == i) return p;
  return -1;
}

/* Inverse of one 4x4 block by GJE on [A | I]. */
static int inv4(const double *a, double *out) {
  double L[4][4], R[16];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) { L[r][c] = a[4 * r + c]; R[4 * r + c] = (r == c) ? 1.0 : 0.0; }
  int st = gje4(L, R, 4);
  if (st == OR_OK) memcpy(out, R, sizeof(R));
  return st;
}

/* Decoupling as a left scaling (D^{-1} A) x = D^{-1} b (Eq. decoupled-eq).
 *  ABF (Eq. decoupled-abf): D = diag(A_11, ..., A_nn).  Computed by GJE on
 *    the block row [A_ii | A_i,j (j != i) | I]: the result gives
 *    A~_ij = A_ii^{-1} A_ij and D_i^{-1} = A_ii^{-1}; A~_ii is set to I.
 *  Quasi-IMPES (named in the paper only): w_i solves A_ii^T w_i = e_0 (GJE
 *    on [A_ii^T | e_0]); row 0 of every block in row i becomes w_i^T A_ij,
 *    rows 1-3 are unchanged; D_i^{-1} = [w_i^T; e_1^T; e_2^T; e_3^T].
 *  FRS (Eq. decoupled-frs): D_i^{-1} = F, the 4x4 matrix with ones in row
 *    0 and on the diagonal, zeros elsewhere: row 0 of every block (and of
 *    the right-hand side) becomes the sum of its four rows, summed in row
 *    order; rows 1-3 are unchanged.
 *  FRS+ABF (the two-stage decoupling of the same section): FRS first, then
 *    ABF on the result, i.e. GJE on [F A_ii | F A_i,j | F]:
 *    A~_ij = (F A_ii)^{-1} F A_ij, D_i^{-1} = (F A_ii)^{-1} F.  In exact
 *    arithmetic this equals ABF alone, since (F A_ii)^{-1} F = A_ii^{-1}.
 * vt receives the decoupled blocks (same pattern), dinv the 4x4 D_i^{-1}.
 * Pinned by the dense product blockdiag(A)^{-1} A, by A~_ii = I, by the
 * quasi-IMPES pressure row equalling the ABF one, by D^{-1}A x = D^{-1}b
 * sharing the solution of A x = b, by FRS equalling blockdiag(F) A, and by
 * FRS+ABF equalling ABF to rounding. */
int or_decouple(int n, const int *rp, const int *ci, const double *v, int method,
                double *vt, double *dinv) {
  int maxw = 0;
  for (int64_t i = 0; i < n; ++i) {
    int w = (rp[i + 1] - rp[i]) * 4;
    if (w > maxw) maxw = w;
  }
  double *R = (double *)malloc(sizeof(double) * 4 * (size_t)(maxw + 4));
  if (!R) return OR_E_ARG;
  int status = OR_OK;
  for (int64_t i = 0; i < n && status == OR_OK; ++i) {
    int64_t pd = diag_pos(rp, ci, i);
    if (pd < 0) { status = OR_E_ARG; break; }
    const double *Aii = &v[16 * pd];
    int nb = rp[i + 1] - rp[i];
    if (method == OR_ABF || method == OR_FRS_ABF) {
      int w = 4 * nb + 4;     /* every block of the row, then I (F for FRS+ABF) */
      double L[4][4];
      for (int r = 0; r < 4; ++r) {
        for (int c = 0; c < 4; ++c) L[r][c] = Aii[4 * r + c];
        for (int b = 0; b < nb; ++b)
          for (int c = 0; c < 4; ++c) R[r * w + 4 * b + c] = v[16 * (rp[i] + b) + 4 * r + c];
        for (int c = 0; c < 4; ++c) R[r * w + 4 * nb + c] = (r == c) ? 1.0 : 0.0;
      }
      if (method == OR_FRS_ABF) {
        for (int c = 0; c < 4; ++c) L[0][c] = ((L[0][c] + L[1][c]) + L[2][c]) + L[3][c];
        for (int c = 0; c < w; ++c) R[c] = ((R[c] + R[w + c]) + R[2 * w + c]) + R[3 * w + c];
      }
      status = gje4(L, R, w);
      if (status != OR_OK) break;
      for (int b = 0; b < nb; ++b) {
        double *o = &vt[16 * (rp[i] + b)];
        if (rp[i] + b == pd) {
          for (int e = 0; e < 16; ++e) o[e] = (e % 5 == 0) ? 1.0 : 0.0;
        } else {
          for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) o[4 * r + c] = R[r * w + 4 * b + c];
        }
      }
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) dinv[16 * i + 4 * r + c] = R[r * w + 4 * nb + c];
    } else if (method == OR_QIMPES) {
      double L[4][4], e0[4] = {1.0, 0.0, 0.0, 0.0};
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) L[r][c] = Aii[4 * c + r];   /* A_ii^T */
      status = gje4(L, e0, 1);
      if (status != OR_OK) break;
      for (int b = 0; b < nb; ++b) {
        const double *a = &v[16 * (rp[i] + b)];
        double *o = &vt[16 * (rp[i] + b)];
        for (int c = 0; c < 4; ++c) {
          double s = 0.0;
          for (int m = 0; m < 4; ++m) s = s + e0[m] * a[4 * m + c];
          o[c] = s;
        }
        for (int e = 4; e < 16; ++e) o[e] = a[e];
      }
      double *d = &dinv[16 * i];
      for (int e = 0; e < 16; ++e) d[e] = 0.0;
      for (int c = 0; c < 4; ++c) d[c] = e0[c];
      d[5] = d[10] = d[15] = 1.0;
    } else if (method == OR_FRS) {
      for (int b = 0; b < nb; ++b) {
        const double *a = &v[16 * (rp[i] + b)];
        double *o = &vt[16 * (rp[i] + b)];
        for (int c = 0; c < 4; ++c) o[c] = ((a[c] + a[4 + c]) + a[8 + c]) + a[12 + c];
        for (int e = 4; e < 16; ++e) o[e] = a[e];
      }
      double *d = &dinv[16 * i];
      for (int e = 0; e < 16; ++e) d[e] = (e < 4 || e % 5 == 0) ? 1.0 : 0.0;
    } else {
      status = OR_E_ARG;
    }
  }
  free(R);
  return status;
}

/* Pressure sub-matrix ("getting sub-matrix (for CPR-type preconditioners)",
 * Section "Linear Solver"): A_p[i][j] = A~_ij[0][0], same pattern.
 * Pinned by brute-force indexing of the dense decoupled matrix. */
void or_extract_pressure(int64_t nnzb, const double *vt, double *ap) {
  for (int64_t p = 0; p < nnzb; ++p) ap[p] = vt[16 * p];
}

/* Block-Jacobi: restricted additive Schwarz with overlap 0 on one subdomain
 * per block (Section "Preconditioners": overlap 0 is block Jacobi).
 * z_i = A~_ii^{-1} r_i.  Under ABF A~_ii = I and this is the identity. */
int or_bj_setup(int n, const int *rp, const int *ci, const double *vt, double *dinv2) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t pd = diag_pos(rp, ci, i);
    if (pd < 0) return OR_E_ARG;
    int st = inv4(&vt[16 * pd], &dinv2[16 * i]);
    if (st != OR_OK) return st;
  }
  return OR_OK;
}

static void matvec4(const double *a, const double *x, double *y) {
  for (int r = 0; r < 4; ++r) {
    double s = 0.0;
    for (int c = 0; c < 4; ++c) s = s + a[4 * r + c] * x[c];
    y[r] = s;
  }
}

void or_bj_apply(int n, const double *dinv2, const double *r, double *z) {
  for (int64_t i = 0; i < n; ++i) matvec4(&dinv2[16 * i], &r[4 * i], &z[4 * i]);
}

/* Block ILU(0) in natural (cell) order, the local solver named for RAS
 * (Section "Preconditioners": ILU(k) or block ILU(k); k = 0 here).  On a
 * 7-point block pattern no fill position of ILU(0) lies on the pattern, so
 * only the diagonal blocks change (DILU):
 *    D_i = A~_ii - sum_{k < i, (i,k) stored} A~_ik D_k^{-1} A~_ki,
 * stored as D_i^{-1}.  Pinned by the ILU(0) identity (L U)_ij = A~_ij on
 * the pattern with L = (D + A~_lower) D^{-1}, U = D + A~_upper. */
int or_dilu_setup(int n, const int *rp, const int *ci, const double *vt, double *dinv2) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t pd = diag_pos(rp, ci, i);
    if (pd < 0) return OR_E_ARG;
    double D[16];
    memcpy(D, &vt[16 * pd], sizeof(D));
    for (int64_t p = rp[i]; p < pd; ++p) {
      int64_t k = ci[p];
      int64_t q = -1;                       /* position of (k, i) */
      for (int64_t t = rp[k]; t < rp[k + 1]; ++t)
        if (ci[t] == i) { q = t; break; }
      if (q < 0) return OR_E_ARG;
      double T1[16], T2[16];               /* T1 = D_k^{-1} A~_ki, T2 = A~_ik T1 */
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          double s = 0.0;
          for (int m = 0; m < 4; ++m) s = s + dinv2[16 * k + 4 * r + m] * vt[16 * q + 4 * m + c];
          T1[4 * r + c] = s;
        }
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          double s = 0.0;
          for (int m = 0; m < 4; ++m) s = s + vt[16 * p + 4 * r + m] * T1[4 * m + c];
          T2[4 * r + c] = s;
        }
      for (int e = 0; e < 16; ++e) D[e] = D[e] - T2[e];
    }
    int st = inv4(D, &dinv2[16 * i]);
    if (st != OR_OK) return st;
  }
  return OR_OK;
}

/* DILU solve z = M^{-1} r with M = (D + A~_lower) D^{-1} (D + A~_upper):
 * forward  y_i = D_i^{-1} (r_i - sum_{k<i} A~_ik y_k),
 * backward z_i = y_i - D_i^{-1} sum_{j>i} A~_ij z_j.
 * Pinned by dense triangular solves with the same factors. */
void or_dilu_apply(int n, const int *rp, const int *ci, const double *vt,
                   const double *dinv2, const double *r, double *z) {
  double *y = z;
  for (int64_t i = 0; i < n; ++i) {
    double s[4];
    for (int c = 0; c < 4; ++c) s[c] = r[4 * i + c];
    for (int64_t p = rp[i]; p < rp[i + 1] && ci[p] < i; ++p) {
      double t[4];
      matvec4(&vt[16 * p], &y[4 * (int64_t)ci[p]], t);
      for (int c = 0; c < 4; ++c) s[c] = s[c] - t[c];
    }
    matvec4(&dinv2[16 * i], s, &y[4 * i]);
  }
  for (int64_t i = (int64_t)n - 1; i >= 0; --i) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      if (ci[p] <= i) continue;
      double t[4];
      matvec4(&vt[16 * p], &z[4 * (int64_t)ci[p]], t);
      for (int c = 0; c < 4; ++c) s[c] = s[c] + t[c];
    }
    double u[4];
    matvec4(&dinv2[16 * i], s, u);
    for (int c = 0; c < 4; ++c) z[4 * i + c] = y[4 * i + c] - u[c];
  }
}

/* Restricted additive Schwarz with zero overlap (Section "Preconditioners":
 * with overlap 0 RAS is block Jacobi over the subdomains) and block ILU(0)
 * as the subdomain solver (BILU(k), k = 0, named in the same section).
 * Subdomain of cell i is floor(i / sub); with cells numbered i fastest and
 * sub = nx*ny the subdomains are the xy-layers of the grid.  Block Jacobi over
 * subdomains means every block that couples two subdomains is left out, so
 * the preconditioner is the DILU of the restricted matrix built here.
 * Returns a new CSR pattern and values (caller frees *rp2, *ci2, *vt2).
 * Pinned by: sub >= n gives the global DILU; each subdomain solved on its
 * own extracted matrix gives the same result; the dense product
 * (D+L)D^{-1}(D+U) equals the restricted matrix on its pattern. */
int or_ras_restrict(int n, int64_t sub, const int *rp, const int *ci, const double *vt,
                    int **rp2, int **ci2, double **vt2) {
  if (sub < 1) return OR_E_ARG;
  int64_t keep = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
      if (ci[p] / sub == i / sub) ++keep;
  *rp2 = (int *)malloc(sizeof(int) * ((size_t)n + 1));
  *ci2 = (int *)malloc(sizeof(int) * (size_t)(keep > 0 ? keep : 1));
  *vt2 = (double *)malloc(sizeof(double) * 16 * (size_t)(keep > 0 ? keep : 1));
  int64_t q = 0;
  (*rp2)[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      if (ci[p] / sub != i / sub) continue;
      (*ci2)[q] = ci[p];
      memcpy(&(*vt2)[16 * q], &vt[16 * p], 16 * sizeof(double));
      ++q;
    }
    (*rp2)[i + 1] = (int)q;
  }
  return OR_OK;
}

void or_free(void *p) { free(p); }
