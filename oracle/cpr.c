/* cpr.c -- two-stage CPR preconditioner, restarted flexible GMRES and the
 * adjoint gradient with respect to log-permeability.  FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

struct or_cpr {
  int n, smoother, stages;
  int64_t nnzb;
  const int *rp, *ci;      /* borrowed pattern */
  int *rpc, *cic;          /* own copy of the pattern */
  double *vt;              /* decoupled blocks */
  double *dinv;            /* decoupling D_i^{-1} */
  double *ap;              /* pressure matrix values */
  double *dinv2;           /* second-stage block inverses */
  int *rp2, *ci2;          /* RAS: pattern restricted to the subdomains */
  double *vt2;             /* RAS: decoupled blocks on that pattern */
  or_rasov *ras;           /* RAS with overlap 1 */
  or_amg *amg;
};

/* CPR of pressure-then-full type (stages = 2) or the three-stage CPR-FPF
 * (stages = 3) of Section "Preconditioners" (Algorithm pc-fpf).  The printed
 * algorithm repeats its first step as its third; the text around it gives
 * five steps, which are what stages = 3 computes, on the decoupled system:
 *    f   = D^{-1} r                          (decoupling, Eq. decoupled-eq)
 *    1.  y = M2^{-1} f                       (full-system stage)
 *    2.  q = f - A~ y
 *    3.  y = y + Pi_p Vcycle(A_p, Pi_r q)    (pressure stage)
 *    4.  q = f - A~ y
 *    5.  y = y + M2^{-1} q                   (full-system stage)
 * M2 is block Jacobi, DILU, or RAS with DILU in each subdomain (overlap 0,
 * or overlap 1: ras.c), on A~; Pi_r takes unknown 0, Pi_p injects into
 * unknown 0.
 * stages = 2 keeps steps 3-5 with y = 0:
 *    x_p = Vcycle(A_p, Pi_r f),  z = M2^{-1}(f - A~ Pi_p x_p) + Pi_p x_p.
 * Pinned by the dense compositions, with S = M2^{-1} and
 * C = Pi_p A_p^{-1} Pi_r when the AMG is a single exact level:
 *    two-stage    [C + S(I - A~ C)] D^{-1}
 *    three-stage  [S + (C + S(I - A~ C))(I - A~ S)] D^{-1},
 * the latter also through its error propagation
 *    I - A~ M^{-1} D = (I - A~ S)(I - A~ C)(I - A~ S). */
or_cpr *or_cpr_setup(int n, const int *rp, const int *ci, const double *v,
                     int method, int smoother, int64_t sub, int stages,
                     const or_amg_opts *ao, int *status) {
  or_cpr *M = (or_cpr *)calloc(1, sizeof(or_cpr));
  int64_t nnzb = rp[n];
  M->n = n; M->smoother = smoother; M->nnzb = nnzb; M->stages = stages;
  if (stages != 2 && stages != 3) { *status = OR_E_ARG; return M; }
  M->rpc = (int *)malloc(sizeof(int) * ((size_t)n + 1));
  M->cic = (int *)malloc(sizeof(int) * (size_t)nnzb);
  memcpy(M->rpc, rp, sizeof(int) * ((size_t)n + 1));
  memcpy(M->cic, ci, sizeof(int) * (size_t)nnzb);
  M->rp = M->rpc; M->ci = M->cic;
  M->vt = (double *)malloc(sizeof(double) * 16 * (size_t)nnzb);
  M->dinv = (double *)malloc(sizeof(double) * 16 * (size_t)n);
  M->ap = (double *)malloc(sizeof(double) * (size_t)nnzb);
  M->dinv2 = (double *)malloc(sizeof(double) * 16 * (size_t)n);
  *status = or_decouple(n, rp, ci, v, method, M->vt, M->dinv);
  if (*status != OR_OK) return M;
  or_extract_pressure(nnzb, M->vt, M->ap);
  if (smoother == OR_SM_RAS) {
    *status = or_ras_restrict(n, sub, rp, ci, M->vt, &M->rp2, &M->ci2, &M->vt2);
    if (*status == OR_OK) *status = or_dilu_setup(n, M->rp2, M->ci2, M->vt2, M->dinv2);
  } else if (smoother == OR_SM_RAS1) {
    M->ras = or_rasov_setup(n, rp, ci, M->vt, sub, 1, status);
    if (*status == OR_OK) or_rasov_owned_dinv(M->ras, M->dinv2);
  } else {
    *status = (smoother == OR_SM_DILU) ? or_dilu_setup(n, rp, ci, M->vt, M->dinv2)
                                       : or_bj_setup(n, rp, ci, M->vt, M->dinv2);
  }
  if (*status != OR_OK) return M;
  M->amg = or_amg_setup(n, rp, ci, M->ap, ao, status);
  return M;
}

static void m2_apply(const or_cpr *M, const double *r, double *z) {
  int n = M->n;
  if (M->smoother == OR_SM_DILU) or_dilu_apply(n, M->rp, M->ci, M->vt, M->dinv2, r, z);
  else if (M->smoother == OR_SM_RAS) or_dilu_apply(n, M->rp2, M->ci2, M->vt2, M->dinv2, r, z);
  else if (M->smoother == OR_SM_RAS1) or_rasov_apply(M->ras, M->vt, r, z);
  else or_bj_apply(n, M->dinv2, r, z);
}

void or_cpr_apply(const or_cpr *M, const double *r, double *z) {
  int n = M->n;
  int64_t N = 4 * (int64_t)n;
  double *f = (double *)malloc(sizeof(double) * (size_t)N);
  double *q = (double *)malloc(sizeof(double) * (size_t)N);
  double *w = (double *)malloc(sizeof(double) * (size_t)N);
  double *bp = (double *)malloc(sizeof(double) * (size_t)n);
  double *xp = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 4; ++a) {
      double s = 0.0;
      for (int c = 0; c < 4; ++c) s = s + M->dinv[16 * i + 4 * a + c] * r[4 * i + c];
      f[4 * i + a] = s;
    }
  if (M->stages == 2) {
    for (int64_t i = 0; i < n; ++i) bp[i] = f[4 * i];
    or_amg_vcycle(M->amg, bp, xp);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p) {
        double xj = xp[M->ci[p]];
        for (int a = 0; a < 4; ++a) f[4 * i + a] = f[4 * i + a] - M->vt[16 * p + 4 * a] * xj;
      }
    m2_apply(M, f, z);
    for (int64_t i = 0; i < n; ++i) z[4 * i] = z[4 * i] + xp[i];
  } else {
    m2_apply(M, f, z);                                            /* 1 */
    or_spmv(n, M->rp, M->ci, M->vt, z, q);                        /* 2 */
    for (int64_t t = 0; t < N; ++t) q[t] = f[t] - q[t];
    for (int64_t i = 0; i < n; ++i) bp[i] = q[4 * i];             /* 3 */
    or_amg_vcycle(M->amg, bp, xp);
    for (int64_t i = 0; i < n; ++i) z[4 * i] = z[4 * i] + xp[i];
    or_spmv(n, M->rp, M->ci, M->vt, z, q);                        /* 4 */
    for (int64_t t = 0; t < N; ++t) q[t] = f[t] - q[t];
    m2_apply(M, q, w);                                            /* 5 */
    for (int64_t t = 0; t < N; ++t) z[t] = z[t] + w[t];
  }
  free(f); free(q); free(w); free(bp); free(xp);
}

const double *or_cpr_decoupled(const or_cpr *M) { return M->vt; }
const double *or_cpr_dinv(const or_cpr *M) { return M->dinv; }
const double *or_cpr_dinv2(const or_cpr *M) { return M->dinv2; }
const double *or_cpr_pressure(const or_cpr *M) { return M->ap; }
const or_amg *or_cpr_amg(const or_cpr *M) { return M->amg; }

void or_cpr_free(or_cpr *M) {
  if (!M) return;
  free(M->rpc); free(M->cic); free(M->vt); free(M->dinv); free(M->ap); free(M->dinv2);
  free(M->rp2); free(M->ci2); free(M->vt2);
  or_rasov_free(M->ras);
  or_amg_free(M->amg);
  free(M);
}

static double dot(int64_t m, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i) s = s + a[i] * b[i];
  return s;
}

/* Restarted, right-preconditioned flexible GMRES(m) for A x = b (the Krylov
 * solver of Section "Linear Solver"; the paper names GMRES without details).
 * Arnoldi with classical Gram-Schmidt applied twice; Givens rotations via
 * hypot; the cycle stops when the rotated residual |g_{j+1}| <= rtol*||b||,
 * on breakdown h_{j+1,j} <= 1e-14*||A z_j||, or at maxit; x += Z y; a new
 * cycle starts from the true residual until ||b - A x|| <= rtol*||b|| or
 * maxit Arnoldi steps have run.  M == NULL means no preconditioner.
 * hist (optional) receives the rotated residual estimate per step.
 * Pinned by: convergence in at most N steps when restart >= N, the dense-LU
 * solution on small grids, and the closed-form DCT solution of the
 * separable (homogeneous) problem. */
int or_gmres(int n, const int *rp, const int *ci, const double *v, const or_cpr *M,
             const double *b, double *x, int restart, double rtol, int maxit,
             or_info *info, double *hist, int hist_len) {
  int64_t N = 4 * (int64_t)n;
  int m = restart;
  if (m < 1 || m > 63 || n < 1) return OR_E_ARG;
  double *V = (double *)malloc(sizeof(double) * (size_t)N * (size_t)(m + 1));
  double *Z = (double *)malloc(sizeof(double) * (size_t)N * (size_t)m);
  double *w = (double *)malloc(sizeof(double) * (size_t)N);
  double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * (size_t)m);
  double *sn = (double *)malloc(sizeof(double) * (size_t)m);
  double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *y = (double *)malloc(sizeof(double) * (size_t)m);
  double *h = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double bnorm = sqrt(dot(N, b, b));
  int iters = 0, cycles = 0, status = 1;
  double relres = 0.0;
  if (!(bnorm == bnorm) || isinf(bnorm)) { status = OR_E_NONFINITE; goto done; }
  if (bnorm == 0.0) { for (int64_t i = 0; i < N; ++i) x[i] = 0.0; status = 0; goto done; }
  for (;;) {
    or_spmv(n, rp, ci, v, x, w);
    for (int64_t i = 0; i < N; ++i) w[i] = b[i] - w[i];
    double beta = sqrt(dot(N, w, w));
    relres = beta / bnorm;
    if (beta <= rtol * bnorm) { status = 0; break; }
    if (iters >= maxit) { status = 1; break; }
    for (int64_t i = 0; i < N; ++i) V[i] = w[i] / beta;
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    int k = 0;
    ++cycles;
    for (int j = 0; j < m; ++j) {
      double *vj = &V[(size_t)j * N], *zj = &Z[(size_t)j * N];
      if (M) or_cpr_apply(M, vj, zj); else memcpy(zj, vj, sizeof(double) * (size_t)N);
      or_spmv(n, rp, ci, v, zj, w);
      double wn0 = sqrt(dot(N, w, w));
      for (int i = 0; i <= j; ++i) h[i] = 0.0;
      for (int pass = 0; pass < 2; ++pass) {
        double hh[64];
        for (int i = 0; i <= j; ++i) hh[i] = dot(N, &V[(size_t)i * N], w);
        for (int i = 0; i <= j; ++i) {
          const double *vi = &V[(size_t)i * N];
          for (int64_t t = 0; t < N; ++t) w[t] = w[t] - hh[i] * vi[t];
        }
        for (int i = 0; i <= j; ++i) h[i] = h[i] + hh[i];
      }
      double hn = sqrt(dot(N, w, w));
      for (int i = 0; i <= j; ++i) H[i * m + j] = h[i];
      H[(j + 1) * m + j] = hn;
      ++iters;
      k = j + 1;
      for (int i = 0; i < j; ++i) {
        double a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      double a = H[j * m + j], c = H[(j + 1) * m + j];
      double d = hypot(a, c);
      cs[j] = a / d; sn[j] = c / d;
      H[j * m + j] = d; H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      if (hist && iters - 1 < hist_len) hist[iters - 1] = fabs(g[j + 1]) / bnorm;
      if (hn <= 1e-14 * wn0) break;                        /* happy breakdown */
      for (int64_t t = 0; t < N; ++t) V[(size_t)(j + 1) * N + t] = w[t] / hn;
      if (fabs(g[j + 1]) <= rtol * bnorm || iters >= maxit) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < k; ++c) s = s - H[i * m + c] * y[c];
      y[i] = s / H[i * m + i];
    }
    for (int i = 0; i < k; ++i) {
      const double *zi = &Z[(size_t)i * N];
      for (int64_t t = 0; t < N; ++t) x[t] = x[t] + y[i] * zi[t];
    }
  }
done:
  if (info) { info->iters = iters; info->cycles = cycles; info->status = status; info->relres = relres; }
  free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y); free(h);
  return status;
}

/* Right-preconditioned BiCGSTAB (van der Vorst, 1992) for A x = b.  The
 * paper names BiCGSTAB beside GMRES in Section "Linear Solver" and runs every
 * experiment with it, without further detail; this is the textbook method
 * with M applied on the right (p^ = M^{-1} p, s^ = M^{-1} s), so the
 * residual it updates is that of the original system:
 *   r = b - A x, shadow r^ = r, rho_0 = alpha = omega = 1, p = v = 0
 *   iteration i:
 *     rho_i = (r^, r)                          breakdown if rho_i == 0
 *     p     = r + (rho_i / rho_{i-1})(alpha / omega) (p - omega v)
 *     v     = A p^,  alpha = rho_i / (r^, v)   breakdown if (r^, v) == 0
 *     s     = r - alpha v
 *     if ||s|| <= rtol ||b||:  x += alpha p^, leave the loop
 *     t     = A s^,  omega = (t, s) / (t, t)   breakdown if (t, t) == 0
 *     x    += alpha p^ + omega s^,  r = s - omega t
 *     leave the loop if ||r|| <= rtol ||b||;  breakdown if omega == 0
 * (With p = v = 0 the first iteration gives p = r.)  When the loop is left
 * (estimate met, breakdown, or maxit iterations) the true residual b - A x is
 * recomputed; if it misses rtol and iterations remain, the method starts
 * again from it with r^ = r.  A breakdown in the first iteration after a
 * start ends the solve.  maxit counts iterations (two products with A and
 * two applications of M each; one of each when it stops at s).
 * M == NULL means no preconditioner.  hist (optional) receives ||r||/||b||
 * (||s||/||b|| for an iteration that stops at s) per iteration.
 * Pinned by: the iterates of an independent implementation of the same
 * recurrence, convergence in one half-iteration when A is a multiple of I,
 * the agreement of the updated and the recomputed residual, and the
 * dense-LU solution on small grids. */
int or_bicgstab(int n, const int *rp, const int *ci, const double *v, const or_cpr *M,
                const double *b, double *x, double rtol, int maxit, or_info *info,
                double *hist, int hist_len) {
  int64_t N = 4 * (int64_t)n;
  if (n < 1 || maxit < 0) return OR_E_ARG;
  double *r = (double *)malloc(sizeof(double) * (size_t)N);
  double *rh = (double *)malloc(sizeof(double) * (size_t)N);
  double *p = (double *)malloc(sizeof(double) * (size_t)N);
  double *vv = (double *)malloc(sizeof(double) * (size_t)N);
  double *ph = (double *)malloc(sizeof(double) * (size_t)N);
  double *sh = (double *)malloc(sizeof(double) * (size_t)N);
  double *t = (double *)malloc(sizeof(double) * (size_t)N);
  double bnorm = sqrt(dot(N, b, b));
  int iters = 0, cycles = 0, status = 1;
  double relres = 0.0;
  if (!(bnorm == bnorm) || isinf(bnorm)) { status = OR_E_NONFINITE; goto done; }
  if (bnorm == 0.0) { for (int64_t i = 0; i < N; ++i) x[i] = 0.0; status = 0; goto done; }
  for (;;) {
    or_spmv(n, rp, ci, v, x, r);
    for (int64_t i = 0; i < N; ++i) r[i] = b[i] - r[i];
    double rn = sqrt(dot(N, r, r));
    relres = rn / bnorm;
    if (!(rn == rn) || isinf(rn)) { status = OR_E_NONFINITE; break; }
    if (rn <= rtol * bnorm) { status = 0; break; }
    if (iters >= maxit) { status = 1; break; }
    ++cycles;
    memcpy(rh, r, sizeof(double) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) { p[i] = 0.0; vv[i] = 0.0; }
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    int first = 1, stop_early = 0;
    while (iters < maxit) {
      double rho = dot(N, rh, r);
      if (rho == 0.0) { stop_early = first; break; }
      double beta = (rho / rho_prev) * (alpha / omega);
      for (int64_t i = 0; i < N; ++i) p[i] = r[i] + beta * (p[i] - omega * vv[i]);
      if (M) or_cpr_apply(M, p, ph); else memcpy(ph, p, sizeof(double) * (size_t)N);
      or_spmv(n, rp, ci, v, ph, vv);
      double rv = dot(N, rh, vv);
      if (rv == 0.0) { stop_early = first; break; }
      alpha = rho / rv;
      ++iters;
      for (int64_t i = 0; i < N; ++i) r[i] = r[i] - alpha * vv[i];   /* r holds s */
      double sn = sqrt(dot(N, r, r));
      if (sn <= rtol * bnorm) {
        for (int64_t i = 0; i < N; ++i) x[i] = x[i] + alpha * ph[i];
        if (hist && iters - 1 < hist_len) hist[iters - 1] = sn / bnorm;
        break;
      }
      if (M) or_cpr_apply(M, r, sh); else memcpy(sh, r, sizeof(double) * (size_t)N);
      or_spmv(n, rp, ci, v, sh, t);
      double tt = dot(N, t, t);
      if (tt == 0.0) {
        for (int64_t i = 0; i < N; ++i) x[i] = x[i] + alpha * ph[i];
        stop_early = first;
        break;
      }
      omega = dot(N, t, r) / tt;
      for (int64_t i = 0; i < N; ++i) {
        x[i] = x[i] + alpha * ph[i] + omega * sh[i];
        r[i] = r[i] - omega * t[i];
      }
      double rnn = sqrt(dot(N, r, r));
      if (hist && iters - 1 < hist_len) hist[iters - 1] = rnn / bnorm;
      rho_prev = rho;
      first = 0;
      if (!(rnn == rnn) || isinf(rnn)) break;
      if (rnn <= rtol * bnorm || omega == 0.0) break;
    }
    if (stop_early) {
      or_spmv(n, rp, ci, v, x, r);
      for (int64_t i = 0; i < N; ++i) r[i] = b[i] - r[i];
      relres = sqrt(dot(N, r, r)) / bnorm;
      status = relres <= rtol ? 0 : 1;
      break;
    }
  }
done:
  if (info) { info->iters = iters; info->cycles = cycles; info->status = status; info->relres = relres; }
  free(r); free(rh); free(p); free(vv); free(ph); free(sh); free(t);
  return status;
}

/* Gradient of J = w^T x, A(theta) x = b, with respect to theta = log k, given
 * the adjoint state lambda (A^T lambda = w) and the solution x:
 *   dJ/dtheta_c = -lambda^T (dA/dtheta_c) x.
 * A depends on theta through the face transmissibilities T_ab (harmonic
 * mean of the directional permeabilities, Section "Numerical Methods") and
 * through the well terms u_c*k_c*I.  Differentiating the assembly:
 *   face (a,b): d/dT of lambda^T A x = lambda_a^T M_ab (x_a - x_b)
 *                                     + lambda_b^T M_ba (x_b - x_a),
 *     dT/dtheta_a = s * 2 k_a k_b^2 / (k_a + k_b)^2  (s = tscale*kv/kh on z
 *     faces, tscale otherwise; symmetric in a <-> b);
 *   well cell c:  lambda_c^T (u_c k_c) x_c.
 * Pinned by central finite differences of J through dense solves and by the
 * duality lambda^T b = w^T x. */
int or_grad_logk(int nx, int ny, int nz, const double *logk, double kvkh, double tscale,
                 const double *Mf, const double *Mb, int nw, const int *wcell,
                 const double *wu, const double *lam, const double *x, double *g) {
  int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
  double *k = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t c = 0; c < n; ++c) { k[c] = exp(logk[c]); g[c] = 0.0; }
  for (int64_t c = 0; c < n; ++c) {
    int i = (int)(c % nx), j = (int)((c / nx) % ny), kk = (int)(c / nxy);
    for (int d = 0; d < 3; ++d) {
      int64_t b;
      if (d == 0) { if (i == nx - 1) continue; b = c + 1; }
      else if (d == 1) { if (j == ny - 1) continue; b = c + nx; }
      else { if (kk == nz - 1) continue; b = c + nxy; }
      double s = tscale * ((d == 2) ? kvkh : 1.0);
      double ka = k[c], kb = k[b];
      double den = (ka + kb) * (ka + kb);
      double dTa = s * 2.0 * ka * kb * kb / den;
      double dTb = s * 2.0 * kb * ka * ka / den;
      const double *Mab = &Mf[(d * n + c) * 16], *Mba = &Mb[(d * n + c) * 16];
      double e = 0.0;
      for (int r = 0; r < 4; ++r)
        for (int q = 0; q < 4; ++q) {
          e = e + lam[4 * c + r] * Mab[4 * r + q] * (x[4 * c + q] - x[4 * b + q]);
          e = e + lam[4 * b + r] * Mba[4 * r + q] * (x[4 * b + q] - x[4 * c + q]);
        }
      g[c] = g[c] - dTa * e;
      g[b] = g[b] - dTb * e;
    }
  }
  for (int t = 0; t < nw; ++t) {
    int64_t c = wcell[t];
    double e = 0.0;
    for (int r = 0; r < 4; ++r) e = e + lam[4 * c + r] * x[4 * c + r];
    g[c] = g[c] - wu[t] * k[c] * e;
  }
  free(k);
  return OR_OK;
}
