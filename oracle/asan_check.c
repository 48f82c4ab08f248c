/* asan_check.c -- memory-safety check program for the oracle (test infrastructure).
 *
 * Built by the CPU test suite together with the oracle's sources under
 * gcc -fsanitize=address,undefined, it reads one small seeded problem (raw
 * little-endian arrays written by the test) and calls every entry point of
 * oracle.h once or more: pattern and assembly, SpMV and transpose, the four
 * decouplings, the second-stage set-ups and applications, RAS with overlap,
 * the AMG hierarchy (piecewise-constant and smoothed prolongators) with a
 * direct and an l1-Jacobi coarsest level, CPR in two
 * and three stages, GMRES (with restarts), BiCGSTAB, the gradient and the
 * thermal residual and Jacobian.  It does no arithmetic of its own beyond
 * checking return codes and finiteness; the sanitizers do the checking.
 *
 * usage: asan_check DIR   (DIR holds dims.i32 and the .f64/.i32 arrays)
 * prints "asan_check ok" and exits 0 when every call succeeded.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static void *load(const char *dir, const char *name, size_t elem, size_t count) {
  char path[1024];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE *f = fopen(path, "rb");
  if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
  void *p = malloc(elem * (count ? count : 1));
  size_t got = fread(p, elem, count, f);
  fclose(f);
  if (got != count) { fprintf(stderr, "%s: %zu of %zu elements\n", path, got, count); exit(2); }
  return p;
}

static int fails = 0;
#define CHECK(expr)                                                        \
  do {                                                                     \
    int st_ = (expr);                                                      \
    if (st_ != 0) { fprintf(stderr, "%s -> %d\n", #expr, st_); ++fails; } \
  } while (0)

static void finite_or_fail(const char *what, const double *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) { fprintf(stderr, "%s[%zu] not finite\n", what, i); ++fails; return; }
}

int main(int argc, char **argv) {
  if (argc != 2) { fprintf(stderr, "usage: %s DIR\n", argv[0]); return 2; }
  const char *dir = argv[1];
  int *dims = load(dir, "dims.i32", sizeof(int), 4);
  const int nx = dims[0], ny = dims[1], nz = dims[2], nw = dims[3];
  const int n = nx * ny * nz;
  const int N = 4 * n;
  double *logk = load(dir, "logk.f64", 8, n);
  double *par = load(dir, "par.f64", 8, 3);         /* kvkh, tscale, dt */
  double *Mf = load(dir, "mf.f64", 8, (size_t)3 * n * 16);
  double *Mb = load(dir, "mb.f64", 8, (size_t)3 * n * 16);
  double *B = load(dir, "b.f64", 8, (size_t)n * 16);
  int *wcell = load(dir, "wcell.i32", sizeof(int), nw);
  double *wu = load(dir, "wu.f64", 8, nw);
  double *rhs = load(dir, "rhs.f64", 8, N);

  /* pattern and assembly */
  int64_t nnzb = or_nnzb(nx, ny, nz);
  int *rp = malloc(sizeof(int) * (n + 1));
  int *ci = malloc(sizeof(int) * nnzb);
  CHECK(or_pattern(nx, ny, nz, rp, ci));
  double *v = calloc((size_t)nnzb * 16, 8);
  CHECK(or_assemble(nx, ny, nz, logk, par[0], par[1], Mf, Mb, B, par[2], nw, wcell, wu, rp, ci, v));
  finite_or_fail("A", v, (size_t)nnzb * 16);

  /* SpMV and transpose */
  double *y = calloc(N, 8), *vt = calloc((size_t)nnzb * 16, 8);
  or_spmv(n, rp, ci, v, rhs, y);
  finite_or_fail("Ax", y, N);
  CHECK(or_transpose(n, rp, ci, v, vt));

  /* decouplings, pressure extraction, second stages */
  double *dinv = calloc((size_t)n * 16, 8), *dinv2 = calloc((size_t)n * 16, 8);
  double *ap = calloc(nnzb, 8), *z = calloc(N, 8);
  for (int m = OR_ABF; m <= OR_FRS_ABF; ++m) {
    CHECK(or_decouple(n, rp, ci, v, m, vt, dinv));
    or_extract_pressure(nnzb, vt, ap);
    CHECK(or_bj_setup(n, rp, ci, vt, dinv2));
    or_bj_apply(n, dinv2, rhs, z);
    CHECK(or_dilu_setup(n, rp, ci, vt, dinv2));
    or_dilu_apply(n, rp, ci, vt, dinv2, rhs, z);
    finite_or_fail("dilu z", z, N);
    int *rp2 = NULL, *ci2 = NULL;
    double *vt2 = NULL;
    CHECK(or_ras_restrict(n, (int64_t)nx * ny, rp, ci, vt, &rp2, &ci2, &vt2));
    or_free(rp2); or_free(ci2); or_free(vt2);
    for (int ov = 0; ov <= 2; ++ov) {
      int st = 0;
      or_rasov *R = or_rasov_setup(n, rp, ci, vt, (int64_t)nx * ny, ov, &st);
      CHECK(st);
      if (R) {
        or_rasov_apply(R, vt, rhs, z);
        finite_or_fail("ras z", z, N);
        or_rasov_owned_dinv(R, dinv2);
        int ne = or_rasov_ext(R, 0, NULL);
        int *ext = malloc(sizeof(int) * (ne ? ne : 1));
        double *ed = malloc(sizeof(double) * 16 * (ne ? ne : 1));
        or_rasov_ext(R, 0, ext);
        or_rasov_ext_dinv(R, 0, ed);
        free(ext); free(ed);
        or_rasov_free(R);
      }
    }
  }

  /* AMG on the ABF pressure matrix: direct and l1-Jacobi coarsest level */
  CHECK(or_decouple(n, rp, ci, v, OR_ABF, vt, dinv));
  or_extract_pressure(nnzb, vt, ap);
  double *bp = calloc(n, 8), *xp = calloc(n, 8);
  for (int i = 0; i < n; ++i) bp[i] = rhs[4 * i];
  for (int variant = 0; variant < 4; ++variant) {
    or_amg_opts o;
    or_amg_defaults(&o);
    if (variant & 1) { o.lu_max = 1; o.coarse_n = 1; }
    if (variant & 2) { o.smooth = 1; o.max_row_sum = 1e30; }
    int st = 0;
    or_amg *h = or_amg_setup(n, rp, ci, ap, &o, &st);
    CHECK(st);
    if (h) {
      for (int l = 0; l < or_amg_nlevels(h); ++l) {
        int nl = or_amg_level_n(h, l);
        int64_t nnz = or_amg_level_nnz(h, l);
        int *lrp = malloc(sizeof(int) * (nl + 1)), *lci = malloc(sizeof(int) * (nnz ? nnz : 1));
        double *la = malloc(sizeof(double) * (nnz ? nnz : 1)), *ld = malloc(sizeof(double) * nl);
        int *agg = malloc(sizeof(int) * nl), *strong = malloc(sizeof(int) * (nnz ? nnz : 1));
        or_amg_level_get(h, l, lrp, lci, la, ld, agg, strong);
        free(lrp); free(lci); free(la); free(ld); free(agg); free(strong);
        int64_t pn = or_amg_level_p(h, l, NULL, NULL, NULL);
        if (pn >= 0) {
          int *prp = malloc(sizeof(int) * (nl + 1)), *pci = malloc(sizeof(int) * (pn ? pn : 1));
          double *pv = malloc(sizeof(double) * (pn ? pn : 1));
          or_amg_level_p(h, l, prp, pci, pv);
          finite_or_fail("P", pv, (size_t)pn);
          free(prp); free(pci); free(pv);
        }
      }
      (void)or_amg_coarsest_is_lu(h);
      or_amg_vcycle(h, bp, xp);
      finite_or_fail("vcycle", xp, n);
      or_amg_free(h);
    }
  }

  /* CPR, GMRES (restart 3 so that cycles restart), BiCGSTAB */
  double *x = calloc(N, 8), *hist = calloc(64, 8);
  or_amg_opts ao;
  or_amg_defaults(&ao);
  for (int sm = OR_SM_BJ; sm <= OR_SM_RAS1; ++sm)
    for (int stages = 2; stages <= 3; ++stages) {
      int st = 0;
      or_cpr *M = or_cpr_setup(n, rp, ci, v, OR_ABF, sm, (int64_t)nx * ny, stages, &ao, &st);
      CHECK(st);
      if (!M) continue;
      or_cpr_apply(M, rhs, z);
      finite_or_fail("cpr z", z, N);
      (void)or_cpr_decoupled(M); (void)or_cpr_dinv(M); (void)or_cpr_dinv2(M);
      (void)or_cpr_pressure(M); (void)or_cpr_amg(M);
      or_info info;
      memset(x, 0, sizeof(double) * N);
      int rc = or_gmres(n, rp, ci, v, M, rhs, x, 3, 1e-8, 40, &info, hist, 64);
      if (rc < 0) { fprintf(stderr, "or_gmres -> %d\n", rc); ++fails; }
      memset(x, 0, sizeof(double) * N);
      rc = or_bicgstab(n, rp, ci, v, M, rhs, x, 1e-8, 40, &info, hist, 64);
      if (rc < 0) { fprintf(stderr, "or_bicgstab -> %d\n", rc); ++fails; }
      finite_or_fail("x", x, N);
      or_cpr_free(M);
    }

  /* gradient with respect to log k */
  double *g = calloc(n, 8);
  CHECK(or_grad_logk(nx, ny, nz, logk, par[0], par[1], Mf, Mb, nw, wcell, wu, rhs, y, g));
  finite_or_fail("grad", g, n);

  /* thermal residual and Jacobian around a plausible state */
  or_thermal_params q;
  or_thermal_defaults(&q);
  double *p = malloc(8 * n), *sw = malloc(8 * n), *so = malloc(8 * n), *t = malloc(8 * n);
  for (int c = 0; c < n; ++c) {
    p[c] = 80.0 + (c % 7); sw[c] = 0.5 + 0.01 * (c % 11); so[c] = 1.0 - sw[c]; t[c] = 150.0 + 3.0 * (c % 13);
  }
  double *u = malloc(8 * N), *u0 = malloc(8 * N), *res = malloc(8 * N);
  or_thermal_state(&q, n, p, sw, so, t, u);
  for (int c = 0; c < n; ++c) { p[c] -= 1.0; t[c] -= 2.0; }
  or_thermal_state(&q, n, p, sw, so, t, u0);
  double *kx = malloc(8 * n), *kz = malloc(8 * n);
  for (int c = 0; c < n; ++c) { kx[c] = exp(logk[c]); kz[c] = par[0] * kx[c]; }
  int *wkind = malloc(sizeof(int) * (nw ? nw : 1));
  double *wval = malloc(8 * (nw ? nw : 1));
  for (int w = 0; w < nw; ++w) { wkind[w] = (w & 1) ? -1 : 1; wval[w] = (w & 1) ? 1.0e4 : 10.0; }
  CHECK(or_thermal_assemble(nx, ny, nz, &q, kx, kx, kz, u, u0, nw, wcell, wkind, wval, rp, ci, v, res));
  finite_or_fail("thermal J", v, (size_t)nnzb * 16);
  finite_or_fail("thermal r", res, N);
  CHECK(or_thermal_assemble(nx, ny, nz, &q, kx, kx, kz, u, u0, nw, wcell, wkind, wval, rp, ci, NULL, res));
  double props[9];
  or_thermal_props(&q, u, props);

  free(dims); free(logk); free(par); free(Mf); free(Mb); free(B); free(wcell); free(wu); free(rhs);
  free(rp); free(ci); free(v); free(y); free(vt); free(dinv); free(dinv2); free(ap); free(z);
  free(bp); free(xp); free(x); free(hist); free(g); free(p); free(sw); free(so); free(t);
  free(u); free(u0); free(res); free(kx); free(kz); free(wkind); free(wval);
  if (fails) { fprintf(stderr, "asan_check: %d failures\n", fails); return 1; }
  printf("asan_check ok\n");
  return 0;
}
