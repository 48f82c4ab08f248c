// assemble.hip -- the synthetic Jacobian on the device, and the chain rule
// back from dJ/dA to dJ/dlog k for the adjoint.
//
// Face transmissibility is tscale times the harmonic mean of the two cells'
// directional permeabilities (Section "Numerical Methods": harmonic
// averaging of the geometric part, one value shared by both cells of a
// face, zero on no-flow boundary faces).  Each row's diagonal block is the
// accumulation block over dt, plus T*M for every face of the row (the
// negated off-diagonal blocks), plus u*k*I in perforated cells (Peaceman
// form, well index proportional to k; Section "Well Modeling").
// FMA contraction is off so the blocks are the same products and sums as in
// a plain FP64 evaluation.
#pragma clang fp contract(off)
#include "rs_internal.h"
#include <math.h>

namespace {

__device__ __forceinline__ int64_t nbr_of(int64_t c, int s, int64_t nx, int64_t nxy) {
  switch (s) {
    case 0: return c - nxy;
    case 1: return c - nx;
    case 2: return c - 1;
    case 3: return c;
    case 4: return c + 1;
    case 5: return c + nx;
    default: return c + nxy;
  }
}
__device__ __forceinline__ bool in_grid(int s, int i, int j, int k, int nx, int ny, int nz) {
  switch (s) {
    case 0: return k > 0;
    case 1: return j > 0;
    case 2: return i > 0;
    case 3: return true;
    case 4: return i < nx - 1;
    case 5: return j < ny - 1;
    default: return k < nz - 1;
  }
}
__device__ __forceinline__ int axis_of(int s) { return s == 0 || s == 6 ? 2 : (s == 1 || s == 5 ? 1 : 0); }

// index of cell c in the ascending well list, or -1
__device__ __forceinline__ int well_of(int nw, const int32_t *__restrict__ wc, int64_t c) {
  int lo = 0, hi = nw - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    if (wc[mid] == c) return mid;
    if (wc[mid] < c) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// position of stencil slot s in the caller row of cell c
__device__ __forceinline__ int64_t pos_of(const int32_t *__restrict__ rp, int64_t c, int s, int i, int j,
                                          int k, int nx, int ny, int nz) {
  int64_t p = rp[c];
  for (int t = 0; t < s; ++t) p += in_grid(t, i, j, k, nx, ny, nz) ? 1 : 0;
  return p;
}

__global__ void k_assemble(int nx, int ny, int nz, const double *__restrict__ logk, double kvkh, double tscale,
                           const double *__restrict__ Mf, const double *__restrict__ Mb,
                           const double *__restrict__ B, double dt, int nw, const int32_t *__restrict__ wc,
                           const double *__restrict__ wu, const int32_t *__restrict__ rp,
                           double *__restrict__ vals) {
  int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = B[16 * c + e] / dt;
  int64_t p = rp[c], diagpos = p;
  for (int s = 0; s < 7; ++s) {
    if (!in_grid(s, i, j, k, nx, ny, nz)) continue;
    if (s == 3) { diagpos = p++; continue; }
    int64_t q = nbr_of(c, s, nx, nxy);
    int d = axis_of(s);
    int64_t lo = q < c ? q : c, hi = q < c ? c : q;
    double pa = exp(logk[lo]), pb = exp(logk[hi]);
    if (d == 2) { pa = kvkh * pa; pb = kvkh * pb; }
    double T = tscale * (((2.0 * pa) * pb) / (pa + pb));
    const double *M = (q > c) ? Mf + (d * n + c) * 16 : Mb + (d * n + q) * 16;
    double *o = vals + 16 * p;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double t = T * M[e];
      o[e] = -t;
      acc[e] = acc[e] + t;
    }
    ++p;
  }
  int w = well_of(nw, wc, c);
  if (w >= 0) {
    double ws = wu[w] * exp(logk[c]);
    if (ws != 0.0)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[5 * r] = acc[5 * r] + ws;
  }
  double *o = vals + 16 * diagpos;
#pragma unroll
  for (int e = 0; e < 16; ++e) o[e] = acc[e];
}

// G = -lambda_i x_j^T for every stored block (i,j), caller layout
__global__ void k_grad_vals(int64_t n, int64_t nx, int64_t nxy, const int64_t *__restrict__ pos7,
                            const double *__restrict__ lam, const double *__restrict__ x,
                            double *__restrict__ G) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 7 * n * 16) return;
  int64_t sc = t >> 4;
  int64_t p = pos7[sc];
  if (p < 0) return;
  int e = (int)(t & 15), r = e >> 2, col = e & 3;
  int s = (int)(sc / n);
  int64_t c = sc - (int64_t)s * n;
  int64_t q = nbr_of(c, s, nx, nxy);
  G[16 * p + e] = -(lam[4 * c + r] * x[4 * q + col]);
}

// dJ/dlog k_c = sum over the faces of c of dT/dlog k_c * (G : dA/dT)
//             + u_c k_c trace(G_cc) at wells
__global__ void k_grad_logk(int nx, int ny, int nz, const double *__restrict__ logk, double kvkh,
                            double tscale, const double *__restrict__ Mf, const double *__restrict__ Mb,
                            int nw, const int32_t *__restrict__ wc, const double *__restrict__ wu,
                            const int32_t *__restrict__ rp, const double *__restrict__ G,
                            double *__restrict__ g) {
  int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
  double kc = exp(logk[c]);
  const double *Gcc = G + 16 * pos_of(rp, c, 3, i, j, k, nx, ny, nz);
  double acc = 0.0;
  for (int s = 0; s < 7; ++s) {
    if (s == 3 || !in_grid(s, i, j, k, nx, ny, nz)) continue;
    int64_t q = nbr_of(c, s, nx, nxy);
    int d = axis_of(s);
    int iq = (int)(q % nx), jq = (int)((q / nx) % ny), kq = (int)(q / nxy);
    double kq_ = exp(logk[q]);
    double sc = tscale * (d == 2 ? kvkh : 1.0);
    double den = (kc + kq_) * (kc + kq_);
    double dT = sc * 2.0 * kc * kq_ * kq_ / den;
    const double *Mcq = (q > c) ? Mf + (d * n + c) * 16 : Mb + (d * n + q) * 16;
    const double *Mqc = (q > c) ? Mb + (d * n + c) * 16 : Mf + (d * n + q) * 16;
    const double *Gcq = G + 16 * pos_of(rp, c, s, i, j, k, nx, ny, nz);
    const double *Gqc = G + 16 * pos_of(rp, q, 6 - s, iq, jq, kq, nx, ny, nz);
    const double *Gqq = G + 16 * pos_of(rp, q, 3, iq, jq, kq, nx, ny, nz);
    double e = 0.0;
    for (int t = 0; t < 16; ++t)
      e = e + (Gcc[t] - Gcq[t]) * Mcq[t] + (Gqq[t] - Gqc[t]) * Mqc[t];
    acc = acc + dT * e;
  }
  int w = well_of(nw, wc, c);
  if (w >= 0) acc = acc + wu[w] * kc * (Gcc[0] + Gcc[5] + Gcc[10] + Gcc[15]);
  g[c] = acc;
}

}  // namespace

extern "C" rs_status rs_assemble(int nx, int ny, int nz, const double *d_logk, double kvkh, double tscale,
                                 const double *d_Mf, const double *d_Mb, const double *d_B, double dt,
                                 int nw, const int32_t *d_wcell, const double *d_wu,
                                 const int32_t *d_row_ptr, double *d_vals, void *stream) {
  if (!rs_grid_dims_ok(nx, ny, nz) || nw < 0 || !d_logk || !d_Mf || !d_Mb || !d_B || !d_row_ptr || !d_vals ||
      (nw > 0 && (!d_wcell || !d_wu)) || !(dt > 0.0))
    return RS_E_ARG;
  int64_t n = (int64_t)nx * ny * nz;
  k_assemble<<<rs_grid(n), RS_BLOCK, 0, rs_stream(stream)>>>(nx, ny, nz, d_logk, kvkh, tscale, d_Mf, d_Mb, d_B,
                                                             dt, nw, d_wcell, d_wu, d_row_ptr, d_vals);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

extern "C" rs_status rs_grad_vals(rs_bsr A, const double *d_lambda, const double *d_x, double *d_G,
                                  void *stream) {
  if (!A || !d_lambda || !d_x || !d_G) return RS_E_ARG;
  int64_t n = A->g.n;
  k_grad_vals<<<rs_grid(7 * n * 16), RS_BLOCK, 0, rs_stream(stream)>>>(n, A->g.nx, A->g.nxy, A->pos7.as<int64_t>(),
                                                                       d_lambda, d_x, d_G);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

extern "C" rs_status rs_grad_logk(int nx, int ny, int nz, const double *d_logk, double kvkh, double tscale,
                                  const double *d_Mf, const double *d_Mb, int nw, const int32_t *d_wcell,
                                  const double *d_wu, const int32_t *d_row_ptr, const double *d_G,
                                  double *d_g, void *stream) {
  if (!rs_grid_dims_ok(nx, ny, nz) || nw < 0 || !d_logk || !d_Mf || !d_Mb || !d_row_ptr || !d_G || !d_g ||
      (nw > 0 && (!d_wcell || !d_wu)))
    return RS_E_ARG;
  int64_t n = (int64_t)nx * ny * nz;
  k_grad_logk<<<rs_grid(n), RS_BLOCK, 0, rs_stream(stream)>>>(nx, ny, nz, d_logk, kvkh, tscale, d_Mf, d_Mb, nw,
                                                              d_wcell, d_wu, d_row_ptr, d_G, d_g);
  RS_HIP(hipGetLastError());
  return RS_OK;
}
