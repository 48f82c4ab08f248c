// block4.h -- 4x4 block helpers shared by the decoupling and the second-stage
// setup: Gauss-Jordan elimination with row pivoting and block loads.
// Include after `#pragma clang fp contract(off)` where the operation order
// must be kept (one multiply and one subtract per update).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define RSF_SINGULAR 1
#define RSF_NONFINITE 2

template <int W>
__device__ __forceinline__ void swap_rows(double (&L)[4][4], double (&R)[4][W], int p, int piv) {
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    if (r > p && r == piv) {
#pragma unroll
      for (int c = 0; c < 4; ++c) { double t = L[p][c]; L[p][c] = L[r][c]; L[r][c] = t; }
#pragma unroll
      for (int c = 0; c < W; ++c) { double t = R[p][c]; R[p][c] = R[r][c]; R[r][c] = t; }
    }
  }
}

// GJE on [L | R]: R <- L^{-1} R.  Returns a RSF_* flag (0 = fine).
template <int W>
__device__ __forceinline__ int gje4(double (&L)[4][4], double (&R)[4][W]) {
  double amax = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) amax = fmax(amax, fabs(L[r][c]));
  if (!isfinite(amax)) return RSF_NONFINITE;
  int flag = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    int piv = p;
    double best = fabs(L[p][p]);
#pragma unroll
    for (int r = p + 1; r < 4; ++r)
      if (fabs(L[r][p]) > best) { best = fabs(L[r][p]); piv = r; }
    swap_rows<W>(L, R, p, piv);
    double pv = L[p][p];
    if (fabs(pv) <= 1e-300 || fabs(pv) <= 1e-14 * amax) { flag = RSF_SINGULAR; pv = 1.0; }
    double inv = 1.0 / pv;
#pragma unroll
    for (int c = p + 1; c < 4; ++c) L[p][c] = L[p][c] * inv;
#pragma unroll
    for (int c = 0; c < W; ++c) R[p][c] = R[p][c] * inv;
    L[p][p] = 1.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q == p) continue;
      double f = L[q][p];
#pragma unroll
      for (int c = p + 1; c < 4; ++c) L[q][c] = L[q][c] - f * L[p][c];
#pragma unroll
      for (int c = 0; c < W; ++c) R[q][c] = R[q][c] - f * R[p][c];
      L[q][p] = 0.0;
    }
  }
  return flag;
}

__device__ __forceinline__ void load16(const double *__restrict__ p, double (&M)[4][4]) {
  const double2 *q = (const double2 *)p;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double2 a = q[2 * r], b = q[2 * r + 1];
    M[r][0] = a.x; M[r][1] = a.y; M[r][2] = b.x; M[r][3] = b.y;
  }
}

