// ras.hip -- second stage as zero-overlap restricted additive Schwarz (RAS)
// with the xy-layers of the grid as subdomains and block ILU(0) inside each
// layer (Section "Preconditioners": RAS with overlap 0 is block Jacobi over
// the subdomains; the subdomain problems are solved by ILU(k) or block
// ILU(k), here k = 0).  On the 7-point block pattern in natural order block
// ILU(0) only modifies the diagonal blocks, so it is DILU; restricted to a
// layer the stencil is the in-plane 5-point one.
//
// Layers are independent.  Inside a layer the recurrences run over the lines
// i + j = lambda (nx + ny - 1 levels): the thread group of line j handles
// cell (lambda - j, j) at level lambda, reads the previous level's values of
// its own line and of line j-1 (j+1 backward) from LDS, and one barrier
// separates the levels.  The factorisation and the FP64 sweeps give each
// layer one workgroup, which never waits on another; the FP32 sweeps split a
// layer into strips of lines, one workgroup each, that hand the boundary
// line's values to the next strip level by level (see the strip sweeps).
// The factorisation uses a quad of lanes per cell in FP64.
//
// The sweeps are written with D^{-1} folded in, which is the same operator
// in exact arithmetic:
//   forward   y = rh - Lh_y y_{c-nx} - Lh_x y_{c-1},   rh = D^{-1} r~2,
//   backward  z = y  - Uh_x z_{c+1}  - Uh_y z_{c+nx},
// with Lh = D^{-1} L and Uh = D^{-1} U formed once at set-up.  Their operands
// are stored level by level ("wavefront order": within a layer, by lambda,
// then by j), so the cells of one level are contiguous in memory; rh is
// formed (and permuted) by an elementwise pass over the whole grid.
//
// Layout: A~ blocks by stencil slot t7[7][n][16] (slots -z -y -x self +x +y
// +z, zeros off-grid), D^{-1} blocks dinv2[n][16]; scaled blocks
// blk[4][n][16] (Lh_y, Lh_x, Uh_x, Uh_y) in wavefront order; vectors [n][4];
// all in the preconditioner's precision.
#include "rs_internal.h"
#include <math.h>
#include <algorithm>
#include <functional>

namespace {
#pragma clang fp contract(off)
#include "block4.h"
#pragma clang fp contract(fast)
#include "quad4.h"

// ---- wavefront order --------------------------------------------------------
// Number of cells (i, j) of an nx x ny layer with i + j < lambda.
__device__ __forceinline__ int64_t tri(int64_t x) { return x > 0 ? x * (x + 1) / 2 : 0; }
__device__ __forceinline__ int64_t wf_off(int lam, int nx, int ny) {
  return tri(lam) - tri(lam - nx) - tri(lam - ny) + tri(lam - nx - ny);
}
__device__ __forceinline__ int wf_jlo(int lam, int nx) { return max(0, lam - nx + 1); }
// position of cell (i, j) of its layer in wavefront order
__device__ __forceinline__ int64_t wf_pos(int i, int j, int nx, int ny) {
  return wf_off(i + j, nx, ny) + (j - wf_jlo(i + j, nx));
}

// ---- right-hand side of the forward sweep, per (cell, block row) ------------
// rh = D^{-1} (r~ - A~[:,0] x_p) in wavefront order, and x_p permuted alike.
// x_p carries nx*ny zero guard entries on each side, so every stencil
// neighbour is in bounds, and off-grid column-0 entries are zero.
// Per tile of RI x RJ cells of a layer (4 lanes per cell, one workgroup of
// 4*RI*RJ threads): the results are staged in LDS in the tile's own
// wavefront order, in which the cells of one anti-diagonal of the tile are
// consecutive in the layer's wavefront order too, and written back as runs
// of up to min(RI, RJ) cells instead of one scattered cell per quad.
// tickets (optional): the FP32 sweeps' two ticket counters, zeroed here for
// the forward and backward sweeps that follow on the stream.
constexpr int RI = 16, RJ = 16;
template <class T>
__global__ __launch_bounds__(4 * RI * RJ) void k_ras_in_tile(int nx, int ny, int64_t n, const T *__restrict__ rt,
                                                             const T *__restrict__ col0, const T *__restrict__ xp,
                                                             const T *__restrict__ dinv2, T *__restrict__ rh,
                                                             T *__restrict__ xpw, int *__restrict__ tickets) {
  __shared__ T so[RI * RJ][4];
  if (tickets && blockIdx.x == 0 && threadIdx.x < 2) tickets[threadIdx.x] = 0;
  __shared__ T sx[RI * RJ];
  __shared__ int sab[RI * RJ];
  const int tx = (nx + RI - 1) / RI, ty = (ny + RJ - 1) / RJ;
  const int layer = blockIdx.x / (tx * ty), tt = blockIdx.x - layer * (tx * ty);
  const int i0 = (tt % tx) * RI, j0 = (tt / tx) * RJ;
  const int ni = min(RI, nx - i0), nj = min(RJ, ny - j0);      // this tile's extent
  const int64_t nxy = (int64_t)nx * ny;
  const int tid = threadIdx.x, row = tid & 3, q = tid >> 2;
  const int a = q % RI, b = q / RI;
  if (a < ni && b < nj) {
    const int64_t c = layer * nxy + (int64_t)(j0 + b) * nx + (i0 + a);
    const int64_t off[7] = {-nxy, -(int64_t)nx, -1, 0, 1, (int64_t)nx, nxy};
    T col[8], dv[4];
    ld8v(col0 + c * 32 + 8 * row, col);
    ld4v(dinv2 + c * 16 + 4 * row, dv);
    T v = rt[4 * c + row];
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) v = v - col[sl] * xp[c + off[sl]];
    const T o = quad_mv<T>(dv, v);
    const int w = (int)wf_pos(a, b, ni, nj);                   // tile-local wavefront index
    so[w][row] = o;
    if (row == 0) {
      sx[w] = xp[c];
      sab[w] = a | (b << 16);
    }
  }
  __syncthreads();
  if (q < ni * nj) {
    const int ab = sab[q], aa = ab & 0xffff, bb = ab >> 16;
    const int64_t p = layer * nxy + wf_pos(i0 + aa, j0 + bb, nx, ny);
    rh[4 * p + row] = so[q][row];
    if (row == 0) xpw[p] = sx[q];
  }
}

// ---- scaled blocks for the sweeps, per (cell, block row) ---------------------
// blk[b][p] = D_c^{-1} A~_{c, nb(b)} for b = 0..3: -y, -x, +x, +y (slots 1, 2,
// 4, 5), at the cell's wavefront position p; FP64 products rounded once.
template <class T>
__global__ __launch_bounds__(256) void k_ras_scale(int nx, int ny, int64_t n, const T *__restrict__ t7,
                                                   const T *__restrict__ dinv2, T *__restrict__ blk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  const int64_t nxy = (int64_t)nx * ny, c = t >> 2;
  const int row = (int)(t & 3);
  double dv[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) dv[m] = (double)dinv2[c * 16 + 4 * row + m];
  const int64_t k = c / nxy, rem = c - k * nxy;
  const int j = (int)(rem / nx), i = (int)(rem - (int64_t)j * nx);
  const int64_t p = k * nxy + wf_pos(i, j, nx, ny);
  const int slot[4] = {1, 2, 4, 5};
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const T *a = t7 + ((int64_t)slot[b] * n + c) * 16;
    T o[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) v = fma(dv[m], (double)a[4 * m + cc], v);
      o[cc] = (T)v;
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) blk[((int64_t)b * n + p) * 16 + 4 * row + cc] = o[cc];
  }
}

// ---- sweeps ----------------------------------------------------------------
// A sweep workgroup has 4*LW compute lanes (lines j = q + LW*u, q = lane/4,
// U passes per level) and one writer wave.  Compute waves only load from
// global memory and keep the loads of the next P levels in flight in
// registers; their results go to an LDS ring of two levels.  The writer wave
// only stores: during level lambda it copies the outputs of level lambda-1
// from the ring to global memory.  On this architecture one counter tracks
// both loads and stores of a wave, and with both kinds in flight a wave can
// only wait for all of them; keeping them in different waves lets a compute
// wave wait for just the oldest of its prefetched loads.
template <class T> struct vec4t;
template <> struct vec4t<float> { typedef float4 type; };
template <> struct vec4t<double> { typedef double4 type; };

// copy the outputs of level m (lines j with 0 <= m - j < nx) from an LDS ring
// buffer [ny][4] to out: in wavefront order (WF) or natural order
template <class T, bool WF>
__device__ __forceinline__ void ras_write_level(int m, int nx, int ny, int64_t cl, const T *__restrict__ src,
                                                T *__restrict__ out, int w, int nw) {
  if (m < 0) return;
  const int jlo = max(0, m - nx + 1), jhi = min(ny - 1, m);
  const int64_t base = cl + (WF ? wf_off(m, nx, ny) - jlo : 0);
  for (int j = jlo + w; j <= jhi; j += nw) {
    const int64_t c = WF ? base + j : cl + (int64_t)j * nx + (m - j);
    *(typename vec4t<T>::type *)(out + 4 * c) = *(const typename vec4t<T>::type *)(src + 4 * j);
  }
}

// The loads that refill a level's registers must come after the level's last
// use of them.  Loads from read-only restrict arguments are free to move, and
// once hoisted above that use the registers rotate through copies that wait
// for every load in flight; an empty asm statement that takes the level's
// result and "changes" the refill's line index pins the order (it emits no
// instruction).
template <class T> __device__ __forceinline__ void order_after(int &idx, T tok) {
  asm volatile("" : "+v"(idx) : "v"(tok));
}

// ---- factorisation, per layer: D_c = A~_cc - sum_{q in {c-nx, c-1}} A~_cq D_q^{-1} A~_qc
// A quad of lanes per cell, lane r holding block row r, computes in FP64
// (lines j = q + LW*u for quad q, U passes).  Each lane forms row r of
// T = D_q^{-1} A~_qc and of the Schur update; the other rows of A~_qc and T
// come from the quad by DPP.  The inverse is the Gauss-Jordan elimination
// with row pivoting of the single-thread form, element by element the same
// operations: the quad tracks the row permutation instead of moving rows
// (every lane takes the same pivot decision from the broadcast column), and
// each lane scales the pivot row, read from its lane, itself.  D^{-1} blocks
// are rounded to the stored precision before the next cells use them; both
// neighbours' D^{-1} (cell before in x: same line, previous level; before in
// y: line j-1) come from an LDS slot per line, with a barrier after the
// reads of a level and one after its writes.  One writer wave copies the
// D^{-1} blocks of level lambda-1 from LDS to global memory while level
// lambda is computed.
// diag (optional, [n][16]) replaces the diagonal blocks A~_cc of t7: the
// overlapping RAS factors a layer whose diagonal already carries the Schur
// term of the layer below.
template <class T, int U>
__global__ __launch_bounds__(1024) void k_ras_setup(int nx, int ny, int64_t n, int LW, const T *__restrict__ t7,
                                                    const T *__restrict__ diag, T *__restrict__ dinv2,
                                                    int *__restrict__ flag) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char smem[];
  T *ring = (T *)smem;                                  // [ny][16]
  const int tid = threadIdx.x;
  const bool compute = tid < 4 * LW;                    // wave-uniform (4 LW is a multiple of 64)
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * blockIdx.x;
  const int Lv = nx + ny - 1;
  if (!compute) {
    const int w = tid - 4 * LW;
    auto write_level = [&](int m) {
      if (m < 0 || m >= Lv) return;
      const int jlo = max(0, m - nx + 1), jhi = min(ny - 1, m);
      for (int j = jlo + w; j <= jhi; j += 64) {
        const int64_t c = cl + (int64_t)j * nx + (m - j);
#pragma unroll
        for (int e = 0; e < 16; e += 4)
          *(typename vec4t<T>::type *)(dinv2 + c * 16 + e) = *(const typename vec4t<T>::type *)(ring + j * 16 + e);
      }
    };
    for (int lam = 0; lam < Lv; ++lam) {
      write_level(lam - 1);
      __syncthreads();
      __syncthreads();
    }
    write_level(Lv - 1);
    return;
  }
  const int q = tid >> 2, r = tid & 3, wq = (tid & 63) & ~3;
  const T *Ad = diag ? diag : t7 + 3 * n * 16, *Ay = t7 + 1 * n * 16, *Ax = t7 + 2 * n * 16;
  const T *Upx = t7 + 4 * n * 16, *Upy = t7 + 5 * n * 16;
  // this lane's row of A~_cc, A~_{c,c-nx}, A~_{c,c-1}, A~_{c-nx,c}, A~_{c-1,c}:
  // one level ahead with one pass, loaded at use with several
  T pre[5][4];
  auto load = [&](int lam, int u, T (&p)[5][4]) {
    const int j = min(q + LW * u, ny - 1);
    const int i = min(max(lam - j, 0), nx - 1);
    const int64_t c = cl + (int64_t)j * nx + i;
    const int64_t qy = j > 0 ? c - nx : c, qx = i > 0 ? c - 1 : c;
    ld4v(Ad + c * 16 + 4 * r, p[0]);
    ld4v(Ay + c * 16 + 4 * r, p[1]);
    ld4v(Ax + c * 16 + 4 * r, p[2]);
    ld4v(Upy + qy * 16 + 4 * r, p[3]);
    ld4v(Upx + qx * 16 + 4 * r, p[4]);
  };
  if constexpr (U == 1) load(0, 0, pre);
  int bad = 0;
  T orow[U][4];
  int ok[U];
  for (int lam = 0; lam < Lv; ++lam) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = q + LW * u, i = lam - j;
      T a[5][4];
      if constexpr (U == 1) {
#pragma unroll
        for (int b = 0; b < 5; ++b)
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) a[b][cc] = pre[b][cc];
      } else {
        load(lam, u, a);
      }
      if (j < ny && i >= 0 && i < nx) {                 // the same for the four lanes of the cell
        double Lr[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) Lr[cc] = (double)a[0][cc];
#pragma unroll
        for (int s = 0; s < 2; ++s) {                   // -y, then -x (ascending column)
          if (s == 0 ? j == 0 : i == 0) continue;
          const T *dq = ring + (s == 0 ? j - 1 : j) * 16 + 4 * r;
          double Aqc[4][4], t[4], Tm[4][4];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const T v = a[s == 0 ? 3 : 4][cc];
            Aqc[0][cc] = (double)qb<0>(v); Aqc[1][cc] = (double)qb<1>(v);
            Aqc[2][cc] = (double)qb<2>(v); Aqc[3][cc] = (double)qb<3>(v);
          }
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) v = v + (double)dq[m] * Aqc[m][cc];
            t[cc] = v;
          }
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            Tm[0][cc] = qb<0>(t[cc]); Tm[1][cc] = qb<1>(t[cc]);
            Tm[2][cc] = qb<2>(t[cc]); Tm[3][cc] = qb<3>(t[cc]);
          }
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) v = v + (double)a[s == 0 ? 1 : 2][m] * Tm[m][cc];
            Lr[cc] = Lr[cc] - v;
          }
        }
        // Gauss-Jordan on [L | I]; lane `mine` holds logical row `mine`
        double Rr[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) Rr[cc] = cc == r ? 1.0 : 0.0;
        double rmax = 0.0;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) rmax = fmax(rmax, fabs(Lr[cc]));
        const double amax = fmax(fmax(fmax(fmax(0.0, qb<0>(rmax)), qb<1>(rmax)), qb<2>(rmax)), qb<3>(rmax));
        int mine = r;
        if (!isfinite(amax)) {
          bad |= RSF_NONFINITE;
        } else {
          unsigned perm = 0xE4u;                        // 2 bits per logical row k: its lane
          auto lane_of = [&](int k) { return (int)((perm >> (2 * k)) & 3u); };
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const double c0 = qb<0>(Lr[p]), c1 = qb<1>(Lr[p]), c2 = qb<2>(Lr[p]), c3 = qb<3>(Lr[p]);
            auto col = [&](int l) { return l == 0 ? c0 : (l == 1 ? c1 : (l == 2 ? c2 : c3)); };
            int piv = p;
            double best = fabs(col(lane_of(p)));
#pragma unroll
            for (int k = p + 1; k < 4; ++k)
              if (fabs(col(lane_of(k))) > best) { best = fabs(col(lane_of(k))); piv = k; }
            const unsigned lp = (unsigned)lane_of(p), lq = (unsigned)lane_of(piv);
            perm = (perm & ~(3u << (2 * p)) & ~(3u << (2 * piv))) | (lq << (2 * p)) | (lp << (2 * piv));
            mine = mine == p ? piv : (mine == piv ? p : mine);
            const int src = wq + (int)lq;
            double pv = col((int)lq);
            if (fabs(pv) <= 1e-300 || fabs(pv) <= 1e-14 * amax) { bad |= RSF_SINGULAR; pv = 1.0; }
            const double inv = 1.0 / pv;
            double pL[4], pR[4];
#pragma unroll
            for (int cc = p + 1; cc < 4; ++cc) pL[cc] = __shfl(Lr[cc], src, 64) * inv;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) pR[cc] = __shfl(Rr[cc], src, 64) * inv;
            if (mine == p) {
#pragma unroll
              for (int cc = p + 1; cc < 4; ++cc) Lr[cc] = pL[cc];
#pragma unroll
              for (int cc = 0; cc < 4; ++cc) Rr[cc] = pR[cc];
              Lr[p] = 1.0;
            } else {
              const double f = Lr[p];
#pragma unroll
              for (int cc = p + 1; cc < 4; ++cc) Lr[cc] = Lr[cc] - f * pL[cc];
#pragma unroll
              for (int cc = 0; cc < 4; ++cc) Rr[cc] = Rr[cc] - f * pR[cc];
              Lr[p] = 0.0;
            }
          }
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) orow[u][cc] = (T)Rr[cc];
        ok[u] = mine;
      }
      if constexpr (U == 1) load(lam + 1, 0, pre);
    }
    __syncthreads();                                    // level lam-1 reads done
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = q + LW * u, i = lam - j;
      if (j < ny && i >= 0 && i < nx) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) ring[j * 16 + 4 * ok[u] + cc] = orow[u][cc];
      }
    }
    __syncthreads();                                    // level lam visible
  }
  if (bad) atomicOr(flag, bad);
}

// wavefront index (within the grid) of line j at level lam, clamped to the
// level's cells and the level to the layer's levels: always in bounds
__device__ __forceinline__ int64_t wf_clamped(int64_t cl, int lam, int j, int nx, int ny) {
  lam = min(max(lam, 0), nx + ny - 2);
  const int jlo = wf_jlo(lam, nx), jhi = min(ny - 1, lam);
  return cl + wf_off(lam, nx, ny) + (min(max(j, jlo), jhi) - jlo);
}

// forward, per layer: y = rh - Lh_y y_{c-nx} - Lh_x y_{c-1}
// The level count is padded to a multiple of P and every load and LDS read is
// issued unconditionally at clamped (in-bounds) addresses, with the terms of
// inactive cells dropped by selects: then every path through a level issues
// the same loads, and the compiler waits only for the level's own data.
template <class T> struct ras_fpre { T r, a1[4], a2[4]; };

template <class T, int U, int P>
__global__ __launch_bounds__(1024) void k_ras_fwd(int nx, int ny, int64_t n, int LW, const T *__restrict__ blk,
                                                  const T *__restrict__ rh, T *__restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *ring = (T *)smem;                                  // [2][ny][4]
  const int q = threadIdx.x >> 2, row = threadIdx.x & 3;
  const bool compute = (int)threadIdx.x < 4 * LW;       // wave-uniform (LW is a multiple of 16)
  const int w = threadIdx.x - 4 * LW, nw = blockDim.x - 4 * LW;
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * blockIdx.x;
  const int Lv = nx + ny - 1, Lpad = (Lv + P - 1) / P * P;
  if (!compute) {
    // the writer wave: its own level loop with one barrier per level, like
    // the compute waves, so that no path mixes its stores with the loads
    for (int lam = 0; lam < Lpad; ++lam) {
      ras_write_level<T, true>(lam - 1, nx, ny, cl, ring + ((lam & 1) ^ 1) * ny * 4, y, w, nw);
      __syncthreads();
    }
    ras_write_level<T, true>(Lpad - 1, nx, ny, cl, ring + ((Lpad - 1) & 1) * ny * 4, y, w, nw);
    return;
  }
  const T *By = blk, *Bx = blk + n * 16;
  ras_fpre<T> R[P][U];
  auto load = [&](int lam, ras_fpre<T> &p, int u, T tok) {
    int j = q + LW * u;
    order_after(j, tok);
    const int64_t c = wf_clamped(cl, lam, j, nx, ny);
    p.r = rh[4 * c + row];
    ld4v(By + c * 16 + 4 * row, p.a1);
    ld4v(Bx + c * 16 + 4 * row, p.a2);
  };
#pragma unroll
  for (int d = 0; d < P; ++d)
#pragma unroll
    for (int u = 0; u < U; ++u) load(d, R[d][u], u, (T)0);
  for (int lam0 = 0; lam0 < Lpad; lam0 += P) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
      const int lam = lam0 + d;
      T *cur = ring + (lam & 1) * ny * 4;
      const T *prv = ring + ((lam & 1) ^ 1) * ny * 4;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = q + LW * u, i = lam - j;
        const bool act = j < ny && i >= 0 && i < nx;
        const int jr = min(j, ny - 1);
        T yy[4], yx[4];
        ld4v(prv + 4 * max(jr - 1, 0), yy);
        ld4v(prv + 4 * jr, yx);
        const T ty = dot4(R[d][u].a1, yy), tx = dot4(R[d][u].a2, yx);
        T v = R[d][u].r;
        v = (act && j > 0) ? v - ty : v;
        v = (act && i > 0) ? v - tx : v;
        if (act) cur[4 * j + row] = v;
        load(lam + P, R[d][u], u, v);
      }
      __syncthreads();
    }
  }
}

// backward, per layer: z = y - Uh_x z_{c+1} - Uh_y z_{c+nx}, output z + Pi_p x_p
// (x_p added to unknown 0) in natural order through a second LDS ring
template <class T> struct ras_bpre { T yc, xpc, a4[4], a5[4]; };

template <class T, int U, int P>
__global__ __launch_bounds__(1024) void k_ras_bwd(int nx, int ny, int64_t n, int LW, const T *__restrict__ blk,
                                                  const T *__restrict__ y, const T *__restrict__ xpw,
                                                  T *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *ring = (T *)smem;                                  // [2][ny][4]: z
  T *oring = ring + 2 * ny * 4;                         // [2][ny][4]: output
  const int q = threadIdx.x >> 2, row = threadIdx.x & 3;
  const bool compute = (int)threadIdx.x < 4 * LW;
  const int w = threadIdx.x - 4 * LW, nw = blockDim.x - 4 * LW;
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * blockIdx.x;
  const int Lv = nx + ny - 1, Lpad = (Lv + P - 1) / P * P;
  if (!compute) {
    // step s handles level Lv-1-s; the writer copies the previous step's
    for (int step = 0; step < Lpad; ++step) {
      ras_write_level<T, false>(step >= 1 ? Lv - step : -1, nx, ny, cl, oring + ((step & 1) ^ 1) * ny * 4, out, w,
                                nw);
      __syncthreads();
    }
    ras_write_level<T, false>(Lv - Lpad, nx, ny, cl, oring + ((Lpad - 1) & 1) * ny * 4, out, w, nw);
    return;
  }
  const T *Bx = blk + 2 * n * 16, *By = blk + 3 * n * 16;
  ras_bpre<T> R[P][U];
  auto load = [&](int step, ras_bpre<T> &p, int u, T tok) {
    int j = q + LW * u;
    order_after(j, tok);
    const int64_t c = wf_clamped(cl, Lv - 1 - step, j, nx, ny);
    p.yc = y[4 * c + row];
    p.xpc = xpw[c];
    ld4v(Bx + c * 16 + 4 * row, p.a4);
    ld4v(By + c * 16 + 4 * row, p.a5);
  };
#pragma unroll
  for (int d = 0; d < P; ++d)
#pragma unroll
    for (int u = 0; u < U; ++u) load(d, R[d][u], u, (T)0);
  for (int s0 = 0; s0 < Lpad; s0 += P) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
      const int step = s0 + d;
      const int lam = Lv - 1 - step;
      const int cb = (step & 1) * ny * 4, pb = ((step & 1) ^ 1) * ny * 4;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = q + LW * u, i = lam - j;
        const bool act = j < ny && i >= 0 && i < nx;
        const int jr = min(j, ny - 1);
        T zx[4], zy[4];
        ld4v(ring + pb + 4 * jr, zx);
        ld4v(ring + pb + 4 * min(jr + 1, ny - 1), zy);
        const T tx = dot4(R[d][u].a4, zx), ty = dot4(R[d][u].a5, zy);
        T zc = R[d][u].yc;
        zc = (act && i < nx - 1) ? zc - tx : zc;
        zc = (act && j < ny - 1) ? zc - ty : zc;
        if (act) {
          ring[cb + 4 * j + row] = zc;
          oring[cb + 4 * j + row] = row == 0 ? zc + R[d][u].xpc : zc;
        }
        load(step + P, R[d][u], u, zc);
      }
      __syncthreads();
    }
  }
}

// ---- sweeps with one lane per cell, layers split into strips (FP32) ---------
// One lane per line handles all four block rows of its cell (per cell the
// same arithmetic sequence as the four-lane form; a quarter of the lanes).
// A workgroup keeps a layer's lines streamed through one CU, which bounds it
// at that CU's memory stream, so each layer is further split into S strips
// of H consecutive lines, one workgroup each.  A strip needs, at every level,
// the value of the line just before it (after it, backward) computed one
// level earlier by the neighbouring strip:
//   - the producer's writer wave publishes its boundary line, level by level,
//     as 64-bit words (launch tag << 32 | FP32 bits), one per block row,
//     with device-scope stores;
//   - the consumer's writer wave polls those words with device-scope loads
//     until the tag matches and puts the value into a ghost slot of its LDS
//     ring, ready for the next level;
//   - workgroups take tickets in dependency order (every strip of a layer
//     after the one it reads), so a workgroup only waits on workgroups that
//     are already running; every wait is bounded, and a time-out latches an
//     error word (ctl[2]) that the host turns into RS_E_HIP.
// Compute waves only load; the writer wave stores (see above).
constexpr int RAS_SPIN_LIMIT = 1 << 20;     // polls with a short sleep: about a second

__device__ __forceinline__ void ras_put(uint64_t *p, float v, uint32_t tag) {
  __hip_atomic_store(p, ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// value of the word at p once its tag is `tag`; false on time-out
__device__ __forceinline__ bool ras_get(const uint64_t *p, uint32_t tag, float &v, bool &failed) {
  int spins = 0;
  for (;;) {
    uint64_t w = __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(w >> 32) == tag) { v = __uint_as_float((uint32_t)w); return true; }
    if (failed || ++spins > RAS_SPIN_LIMIT) { failed = true; return false; }
    __builtin_amdgcn_s_sleep(1);
  }
}

// A value in FP64 crosses strips as two such words, high half first, each
// with the tag: words of value r of line i: [W r, W r + W), W = 1 or 2.
template <class T> struct ras_nw { static constexpr int W = sizeof(T) / 4; };
__device__ __forceinline__ void ras_put_v(uint64_t *p, float v, uint32_t tag) { ras_put(p, v, tag); }
__device__ __forceinline__ void ras_put_v(uint64_t *p, double v, uint32_t tag) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  __hip_atomic_store(p, ((uint64_t)tag << 32) | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, ((uint64_t)tag << 32) | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// value from its words once every tag is `tag`; w holds the words as loaded
// earlier, re-read (bounded) until they match; false on time-out
__device__ __forceinline__ bool ras_get_v(const uint64_t *p, const uint64_t (&w)[1], uint32_t tag, float &v,
                                          bool &failed) {
  if ((uint32_t)(w[0] >> 32) == tag) { v = __uint_as_float((uint32_t)w[0]); return true; }
  return ras_get(p, tag, v, failed);
}
__device__ __forceinline__ bool ras_get_v(const uint64_t *p, const uint64_t (&w)[2], uint32_t tag, double &v,
                                          bool &failed) {
  uint32_t h[2];
  for (int q = 0; q < 2; ++q) {
    uint64_t x = w[q];
    int spins = 0;
    while ((uint32_t)(x >> 32) != tag) {
      if (failed || ++spins > RAS_SPIN_LIMIT) { failed = true; return false; }
      __builtin_amdgcn_s_sleep(1);
      x = __hip_atomic_load(const_cast<uint64_t *>(p + q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    h[q] = (uint32_t)x;
  }
  v = __longlong_as_double((long long)(((uint64_t)h[0] << 32) | h[1]));
  return true;
}

// store the outputs of level lam (own lines [j0, j1)) from an LDS ring
// buffer [H+2][4] (slot of line j: j - j0 + 1) to out, in wavefront order
// (WF) or natural order
template <bool WF, class T = float>
__device__ __forceinline__ void ras_write_strip(int lam, int nx, int ny, int j0, int j1, int64_t cl,
                                                const T *__restrict__ src, T *__restrict__ out, int w, int nw) {
  if (lam < 0 || lam > nx + ny - 2) return;
  const int jlo = max(j0, lam - nx + 1), jhi = min(j1 - 1, lam);
  const int64_t base = WF ? cl + wf_off(lam, nx, ny) - max(0, lam - nx + 1) : 0;
  for (int j = jlo + w; j <= jhi; j += nw) {
    const int64_t c = WF ? base + j : cl + (int64_t)j * nx + (lam - j);
    *(typename vec4t<T>::type *)(out + 4 * c) = *(const typename vec4t<T>::type *)(src + 4 * (j - j0 + 1));
  }
}

// word of the boundary value (row r) of strip s of layer k at column i
__device__ __forceinline__ int64_t ras_xword(int k, int s, int S, int nx, int i) {
  return (((int64_t)k * S + s) * nx + i) * 4;
}

template <class T> struct ras_f1 { T r[4], a1[16], a2[16]; };

template <int U, int P>
__global__ __launch_bounds__(320) void k_ras_fwd1(int nx, int ny, int nz, int S, int H, int64_t n, int LW,
                                                  const float *__restrict__ blk, const float *__restrict__ rh,
                                                  float *__restrict__ y, int *__restrict__ ctl,
                                                  uint64_t *__restrict__ xw, uint32_t tag) {
  extern __shared__ __align__(16) unsigned char smem[];
  float *ring = (float *)smem;                          // [2][H+2][4]
  __shared__ int s_t;
  __shared__ float gh[32][4];                           // ghost line j0-1, by level mod 32
  const int tid = threadIdx.x;
  if (tid == 0) s_t = atomicAdd(&ctl[0], 1);
  __syncthreads();
  const int s = s_t / nz, k = s_t - (s_t / nz) * nz;
  const int j0 = s * H, j1 = min(ny, j0 + H), RS = H + 2;
  const bool compute = tid < LW;                        // wave-uniform (LW is a multiple of 64)
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * k;
  const int Lw = nx + (j1 - j0) - 1, Lpad = (Lw + P - 1) / P * P;   // levels j0 .. j0+Lw-1
  if (!compute) {
    const int w = tid - LW, nw = blockDim.x - LW;
    bool failed = false;
    // ghost line j0-1 for local level m (cell i = m) goes to gh[m % 32]; the
    // writer loads 16 levels at a time (64 lanes: level offset, block row),
    // issued 8 levels before the first of them is needed and checked one
    // level before it, so the neighbour's words are normally published by
    // the time they are loaded and the load latency is hidden behind 7
    // levels; a word not yet published is polled
    auto issue16 = [&](int m16, uint64_t &slot) {
      const int m = m16 + (w >> 2), r = w & 3;
      if (s == 0 || w >= 64 || m >= nx) return;
      slot = __hip_atomic_load(xw + ras_xword(k, s - 1, S, nx, m) + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto finish16 = [&](int m16, uint64_t slot) {
      const int m = m16 + (w >> 2), r = w & 3;
      if (s == 0 || w >= 64 || m >= nx) return;
      float v;
      if ((uint32_t)(slot >> 32) == tag) v = __uint_as_float((uint32_t)slot);
      else if (!ras_get(xw + ras_xword(k, s - 1, S, nx, m) + r, tag, v, failed)) atomicOr(&ctl[2], 1);
      gh[m & 31][r] = v;
    };
    // own last line j1-1 at local level m (cell i = m + j0 - (j1-1)), buffer m&1
    auto publish = [&](int m) {
      if (s == S - 1 || w >= 4 || m < 0) return;
      const int i = m + j0 - (j1 - 1);
      if (i < 0 || i >= nx) return;
      ras_put(xw + ras_xword(k, s, S, nx, i) + w, ring[(m & 1) * RS * 4 + (j1 - j0) * 4 + w], tag);
    };
    uint64_t pend = 0;
    issue16(0, pend);
    finish16(0, pend);
    __syncthreads();
    for (int m = 0; m < Lpad; ++m) {
      if ((m & 15) == 8) issue16(m + 8, pend);          // the next batch, 8 levels ahead
      ras_write_strip<true>(j0 + m - 1, nx, ny, j0, j1, cl, ring + ((m + 1) & 1) * RS * 4, y, w, nw);
      publish(m - 1);
      if ((m & 15) == 15) finish16(m + 1, pend);        // levels m+1 .. m+16
      __syncthreads();
    }
    ras_write_strip<true>(j0 + Lpad - 1, nx, ny, j0, j1, cl, ring + ((Lpad + 1) & 1) * RS * 4, y, w, nw);
    publish(Lpad - 1);
    return;
  }
  __syncthreads();
  const float *By = blk, *Bx = blk + n * 16;
  ras_f1<float> R[P][U];
  auto load = [&](int m, ras_f1<float> &p, int u, float tok) {
    int j = j0 + tid + LW * u;
    order_after(j, tok);
    const int64_t c = wf_clamped(cl, j0 + m, j, nx, ny);
    ld4v(rh + 4 * c, p.r);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float t4[4];
      ld4v(By + c * 16 + 4 * q, t4);
#pragma unroll
      for (int e = 0; e < 4; ++e) p.a1[4 * q + e] = t4[e];
      ld4v(Bx + c * 16 + 4 * q, t4);
#pragma unroll
      for (int e = 0; e < 4; ++e) p.a2[4 * q + e] = t4[e];
    }
  };
  // slot d of R holds level m0 + d; the slot of the previous level is
  // refilled at the start of each level (before its LDS reads, so that the
  // load issue overlaps their latency), keeping P-1 levels in flight
#pragma unroll
  for (int d = 0; d < P - 1; ++d)
#pragma unroll
    for (int u = 0; u < U; ++u) load(d, R[d][u], u, 0.f);
  float tok[U];
#pragma unroll
  for (int u = 0; u < U; ++u) tok[u] = 0.f;
  for (int m0 = 0; m0 < Lpad; m0 += P) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
      const int m = m0 + d, lam = j0 + m;
      float *cur = ring + (m & 1) * RS * 4;
      const float *prv = ring + ((m + 1) & 1) * RS * 4;
#pragma unroll
      for (int u = 0; u < U; ++u) load(m + P - 1, R[(d + P - 1) % P][u], u, tok[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + tid + LW * u, i = lam - j;
        const bool act = j < j1 && i >= 0 && i < nx;
        const int sl = min(j, j1 - 1) - j0 + 1;         // slot of line j
        float yy[4], yx[4], v[4];
        ld4v(sl == 1 ? &gh[m & 31][0] : prv + 4 * (sl - 1), yy);   // line j0-1: the ghost
        ld4v(prv + 4 * sl, yx);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float a1r[4] = {R[d][u].a1[4 * r], R[d][u].a1[4 * r + 1], R[d][u].a1[4 * r + 2], R[d][u].a1[4 * r + 3]};
          float a2r[4] = {R[d][u].a2[4 * r], R[d][u].a2[4 * r + 1], R[d][u].a2[4 * r + 2], R[d][u].a2[4 * r + 3]};
          const float ty = dot4(a1r, yy), tx = dot4(a2r, yx);
          float vr = R[d][u].r[r];
          vr = (act && j > 0) ? vr - ty : vr;
          vr = (act && i > 0) ? vr - tx : vr;
          v[r] = vr;
        }
        if (act) *(float4 *)(cur + 4 * sl) = make_float4(v[0], v[1], v[2], v[3]);
        tok[u] = v[3];
      }
      __syncthreads();
    }
  }
}

template <class T> struct ras_b1 { T yc[4], xpc, a4[16], a5[16]; };

template <int U, int P>
__global__ __launch_bounds__(320) void k_ras_bwd1(int nx, int ny, int nz, int S, int H, int64_t n, int LW,
                                                  const float *__restrict__ blk, const float *__restrict__ y,
                                                  const float *__restrict__ xpw, float *__restrict__ out,
                                                  int *__restrict__ ctl, uint64_t *__restrict__ xw, uint32_t tag) {
  extern __shared__ __align__(16) unsigned char smem[];
  float *ring = (float *)smem;                          // [2][H+2][4]: z
  __shared__ int s_t;
  __shared__ float gh[32][4];                           // ghost line j1, by step mod 32
  const int tid = threadIdx.x;
  if (tid == 0) s_t = atomicAdd(&ctl[1], 1);
  __syncthreads();
  const int st = s_t / nz, k = s_t - st * nz, s = S - 1 - st;   // last strip first
  const int j0 = s * H, j1 = min(ny, j0 + H), RS = H + 2, nl = j1 - j0;
  float *oring = ring + 2 * RS * 4;                     // [2][H+2][4]: output
  const bool compute = tid < LW;
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * k;
  const int Lw = nx + nl - 1, Lpad = (Lw + P - 1) / P * P;
  const int ltop = j1 - 1 + nx - 1;                     // step m handles level ltop - m
  if (!compute) {
    const int w = tid - LW, nw = blockDim.x - LW;
    bool failed = false;
    // ghost line j1 for step m (cell i = ltop - m - (j1-1)) goes to gh[m % 32],
    // loaded 16 steps at a time as in the forward sweep
    auto issue16 = [&](int m16, uint64_t &slot) {
      const int m = m16 + (w >> 2), r = w & 3;
      const int i = ltop - m - (j1 - 1);
      if (s == S - 1 || w >= 64 || i < 0 || i >= nx) return;
      slot = __hip_atomic_load(xw + ras_xword(k, s + 1, S, nx, i) + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto finish16 = [&](int m16, uint64_t slot) {
      const int m = m16 + (w >> 2), r = w & 3;
      const int i = ltop - m - (j1 - 1);
      if (s == S - 1 || w >= 64 || i < 0 || i >= nx) return;
      float v;
      if ((uint32_t)(slot >> 32) == tag) v = __uint_as_float((uint32_t)slot);
      else if (!ras_get(xw + ras_xword(k, s + 1, S, nx, i) + r, tag, v, failed)) atomicOr(&ctl[2], 1);
      gh[m & 31][r] = v;
    };
    // own first line j0 at step m (cell i = ltop - m - j0), buffer m&1, slot 1
    auto publish = [&](int m) {
      if (s == 0 || w >= 4 || m < 0) return;
      const int i = ltop - m - j0;
      if (i < 0 || i >= nx) return;
      ras_put(xw + ras_xword(k, s, S, nx, i) + w, ring[(m & 1) * RS * 4 + 4 + w], tag);
    };
    uint64_t pend = 0;
    issue16(0, pend);
    finish16(0, pend);
    __syncthreads();
    for (int m = 0; m < Lpad; ++m) {
      if ((m & 15) == 8) issue16(m + 8, pend);          // the next batch, 8 levels ahead
      if (m >= 1) ras_write_strip<false>(ltop - m + 1, nx, ny, j0, j1, cl, oring + ((m + 1) & 1) * RS * 4, out, w, nw);
      publish(m - 1);
      if ((m & 15) == 15) finish16(m + 1, pend);        // steps m+1 .. m+16
      __syncthreads();
    }
    ras_write_strip<false>(ltop - Lpad + 1, nx, ny, j0, j1, cl, oring + ((Lpad + 1) & 1) * RS * 4, out, w, nw);
    publish(Lpad - 1);
    return;
  }
  __syncthreads();
  const float *Bx = blk + 2 * n * 16, *By = blk + 3 * n * 16;
  ras_b1<float> R[P][U];
  auto load = [&](int m, ras_b1<float> &p, int u, float tok) {
    int j = j0 + tid + LW * u;
    order_after(j, tok);
    const int64_t c = wf_clamped(cl, ltop - m, j, nx, ny);
    ld4v(y + 4 * c, p.yc);
    p.xpc = xpw[c];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float t4[4];
      ld4v(Bx + c * 16 + 4 * q, t4);
#pragma unroll
      for (int e = 0; e < 4; ++e) p.a4[4 * q + e] = t4[e];
      ld4v(By + c * 16 + 4 * q, t4);
#pragma unroll
      for (int e = 0; e < 4; ++e) p.a5[4 * q + e] = t4[e];
    }
  };
#pragma unroll
  for (int d = 0; d < P - 1; ++d)
#pragma unroll
    for (int u = 0; u < U; ++u) load(d, R[d][u], u, 0.f);
  float tok[U];
#pragma unroll
  for (int u = 0; u < U; ++u) tok[u] = 0.f;
  for (int m0 = 0; m0 < Lpad; m0 += P) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
      const int m = m0 + d, lam = ltop - m;
      const int cb = (m & 1) * RS * 4, pb = ((m + 1) & 1) * RS * 4;
#pragma unroll
      for (int u = 0; u < U; ++u) load(m + P - 1, R[(d + P - 1) % P][u], u, tok[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + tid + LW * u, i = lam - j;
        const bool act = j < j1 && i >= 0 && i < nx;
        const int sl = min(j, j1 - 1) - j0 + 1;
        float zx[4], zy[4], z[4];
        ld4v(ring + pb + 4 * sl, zx);
        ld4v(sl == nl ? &gh[m & 31][0] : ring + pb + 4 * (sl + 1), zy);   // line j1: the ghost
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float a4r[4] = {R[d][u].a4[4 * r], R[d][u].a4[4 * r + 1], R[d][u].a4[4 * r + 2], R[d][u].a4[4 * r + 3]};
          float a5r[4] = {R[d][u].a5[4 * r], R[d][u].a5[4 * r + 1], R[d][u].a5[4 * r + 2], R[d][u].a5[4 * r + 3]};
          const float tx = dot4(a4r, zx), ty = dot4(a5r, zy);
          float zr = R[d][u].yc[r];
          zr = (act && i < nx - 1) ? zr - tx : zr;
          zr = (act && j < ny - 1) ? zr - ty : zr;
          z[r] = zr;
        }
        if (act) {
          *(float4 *)(ring + cb + 4 * sl) = make_float4(z[0], z[1], z[2], z[3]);
          *(float4 *)(oring + cb + 4 * sl) = make_float4(z[0] + R[d][u].xpc, z[1], z[2], z[3]);
        }
        tok[u] = z[3];
      }
      __syncthreads();
    }
  }
}

// ---- sweeps with a quad of lanes per cell on strips (FP32 and FP64) ---------
// The strips, tickets and boundary words of the sweeps above, with the
// compute of the one-workgroup-per-layer sweeps: lane r of a cell's quad owns
// block row r and keeps its rows of the next P levels in flight in registers
// (three loads per level: its rh or y entry and its rows of the two scaled
// blocks, plus x_p backward), so a level's loads are spread over four times
// as many lanes as with one lane per line.  The waves each have one kind of
// memory traffic: compute waves only load; the writer wave only stores
// (outputs and published boundary words); a poller wave only loads the
// neighbour strip's words, so no wait for a load ever waits for a store.
// Strips of up to 224 lines (one pass).
template <class T, int P>
__global__ __launch_bounds__(1024) void k_ras_fwd3(int nx, int ny, int nz, int S, int H, int64_t n, int LWq,
                                                   const T *__restrict__ blk, const T *__restrict__ rh,
                                                   T *__restrict__ y, int *__restrict__ ctl,
                                                   uint64_t *__restrict__ xw, uint32_t tag) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *ring = (T *)smem;                                  // [2][H+2][4]
  __shared__ int s_t;
  __shared__ T gh[32][4];                               // ghost line j0-1, by level mod 32
  const int tid = threadIdx.x, NC = 4 * LWq;
  constexpr int W = ras_nw<T>::W;                       // boundary words per value
  if (tid == 0) s_t = atomicAdd(&ctl[0], 1);
  __syncthreads();
  const int s = s_t / nz, k = s_t - (s_t / nz) * nz;
  const int j0 = s * H, j1 = min(ny, j0 + H), RS = H + 2;
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * k;
  const int Lw = nx + (j1 - j0) - 1, Lpad = (Lw + P - 1) / P * P;
  if (tid >= NC + 64) {
    // poller wave
    const int w = tid - NC - 64;
    bool failed = false;
    auto wp = [&](int m, int r) { return xw + W * (ras_xword(k, s - 1, S, nx, m) + r); };
    auto issue16 = [&](int m16, uint64_t (&slot)[W]) {
      const int m = m16 + (w >> 2), r = w & 3;
      if (s == 0 || m >= nx) return;
#pragma unroll
      for (int q = 0; q < W; ++q)
        slot[q] = __hip_atomic_load(wp(m, r) + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto finish16 = [&](int m16, const uint64_t (&slot)[W]) {
      const int m = m16 + (w >> 2), r = w & 3;
      if (s == 0 || m >= nx) return;
      T v = 0;
      if (!ras_get_v(wp(m, r), slot, tag, v, failed)) atomicOr(&ctl[2], 1);
      gh[m & 31][r] = v;
    };
    uint64_t pend[W] = {};
    issue16(0, pend);
    finish16(0, pend);
    __syncthreads();
    for (int m = 0; m < Lpad; ++m) {
      if ((m & 15) == 8) issue16(m + 8, pend);
      if ((m & 15) == 15) finish16(m + 1, pend);
      __syncthreads();
    }
    return;
  }
  if (tid >= NC) {
    // writer wave: stores only
    const int w = tid - NC, nw = 64;
    auto publish = [&](int m) {
      if (s == S - 1 || w >= 4 || m < 0) return;
      const int i = m + j0 - (j1 - 1);
      if (i < 0 || i >= nx) return;
      ras_put_v(xw + W * (ras_xword(k, s, S, nx, i) + w), ring[(m & 1) * RS * 4 + (j1 - j0) * 4 + w], tag);
    };
    __syncthreads();
    for (int m = 0; m < Lpad; ++m) {
      ras_write_strip<true, T>(j0 + m - 1, nx, ny, j0, j1, cl, ring + ((m + 1) & 1) * RS * 4, y, w, nw);
      publish(m - 1);
      __syncthreads();
    }
    ras_write_strip<true, T>(j0 + Lpad - 1, nx, ny, j0, j1, cl, ring + ((Lpad + 1) & 1) * RS * 4, y, w, nw);
    publish(Lpad - 1);
    return;
  }
  __syncthreads();
  const int row = tid & 3, j = j0 + (tid >> 2);
  const int sl = min(j, j1 - 1) - j0 + 1;               // slot of line j in the ring
  const T *By = blk, *Bx = blk + n * 16;
  ras_fpre<T> R[P];
  auto load = [&](int m, ras_fpre<T> &p, T tok) {
    int jj = j;
    order_after(jj, tok);
    const int64_t c = wf_clamped(cl, j0 + m, jj, nx, ny);
    p.r = rh[4 * c + row];
    ld4v(By + c * 16 + 4 * row, p.a1);
    ld4v(Bx + c * 16 + 4 * row, p.a2);
  };
#pragma unroll
  for (int d = 0; d < P; ++d) load(d, R[d], (T)0);
  for (int m0 = 0; m0 < Lpad; m0 += P) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
      const int m = m0 + d, i = j0 + m - j;
      const bool act = j < j1 && i >= 0 && i < nx;
      T *cur = ring + (m & 1) * RS * 4;
      const T *prv = ring + ((m + 1) & 1) * RS * 4;
      T yy[4], yx[4];
      ld4v(sl == 1 ? &gh[m & 31][0] : prv + 4 * (sl - 1), yy);   // line j0-1: the ghost
      ld4v(prv + 4 * sl, yx);
      const T ty = dot4(R[d].a1, yy), tx = dot4(R[d].a2, yx);
      T v = R[d].r;
      v = (act && j > 0) ? v - ty : v;
      v = (act && i > 0) ? v - tx : v;
      if (act) cur[4 * sl + row] = v;
      load(m + P, R[d], v);
      __syncthreads();
    }
  }
}

template <class T, int P>
__global__ __launch_bounds__(1024) void k_ras_bwd3(int nx, int ny, int nz, int S, int H, int64_t n, int LWq,
                                                   const T *__restrict__ blk, const T *__restrict__ y,
                                                   const T *__restrict__ xpw, T *__restrict__ out,
                                                   int *__restrict__ ctl, uint64_t *__restrict__ xw, uint32_t tag) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *ring = (T *)smem;                                  // [2][H+2][4]: z
  __shared__ int s_t;
  __shared__ T gh[32][4];                               // ghost line j1, by step mod 32
  const int tid = threadIdx.x, NC = 4 * LWq;
  constexpr int W = ras_nw<T>::W;                       // boundary words per value
  if (tid == 0) s_t = atomicAdd(&ctl[1], 1);
  __syncthreads();
  const int st = s_t / nz, k = s_t - st * nz, s = S - 1 - st;   // last strip first
  const int j0 = s * H, j1 = min(ny, j0 + H), RS = H + 2, nl = j1 - j0;
  T *oring = ring + 2 * RS * 4;                         // [2][H+2][4]: output
  const int64_t nxy = (int64_t)nx * ny, cl = nxy * k;
  const int Lw = nx + nl - 1, Lpad = (Lw + P - 1) / P * P;
  const int ltop = j1 - 1 + nx - 1;                     // step m handles level ltop - m
  if (tid >= NC + 64) {
    const int w = tid - NC - 64;
    bool failed = false;
    auto wp = [&](int i, int r) { return xw + W * (ras_xword(k, s + 1, S, nx, i) + r); };
    auto issue16 = [&](int m16, uint64_t (&slot)[W]) {
      const int m = m16 + (w >> 2), r = w & 3;
      const int i = ltop - m - (j1 - 1);
      if (s == S - 1 || i < 0 || i >= nx) return;
#pragma unroll
      for (int q = 0; q < W; ++q)
        slot[q] = __hip_atomic_load(wp(i, r) + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto finish16 = [&](int m16, const uint64_t (&slot)[W]) {
      const int m = m16 + (w >> 2), r = w & 3;
      const int i = ltop - m - (j1 - 1);
      if (s == S - 1 || i < 0 || i >= nx) return;
      T v = 0;
      if (!ras_get_v(wp(i, r), slot, tag, v, failed)) atomicOr(&ctl[2], 1);
      gh[m & 31][r] = v;
    };
    uint64_t pend[W] = {};
    issue16(0, pend);
    finish16(0, pend);
    __syncthreads();
    for (int m = 0; m < Lpad; ++m) {
      if ((m & 15) == 8) issue16(m + 8, pend);
      if ((m & 15) == 15) finish16(m + 1, pend);
      __syncthreads();
    }
    return;
  }
  if (tid >= NC) {
    const int w = tid - NC, nw = 64;
    auto publish = [&](int m) {
      if (s == 0 || w >= 4 || m < 0) return;
      const int i = ltop - m - j0;
      if (i < 0 || i >= nx) return;
      ras_put_v(xw + W * (ras_xword(k, s, S, nx, i) + w), ring[(m & 1) * RS * 4 + 4 + w], tag);
    };
    __syncthreads();
    for (int m = 0; m < Lpad; ++m) {
      if (m >= 1) ras_write_strip<false, T>(ltop - m + 1, nx, ny, j0, j1, cl, oring + ((m + 1) & 1) * RS * 4, out, w, nw);
      publish(m - 1);
      __syncthreads();
    }
    ras_write_strip<false, T>(ltop - Lpad + 1, nx, ny, j0, j1, cl, oring + ((Lpad + 1) & 1) * RS * 4, out, w, nw);
    publish(Lpad - 1);
    return;
  }
  __syncthreads();
  const int row = tid & 3, j = j0 + (tid >> 2);
  const int sl = min(j, j1 - 1) - j0 + 1;
  const T *Bx = blk + 2 * n * 16, *By = blk + 3 * n * 16;
  ras_bpre<T> R[P];
  auto load = [&](int m, ras_bpre<T> &p, T tok) {
    int jj = j;
    order_after(jj, tok);
    const int64_t c = wf_clamped(cl, ltop - m, jj, nx, ny);
    p.yc = y[4 * c + row];
    p.xpc = xpw[c];
    ld4v(Bx + c * 16 + 4 * row, p.a4);
    ld4v(By + c * 16 + 4 * row, p.a5);
  };
#pragma unroll
  for (int d = 0; d < P; ++d) load(d, R[d], (T)0);
  for (int m0 = 0; m0 < Lpad; m0 += P) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
      const int m = m0 + d, i = ltop - m - j;
      const bool act = j < j1 && i >= 0 && i < nx;
      const int cb = (m & 1) * RS * 4, pb = ((m + 1) & 1) * RS * 4;
      T zx[4], zy[4];
      ld4v(ring + pb + 4 * sl, zx);
      ld4v(sl == nl ? &gh[m & 31][0] : ring + pb + 4 * (sl + 1), zy);   // line j1: the ghost
      const T tx = dot4(R[d].a4, zx), ty = dot4(R[d].a5, zy);
      T zc = R[d].yc;
      zc = (act && i < nx - 1) ? zc - tx : zc;
      zc = (act && j < ny - 1) ? zc - ty : zc;
      if (act) {
        ring[cb + 4 * sl + row] = zc;
        oring[cb + 4 * sl + row] = row == 0 ? zc + R[d].xpc : zc;
      }
      load(m + P, R[d], zc);
      __syncthreads();
    }
  }
}

// ---- RAS with overlap 1 over the layers -------------------------------------
// The extension of layer k is the layers k-1, k, k+1; its block ILU(0) in
// natural order factors them one after another: the first with the plain
// layer factors P0, the next two with their diagonals reduced by the Schur
// term of the layer below (P1 for layer k, P2 for layer k+1).  The sweeps of
// one extension are layer sweeps joined by the couplings across z:
//   y0 = fwd(P0, r2)                            on layer k-1
//   y1 = fwd(P1, r2 - A~_{-z} y0)               on layer k
//   y2 = fwd(P2, r2 - A~_{-z} y1)               on layer k+1
//   z2 = bwd(P2, y2)                            on layer k+1
//   z  = bwd(P1, y1 - P1^{-1} A~_{+z} z2)       on layer k (kept)
// so every layer is swept three times forward and twice backward, each sweep
// over all layers at once.

// E_c = A~_cc - A~_{c,c-nxy} P_{c-nxy} A~_{c-nxy,c} (A~_cc on the first
// layer), per (cell, block row), in FP64 with the DILU's operations in its
// order: T1 = P_{c-nxy} A~_{c-nxy,c}, then row r of A~_{c,c-nxy} T1, then the
// subtraction.
template <class T>
__global__ __launch_bounds__(256) void k_ras_zdiag(int64_t n, int64_t nxy, const T *__restrict__ t7,
                                                   const T *__restrict__ P, T *__restrict__ E) {
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  const int64_t c = t >> 2;
  const int r = (int)(t & 3);
  const T *Acc = t7 + (3 * n + c) * 16;
  if (c < nxy) {
#pragma unroll
    for (int b = 0; b < 4; ++b) E[c * 16 + 4 * r + b] = Acc[4 * r + b];
    return;
  }
  const int64_t q = c - nxy;
  const T *Pq = P + q * 16, *Aqc = t7 + (6 * n + q) * 16, *Acq = t7 + c * 16;
  double T1[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) v = v + (double)Pq[4 * a + m] * (double)Aqc[4 * m + b];
      T1[a][b] = v;
    }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) v = v + (double)Acq[4 * r + m] * T1[m][b];
    E[c * 16 + 4 * r + b] = (T)((double)Acc[4 * r + b] - v);
  }
}

// rh = P^{-1} (r~ - A~[:,0] x_p - A~_{c,c-nxy} yb_{c-nxy}) in wavefront order,
// with yb the forward result of the layer below (wavefront order) and no
// z term on the first layer; x_p carries nx*ny zero guards on each side.
template <class T>
__global__ __launch_bounds__(256) void k_ras1_rhs(int nx, int ny, int64_t n, const T *__restrict__ rt,
                                                  const T *__restrict__ col0, const T *__restrict__ xp,
                                                  const T *__restrict__ t7, const T *__restrict__ yb,
                                                  const T *__restrict__ P, T *__restrict__ rh) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;                               // whole quads
  const int64_t nxy = (int64_t)nx * ny, c = t >> 2;
  const int row = (int)(t & 3);
  const int64_t off[7] = {-nxy, -(int64_t)nx, -1, 0, 1, (int64_t)nx, nxy};
  T col[8], dv[4];
  ld8v(col0 + c * 32 + 8 * row, col);
  ld4v(P + c * 16 + 4 * row, dv);
  T v = rt[t];
#pragma unroll
  for (int s = 0; s < 7; ++s) v = v - col[s] * xp[c + off[s]];
  const int64_t k = c / nxy, rem = c - k * nxy;
  const int j = (int)(rem / nx), i = (int)(rem - (int64_t)j * nx);
  const int64_t p = k * nxy + wf_pos(i, j, nx, ny);
  if (k > 0) {
    T a[4], yv[4];
    ld4v(t7 + c * 16 + 4 * row, a);                     // slot 0: A~_{c,c-nxy}
    ld4v(yb + 4 * (p - nxy), yv);
    v = v - dot4(a, yv);
  }
  rh[4 * p + row] = quad_mv<T>(dv, v);
}

// y = y - P^{-1} A~_{c,c+nxy} za_{c+nxy} on every layer but the last; y in
// wavefront order, za (the backward result of the layer above) natural.
template <class T>
__global__ __launch_bounds__(256) void k_ras1_up(int nx, int ny, int nz, int64_t n, const T *__restrict__ t7,
                                                 const T *__restrict__ za, const T *__restrict__ P,
                                                 T *__restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;                               // whole quads
  const int64_t nxy = (int64_t)nx * ny, c = t >> 2;
  const int row = (int)(t & 3);
  const int64_t k = c / nxy;
  if (k >= nz - 1) return;                              // the same for the quad
  const int64_t rem = c - k * nxy;
  const int j = (int)(rem / nx), i = (int)(rem - (int64_t)j * nx);
  const int64_t p = k * nxy + wf_pos(i, j, nx, ny);
  T a[4], zv[4], dv[4];
  ld4v(t7 + (6 * n + c) * 16 + 4 * row, a);             // slot 6: A~_{c,c+nxy}
  ld4v(za + 4 * (c + nxy), zv);
  ld4v(P + c * 16 + 4 * row, dv);
  const T u = dot4(a, zv);
  y[4 * p + row] = y[4 * p + row] - quad_mv<T>(dv, u);
}

template <class T>
__global__ void k_ras_zero(int64_t m, T *__restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) v[t] = (T)0;
}

__global__ void k_ras_reset(int *__restrict__ ctl) {
  if (threadIdx.x < 2) ctl[threadIdx.x] = 0;
}

// launch shape of the sweeps: LW lines per pass (a multiple of 16, so whole
// waves), U passes per level
struct sweep_shape { int lw, u; };
static sweep_shape ras_sweep_shape(int ny) {
  int u = 1;
  while ((ny + u - 1) / u > 240) u *= 2;
  int lw = (ny + u - 1) / u;
  lw = (lw + 15) / 16 * 16;
  return {lw, u};
}

}  // namespace

// ---------------------------------------------------------------------------
rs_status rs_ras_check_shape(const grid3 &g, int prec) {
  // sweeps: at most 240 lines per pass and 2 passes (FP64) or 4 (FP32);
  // LDS: the factorisation keeps one D^{-1} block per line, the backward
  // sweep four 4-vectors per line, both within 64 KiB
  int max_ny = prec == 64 ? 480 : 960;
  if (g.ny < 1 || g.ny > max_ny || g.nx < 1 || g.nz < 1) return RS_E_ARG;
  return RS_OK;
}

rs_status rs_ras_setup_run(rs_cpr_s *M, int *flag, hipStream_t s) {
  const grid3 &g = M->A->g;
  RS_TRY(rs_ras_check_shape(g, M->prec));
  const bool ov1 = M->o.smoother == RS_SM_RAS1;
  // a quad of lanes per line, at most 240 lines per pass (U passes), and
  // one writer wave: at most 1024 threads
  int u = 1;
  while ((g.ny + u - 1) / u > 240) u *= 2;            // 1, 2 or 4
  const int lw = ((g.ny + u - 1) / u + 15) / 16 * 16;
  size_t es = M->prec == 64 ? sizeof(double) : sizeof(float);
  size_t lds = es * 16 * (size_t)g.ny;
  RS_TRY(M->rblk.alloc(es * 4 * 16 * (size_t)g.n));
  RS_TRY(M->rxp.alloc(es * (size_t)g.n));
  if (ov1) {
    RS_TRY(M->rdv0.alloc(es * 16 * (size_t)g.n));
    RS_TRY(M->rdv2.alloc(es * 16 * (size_t)g.n));
    RS_TRY(M->rblk1.alloc(es * 4 * 16 * (size_t)g.n));
    RS_TRY(M->rblk2.alloc(es * 4 * 16 * (size_t)g.n));
    RS_TRY(M->ry1.alloc(es * 4 * (size_t)g.n));
    RS_TRY(M->rz2.alloc(es * 4 * (size_t)g.n));
    RS_TRY(M->rzero.alloc(es * (size_t)g.n));
  }
  {
    // strips per layer: enough workgroups for the CUs, at least 32 lines each
    int S = std::max(1, std::min(256 / std::max(g.nz, 1), (g.ny + 31) / 32));
    int H = (g.ny + S - 1) / S;
    S = (g.ny + H - 1) / H;                          // every strip non-empty
    M->rs_strips = S; M->rs_h = H;
    const size_t words = (size_t)g.nz * S * g.nx * 4 * (M->prec == 64 ? 2 : 1);
    RS_TRY(M->rxw.alloc(sizeof(uint64_t) * words));
    RS_TRY(M->rctl.alloc(sizeof(int) * 4));
    RS_HIP(hipMemsetAsync(M->rxw.p, 0, sizeof(uint64_t) * words, s));
    RS_HIP(hipMemsetAsync(M->rctl.p, 0, sizeof(int) * 4, s));
    M->repoch = 0;
  }
  auto run = [&](auto tag) -> rs_status {
    using T = decltype(tag);
    const T *t7 = M->D->t7.as<T>();
    auto factor = [&](const T *diag, T *dinv) {
      if constexpr (sizeof(T) == 8) {
        if (u == 1) k_ras_setup<T, 1><<<g.nz, 4 * lw + 64, lds, s>>>(g.nx, g.ny, g.n, lw, t7, diag, dinv, flag);
        else k_ras_setup<T, 2><<<g.nz, 4 * lw + 64, lds, s>>>(g.nx, g.ny, g.n, lw, t7, diag, dinv, flag);
      } else {
        if (u == 1) k_ras_setup<T, 1><<<g.nz, 4 * lw + 64, lds, s>>>(g.nx, g.ny, g.n, lw, t7, diag, dinv, flag);
        else if (u == 2) k_ras_setup<T, 2><<<g.nz, 4 * lw + 64, lds, s>>>(g.nx, g.ny, g.n, lw, t7, diag, dinv, flag);
        else k_ras_setup<T, 4><<<g.nz, 4 * lw + 64, lds, s>>>(g.nx, g.ny, g.n, lw, t7, diag, dinv, flag);
      }
    };
    auto scale = [&](const T *dinv, T *blk) {
      k_ras_scale<T><<<rs_grid(4 * g.n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.n, t7, dinv, blk);
    };
    if (!ov1) {
      factor(nullptr, M->dinv2.as<T>());
      scale(M->dinv2.as<T>(), M->rblk.as<T>());
    } else {
      // P0 (plain layers), P1 (middle of each extension, the owned cells':
      // dinv2), P2 (top of each extension).  The reduced diagonals E live in
      // the P2 scaled blocks' buffer (16 n of its 64 n entries), written only
      // after the last factorisation has read E: no pool memory is released
      // while this stream (possibly a side stream) still uses it.
      T *E = M->rblk2.as<T>();
      factor(nullptr, M->rdv0.as<T>());
      k_ras_zdiag<T><<<rs_grid(4 * g.n), RS_BLOCK, 0, s>>>(g.n, g.nxy, t7, M->rdv0.as<T>(), E);
      factor(E, M->dinv2.as<T>());
      k_ras_zdiag<T><<<rs_grid(4 * g.n), RS_BLOCK, 0, s>>>(g.n, g.nxy, t7, M->dinv2.as<T>(), E);
      factor(E, M->rdv2.as<T>());
      scale(M->rdv0.as<T>(), M->rblk.as<T>());
      scale(M->dinv2.as<T>(), M->rblk1.as<T>());
      scale(M->rdv2.as<T>(), M->rblk2.as<T>());
      k_ras_zero<T><<<rs_grid(g.n), RS_BLOCK, 0, s>>>(g.n, M->rzero.as<T>());
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
  };
  if (M->prec == 64) return run(double{});
  return run(float{});
}

template <class T>
rs_status rs_ras_apply_run(rs_cpr_s *M, const T *xp, T *out, hipStream_t s) {
  const grid3 &g = M->A->g;
  const rs_dcpl_s *D = M->D;
  const bool ov1 = M->o.smoother == RS_SM_RAS1;
  // rh goes to zt, the forward result (wavefront order) to yv
  T *rh = M->zt.as<T>(), *y = M->yv.as<T>(), *xpw = M->rxp.as<T>();
  // the layer factors of the first forward sweep: P0 (dinv2 for overlap 0)
  const T *P0 = ov1 ? M->rdv0.as<T>() : M->dinv2.as<T>();
  {
    const int64_t tiles = (int64_t)g.nz * ((g.nx + RI - 1) / RI) * ((g.ny + RJ - 1) / RJ);
    // the tickets of the sweeps below are zeroed here (overlap 0); the
    // overlapping form sweeps several times and zeroes them before each
    int *tk = !ov1 ? M->rctl.as<int>() : nullptr;
    k_ras_in_tile<T><<<(unsigned)tiles, 4 * RI * RJ, 0, s>>>(g.nx, g.ny, g.n, M->rt.as<T>(), D->col0.as<T>(), xp,
                                                             P0, rh, xpw, tk);
  }
  RS_HIP(hipGetLastError());
  const sweep_shape sh = ras_sweep_shape(g.ny);
  // compute lanes (at most 960) + one writer wave
  const int nt = 4 * sh.lw + 64;
  const size_t ring_bytes = sizeof(T) * 8 * (size_t)g.ny;     // two levels of [ny][4]
  // one forward sweep over all layers: blocks blk, rhs r (wavefront), result yo (wavefront)
  std::function<void(const T *, const T *, T *)> fwd;
  // one backward sweep: result + x_p (x_p in wavefront order) in natural order
  std::function<void(const T *, const T *, const T *, T *)> bwd;
  // strips of H lines (the tickets restart at every launch)
  const int S = M->rs_strips, H = M->rs_h;
  int *ctl = M->rctl.as<int>();
  uint64_t *xw = M->rxw.as<uint64_t>();
  const unsigned nwg = (unsigned)(g.nz * S);
  if (H <= 224) {
    // strips of at most 224 lines: a quad of lanes per cell (one pass)
    const int lwq = (H + 15) / 16 * 16, ntq = 4 * lwq + 128;
    const size_t rb3 = sizeof(T) * 8 * (size_t)(H + 2);
    fwd = [=](const T *blk, const T *r, T *yo) {
      if (ov1) k_ras_reset<<<1, 64, 0, s>>>(ctl);
      const uint32_t tag = ++M->repoch;
      k_ras_fwd3<T, 4><<<nwg, ntq, rb3, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lwq, blk, r, yo, ctl, xw, tag);
    };
    bwd = [=](const T *blk, const T *yi, const T *xw_p, T *o) {
      if (ov1) k_ras_reset<<<1, 64, 0, s>>>(ctl);
      const uint32_t tag = ++M->repoch;
      k_ras_bwd3<T, 4><<<nwg, ntq, 2 * rb3, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lwq, blk, yi, xw_p, o, ctl, xw, tag);
    };
  } else if constexpr (sizeof(T) == 4) {
    // taller strips (FP32): one lane per line (at most 256 per pass, U passes)
    const int u1 = H <= 256 ? 1 : (H <= 512 ? 2 : 4);
    const int lw1 = ((H + u1 - 1) / u1 + 63) / 64 * 64, nt1 = lw1 + 64;
    const size_t rb = sizeof(float) * 8 * (size_t)(H + 2);
    fwd = [=](const T *blk, const T *r, T *yo) {
      if (ov1) k_ras_reset<<<1, 64, 0, s>>>(ctl);
      const uint32_t tag = ++M->repoch;
      if (u1 == 1) k_ras_fwd1<1, 5><<<nwg, nt1, rb, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lw1, blk, r, yo, ctl, xw, tag);
      else if (u1 == 2) k_ras_fwd1<2, 3><<<nwg, nt1, rb, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lw1, blk, r, yo, ctl, xw, tag);
      else k_ras_fwd1<4, 2><<<nwg, nt1, rb, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lw1, blk, r, yo, ctl, xw, tag);
    };
    bwd = [=](const T *blk, const T *yi, const T *xw_p, T *o) {
      if (ov1) k_ras_reset<<<1, 64, 0, s>>>(ctl);
      const uint32_t tag = ++M->repoch;
      if (u1 == 1) k_ras_bwd1<1, 5><<<nwg, nt1, 2 * rb, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lw1, blk, yi, xw_p, o, ctl, xw, tag);
      else if (u1 == 2) k_ras_bwd1<2, 3><<<nwg, nt1, 2 * rb, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lw1, blk, yi, xw_p, o, ctl, xw, tag);
      else k_ras_bwd1<4, 2><<<nwg, nt1, 2 * rb, s>>>(g.nx, g.ny, g.nz, S, H, g.n, lw1, blk, yi, xw_p, o, ctl, xw, tag);
    };
  } else {
    // taller layers (FP64): one workgroup per layer, a quad of lanes per cell
    fwd = [=](const T *blk, const T *r, T *yo) {
      if (sh.u == 1) k_ras_fwd<T, 1, 4><<<g.nz, nt, ring_bytes, s>>>(g.nx, g.ny, g.n, sh.lw, blk, r, yo);
      else k_ras_fwd<T, 2, 2><<<g.nz, nt, ring_bytes, s>>>(g.nx, g.ny, g.n, sh.lw, blk, r, yo);
    };
    bwd = [=](const T *blk, const T *yi, const T *xw_p, T *o) {
      if (sh.u == 1) k_ras_bwd<T, 1, 4><<<g.nz, nt, 2 * ring_bytes, s>>>(g.nx, g.ny, g.n, sh.lw, blk, yi, xw_p, o);
      else k_ras_bwd<T, 2, 2><<<g.nz, nt, 2 * ring_bytes, s>>>(g.nx, g.ny, g.n, sh.lw, blk, yi, xw_p, o);
    };
  }
  const T *blk = M->rblk.as<T>();
  if (!ov1) {
    fwd(blk, rh, y);
    RS_HIP(hipGetLastError());
    bwd(blk, y, xpw, out);
    RS_HIP(hipGetLastError());
    return RS_OK;
  }
  const T *t7 = D->t7.as<T>();
  T *y1 = M->ry1.as<T>(), *z2 = M->rz2.as<T>();
  const unsigned gq = rs_grid(4 * g.n);
  fwd(blk, rh, y);                                                       // y0
  k_ras1_rhs<T><<<gq, RS_BLOCK, 0, s>>>(g.nx, g.ny, g.n, M->rt.as<T>(), D->col0.as<T>(), xp, t7, y,
                                        M->dinv2.as<T>(), rh);
  fwd(M->rblk1.as<T>(), rh, y1);                                         // y1
  k_ras1_rhs<T><<<gq, RS_BLOCK, 0, s>>>(g.nx, g.ny, g.n, M->rt.as<T>(), D->col0.as<T>(), xp, t7, y1,
                                        M->rdv2.as<T>(), rh);
  fwd(M->rblk2.as<T>(), rh, y);                                          // y2
  bwd(M->rblk2.as<T>(), y, M->rzero.as<T>(), z2);                        // z2 (natural order)
  k_ras1_up<T><<<gq, RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, g.n, t7, z2, M->dinv2.as<T>(), y1);
  bwd(M->rblk1.as<T>(), y1, xpw, out);                                   // z of the owned layer
  RS_HIP(hipGetLastError());
  return RS_OK;
}

template rs_status rs_ras_apply_run<double>(rs_cpr_s *, const double *, double *, hipStream_t);
template rs_status rs_ras_apply_run<float>(rs_cpr_s *, const float *, float *, hipStream_t);
