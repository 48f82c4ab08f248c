// dilu.hip -- block ILU(0) (DILU on the 7-point block pattern) in natural
// order: factorisation and forward/backward sweeps as persistent, pipelined
// kernels.
//
// The recurrences run over hyperplanes i+j+k = const.  One launch per
// hyperplane costs a few microseconds of launch and drain each (about 1000
// launches per application at 200x200x100), so instead the grid is cut into
// bricks of B x B x-lines (j, k) running along the whole x extent, and one
// workgroup walks its brick hyperplane by hyperplane (local level
// lambda = i + j_local + k_local): four lanes per cell (one block row each),
// the previous level of the brick in an LDS ring, one barrier per level.
// A brick needs, at level lambda, the face values of the bricks before it in
// j and in k at their level lambda + B - 1, published through per-brick
// progress counters.
//
// Progress and visibility across workgroups (and across XCDs, whose L2 caches
// are not coherent with each other):
//   - the only values other bricks read are the brick's outgoing faces; all
//     of them are mapped into wave 0 and stored with device-scope stores;
//   - wave 0 waits for its stores to complete (s_waitcnt vmcnt(0)), then
//     lane 0 stores the level counter with a device-scope store;
//   - a consumer polls the counter with device-scope loads and reads the
//     face values with device-scope loads, after a barrier that follows the
//     poll.
//   - bricks are handed out by a ticket counter in an order where every
//     brick comes after the bricks it waits on, so a waiting workgroup only
//     ever waits on workgroups that are already running: no deadlock,
//     whatever the residency.  Each wait is bounded; on time-out the kernel
//     records an error and finishes (the host reports RS_E_HIP).
// The arithmetic per cell is the same sequence of operations as the
// definition, so results are bitwise reproducible.
#include "rs_internal.h"
#include <math.h>
#include <algorithm>
#include <stdlib.h>

namespace {
#pragma clang fp contract(off)
#include "block4.h"
#pragma clang fp contract(fast)
#include "quad4.h"

constexpr int SPIN_LIMIT = 1 << 22;     // about a quarter of a second of polling
constexpr int XSPIN_LIMIT = 1 << 20;    // face-word polls (each a device-scope load): about a second

// Wait until *flag >= need.  After one time-out in a workgroup (recorded in
// *err and in `failed`) it stops waiting altogether, so a failure costs one
// time-out, not one per level.
__device__ __forceinline__ int poll_until(const int *flag, int need, int seen, int *err, bool &failed) {
  int spins = 0;
  while (seen < need && !failed) {
    seen = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (seen >= need) break;
    __builtin_amdgcn_s_sleep(2);
    if (++spins > SPIN_LIMIT) { atomicOr(err, 1); failed = true; }
  }
  return seen;
}

template <class T>
__device__ __forceinline__ void st_dev(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <class T>
__device__ __forceinline__ T ld_dev(const T *p) { return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// cell slot of a brick: faces first (so that they all land in wave 0).
// fwd: outgoing faces are jl == B-1 and kl == B-1; bwd: jl == 0 and kl == 0.
template <int B, bool FWD>
__device__ __forceinline__ void cell_of(int cl, int &jl, int &kl) {
  int f = FWD ? B - 1 : 0;
  if (cl < B) { jl = f; kl = cl; return; }
  if (cl < 2 * B - 1) {
    int t = cl - B;                         // 0 .. B-2
    kl = f;
    jl = FWD ? t : t + 1;
    return;
  }
  int m = cl - (2 * B - 1);                 // interior (B-1)^2
  jl = m % (B - 1);
  kl = m / (B - 1);
  if (!FWD) { jl += 1; kl += 1; }
}

__global__ void k_pipe_reset(int nb, int *__restrict__ done, int *__restrict__ ticket) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nb) done[t] = 0;
  if (t == 0) *ticket = 0;
}

template <class T>
__device__ __forceinline__ T group_mv(const T *__restrict__ Mrow, T v) {
  int base = (threadIdx.x & 63) & ~3;
  T out = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) out = fma(Mrow[m], __shfl(v, base + m, 64), out);
  return out;
}

// ---- tagged exchange of brick faces ------------------------------------------
// A face value travels as 64-bit words (tag << 32 | 32 data bits): one word
// per FP32 value, two (low, high halves) per FP64 value.  The tag is the
// launch's epoch, so a consumer that reads its word with a device-scope load
// knows the data is current when the tag matches; stale words from earlier
// launches carry older epochs and no reset is needed.
template <class T> struct xw;
template <> struct xw<float> {
  static constexpr int W = 1;
  __device__ static void put(uint64_t *p, float v, uint32_t tag) {
    st_dev(p, (uint64_t)(((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v)));
  }
  // spins until the tag matches; returns false on time-out
  __device__ static bool get(const uint64_t *p, uint64_t &w0, uint64_t &, uint32_t tag, float &v, bool &failed) {
    int spins = 0;
    while ((uint32_t)(w0 >> 32) != tag && !failed) {
      if (++spins > XSPIN_LIMIT) { failed = true; return false; }
      __builtin_amdgcn_s_sleep(1);
      w0 = ld_dev(p);
    }
    v = __uint_as_float((uint32_t)w0);
    return true;
  }
  __device__ static void pre(const uint64_t *p, uint64_t &w0, uint64_t &) { w0 = ld_dev(p); }
};
template <> struct xw<double> {
  static constexpr int W = 2;
  __device__ static void put(uint64_t *p, double v, uint32_t tag) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    st_dev(p, (uint64_t)(((uint64_t)tag << 32) | (b & 0xffffffffull)));
    st_dev(p + 1, (uint64_t)(((uint64_t)tag << 32) | (b >> 32)));
  }
  __device__ static bool get(const uint64_t *p, uint64_t &w0, uint64_t &w1, uint32_t tag, double &v, bool &failed) {
    int spins = 0;
    while (((uint32_t)(w0 >> 32) != tag || (uint32_t)(w1 >> 32) != tag) && !failed) {
      if (++spins > XSPIN_LIMIT) { failed = true; return false; }
      __builtin_amdgcn_s_sleep(1);
      w0 = ld_dev(p);
      w1 = ld_dev(p + 1);
    }
    v = __longlong_as_double((long long)(((w1 & 0xffffffffull) << 32) | (w0 & 0xffffffffull)));
    return true;
  }
  __device__ static void pre(const uint64_t *p, uint64_t &w0, uint64_t &w1) { w0 = ld_dev(p); w1 = ld_dev(p + 1); }
};

// word offset of the value (row r) of face cell (face f, position pos, i) of brick b
template <class T, int B>
__device__ __forceinline__ int64_t xslot(int b, int f, int pos, int i, int nx, int r) {
  return ((((int64_t)b * 2 + f) * B + pos) * nx + i) * (4 * xw<T>::W) + r * xw<T>::W;
}

// ---- forward sweep: y_c = D_c^{-1} (r~2_c - sum_{lower k} A~_ck y_k) --------
// Bricks of 4 x 4 x-lines, so one level of a brick is 16 cells x 4 block rows
// = one wave.  The workgroup's NW waves take the levels in turn: wave w
// computes levels w, w+NW, ...; right after computing a level it issues
// every load of its next one (blocks, D^{-1} row, residual and correction
// terms, and the neighbour bricks' face values).  A wave therefore only ever
// has its own next level's loads in flight, which get NW-1 level-times to
// land.  The previous level passes between waves through an LDS ring; one
// barrier per level.  The per-level critical path is kept short: addresses
// are a uniform per-array base plus one 32-bit lane offset, the 4-vectors of
// neighbours are read whole from LDS (or were prefetched whole from the
// exchange buffer), and the 4x4 products gather the other rows of the cell
// with quad-broadcast DPP moves instead of LDS permutes.
constexpr int BR = 4;                    // brick edge (x-lines per side)

template <class T> __device__ __forceinline__ const T *at(const T *base, uint32_t byte_off) {
  return (const T *)((const char *)base + byte_off);
}

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// all 4 values of a neighbour cell from the exchange buffer (words prefetched
// in w[]; re-polled while the tag is stale)
// The exchange buffer is read through a buffer resource: 16-byte loads with
// device scope (sc1), which return zero instead of faulting out of range.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int RS_CPOL_SC1 = 16;          // cache policy: device scope
__device__ __forceinline__ __amdgpu_buffer_rsrc_t xrsrc(const uint64_t *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}

template <class T> struct xcell {
  static constexpr int NWD = 4 * xw<T>::W;
  // words w[] of the cell starting at word index `word` (16-byte aligned):
  // each 64-bit word is read whole, tag and data together
  __device__ static void pre(__amdgpu_buffer_rsrc_t r, int64_t word, uint64_t (&w)[NWD]) {
#pragma unroll
    for (int e = 0; e < NWD; e += 2) {
      u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, (uint32_t)((word + e) * 8), 0, RS_CPOL_SC1);
      w[e] = ((uint64_t)q.y << 32) | q.x;
      w[e + 1] = ((uint64_t)q.w << 32) | q.z;
    }
  }
  __device__ static bool get(__amdgpu_buffer_rsrc_t r, int64_t word, uint64_t (&w)[NWD], uint32_t tag, T (&out)[4],
                             bool &failed) {
    int spins = 0;
    for (;;) {
      bool ok = true;
#pragma unroll
      for (int e = 0; e < NWD; ++e) ok = ok && (uint32_t)(w[e] >> 32) == tag;
      if (ok || failed) break;
      if (++spins > XSPIN_LIMIT) { failed = true; return false; }
      __builtin_amdgcn_s_sleep(1);
      pre(r, word, w);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (xw<T>::W == 1) {
        out[m] = (T)__uint_as_float((uint32_t)w[m]);
      } else {
        uint64_t lo = w[2 * m] & 0xffffffffull, hi = w[2 * m + 1] & 0xffffffffull;
        out[m] = (T)__longlong_as_double((long long)((hi << 32) | lo));
      }
    }
    return true;
  }
};

template <class T> struct fwd_pre {
  T rt, col[8], xq[7], a[3][4], dv[4];
  uint64_t ez[4 * xw<T>::W], ey[4 * xw<T>::W];      // face words (-z, -y)
};

template <class T, int NW>
__global__ __launch_bounds__(64 * NW) void k_fwd_pipe(
    int nx, int ny, int nz, int NJ, const int *__restrict__ ord, int *__restrict__ ticket,
    int *__restrict__ err, uint32_t tag, uint64_t *__restrict__ xch, uint32_t xbytes, const T *__restrict__ t7,
    const T *__restrict__ dinv2, const T *__restrict__ rt, const T *__restrict__ col0,
    const T *__restrict__ xp, T *__restrict__ y) {
  constexpr int B = BR;
  __shared__ T ring[2][B][B][4];
  __shared__ int s_b;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int row = lane & 3, cl = lane >> 2;
  const int jl = cl % B, kl = cl / B;
  if (tid == 0) s_b = ord[atomicAdd(ticket, 1)];
  __syncthreads();
  const int b = s_b, J = b % NJ, K = b / NJ;
  const int j = J * B + jl, k = K * B + kl;
  const bool line = j < ny && k < nz;
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  const int L = nx + 2 * B - 2;
  const bool ext_z = kl == 0 && k > 0, ext_y = jl == 0 && j > 0;
  const uint32_t c0 = line ? (uint32_t)(nx * (j + (int64_t)ny * k)) : 0u;
  const int64_t off[7] = {-nxy, -(int64_t)nx, -1, 0, 1, (int64_t)nx, nxy};
  const __amdgpu_buffer_rsrc_t xr = xrsrc(xch, xbytes);
  bool failed = false;
  auto load = [&](int lam, fwd_pre<T> &P) {
    const int i = lam - jl - kl;
    const uint32_t c = c0 + (uint32_t)min(max(i, 0), nx - 1);
    const uint32_t o4 = c * 4u * sizeof(T), o16 = c * 16u * sizeof(T), o1 = c * (uint32_t)sizeof(T);
    const uint32_t r1 = row * (uint32_t)sizeof(T), r4 = row * 4u * (uint32_t)sizeof(T);
    P.rt = *at(rt, o4 + r1);
    ld8v(at(col0, 2 * o16 + 2 * r4), P.col);
#pragma unroll
    for (int s = 0; s < 7; ++s) P.xq[s] = *at(xp + off[s], o1);   // x_p carries zero guard planes
#pragma unroll
    for (int s = 0; s < 3; ++s) ld4v(at(t7 + (int64_t)s * n * 16, o16 + r4), P.a[s]);
    ld4v(at(dinv2, o16 + r4), P.dv);
    const bool act = line && i >= 0 && i < nx;
    // lanes without an external neighbour load their own brick's face words
    // instead (distinct addresses, never used) so that the load count stays fixed
    const int ic = min(max(i, 0), nx - 1);
    xcell<T>::pre(xr, (act && ext_z) ? xslot<T, B>(b - NJ, 1, jl, i, nx, 0) : xslot<T, B>(b, 1, jl, ic, nx, 0), P.ez);
    xcell<T>::pre(xr, (act && ext_y) ? xslot<T, B>(b - 1, 0, kl, i, nx, 0) : xslot<T, B>(b, 0, kl, ic, nx, 0), P.ey);
  };
  fwd_pre<T> P;
  if (wave < L) load(wave, P);
  for (int lam = 0; lam < L; ++lam) {
    __syncthreads();
    if (lam % NW != wave) continue;            // wave-uniform
    const int prev = (lam + 1) & 1, cur = lam & 1;
    const int i = lam - jl - kl;
    const bool act = line && i >= 0 && i < nx;
    T v = P.rt;
#pragma unroll
    for (int s = 0; s < 7; ++s) v = v - P.col[s] * P.xq[s];
    T yz[4], yy[4], yx[4];
    if (kl > 0) ld4(&ring[prev][kl - 1][jl][0], yz);
    else if (act && k > 0 && !xcell<T>::get(xr, xslot<T, B>(b - NJ, 1, jl, i, nx, 0), P.ez, tag, yz, failed)) atomicOr(err, 1);
    if (jl > 0) ld4(&ring[prev][kl][jl - 1][0], yy);
    else if (act && j > 0 && !xcell<T>::get(xr, xslot<T, B>(b - 1, 0, kl, i, nx, 0), P.ey, tag, yy, failed)) atomicOr(err, 1);
    ld4(&ring[prev][kl][jl][0], yx);
    if (act && k > 0) v = v - dot4(P.a[0], yz);
    if (act && j > 0) v = v - dot4(P.a[1], yy);
    if (act && i > 0) v = v - dot4(P.a[2], yx);
    const T o = quad_mv<T>(P.dv, v);
    if (act) {
      const uint32_t c = c0 + (uint32_t)i;
      ring[cur][kl][jl][row] = o;
      y[(int64_t)4 * c + row] = o;
      if (jl == B - 1) xw<T>::put(xch + xslot<T, B>(b, 0, kl, i, nx, row), o, tag);
      if (kl == B - 1) xw<T>::put(xch + xslot<T, B>(b, 1, jl, i, nx, row), o, tag);
    }
    if (lam + NW < L) load(lam + NW, P);
  }
}

// ---- backward sweep: z_c = y_c - D_c^{-1} sum_{upper k} A~_ck z_k ------------
template <class T> struct bwd_pre {
  T yc, xpc, a[3][4], dv[4];
  uint64_t ey[4 * xw<T>::W], ez[4 * xw<T>::W];      // face words (+y, +z)
};

template <class T, int NW>
__global__ __launch_bounds__(64 * NW) void k_bwd_pipe(
    int nx, int ny, int nz, int NJ, int NK, const int *__restrict__ ord, int *__restrict__ ticket,
    int *__restrict__ err, uint32_t tag, uint64_t *__restrict__ xch, uint32_t xbytes, const T *__restrict__ t7,
    const T *__restrict__ dinv2, const T *__restrict__ y, const T *__restrict__ xp, T *__restrict__ out) {
  constexpr int B = BR;
  __shared__ T ring[2][B][B][4];
  __shared__ int s_b;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int row = lane & 3, cl = lane >> 2;
  const int jl = cl % B, kl = cl / B;
  const int nb = NJ * NK;
  if (tid == 0) s_b = ord[nb - 1 - atomicAdd(ticket, 1)];
  __syncthreads();
  const int b = s_b, J = b % NJ, K = b / NJ;
  const int j = J * B + jl, k = K * B + kl;
  const bool line = j < ny && k < nz;
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  const int L = nx + 2 * B - 2;
  const bool ext_y = jl == B - 1 && j < ny - 1, ext_z = kl == B - 1 && k < nz - 1;
  const uint32_t c0 = line ? (uint32_t)(nx * (j + (int64_t)ny * k)) : 0u;
  const __amdgpu_buffer_rsrc_t xr = xrsrc(xch, xbytes);
  bool failed = false;
  auto load = [&](int step, bwd_pre<T> &P) {
    const int i = L - 1 - step - jl - kl;
    const uint32_t c = c0 + (uint32_t)min(max(i, 0), nx - 1);
    const uint32_t o4 = c * 4u * sizeof(T), o16 = c * 16u * sizeof(T), o1 = c * (uint32_t)sizeof(T);
    const uint32_t r1 = row * (uint32_t)sizeof(T), r4 = row * 4u * (uint32_t)sizeof(T);
    P.yc = *at(y, o4 + r1);
    P.xpc = *at(xp, o1);
#pragma unroll
    for (int s = 0; s < 3; ++s) ld4v(at(t7 + (int64_t)(s + 4) * n * 16, o16 + r4), P.a[s]);
    ld4v(at(dinv2, o16 + r4), P.dv);
    const bool act = line && i >= 0 && i < nx;
    const int ic = min(max(i, 0), nx - 1);
    xcell<T>::pre(xr, (act && ext_y) ? xslot<T, B>(b + 1, 0, kl, i, nx, 0) : xslot<T, B>(b, 0, kl, ic, nx, 0), P.ey);
    xcell<T>::pre(xr, (act && ext_z) ? xslot<T, B>(b + NJ, 1, jl, i, nx, 0) : xslot<T, B>(b, 1, jl, ic, nx, 0), P.ez);
  };
  bwd_pre<T> P;
  if (wave < L) load(wave, P);
  for (int step = 0; step < L; ++step) {
    __syncthreads();
    if (step % NW != wave) continue;           // wave-uniform
    const int prev = (step + 1) & 1, cur = step & 1;
    const int i = L - 1 - step - jl - kl;
    const bool act = line && i >= 0 && i < nx;
    T zx[4], zy[4], zz[4];
    ld4(&ring[prev][kl][jl][0], zx);
    if (jl < B - 1) ld4(&ring[prev][kl][jl + 1][0], zy);
    else if (act && j < ny - 1 && !xcell<T>::get(xr, xslot<T, B>(b + 1, 0, kl, i, nx, 0), P.ey, tag, zy, failed)) atomicOr(err, 1);
    if (kl < B - 1) ld4(&ring[prev][kl + 1][jl][0], zz);
    else if (act && k < nz - 1 && !xcell<T>::get(xr, xslot<T, B>(b + NJ, 1, jl, i, nx, 0), P.ez, tag, zz, failed)) atomicOr(err, 1);
    T v = 0;
    if (act && i < nx - 1) v = v + dot4(P.a[0], zx);
    if (act && j < ny - 1) v = v + dot4(P.a[1], zy);
    if (act && k < nz - 1) v = v + dot4(P.a[2], zz);
    const T w = quad_mv<T>(P.dv, v);
    if (act) {
      const uint32_t c = c0 + (uint32_t)i;
      const T zc = P.yc - w;
      ring[cur][kl][jl][row] = zc;
      out[(int64_t)4 * c + row] = row == 0 ? zc + P.xpc : zc;
      if (jl == 0) xw<T>::put(xch + xslot<T, B>(b, 0, kl, i, nx, row), zc, tag);
      if (kl == 0) xw<T>::put(xch + xslot<T, B>(b, 1, jl, i, nx, row), zc, tag);
    }
    if (step + NW < L) load(step + NW, P);
  }
}

// ---- factorisation: D_c = A~_cc - sum_{lower k} A~_ck D_k^{-1} A~_kc ----------
// one thread per cell (B*B threads: one wave for B = 8); the previous level's
// D^{-1} blocks of the brick in an LDS ring
template <class T, int B>
__global__ __launch_bounds__(B * B) void k_setup_pipe(
    int nx, int ny, int nz, int NJ, const int *__restrict__ ord, int *__restrict__ ticket,
    int *__restrict__ done, int *__restrict__ err, const T *__restrict__ t7, T *__restrict__ dinv2,
    int *__restrict__ flag) {
#pragma clang fp contract(off)
  __shared__ T ring[2][B][B][16];
  __shared__ int s_b;
  const int tid = threadIdx.x;
  int jl, kl;
  cell_of<B, true>(tid, jl, kl);
  if (tid == 0) s_b = ord[atomicAdd(ticket, 1)];
  __syncthreads();
  const int b = s_b, J = b % NJ, K = b / NJ;
  const int j = J * B + jl, k = K * B + kl;
  const bool line = j < ny && k < nz;
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  const int L = nx + 2 * B - 2;
  const bool face = (jl == B - 1) || (kl == B - 1);
  int seenJ = 0, seenK = 0, bad = 0;
  bool failed = false;
  for (int lam = 0; lam < L; ++lam) {
    const int i = lam - jl - kl;
    const bool act = line && i >= 0 && i < nx;
    const int64_t c = act ? i + nx * (j + (int64_t)ny * k) : 0;
    if (tid == 0) {
      if (J > 0) seenJ = poll_until(done + b - 1, min(lam + B, L), seenJ, err, failed);
      if (K > 0) seenK = poll_until(done + b - NJ, min(lam + B, L), seenK, err, failed);
    }
    __syncthreads();
    const int prev = (lam + 1) & 1, cur = lam & 1;
    if (act) {
      double D[4][4];
#pragma unroll
      for (int e = 0; e < 16; ++e) D[e >> 2][e & 3] = (double)t7[(3 * n + c) * 16 + e];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        bool has = s == 0 ? k > 0 : (s == 1 ? j > 0 : i > 0);
        if (!has) continue;
        int64_t q = c - (s == 0 ? nxy : (s == 1 ? (int64_t)nx : 1));
        double Dq[4][4], Aqc[4][4], Acq[4][4], T1[4][4];
        if (s == 0 && kl == 0) {
#pragma unroll
          for (int e = 0; e < 16; ++e) Dq[e >> 2][e & 3] = (double)ld_dev(dinv2 + q * 16 + e);
        } else if (s == 1 && jl == 0) {
#pragma unroll
          for (int e = 0; e < 16; ++e) Dq[e >> 2][e & 3] = (double)ld_dev(dinv2 + q * 16 + e);
        } else {
          int rk = s == 0 ? kl - 1 : kl, rj = s == 1 ? jl - 1 : jl;
#pragma unroll
          for (int e = 0; e < 16; ++e) Dq[e >> 2][e & 3] = (double)ring[prev][rk][rj][e];
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          Aqc[e >> 2][e & 3] = (double)t7[((int64_t)(6 - s) * n + q) * 16 + e];
          Acq[e >> 2][e & 3] = (double)t7[((int64_t)s * n + c) * 16 + e];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) v = v + Dq[r][m] * Aqc[m][cc];
            T1[r][cc] = v;
          }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) v = v + Acq[r][m] * T1[m][cc];
            D[r][cc] = D[r][cc] - v;
          }
      }
      double R[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) R[r][qq] = (r == qq) ? 1.0 : 0.0;
      bad |= gje4<4>(D, R);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        T v = (T)R[e >> 2][e & 3];
        ring[cur][kl][jl][e] = v;
        if (face) st_dev(dinv2 + c * 16 + e, v);
        else dinv2[c * 16 + e] = v;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (tid == 0) st_dev(done + b, lam + 1);
  }
  if (bad) atomicOr(flag, bad);
}

}  // namespace

// ---------------------------------------------------------------------------
rs_status rs_dilu_prepare(rs_cpr_s *M) {
  const grid3 &g = M->A->g;
  int B = BR;
  int NJ = (g.ny + B - 1) / B, NK = (g.nz + B - 1) / B, nb = NJ * NK;
  M->pb = B; M->pnj = NJ; M->pnk = NK;
  // bricks by increasing J + K (then K): every brick after the ones it waits on
  std::vector<int> ord(nb);
  for (int t = 0; t < nb; ++t) ord[t] = t;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    int da = a % NJ + a / NJ, db = b % NJ + b / NJ;
    return da < db;
  });
  RS_TRY(M->pord.alloc(sizeof(int) * nb));
  RS_TRY(M->pdone.alloc(sizeof(int) * (nb + 1)));
  RS_TRY(M->pctl.alloc(sizeof(int) * 2));     // [0] ticket, [1] error
  // face exchange: 2 faces x B lines x nx cells x 4 values x (1 or 2) words
  size_t words = (size_t)nb * 2 * B * g.nx * 4 * (M->prec == 64 ? 2 : 1);
  if (sizeof(uint64_t) * words >= 0xffffffffull) return RS_E_ARG;   // one buffer resource covers it
  RS_TRY(M->pxch.alloc(sizeof(uint64_t) * words));
  RS_HIP(hipMemset(M->pxch.p, 0, sizeof(uint64_t) * words));
  M->pepoch = 0;
  RS_HIP(hipMemcpy(M->pord.p, ord.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
  RS_HIP(hipMemset(M->pctl.p, 0, sizeof(int) * 2));
  return RS_OK;
}

static void pipe_reset(rs_cpr_s *M, hipStream_t s) {
  int nb = M->pnj * M->pnk;
  k_pipe_reset<<<rs_grid(nb), RS_BLOCK, 0, s>>>(nb, M->pdone.as<int>(), M->pctl.as<int>());
}

rs_status rs_dilu_setup_run(rs_cpr_s *M, int *flag, hipStream_t s) {
  const grid3 &g = M->A->g;
  int nb = M->pnj * M->pnk;
  int *ctl = M->pctl.as<int>();
  pipe_reset(M, s);
#define RS_SETUP(T, BB)                                                                            \
  k_setup_pipe<T, BB><<<nb, BB * BB, 0, s>>>(g.nx, g.ny, g.nz, M->pnj, M->pord.as<int>(), ctl,      \
                                             M->pdone.as<int>(), ctl + 1, M->D->t7.as<T>(),        \
                                             M->dinv2.as<T>(), flag)
  if (M->prec == 64) RS_SETUP(double, BR);
  else RS_SETUP(float, BR);
#undef RS_SETUP
  RS_HIP(hipGetLastError());
  return RS_OK;
}

template <class T>
rs_status rs_dilu_apply_run(rs_cpr_s *M, const T *xp, T *out, hipStream_t s) {
  const grid3 &g = M->A->g;
  int nb = M->pnj * M->pnk;
  int *ctl = M->pctl.as<int>();
  const rs_dcpl_s *D = M->D;
  uint64_t *xch = M->pxch.as<uint64_t>();
  uint32_t xbytes = (uint32_t)M->pxch.bytes;
  const int nw = 6;                   // waves per brick workgroup
  pipe_reset(M, s);
  uint32_t tag = ++M->pepoch;
#define RS_FWD(NW) k_fwd_pipe<T, NW><<<nb, 64 * NW, 0, s>>>(g.nx, g.ny, g.nz, M->pnj, M->pord.as<int>(), ctl, ctl + 1, \
      tag, xch, xbytes, D->t7.as<T>(), M->dinv2.as<T>(), M->rt.as<T>(), D->col0.as<T>(), xp, M->yv.as<T>())
  if (nw == 4) RS_FWD(4); else if (nw == 8) RS_FWD(8); else RS_FWD(6);
#undef RS_FWD
  pipe_reset(M, s);
  tag = ++M->pepoch;
#define RS_BWD(NW) k_bwd_pipe<T, NW><<<nb, 64 * NW, 0, s>>>(g.nx, g.ny, g.nz, M->pnj, M->pnk, M->pord.as<int>(), ctl, \
      ctl + 1, tag, xch, xbytes, D->t7.as<T>(), M->dinv2.as<T>(), M->yv.as<T>(), xp, out)
  if (nw == 4) RS_BWD(4); else if (nw == 8) RS_BWD(8); else RS_BWD(6);
#undef RS_BWD
  RS_HIP(hipGetLastError());
  return RS_OK;
}

template rs_status rs_dilu_apply_run<double>(rs_cpr_s *, const double *, double *, hipStream_t);
template rs_status rs_dilu_apply_run<float>(rs_cpr_s *, const float *, float *, hipStream_t);

// error word of the pipelined kernels (time-out of a bounded wait)
// error words of the pipelined sweeps (DILU bricks, RAS strips): a bounded
// wait that timed out leaves a non-zero word
rs_status rs_dilu_check(rs_cpr_s *M, hipStream_t s) {
  int h = 0, r = 0;
  if (M->pctl.p) RS_TRY(rs_wait_read(&h, M->pctl.as<int>() + 1, sizeof(int), s));
  if (M->rctl.p) RS_TRY(rs_wait_read(&r, M->rctl.as<int>() + 2, sizeof(int), s));
  return (h || r) ? RS_E_HIP : RS_OK;
}
