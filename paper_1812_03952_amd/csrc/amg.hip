// amg.hip -- aggregation AMG for the pressure stage of CPR, set up and
// applied on the device.
//
// The paper solves the pressure sub-problem with one AMG V-cycle using the
// defaults of Fig. fig-ds-amg-par (strength 0.5, max row sum 0.9, one cycle,
// two relaxation sweeps per level visit).  This library keeps those
// parameters and replaces classical coarsening by aggregation, which maps to
// fine-grained parallel work:
//   strength   j strongly influences i if -a_ij >= theta * max_{k!=i}(-a_ik);
//              a row with |sum_j a_ij| > max_row_sum*|a_ii| has none;
//              symmetrised (an edge if either direction is strong).
//   roots      distance-2 maximal independent set with fixed priorities
//              (fmix32 of the index, index in the low word).  Rounds: every
//              undecided vertex that holds the largest priority among the
//              undecided vertices within two strength edges, with no root
//              that close, becomes a root; vertices with a root within two
//              edges drop out.  With fixed priorities this selects exactly
//              the set of the sequential greedy visit in priority order
//              (Blelloch, Fineman & Shun, SPAA 2012), so the result does not
//              depend on scheduling.
//   aggregates roots take their strength neighbours; the rest join the
//              neighbouring first-pass aggregate with the largest |a_ij|,
//              ties to the lowest id; vertices with no strength edge stay
//              unaggregated.
//   Galerkin   A_c = P^T A P for piecewise-constant P, one thread per coarse
//              row, summing members in increasing fine index and each
//              member's row in column order.  Only additions are involved, so
//              coarse matrices are bitwise reproducible.
//   cycle      l1-Jacobi (d_i = sgn(a_ii) sum_j |a_ij|), one sweep before and
//              one after the coarse correction; dense FP64 inverse at the
//              coarsest level.  On the coarser levels the pre-smoothed
//              iterate b/d is not stored (the residual and the post-smoother
//              recompute it); on the fine level, which keeps the 7-point
//              pattern and is stored by stencil slot, it is formed once.
#include "rs_internal.h"
#include <algorithm>
#include <type_traits>
#include <math.h>
#include <mutex>

namespace {

enum : uint8_t { ST_UND = 0, ST_ROOT = 1, ST_OUT = 2, ST_ISO = 3 };

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
__device__ __forceinline__ uint64_t prio(int i, int level) {
  uint32_t h = fmix32((uint32_t)i + 0x9e3779b9u * (uint32_t)(level + 1));
  return ((uint64_t)h << 32) | (uint32_t)i;
}

// ---- scan ------------------------------------------------------------------
__global__ void k_scan_block(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                             int32_t *__restrict__ bsum, int64_t n) {
  __shared__ int32_t s[256];
  int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  int32_t v[4], tsum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) { v[k] = (base + k < n) ? in[base + k] : 0; tsum += v[k]; }
  s[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t ex = s[threadIdx.x] - tsum;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = s[255];
}

__global__ void k_scan_add(int32_t *__restrict__ out, const int32_t *__restrict__ boff, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] += boff[t / 1024];
}

// out = exclusive scan of in (n entries); in may equal out.  The sum goes to
// *total (host: the stream is synchronised) and/or *dtotal (device, stream
// ordered); either may be null.
rs_status scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *total, hipStream_t s,
                   int32_t *dtotal) {
  int64_t nb = (n + 1023) / 1024;
  if (nb < 1) nb = 1;
  dbuf bs, bo;
  RS_TRY(bs.alloc(sizeof(int32_t) * nb));
  k_scan_block<<<(unsigned)nb, 256, 0, s>>>(in, out, bs.as<int32_t>(), n);
  RS_HIP(hipGetLastError());
  if (nb == 1) {
    if (dtotal) RS_HIP(hipMemcpyAsync(dtotal, bs.p, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (total) {
      int32_t t = 0;
      RS_TRY(rs_wait_read(&t, bs.p, sizeof(int32_t), s));
      *total = t;
    }
    return RS_OK;
  }
  RS_TRY(bo.alloc(sizeof(int32_t) * nb));
  RS_TRY(scan_i32(bs.as<int32_t>(), bo.as<int32_t>(), nb, total, s, dtotal));
  k_scan_add<<<rs_grid(n), RS_BLOCK, 0, s>>>(out, bo.as<int32_t>(), n);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

// ---- setup kernels -----------------------------------------------------------
// Fine-level CSR values from the pressure entries by stencil slot: one thread
// per row writes its entries in column (= slot) order.  The pattern is the
// validated 7-point one, so the slots inside the grid are exactly the row.
__global__ __launch_bounds__(256) void k_csr_from7(int nx, int ny, int nz, const int32_t *__restrict__ rp,
                                                   const double *__restrict__ ap7, double *__restrict__ a) {
  const int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
  const bool in[7] = {k > 0, j > 0, i > 0, true, i < nx - 1, j < ny - 1, k < nz - 1};
  int64_t p = rp[c];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl)
    if (in[sl]) a[p++] = ap7[sl * n + c];
}

__global__ void k_strength_dir(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const double *__restrict__ a, double theta, double mrs,
                               uint8_t *__restrict__ dir) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p0 = rp[i], p1 = rp[i + 1];
  double aii = 0.0, nm = 0.0, s = 0.0;
  for (int p = p0; p < p1; ++p) {
    double v = a[p];
    s = s + v;
    if (ci[p] == i) aii = v;
    else if (-v > nm) nm = -v;
  }
  bool weak = fabs(s) > mrs * fabs(aii) || !(nm > 0.0);
  double thr = theta * nm;
  for (int p = p0; p < p1; ++p) dir[p] = (!weak && ci[p] != i && -a[p] >= thr) ? 1 : 0;
}

__device__ __forceinline__ int find_col(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                        int row, int col) {
  int lo = rp[row], hi = rp[row + 1] - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int v = ci[mid];
    if (v == col) return mid;
    if (v < col) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

__global__ void k_strength_sym(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const uint8_t *__restrict__ dir, uint8_t *__restrict__ strong,
                               uint8_t *__restrict__ state) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int deg = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    int j = ci[p];
    uint8_t v = 0;
    if (j != i) {
      int q = find_col(rp, ci, j, i);
      v = dir[p] | (q >= 0 ? dir[q] : (uint8_t)0);
    }
    strong[p] = v;
    deg += v;
  }
  state[i] = deg ? ST_UND : ST_ISO;
}

// A fine-level cell's in-grid flags and neighbours by slot.  The kernels on
// it load every slot's operand unconditionally (from the cell itself where
// the slot is off-grid or masked out) and select afterwards: a load under a
// branch is waited for before the next one issues, while unconditional
// loads are all in flight at once.
struct cell7 {
  int64_t c;
  bool in[7];
  int64_t nb[7];
};
__device__ __forceinline__ cell7 cell7_of(int64_t c, int nx, int ny, int nz) {
  const int64_t nxy = (int64_t)nx * ny;
  const uint32_t cu = (uint32_t)c, t = cu / (uint32_t)nx;   // grids hold fewer than 2^31 cells
  const int i = (int)(cu - t * (uint32_t)nx), j = (int)(t % (uint32_t)ny), k = (int)(t / (uint32_t)ny);
  cell7 e;
  e.c = c;
  e.in[0] = k > 0; e.in[1] = j > 0; e.in[2] = i > 0; e.in[3] = true;
  e.in[4] = i < nx - 1; e.in[5] = j < ny - 1; e.in[6] = k < nz - 1;
  e.nb[0] = c - nxy; e.nb[1] = c - nx; e.nb[2] = c - 1; e.nb[3] = c;
  e.nb[4] = c + 1; e.nb[5] = c + nx; e.nb[6] = c + nxy;
  return e;
}

constexpr int MIS_BATCH = 4;   // MIS rounds per host read

__device__ __forceinline__ uint64_t keyof(uint8_t st, int v, int level) {
  return st == ST_ROOT ? ~0ull : (st == ST_UND ? prio(v, level) : 0ull);
}

// Rounds run in batches without a host read in between; a round whose
// predecessor left no vertex undecided (*prev == 0) has nothing to change
// and returns at once.  prev == nullptr: the predecessor is known to have
// left some.
// und0 (first round of a batch only): the batch's flags, zeroed here
__global__ void k_mis_m1(int n, int level, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const uint8_t *__restrict__ strong, const uint8_t *__restrict__ state,
                         uint64_t *__restrict__ m1, const int *__restrict__ prev, int *__restrict__ und0) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (und0 && u < MIS_BATCH) und0[u] = 0;
  if (u >= n || (prev && *prev == 0)) return;
  const uint8_t su = state[u];
  uint64_t m = keyof(su, u, level);
  bool und = su == ST_UND;
  for (int p = rp[u]; p < rp[u + 1]; ++p)
    if (strong[p]) {
      int w = ci[p];
      const uint8_t sw = state[w];
      uint64_t k = keyof(sw, w, level);
      m = k > m ? k : m;
      und = und || sw == ST_UND;
    }
  if (und) m1[u] = m;                            // as in k_mis7_m1
}

// the distance-2 maximum of an undecided vertex (the largest m1 over its
// closed strong neighbourhood) and its decision; m1 is not written in this
// pass, so the decisions of one round all see the same m1
__global__ void k_mis_m2d(int n, int level, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const uint8_t *__restrict__ strong, const uint64_t *__restrict__ m1,
                          uint8_t *__restrict__ state, int *__restrict__ undecided, const int *__restrict__ prev) {
  if (prev && *prev == 0) return;             // *undecided stays 0
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  int left = 0;
  uint8_t st = ST_ISO;
  if (v < n) st = state[v];
  if (st == ST_UND) {
    uint64_t m = m1[v];
    for (int p = rp[v]; p < rp[v + 1]; ++p)
      if (strong[p]) {
        uint64_t k = m1[ci[p]];
        m = k > m ? k : m;
      }
    if (m == ~0ull) state[v] = ST_OUT;
    else if (m == prio(v, level)) state[v] = ST_ROOT;
    else left = 1;
  }
  // one plain store per block that still has undecided vertices
  if (__syncthreads_or(left) && threadIdx.x == 0) *undecided = 1;
}

// (also zeroes the word *zero1: the aggregation's error flag)
__global__ void k_root_flag(int n, const uint8_t *__restrict__ state, int32_t *__restrict__ f,
                            int *__restrict__ zero1) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) *zero1 = 0;
  if (v < n) f[v] = state[v] == ST_ROOT ? 1 : 0;
}

// (also zeroes z[0 .. nz): the coarse level's per-row counters, nz <= n)
__global__ void k_agg1(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const uint8_t *__restrict__ strong, const uint8_t *__restrict__ state,
                       const int32_t *__restrict__ id, int32_t *__restrict__ agg1, int32_t *__restrict__ z, int nz) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nz) z[v] = 0;
  if (v >= n) return;
  int g = -1;
  uint8_t st = state[v];
  if (st == ST_ROOT) g = id[v];
  else if (st != ST_ISO)
    for (int p = rp[v]; p < rp[v + 1]; ++p)
      if (strong[p] && state[ci[p]] == ST_ROOT) { g = id[ci[p]]; break; }
  agg1[v] = g;
}

__global__ void k_agg2(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const uint8_t *__restrict__ strong, const double *__restrict__ a,
                       const uint8_t *__restrict__ state, const int32_t *__restrict__ agg1,
                       int32_t *__restrict__ agg, int *__restrict__ bad) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int g = agg1[v];
  if (g < 0 && state[v] != ST_ISO) {
    double bw = -1.0;
    for (int p = rp[v]; p < rp[v + 1]; ++p) {
      if (!strong[p]) continue;
      int ag = agg1[ci[p]];
      if (ag < 0) continue;
      double w = fabs(a[p]);
      if (w > bw || (w == bw && ag < g)) { bw = w; g = ag; }
    }
    if (g < 0) atomicOr(bad, 1);     // cannot happen for a maximal distance-2 set
  }
  agg[v] = g;
}

// (also zeroes z[0 .. nz), the fill counters of k_fill_members, nz <= n)
__global__ void k_count_members(int n, const int32_t *__restrict__ agg, int32_t *__restrict__ cnt,
                                int32_t *__restrict__ z, int nz) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nz) z[v] = 0;
  if (v < n && agg[v] >= 0) atomicAdd(&cnt[agg[v]], 1);
}

__global__ void k_fill_members(int n, const int32_t *__restrict__ agg, const int32_t *__restrict__ mptr,
                               int32_t *__restrict__ fill, int32_t *__restrict__ mem) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && agg[v] >= 0) {
    int g = agg[v];
    int k = atomicAdd(&fill[g], 1);
    mem[mptr[g] + k] = v;
  }
}

// atomics fill each member list in arbitrary order: sort it (lists are short)
__global__ void k_sort_members(int nc, const int32_t *__restrict__ mptr, int32_t *__restrict__ mem) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int b = mptr[I], e = mptr[I + 1];
  for (int x = b + 1; x < e; ++x) {
    int v = mem[x], y = x - 1;
    while (y >= b && mem[y] > v) { mem[y + 1] = mem[y]; --y; }
    mem[y + 1] = v;
  }
}

__global__ void k_cand(int nc, const int32_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                       const int32_t *__restrict__ rp, int32_t *__restrict__ cand) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int s = 0;
  for (int x = mptr[I]; x < mptr[I + 1]; ++x) s += rp[mem[x] + 1] - rp[mem[x]];
  cand[I] = s;
}

// Coarse row I: accumulate members' rows into a first-seen list, then sort
// the list by column (insertion sort on the short list).  The list lives in
// LDS (one column per thread: entry s of thread t at [s][t]) while it holds
// at most GAL_CAP distinct coarse columns; a row that needs more starts
// again with the list in the global scratch (sized by the candidate count).
// The additions happen in the same order either way.
constexpr int GAL_BLOCK = 128;
// LDS list length per row source: piecewise-constant aggregation of a
// 7-point (and the next coarser) pattern gives short coarse rows (at most 15
// entries on the grids measured), and a shorter list leaves room for more
// workgroups per CU; the smoothed product's rows are longer
template <class R> struct gal_cap { static constexpr int CAP = 16; };

// Row sources: each(i, agg, f) calls f(agg[col], a) for the entries of
// fine row i in column order and stops when f returns false.
struct rows_csr {
  const int32_t *rp, *ci;
  const double *a;
  template <class F> __device__ __forceinline__ bool each(int i, const int32_t *__restrict__ agg, F &&f) const {
    for (int p = rp[i]; p < rp[i + 1]; ++p)
      if (!f(agg[ci[p]], a[p])) return false;
    return true;
  }
};
struct rows_7 {
  int nx, ny, nz;
  const double *ap7;
  // a row's entries and their columns' aggregates, all 14 loads issued at once
  struct row { double a[7]; int32_t J[7]; unsigned in; };
  __device__ __forceinline__ void fetch(int i, const int32_t *__restrict__ agg, row &w) const {
    const int64_t n = (int64_t)nx * ny * nz;
    const cell7 e = cell7_of(i, nx, ny, nz);
    w.in = 0;
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) {
      int64_t q = e.in[sl] ? e.nb[sl] : (int64_t)i;
      asm volatile("" : "+v"(q));
      w.a[sl] = ap7[sl * n + i];
      w.J[sl] = agg[q];
      w.in |= e.in[sl] ? (1u << sl) : 0u;
    }
  }
  template <class F> __device__ __forceinline__ bool apply(const row &w, F &&f) const {
#pragma unroll
    for (int sl = 0; sl < 7; ++sl)
      if (((w.in >> sl) & 1u) && !f(w.J[sl], w.a[sl])) return false;
    return true;
  }
  template <class F> __device__ __forceinline__ bool each(int i, const int32_t *__restrict__ agg, F &&f) const {
    row w;
    fetch(i, agg, w);
    return apply(w, f);
  }
};

// false when the list would exceed cap entries
template <class R, class K, class V>
__device__ __forceinline__ bool gal_row(int I, const int32_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                                        const R &rows, const int32_t *__restrict__ agg, K key, V val, int cap,
                                        int &m) {
  m = 0;
  int sI = -1;                                   // slot of column I (most entries), once seen
  const int x0 = mptr[I], x1 = mptr[I + 1];
  auto add = [&](int J, double a) -> bool {
      if (J < 0) return true;
      int s;
      if (J == I && sI >= 0) {
        s = sI;
      } else {
        s = 0;
        while (s < m && key(s) != J) ++s;
        if (s == m) {
          if (m == cap) return false;
          key(m) = J;
          val(m) = 0.0;
          ++m;
        }
        if (J == I) sI = s;
      }
      val(s) = val(s) + a;
      return true;
  };
  if constexpr (std::is_same<R, rows_7>::value) {
    // the next member's entries are in flight while a member's are added
    // (member indices two ahead; clamped, so that every fetch is issued
    // unconditionally)
    if (x0 < x1) {
      typename R::row cur, nxt;
      int inx = mem[x0 + 1 < x1 ? x0 + 1 : x0];
      rows.fetch(mem[x0], agg, cur);
      for (int x = x0; x < x1; ++x) {
        const int in2 = mem[x + 2 < x1 ? x + 2 : x1 - 1];
        rows.fetch(inx, agg, nxt);
        if (!rows.apply(cur, add)) return false;
        cur = nxt;
        inx = in2;
      }
    }
  } else {
    for (int x = x0; x < x1; ++x)
      if (!rows.each(mem[x], agg, add)) return false;
  }
  for (int x = 1; x < m; ++x) {
    int k = key(x);
    double v = val(x);
    int y = x - 1;
    while (y >= 0 && key(y) > k) { key(y + 1) = key(y); val(y + 1) = val(y); --y; }
    key(y + 1) = k;
    val(y + 1) = v;
  }
  return true;
}

template <class R, int GAL_CAP = gal_cap<R>::CAP>
__global__ __launch_bounds__(GAL_BLOCK) void k_galerkin(int nc, const int32_t *__restrict__ mptr,
                                                        const int32_t *__restrict__ mem, R rows,
                                                        const int32_t *__restrict__ agg,
                                                        const int32_t *__restrict__ off, int32_t *__restrict__ skey,
                                                        double *__restrict__ sval, int32_t *__restrict__ cnt) {
  __shared__ int32_t lk[GAL_CAP][GAL_BLOCK];
  __shared__ double lv[GAL_CAP][GAL_BLOCK];
  const int t = threadIdx.x;
  const int I = blockIdx.x * blockDim.x + t;
  if (I >= nc) return;
  const int base = off[I], ncand = cnt[I];       // candidate count from k_cand
  int m = 0;
  if (gal_row(I, mptr, mem, rows, agg, [&](int s) -> int32_t & { return lk[s][t]; },
              [&](int s) -> double & { return lv[s][t]; }, GAL_CAP, m)) {
    for (int s = 0; s < m; ++s) { skey[base + s] = lk[s][t]; sval[base + s] = lv[s][t]; }
  } else {
    gal_row(I, mptr, mem, rows, agg, [&](int s) -> int32_t & { return skey[base + s]; },
            [&](int s) -> double & { return sval[base + s]; }, ncand, m);
  }
  cnt[I] = m;
}

// Also the coarse level's l1 diagonal (as k_l1diag, the same additions in
// the same order) and, when cap is given, its FP32 values (as k_cast_f32),
// so the coarse level needs no pass of its own for them.
template <class T>
__global__ void k_galerkin_copy(int nc, const int32_t *__restrict__ off, const int32_t *__restrict__ skey,
                                const double *__restrict__ sval, const int32_t *__restrict__ crp,
                                int32_t *__restrict__ cci, double *__restrict__ ca, float *__restrict__ cap,
                                T *__restrict__ dl1) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int b = off[I], o = crp[I], m = crp[I + 1] - crp[I];
  double sum = 0.0, aii = 0.0;
  for (int sb = 0; sb < m; sb += 8) {            // eight entries' loads in flight at once
    int32_t kv[8];
    double vv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int e = sb + k < m ? sb + k : 0;
      asm volatile("" : "+v"(e));
      kv[k] = skey[b + e];
      vv[k] = sval[b + e];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (sb + k < m) {
        cci[o + sb + k] = kv[k];
        ca[o + sb + k] = vv[k];
        if (cap) cap[o + sb + k] = (float)vv[k];
        sum = sum + fabs(vv[k]);
        if (kv[k] == I) aii = vv[k];
      }
  }
  if (sum == 0.0) sum = 1.0;
  dl1[I] = (T)(aii < 0.0 ? -sum : sum);
}

__global__ void k_set_last(int32_t *__restrict__ p, int64_t idx, const int32_t *__restrict__ v) { p[idx] = *v; }

template <class T>
__global__ void k_l1diag(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ a, T *__restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, aii = 0.0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    s = s + fabs(a[p]);
    if (ci[p] == i) aii = a[p];
  }
  if (s == 0.0) s = 1.0;
  d[i] = (T)(aii < 0.0 ? -s : s);
}

__global__ void k_cast_f32(int64_t m, const double *__restrict__ a, float *__restrict__ b) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) b[t] = (float)a[t];
}

__global__ void k_densify(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const double *__restrict__ a, double *__restrict__ G) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double *row = G + (int64_t)i * 2 * n;
  for (int c = 0; c < 2 * n; ++c) row[c] = (c == n + i) ? 1.0 : 0.0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) row[ci[p]] = a[p];
}

__global__ void k_augment(int n, const double *__restrict__ a, double *__restrict__ G) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * (int64_t)n * n) return;
  const int64_t r = t / (2 * n), c = t - r * 2 * n;
  G[t] = c < n ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
}

// Gauss-Jordan with partial pivoting on [A | I] (n x 2n, row-major), one
// pivot column per pair of launches.
__global__ void k_gj_pivot(int n, int k, double *__restrict__ G, int *__restrict__ bad) {
  __shared__ double sv[256];
  __shared__ int si[256];
  int tid = threadIdx.x;
  double best = -1.0;
  int bi = k;
  for (int r = k + tid; r < n; r += blockDim.x) {
    double v = fabs(G[(int64_t)r * 2 * n + k]);
    if (v > best) { best = v; bi = r; }
  }
  sv[tid] = best; si[tid] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) {
      if (sv[tid + s] > sv[tid] || (sv[tid + s] == sv[tid] && si[tid + s] < si[tid])) {
        sv[tid] = sv[tid + s]; si[tid] = si[tid + s];
      }
    }
    __syncthreads();
  }
  int piv = si[0];
  double *rk = G + (int64_t)k * 2 * n, *rpv = G + (int64_t)piv * 2 * n;
  if (piv != k)
    for (int c = tid; c < 2 * n; c += blockDim.x) { double t = rk[c]; rk[c] = rpv[c]; rpv[c] = t; }
  __syncthreads();
  double pv = rk[k];
  if (tid == 0 && !(fabs(pv) > 0.0)) atomicOr(bad, 1);
  double inv = 1.0 / pv;
  __syncthreads();
  for (int c = tid; c < 2 * n; c += blockDim.x)
    if (c != k) rk[c] = rk[c] * inv;
  __syncthreads();
  if (tid == 0) rk[k] = 1.0;
}

__global__ void k_gj_elim(int n, int k, double *__restrict__ G) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t w = 2 * (int64_t)n - (k + 1);
  if (t >= (int64_t)n * w) return;
  int r = (int)(t / w);
  int c = (int)(t - (int64_t)r * w) + k + 1;
  if (r == k) return;
  double f = G[(int64_t)r * 2 * n + k];
  G[(int64_t)r * 2 * n + c] -= f * G[(int64_t)k * 2 * n + c];
}

// The same elimination for small n in one workgroup, three barriers per
// column: the pivot (largest |value|, lowest row on ties) is reduced per wave
// with shuffles and then across the waves from LDS; the row swap and the
// scaling of the pivot row are one pass (each thread owns whole columns);
// then the elimination.  Every entry gets the same operations as in the
// two-launch form.
constexpr int GJ_FUSED_MAX = 256;
__global__ __launch_bounds__(1024) void k_gj_fused(int n, double *__restrict__ G, int *__restrict__ bad) {
  __shared__ double sv[16], sp[16];
  __shared__ int si[16];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
  const int64_t ld = 2 * (int64_t)n;
  const int tpr = max(1, nt / n);             // threads per row in the elimination
  const int rstep = nt / tpr, r0 = tid / tpr, c0 = tid - r0 * tpr;
  for (int k = 0; k < n; ++k) {
    // pivot: |value| compared, the signed value carried along
    double best = -1.0, bval = 0.0;
    int bi = k;
    for (int r = k + tid; r < n; r += nt) {
      double x = G[(int64_t)r * ld + k], v = fabs(x);
      if (v > best) { best = v; bval = x; bi = r; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_down(best, off, 64), ox = __shfl_down(bval, off, 64);
      int oi = __shfl_down(bi, off, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bval = ox; bi = oi; }
    }
    if (lane == 0) { sv[wv] = best; sp[wv] = bval; si[wv] = bi; }
    __syncthreads();
    best = sv[0]; bval = sp[0]; bi = si[0];
    for (int w = 1; w < nwv; ++w)
      if (sv[w] > best || (sv[w] == best && si[w] < bi)) { best = sv[w]; bval = sp[w]; bi = si[w]; }
    const int piv = bi;
    double *rk = G + (int64_t)k * ld, *rpv = G + (int64_t)piv * ld;
    const double pv = bval;
    if (tid == 0 && !(fabs(pv) > 0.0)) atomicOr(bad, 1);
    const double inv = 1.0 / pv;
    for (int c = tid; c < ld; c += nt) {
      const double vk = rk[c], vp = rpv[c];
      if (piv != k) rpv[c] = vk;
      rk[c] = (c == k) ? 1.0 : vp * inv;
    }
    __syncthreads();
    // thread -> (rows r0 + rstep*m, columns c0 + tpr*q): no divisions per entry
    for (int r = r0; r < n && tid < rstep * tpr; r += rstep) {
      if (r == k) continue;
      const double f = G[(int64_t)r * ld + k];
      double *gr = G + (int64_t)r * ld;
      for (int c = k + 1 + c0; c < ld; c += tpr) gr[c] -= f * rk[c];
    }
    __syncthreads();
  }
}

// Coarsest levels up to GJ_BLK_MAX rows are inverted in one workgroup with
// the n x n matrix in registers, by in-place Gauss-Jordan with implicit
// partial pivoting: rows never move; at step k the pivot is the largest
// |value| of column k among the rows not yet used as pivots (lowest row on
// ties), and column k is then reused to hold the column of the inverse that
// this step creates.  Thread (rg, cg) owns rows rg + nrg*i and columns
// cg + ncg*j of an R x Q tile, so column k = kc + ncg*j0 always sits in
// register slot j0, a compile-time index once the loop over j0 is unrolled.
// Per step:
//   - the owners of column k publish it to LDS (value, and |value| or -1
//     for used rows);
//   - every wave reduces max |value| with DPP and takes the lowest row
//     holding it from a ballot, and its signed value with a readlane;
//   - the owners set column k to e_p (the identity column of pivot row p);
//   - the pivot row's threads publish that row times 1/pivot and zero it;
//   - every row applies g -= f * prow, with f = -1 on the pivot row.
// Each entry gets the operations of Gauss-Jordan on [A | I] with row swaps:
// the same products and fused multiply-adds, in the same order.
// With p_k the pivot row of step k, the final tile X gives
// inverse[k][p_k'] = X[p_k][k'], which the last pass scatters.
constexpr int GJ_BLK_MAX = 156;
template <int CTRL, int RM>
__device__ __forceinline__ double gj_dpp_max(double x) {
  const int a0 = __double2loint(x), a1 = __double2hiint(x);
  const double o = __hiloint2double(__builtin_amdgcn_update_dpp(a1, a1, CTRL, RM, 0xf, false),
                                    __builtin_amdgcn_update_dpp(a0, a0, CTRL, RM, 0xf, false));
  return fmax(x, o);
}
template <int NT, int R, int Q>
__global__ __launch_bounds__(NT) void k_gj_blk(int n, int ld, const double *__restrict__ G0, double *__restrict__ cinv,
                                               int *__restrict__ bad) {
  __shared__ double colk[2][GJ_BLK_MAX + 8], cabs[2][GJ_BLK_MAX + 8], prow[GJ_BLK_MAX + 8];
  __shared__ int pivrow[GJ_BLK_MAX];
  const int tid = threadIdx.x, lane = tid & 63;
  const int nrg = (n + R - 1) / R, ncg = (n + Q - 1) / Q;
  const int rg = tid / ncg, cg = tid - rg * ncg;
  const bool act = rg < nrg;
  double g[R][Q];
  bool used[R];
  int pos[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    used[i] = false;
    pos[i] = 0;
    const int row = rg + nrg * i;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int col = cg + ncg * j;
      g[i][j] = (act && row < n && col < n) ? G0[(int64_t)row * ld + col] : 0.0;
    }
  }
  int b = 0;  // colk / cabs double buffer: step k+1 publishes while step k's f reads finish
#pragma unroll
  for (int j0 = 0; j0 < Q; ++j0) {
    for (int kc = 0; kc < ncg; ++kc) {
      const int k = kc + ncg * j0;
      if (k >= n) break;
      if (act && cg == kc) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = rg + nrg * i;
          colk[b][row] = g[i][j0];
          cabs[b][row] = (used[i] || row >= n) ? -1.0 : fabs(g[i][j0]);
        }
      }
      __syncthreads();
      // pivot: rows lane, lane+64, lane+128
      double a[3], v[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int rr = lane + 64 * m;
        a[m] = -1.0;
        v[m] = 0.0;
        if (rr < n) { a[m] = cabs[b][rr]; v[m] = colk[b][rr]; }
      }
      double mx = fmax(a[0], fmax(a[1], a[2]));
      mx = gj_dpp_max<0xB1, 0xf>(mx);   // quad_perm [1,0,3,2]
      mx = gj_dpp_max<0x4E, 0xf>(mx);   // quad_perm [2,3,0,1]
      mx = gj_dpp_max<0x141, 0xf>(mx);  // row_half_mirror
      mx = gj_dpp_max<0x140, 0xf>(mx);  // row_mirror
      mx = gj_dpp_max<0x142, 0xa>(mx);  // row_bcast:15 into rows 1, 3
      mx = gj_dpp_max<0x143, 0xc>(mx);  // row_bcast:31 into rows 2, 3
      const double gm = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(mx), 63),
                                         __builtin_amdgcn_readlane(__double2loint(mx), 63));
      int p = n - 1;
      double pv = 0.0;
#pragma unroll
      for (int m = 2; m >= 0; --m) {
        const unsigned long long bm = __ballot(a[m] == gm);
        if (bm) {
          const int l = __ffsll(bm) - 1;
          p = 64 * m + l;
          pv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[m]), l),
                                __builtin_amdgcn_readlane(__double2loint(v[m]), l));
        }
      }
      if (tid == 0 && !(fabs(pv) > 0.0)) atomicOr(bad, 1);
      const double inv = 1.0 / pv;
      if (act && cg == kc) {
#pragma unroll
        for (int i = 0; i < R; ++i) g[i][j0] = (rg + nrg * i == p) ? 1.0 : 0.0;
      }
      const int rgp = p % nrg, ip = p / nrg;
      if (act && rg == rgp) {
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (i == ip) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
              prow[cg + ncg * j] = g[i][j] * inv;
              g[i][j] = 0.0;
            }
          }
      }
      if (tid == 0) pivrow[k] = p;
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (rg + nrg * i == p) {
          used[i] = true;
          pos[i] = k;
        }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int row = rg + nrg * i;
          const double f = (row == p) ? -1.0 : colk[b][row];
#pragma unroll
          for (int j = 0; j < Q; ++j) g[i][j] = fma(-f, prow[cg + ncg * j], g[i][j]);
        }
      }
      b ^= 1;
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int row = rg + nrg * i;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const int col = cg + ncg * j;
        if (row < n && col < n) cinv[(int64_t)pos[i] * n + pivrow[col]] = g[i][j];
      }
    }
  }
}

// Tiles of k_gj_blk: R x Q per thread with 1024 threads (2 x 6 up to n = 108,
// 4 x 6 up to 156).
static bool gj_blk_fits(int n, int R, int Q) {
  return n <= GJ_BLK_MAX && (int64_t)((n + R - 1) / R) * ((n + Q - 1) / Q) <= 1024;
}

__global__ void k_extract_inv(int n, const double *__restrict__ G, double *__restrict__ inv) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  int r = (int)(t / n), c = (int)(t % n);
  inv[t] = G[(int64_t)r * 2 * n + n + c];
}

// Inverse of the n x n matrix held in the left half of G (n x 2n, row-major,
// right half the identity; G is overwritten) into cinv (n x n), by the path
// that fits n.  A zero pivot sets *flag.
static rs_status dense_inverse_run(int n, double *G, double *cinv, int *flag, hipStream_t s) {
  if (gj_blk_fits(n, 2, 6)) {
    k_gj_blk<1024, 2, 6><<<1, 1024, 0, s>>>(n, 2 * n, G, cinv, flag);
  } else if (gj_blk_fits(n, 4, 6)) {
    k_gj_blk<1024, 4, 6><<<1, 1024, 0, s>>>(n, 2 * n, G, cinv, flag);
  } else {
    if (n <= GJ_FUSED_MAX) {
      k_gj_fused<<<1, 1024, 0, s>>>(n, G, flag);
    } else {
      for (int k = 0; k < n; ++k) {
        k_gj_pivot<<<1, 256, 0, s>>>(n, k, G, flag);
        int64_t work = (int64_t)n * (2 * (int64_t)n - (k + 1));
        if (work > 0) k_gj_elim<<<rs_grid(work), RS_BLOCK, 0, s>>>(n, k, G);
      }
    }
    k_extract_inv<<<rs_grid((int64_t)n * n), RS_BLOCK, 0, s>>>(n, G, cinv);
  }
  RS_HIP(hipGetLastError());
  return RS_OK;
}

// ---- cycle kernels -----------------------------------------------------------
// r = b - A (b ./ d): residual after one l1-Jacobi sweep from zero.
template <class T>
__global__ __launch_bounds__(256) void k_vc_pre(int n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const T *__restrict__ a,
                                                 const T *__restrict__ d, const T *__restrict__ b,
                                                 T *__restrict__ r) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = rp[i], p1 = rp[i + 1];
  T s = 0;
  // eight entries at a time: their columns, then the gathers, all issued at
  // once (positions past the row read its first entry and are not added)
  for (int pb = p0; pb < p1; pb += 8) {
    int j[8];
    T av[8], bj[8], dj[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int p = pb + k < p1 ? pb + k : p0;
      asm volatile("" : "+v"(p));
      j[k] = ci[p];
      av[k] = a[p];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) { bj[k] = b[j[k]]; dj[k] = d[j[k]]; }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (pb + k < p1) s = fma(av[k], bj[k] / dj[k], s);
  }
  r[i] = b[i] - s;
}

template <class T>
__global__ void k_vc_restrict(int nc, const int32_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                              const T *__restrict__ r, T *__restrict__ bc) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int x0 = mptr[I], x1 = mptr[I + 1];
  T s = 0;
  for (int xb = x0; xb < x1; xb += 8) {          // eight members at a time, as in k_vc_pre
    int m[8];
    T rv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int x = xb + k < x1 ? xb + k : x0;
      asm volatile("" : "+v"(x));
      m[k] = mem[x];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) rv[k] = r[m[k]];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (xb + k < x1) s = s + rv[k];
  }
  bc[I] = s;
}

// x = y + (b - A y) ./ d  with  y = b ./ d + P xc  (prolongation then one
// l1-Jacobi post-sweep).
template <class T>
__global__ __launch_bounds__(256) void k_vc_post(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const T *__restrict__ a,
                                                  const T *__restrict__ d, const int32_t *__restrict__ agg,
                                                  const T *__restrict__ b, const T *__restrict__ xc,
                                                  T *__restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = rp[i], p1 = rp[i + 1];
  const T bi = b[i], di = d[i];
  const int gi = agg[i];
  T s = 0;
  for (int pb = p0; pb < p1; pb += 8) {          // eight entries at a time, as in k_vc_pre
    int j[8], g[8];
    T av[8], bj[8], dj[8], xq[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int p = pb + k < p1 ? pb + k : p0;
      asm volatile("" : "+v"(p));
      j[k] = ci[p];
      av[k] = a[p];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) { bj[k] = b[j[k]]; dj[k] = d[j[k]]; g[k] = agg[j[k]]; }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int gc = g[k] >= 0 ? g[k] : 0;
      asm volatile("" : "+v"(gc));
      xq[k] = xc[gc];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (pb + k >= p1) continue;
      T yj = bj[k] / dj[k];
      if (g[k] >= 0) yj = yj + xq[k];
      s = fma(av[k], yj, s);
    }
  }
  T yi = bi / di;
  if (gi >= 0) yi = yi + xc[gi];
  x[i] = yi + (bi - s) / di;
}


// ---- level 0 on the grid: the pressure matrix keeps the 7-point pattern, so
// its values are stored by stencil slot and the neighbours follow from the
// cell index (no column indices).  Slots run in column order and off-grid
// slots hold zeros, so each sum is the same sequence of operations as the
// row of the CSR form.
template <class T>
__global__ __launch_bounds__(256) void k_cast7(int64_t m, const double *__restrict__ a, T *__restrict__ o) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) o[t] = (T)a[t];
}

__device__ __forceinline__ int nbr7(int i, int s, int n, int nx, int nxy) {
  const int off[7] = {-nxy, -nx, -1, 0, 1, nx, nxy};
  int q = i + off[s];
  return (q < 0 || q >= n) ? i : q;             // off-grid slots hold zero values
}

// Fine-level V-cycle kernels hand out their cells in row bands, one per XCD
// (as the SpMV): workgroup i runs on XCD i % 8 and takes the (i / 8)-th run of
// blockDim.x cells of band i % 8, the rows [b ny / 8, (b + 1) ny / 8) of every
// plane, so a cell's neighbours are mostly read through the same L2.  False
// past the band's end.  Grid: band_grid.
__device__ __forceinline__ bool band_cell(int n, int nx, int nxy, int &c) {
  const int ny = nxy / nx, nz = n / nxy;
  const int xb = (int)(blockIdx.x & 7u);
  const uint32_t m = (blockIdx.x >> 3) * blockDim.x + threadIdx.x;
  const uint32_t j0 = (uint32_t)((int64_t)xb * ny / 8), j1 = (uint32_t)((int64_t)(xb + 1) * ny / 8);
  const uint32_t band = (j1 - j0) * (uint32_t)nx;
  if (band == 0 || m >= band * (uint32_t)nz) return false;
  const uint32_t k = m / band;
  c = (int)(k * (uint32_t)nxy + j0 * (uint32_t)nx + (m - k * band));
  return true;
}
static unsigned band_grid(int nx, int ny, int nz) {
  int64_t most = 0;
  for (int b = 0; b < 8; ++b) most = std::max(most, ((int64_t)(b + 1) * ny / 8 - (int64_t)b * ny / 8) * nx * nz);
  return (unsigned)(8 * ((most + RS_BLOCK - 1) / RS_BLOCK));
}

// pre-smoothing from x = 0 and the residual: y = b ./ d (kept for the
// post-smoothing), r = b - A y with each neighbour's y_q = b_q / d_q formed
// where it is used (the same division, so the same value as a stored y)
template <class T>
__global__ __launch_bounds__(256) void k_vc_pre7(int n, int nx, int nxy, const T *__restrict__ s7,
                                                  const T *__restrict__ d, const T *__restrict__ b,
                                                  T *__restrict__ y, T *__restrict__ r) {
  int i;
  if (!band_cell(n, nx, nxy, i)) return;
  T s = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int q = nbr7(i, k, n, nx, nxy);
    s = fma(s7[(int64_t)k * n + i], b[q] / d[q], s);
  }
  r[i] = b[i] - s;
  y[i] = b[i] / d[i];
}

template <class T>
__global__ __launch_bounds__(256) void k_vc_post7(int n, int nx, int nxy, const T *__restrict__ s7,
                                                   const T *__restrict__ d, const int32_t *__restrict__ agg,
                                                   const T *__restrict__ b, const T *__restrict__ y,
                                                   const T *__restrict__ xc, T *__restrict__ x) {
  int i;
  if (!band_cell(n, nx, nxy, i)) return;
  // two batches of loads, each issued at once: the neighbours' y and
  // aggregates, then their coarse corrections (index 0 for no aggregate)
  T yq[7], xq[7];
  int g[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int q = nbr7(i, k, n, nx, nxy);
    yq[k] = y[q];
    g[k] = agg[q];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    int gc = g[k] >= 0 ? g[k] : 0;
    asm volatile("" : "+v"(gc));
    xq[k] = xc[gc];
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) s = fma(s7[(int64_t)k * n + i], g[k] >= 0 ? yq[k] + xq[k] : yq[k], s);
  const T yi = g[3] >= 0 ? yq[3] + xq[3] : yq[3];     // slot 3 is the cell itself
  x[i] = yi + (b[i] - s) / d[i];
}

template <class T>
__global__ void k_vc_jacobi(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const T *__restrict__ a, const T *__restrict__ d, const T *__restrict__ b,
                            const T *__restrict__ xin, T *__restrict__ xout, int first) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (first) { xout[i] = b[i] / d[i]; return; }
  T s = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) s = fma(a[p], xin[ci[p]], s);
  xout[i] = xin[i] + (b[i] - s) / d[i];
}

template <class T>
__global__ void k_to_f64(int n, const T *__restrict__ a, double *__restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}
template <class T>
__global__ void k_from_f64(int n, const double *__restrict__ a, T *__restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (T)a[i];
}

// ---- structured fine level ---------------------------------------------------
// The fine level is the 7-point grid with its entries by slot (ap7[s][c],
// slots -z -y -x self +x +y +z in ascending column order).  These kernels
// take the CSR kernels' operations in the same order, reading a cell's
// entries from the slot planes: a row's CSR entries are exactly its in-grid
// slots, in slot order.  Strong couplings are a 7-bit mask per cell.
// One pass over a cell's entries: their copy in the preconditioner's
// precision (s7, the operator of the fine-level smoother and residual), the
// l1 diagonal (k_l1diag's operations) and the directed strong couplings,
// dmask bit s: j = nbr(c, s) influences c (k_strength_dir's test).
template <class T>
__global__ void k_fine7(int nx, int ny, int nz, const double *__restrict__ ap7, double theta, double mrs,
                        T *__restrict__ s7, T *__restrict__ d, uint8_t *__restrict__ dmask) {
  const int64_t n = (int64_t)nx * ny * nz, c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const cell7 e = cell7_of(c, nx, ny, nz);
  double v[7];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) v[sl] = ap7[sl * n + c];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) s7[sl * n + c] = (T)v[sl];
  // l1 diagonal: sign of a_ii times the sum of |a_ij| over the row
  double l1 = 0.0;
#pragma unroll
  for (int sl = 0; sl < 7; ++sl)
    if (e.in[sl]) l1 = l1 + fabs(v[sl]);
  const double aii = v[3];
  if (l1 == 0.0) l1 = 1.0;
  d[c] = (T)(aii < 0.0 ? -l1 : l1);
  // strength
  double nm = 0.0, sum = 0.0;
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) {
    if (!e.in[sl]) continue;
    sum = sum + v[sl];
    if (sl != 3 && -v[sl] > nm) nm = -v[sl];
  }
  const bool weak = fabs(sum) > mrs * fabs(aii) || !(nm > 0.0);
  const double thr = theta * nm;
  uint8_t m = 0;
#pragma unroll
  for (int sl = 0; sl < 7; ++sl)
    if (e.in[sl] && sl != 3 && !weak && -v[sl] >= thr) m |= (uint8_t)(1u << sl);
  dmask[c] = m;
}

// symmetrised: smask bit s = dmask(c) bit s | dmask(nbr) bit 6-s
__global__ void k_strength7_sym(int nx, int ny, int nz, const uint8_t *__restrict__ dmask,
                                uint8_t *__restrict__ smask, uint8_t *__restrict__ state) {
  const int64_t n = (int64_t)nx * ny * nz, c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const cell7 e = cell7_of(c, nx, ny, nz);
  uint8_t d[7];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) d[sl] = dmask[e.in[sl] ? e.nb[sl] : c];
  const uint8_t own = d[3];
  uint8_t m = 0;
#pragma unroll
  for (int sl = 0; sl < 7; ++sl)
    if (e.in[sl] && sl != 3 && (((own >> sl) & 1u) || ((d[sl] >> (6 - sl)) & 1u))) m |= (uint8_t)(1u << sl);
  smask[c] = m;
  state[c] = m ? ST_UND : ST_ISO;
}

// Distance-2 MIS round on the grid: m1 as k_mis_m1; m2 and the decision as
// k_mis_m2d, in one kernel that reads only m1 and the cell's own state, so the
// state is updated in place.  Decided cells skip m2.
__global__ void k_mis7_m1(int nx, int ny, int nz, int level, const uint8_t *__restrict__ smask,
                          const uint8_t *__restrict__ state, uint64_t *__restrict__ m1, const int *__restrict__ prev,
                          int *__restrict__ und0) {
  const int64_t n = (int64_t)nx * ny * nz, c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (und0 && c < MIS_BATCH) und0[c] = 0;
  if (c >= n || (prev && *prev == 0)) return;
  const cell7 e = cell7_of(c, nx, ny, nz);
  const uint8_t sm = smask[c];
  int64_t q[7];
  uint8_t st[7];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) {
    q[sl] = ((sm >> sl) & 1u) ? e.nb[sl] : c;
    int64_t a = q[sl];
    asm volatile("" : "+v"(a));   // opaque: keeps the load unconditional
    st[sl] = state[a];
  }
  uint64_t m = keyof(st[3], (int)c, level);
  bool und = st[3] == ST_UND;
#pragma unroll
  for (int sl = 0; sl < 7; ++sl)
    if ((sm >> sl) & 1u) {
      const uint64_t kk = keyof(st[sl], (int)q[sl], level);
      m = kk > m ? kk : m;
      und = und || st[sl] == ST_UND;
    }
  // m1 is read only at undecided vertices and their strong neighbours, so a
  // vertex with no undecided one in its closed neighbourhood (strength is
  // symmetric) skips the store
  if (und) m1[c] = m;
}

__global__ void k_mis7_m2d(int nx, int ny, int nz, int level, const uint8_t *__restrict__ smask,
                           const uint64_t *__restrict__ m1, uint8_t *__restrict__ state,
                           int *__restrict__ undecided, const int *__restrict__ prev) {
  if (prev && *prev == 0) return;             // *undecided stays 0
  const int64_t n = (int64_t)nx * ny * nz, c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int left = 0;
  uint8_t st = ST_ISO, sm = 0;
  if (c < n) {
    st = state[c];
    uint32_t t = smask[c];
    asm volatile("" : "+v"(t));    // both loads issue before the test of st
    sm = (uint8_t)t;
  }
  if (st == ST_UND) {
    const cell7 e = cell7_of(c, nx, ny, nz);
    uint64_t v[7];
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) v[sl] = m1[((sm >> sl) & 1u) ? e.nb[sl] : c];
    uint64_t m = v[3];
#pragma unroll
    for (int sl = 0; sl < 7; ++sl)
      if ((sm >> sl) & 1u) m = v[sl] > m ? v[sl] : m;
    if (m == ~0ull) state[c] = ST_OUT;
    else if (m == prio((int)c, level)) state[c] = ST_ROOT;
    else left = 1;
  }
  // one plain store per block that still has undecided vertices
  if (__syncthreads_or(left) && threadIdx.x == 0) *undecided = 1;
}

// (z, nz as in k_agg1)
__global__ void k_agg1_7(int nx, int ny, int nz, const uint8_t *__restrict__ smask, const uint8_t *__restrict__ state,
                         const int32_t *__restrict__ id, int32_t *__restrict__ agg1, int32_t *__restrict__ z, int nzr) {
  const int64_t n = (int64_t)nx * ny * nz, c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nzr) z[c] = 0;
  if (c >= n) return;
  const cell7 e = cell7_of(c, nx, ny, nz);
  int g = -1;
  const uint8_t sm = smask[c];
  uint8_t st[7];
  int32_t ids[7];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) {
    const int64_t q = ((sm >> sl) & 1u) ? e.nb[sl] : c;
    st[sl] = state[q];
    ids[sl] = id[q];
  }
  if (st[3] == ST_ROOT) g = ids[3];
  else if (st[3] != ST_ISO)
#pragma unroll
    for (int sl = 6; sl >= 0; --sl)               // the first root in slot order wins
      if (((sm >> sl) & 1u) && st[sl] == ST_ROOT) g = ids[sl];
  agg1[c] = g;
}

__global__ void k_agg2_7(int nx, int ny, int nz, const uint8_t *__restrict__ smask, const double *__restrict__ ap7,
                         const uint8_t *__restrict__ state, const int32_t *__restrict__ agg1,
                         int32_t *__restrict__ agg, int *__restrict__ bad) {
  const int64_t n = (int64_t)nx * ny * nz, c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const cell7 e = cell7_of(c, nx, ny, nz);
  const uint8_t sm = smask[c];
  int32_t ags[7];
  double ws[7];
#pragma unroll
  for (int sl = 0; sl < 7; ++sl) {
    ags[sl] = agg1[((sm >> sl) & 1u) ? e.nb[sl] : c];
    ws[sl] = ap7[sl * n + c];
  }
  int g = ags[3];
  if (g < 0 && state[c] != ST_ISO) {
    double bw = -1.0;
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) {
      if (!((sm >> sl) & 1u)) continue;
      const int ag = ags[sl];
      if (ag < 0) continue;
      const double w = fabs(ws[sl]);
      if (w > bw || (w == bw && ag < g)) { bw = w; g = ag; }
    }
    if (g < 0) atomicOr(bad, 1);     // cannot happen for a maximal distance-2 set
  }
  agg[c] = g;
}

__global__ void k_cand7(int nc, int nx, int ny, int nz, const int32_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                        int32_t *__restrict__ cand) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int cnt = 0;
  for (int x = mptr[I]; x < mptr[I + 1]; ++x) {
    const cell7 e = cell7_of(mem[x], nx, ny, nz);
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) cnt += e.in[sl] ? 1 : 0;
  }
  cand[I] = cnt;
}

// x = Cinv b, one wave per row.
template <class T>
__global__ void k_dense_mv(int n, const double *__restrict__ Ci, const T *__restrict__ b, T *__restrict__ x) {
  int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s = fma(Ci[(int64_t)row * n + c], (double)b[c], s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row] = (T)s;
}

// ---- smoothed aggregation -----------------------------------------------------
// Option of the pressure AMG (rs_cpr_opts.smooth): the piecewise-constant
// prolongator P_t of the aggregates is smoothed by one damped Jacobi step,
//   P = (I - omega D^{-1} A) P_t,  D = diag(A),  omega = 4 / (3 rho),
//   rho = max_i sum_j |a_ij| / |a_ii|,
// then truncated as Fig. fig-ds-amg-par's interpolation truncation ("trunc
// error"): weights below trunc times the row's largest |weight| are dropped
// and the kept ones scaled to the row's former sum.  A_c = P^T (A P).  Every
// sum runs in the order of the FP64 oracle and no product is fused into an
// addition, so the hierarchy is the oracle's bit for bit.  Rows of P, of AP
// and of P^T are short (tens of entries), so each is built by one thread in
// its own stretch of memory: P row i at rp[i] + i (a row has at most one
// entry per stored column plus its own aggregate), AP row i at an offset from
// the scan of its candidate count.
#pragma clang fp contract(off)

// rho as the bit pattern of a non-negative double: integer max is float max
__global__ __launch_bounds__(256) void k_sa_rho(int n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ a,
                                                 unsigned long long *__restrict__ rho_bits) {
  __shared__ unsigned long long wm[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double q = 0.0;
  if (i < n) {
    double sm = 0.0, d = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      sm = sm + fabs(a[p]);
      if (ci[p] == i) d = a[p];
    }
    if (d != 0.0) q = sm / fabs(d);
  }
  unsigned long long b = (unsigned long long)__double_as_longlong(q);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(b, off, 64);
    b = o > b ? o : b;
  }
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wm[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = wm[w] > m ? wm[w] : m;
    atomicMax(rho_bits, m);
  }
}

__device__ __forceinline__ void sa_sort(int m, int32_t *__restrict__ k, double *__restrict__ v) {
  for (int x = 1; x < m; ++x) {
    const int32_t kk = k[x];
    const double vv = v[x];
    int y = x - 1;
    while (y >= 0 && k[y] > kk) { k[y + 1] = k[y]; v[y + 1] = v[y]; --y; }
    k[y + 1] = kk;
    v[y + 1] = vv;
  }
}

// Row i of the smoothed, truncated P, in place at pci/pv + rp[i] + i.
__global__ __launch_bounds__(256) void k_sa_p(int n, const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci, const double *__restrict__ a,
                                               const int32_t *__restrict__ agg,
                                               const unsigned long long *__restrict__ rho_bits, double trunc,
                                               int32_t *__restrict__ pcnt, int32_t *__restrict__ pci,
                                               double *__restrict__ pv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double rho = __longlong_as_double((long long)*rho_bits);
  const double omega = rho > 0.0 ? 4.0 / (3.0 * rho) : 0.0;
  const int p0 = rp[i], p1 = rp[i + 1];
  int32_t *cols = pci + p0 + i;
  double *vals = pv + p0 + i;
  int m = 0;
  double d = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int j = ci[p];
    if (j == i) d = a[p];
    const int J = agg[j];
    if (J < 0) continue;
    int t = 0;
    while (t < m && cols[t] != J) ++t;
    if (t == m) { cols[m] = J; vals[m] = 0.0; ++m; }
    vals[t] = vals[t] + a[p];
  }
  const int own = agg[i];
  if (own >= 0) {
    int t = 0;
    while (t < m && cols[t] != own) ++t;
    if (t == m) { cols[m] = own; vals[m] = 0.0; ++m; }
  }
  for (int t = 0; t < m; ++t) {
    const double delta = cols[t] == own ? 1.0 : 0.0;
    vals[t] = d != 0.0 ? delta - omega * (vals[t] / d) : delta;
  }
  sa_sort(m, cols, vals);
  if (trunc > 0.0 && m > 0) {
    double mx = 0.0, sall = 0.0, skeep = 0.0;
    for (int t = 0; t < m; ++t) {
      if (fabs(vals[t]) > mx) mx = fabs(vals[t]);
      sall = sall + vals[t];
    }
    const double thr = trunc * mx;
    int k = 0;
    for (int t = 0; t < m; ++t)
      if (fabs(vals[t]) >= thr) {
        cols[k] = cols[t];
        vals[k] = vals[t];
        skeep = skeep + vals[k];
        ++k;
      }
    if (k < m && skeep != 0.0) {
      const double scale = sall / skeep;
      for (int t = 0; t < k; ++t) vals[t] = vals[t] * scale;
    }
    m = k;
  }
  pcnt[i] = m;
}

// candidates of AP row i: the sum of the P row lengths of its columns
__global__ void k_sa_apcand(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const int32_t *__restrict__ pcnt, int32_t *__restrict__ cand) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) c += pcnt[ci[p]];
  cand[i] = c;
}

// Row i of AP: (AP)_iJ = sum over the row's columns j (ascending) of
// a_ij * p_jJ, then sorted by J; at apci/apv + off[i], apcnt[i] entries.
__global__ __launch_bounds__(256) void k_sa_ap(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const double *__restrict__ a, const int32_t *__restrict__ pcnt,
                                                const int32_t *__restrict__ pci, const double *__restrict__ pv,
                                                const int32_t *__restrict__ off, int32_t *__restrict__ apcnt,
                                                int32_t *__restrict__ apci, double *__restrict__ apv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t *cols = apci + off[i];
  double *vals = apv + off[i];
  int m = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = ci[p];
    const double aij = a[p];
    const int q0 = rp[j] + j, q1 = q0 + pcnt[j];
    for (int q = q0; q < q1; ++q) {
      const int J = pci[q];
      int t = 0;
      while (t < m && cols[t] != J) ++t;
      if (t == m) { cols[m] = J; vals[m] = 0.0; ++m; }
      vals[t] = vals[t] + aij * pv[q];
    }
  }
  sa_sort(m, cols, vals);
  apcnt[i] = m;
}

// P^T: entry counts per coarse column, then a fill in arbitrary order and a
// sort of each column by fine row (deterministic)
__global__ void k_sa_tcount(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ pcnt,
                            const int32_t *__restrict__ pci, int32_t *__restrict__ tcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int q0 = rp[i] + i;
  for (int q = q0; q < q0 + pcnt[i]; ++q) atomicAdd(&tcnt[pci[q]], 1);
}
__global__ void k_sa_tfill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ pcnt,
                           const int32_t *__restrict__ pci, const double *__restrict__ pv,
                           const int32_t *__restrict__ tptr, int32_t *__restrict__ tfill,
                           int32_t *__restrict__ tri, double *__restrict__ trv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int q0 = rp[i] + i;
  for (int q = q0; q < q0 + pcnt[i]; ++q) {
    const int J = pci[q];
    const int at = tptr[J] + atomicAdd(&tfill[J], 1);
    tri[at] = i;
    trv[at] = pv[q];
  }
}
__global__ void k_sa_tsort(int nc, const int32_t *__restrict__ tptr, int32_t *__restrict__ tri,
                           double *__restrict__ trv) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  sa_sort(tptr[I + 1] - tptr[I], tri + tptr[I], trv + tptr[I]);
}
__global__ void k_iota(int m, int32_t *__restrict__ v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) v[t] = t;
}

// candidates of coarse row I: the AP row lengths of its fine rows
__global__ void k_sa_ccand(int nc, const int32_t *__restrict__ tptr, const int32_t *__restrict__ tri,
                           const int32_t *__restrict__ apcnt, int32_t *__restrict__ cand) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int c = 0;
  for (int x = tptr[I]; x < tptr[I + 1]; ++x) c += apcnt[tri[x]];
  cand[I] = c;
}

// Row source of the smoothed Galerkin product for gal_row: "member" x is the
// x-th entry of P^T (fine row tri[x], weight trv[x]); its entries are the
// coarse columns of AP row tri[x] with values trv[x] * (AP)_iJ, so coarse row
// I gets sum over its fine rows (ascending) of p_iI (AP)_iJ.
struct rows_sa {
  const int32_t *tri;
  const double *trv;
  const int32_t *apoff, *apcnt, *apci;
  const double *apv;
  template <class F> __device__ __forceinline__ bool each(int x, const int32_t *__restrict__, F &&f) const {
    const int i = tri[x];
    const double w = trv[x];
    const int q0 = apoff[i], q1 = q0 + apcnt[i];
    for (int q = q0; q < q1; ++q)
      if (!f(apci[q], w * apv[q])) return false;
    return true;
  }
};
template <> struct gal_cap<rows_sa> { static constexpr int CAP = 32; };

#pragma clang fp contract(fast)

template <class T>
__global__ void k_cast_t(int64_t m, const double *__restrict__ a, T *__restrict__ b) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) b[t] = (T)a[t];
}

// cycle: restriction b_c = P^T r, prolongation z = y + P x_c (y = b ./ d, or
// the level's y when given), post-sweep x = z + (b - A z) ./ d
template <class T>
__global__ void k_sa_restrict(int nc, const int32_t *__restrict__ tptr, const int32_t *__restrict__ tri,
                              const T *__restrict__ trv, const T *__restrict__ r, T *__restrict__ bc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  T s = 0;
  for (int x = tptr[I]; x < tptr[I + 1]; ++x) s = fma(trv[x], r[tri[x]], s);
  bc[I] = s;
}
template <class T>
__global__ __launch_bounds__(256) void k_sa_prolong(int n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ pcnt, const int32_t *__restrict__ pci,
                                                     const T *__restrict__ pv, const T *__restrict__ y,
                                                     const T *__restrict__ b, const T *__restrict__ d,
                                                     const T *__restrict__ xc, T *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int q0 = rp[i] + i, q1 = q0 + pcnt[i];
  T s = 0;
  for (int q = q0; q < q1; ++q) s = fma(pv[q], xc[pci[q]], s);
  z[i] = (y ? y[i] : b[i] / d[i]) + s;
}
template <class T>
__global__ __launch_bounds__(256) void k_vc_postz(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const T *__restrict__ a, const T *__restrict__ d,
                                                   const T *__restrict__ b, const T *__restrict__ z, T *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) s = fma(a[p], z[ci[p]], s);
  x[i] = z[i] + (b[i] - s) / d[i];
}
template <class T>
__global__ __launch_bounds__(256) void k_vc_post7z(int n, int nx, int nxy, const T *__restrict__ s7,
                                                    const T *__restrict__ d, const T *__restrict__ b,
                                                    const T *__restrict__ z, T *__restrict__ x) {
  int i;
  if (!band_cell(n, nx, nxy, i)) return;
  T s = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) s = fma(s7[(int64_t)k * n + i], z[nbr7(i, k, n, nx, nxy)], s);
  x[i] = z[i] + (b[i] - s) / d[i];
}

}  // namespace

// ---------------------------------------------------------------------------
rs_status rs_amg_level0_csr(rs_cpr_s *M, hipStream_t s);

static rs_status level_alloc_work(amg_level *L, int prec, int64_t guard, bool csr_values, hipStream_t s) {
  size_t es = prec == 64 ? sizeof(double) : sizeof(float);
  RS_TRY(L->b.alloc(es * (L->n + 1)));
  // the fine level's iterate is read at every stencil neighbour of every cell
  // by the second stage; zero guard planes make those reads in-bounds
  RS_TRY(L->x.alloc(es * (L->n + 1 + 2 * guard)));
  L->xoff = guard;
  if (guard) RS_HIP(hipMemsetAsync(L->x.p, 0, es * (L->n + 1 + 2 * guard), s));
  RS_TRY(L->r.alloc(es * (L->n + 1)));
  // a coarse level's l1 diagonal and FP32 values come with its Galerkin copy
  if (!L->dl1.p) RS_TRY(L->dl1.alloc(es * (L->n + 1)));
  if (prec == 32 && csr_values && !L->ap.p) {
    RS_TRY(L->ap.alloc(sizeof(float) * (L->nnz + 1)));
  }
  return RS_OK;
}

// The fine level was set up by the structured kernels to be coarsened, but no
// aggregate formed (every row weak, or no vertex with a strength edge): it is
// the coarsest level after all, and the coarsest solve (dense inverse or
// l1-Jacobi sweeps) reads its CSR arrays and, in FP32, its FP32 values.
static rs_status level0_as_coarsest(rs_cpr_s *M, hipStream_t s) {
  amg_level *L = M->lev[0];
  RS_TRY(rs_amg_level0_csr(M, s));
  if (M->prec == 32 && !L->ap.p) {
    RS_TRY(L->ap.alloc(sizeof(float) * (L->nnz + 1)));
    k_cast_f32<<<rs_grid(L->nnz), RS_BLOCK, 0, s>>>(L->nnz, L->a.as<double>(), L->ap.as<float>());
    RS_HIP(hipGetLastError());
  }
  return RS_OK;
}

// Build the whole hierarchy; M->lev[0] must hold n and nnz.  The fine level
// is set up by the structured kernels from the pressure entries by slot; its
// CSR arrays are built only when it is also the coarsest level (or when it is
// inspected).
rs_status rs_amg_build(rs_cpr_s *M, hipStream_t s) {
  const rs_cpr_opts &o = M->o;
  int prec = M->prec;
  dbuf flag;                            // [0] error flag, [1] coarse nnz of the level
  RS_TRY(flag.alloc(sizeof(int) * 2));
  for (int l = 0;; ++l) {
    amg_level *L = M->lev[l];
    int n = L->n;
    const bool last = n <= o.coarse_n || (int)M->lev.size() >= o.max_levels;
    const bool st7 = l == 0 && !last;       // structured set-up of the fine level
    if (l == 0 && last) RS_TRY(rs_amg_level0_csr(M, s));
    RS_TRY(level_alloc_work(L, prec, l == 0 ? M->A->g.nxy : 0, !st7, s));
    if (l == 0) {
      size_t es = prec == 64 ? sizeof(double) : sizeof(float);
      RS_TRY(L->s7.alloc(es * 7 * (size_t)n));
      RS_TRY(L->y.alloc(es * ((size_t)n + 1)));
    }
    if (l == 0 && !st7) {
      if (prec == 64) k_cast7<double><<<rs_grid(7 * (int64_t)n), RS_BLOCK, 0, s>>>(7 * (int64_t)n, M->D->ap7.as<double>(), L->s7.as<double>());
      else k_cast7<float><<<rs_grid(7 * (int64_t)n), RS_BLOCK, 0, s>>>(7 * (int64_t)n, M->D->ap7.as<double>(), L->s7.as<float>());
      RS_HIP(hipGetLastError());
    }
    RS_TRY(L->agg.alloc(sizeof(int32_t) * (n + 1)));
    const grid3 &g = M->A->g;
    const double *ap7 = M->D->ap7.as<double>();
    dbuf dir;
    if (st7) {
      RS_TRY(dir.alloc(n));
      if (prec == 64)
        k_fine7<double><<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, ap7, o.theta, o.max_row_sum,
                                                        L->s7.as<double>(), L->dl1.as<double>(), dir.as<uint8_t>());
      else
        k_fine7<float><<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, ap7, o.theta, o.max_row_sum,
                                                       L->s7.as<float>(), L->dl1.as<float>(), dir.as<uint8_t>());
    } else if (l == 0) {
      if (prec == 64) k_l1diag<double><<<rs_grid(n), RS_BLOCK, 0, s>>>(n, L->rp.as<int32_t>(), L->ci.as<int32_t>(), L->a.as<double>(), L->dl1.as<double>());
      else k_l1diag<float><<<rs_grid(n), RS_BLOCK, 0, s>>>(n, L->rp.as<int32_t>(), L->ci.as<int32_t>(), L->a.as<double>(), L->dl1.as<float>());
      if (prec == 32) k_cast_f32<<<rs_grid(L->nnz), RS_BLOCK, 0, s>>>(L->nnz, L->a.as<double>(), L->ap.as<float>());
    }
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemsetAsync(L->agg.p, 0xff, sizeof(int32_t) * (n + 1), s));
    if (last) break;
    // strength: per CSR entry, or a 7-bit mask per cell on the fine level
    dbuf strong, state, m1, und;
    if (!st7) RS_TRY(dir.alloc(L->nnz));
    RS_TRY(strong.alloc(st7 ? n : L->nnz)); RS_TRY(state.alloc(n));
    RS_TRY(m1.alloc(sizeof(uint64_t) * n));
    RS_TRY(und.alloc(sizeof(int) * MIS_BATCH));
    const int32_t *rp = L->rp.as<int32_t>(), *ci = L->ci.as<int32_t>();
    if (st7) {
      k_strength7_sym<<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, dir.as<uint8_t>(), strong.as<uint8_t>(),
                                                      state.as<uint8_t>());
    } else {
      k_strength_dir<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, rp, ci, L->a.as<double>(), o.theta, o.max_row_sum, dir.as<uint8_t>());
      k_strength_sym<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, rp, ci, dir.as<uint8_t>(), strong.as<uint8_t>(), state.as<uint8_t>());
    }
    RS_HIP(hipGetLastError());
    // distance-2 MIS rounds, MIS_BATCH per host read; und[b] = 1 when round b
    // of the batch left undecided vertices
    for (int round = 0;; round += MIS_BATCH) {
      if (round > n + 2) return RS_E_HIP;     // progress is guaranteed; guard anyway
      for (int b = 0; b < MIS_BATCH; ++b) {
        const int *prev = b ? und.as<int>() + b - 1 : nullptr;
        int *und0 = b ? nullptr : und.as<int>();    // zeroed by the batch's first pass
        if (st7) {
          k_mis7_m1<<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, l, strong.as<uint8_t>(), state.as<uint8_t>(),
                                                    m1.as<uint64_t>(), prev, und0);
          k_mis7_m2d<<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, l, strong.as<uint8_t>(), m1.as<uint64_t>(),
                                                     state.as<uint8_t>(), und.as<int>() + b, prev);
        } else {
          k_mis_m1<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, l, rp, ci, strong.as<uint8_t>(), state.as<uint8_t>(),
                                                   m1.as<uint64_t>(), prev, und0);
          k_mis_m2d<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, l, rp, ci, strong.as<uint8_t>(), m1.as<uint64_t>(),
                                                    state.as<uint8_t>(), und.as<int>() + b, prev);
        }
      }
      RS_HIP(hipGetLastError());
      int h = 0;
      RS_TRY(rs_wait_read(&h, und.as<int>() + MIS_BATCH - 1, sizeof(int), s));
      if (h == 0) break;
    }
    // aggregates
    dbuf id, agg1;
    RS_TRY(id.alloc(sizeof(int32_t) * n)); RS_TRY(agg1.alloc(sizeof(int32_t) * n));
    k_root_flag<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, state.as<uint8_t>(), id.as<int32_t>(), flag.as<int>());
    RS_HIP(hipGetLastError());
    int64_t nc64 = 0;
    RS_TRY(scan_i32(id.as<int32_t>(), id.as<int32_t>(), n, &nc64, s, nullptr));
    int nc = (int)nc64;
    if (nc == 0 || nc >= n) {        // no coarsening possible: this level is the coarsest
      if (st7) RS_TRY(level0_as_coarsest(M, s));
      break;
    }
    // per coarse row counters (nc + 1 <= n), zeroed by the first aggregation pass
    dbuf off, skey, sval, cnt;
    RS_TRY(cnt.alloc(sizeof(int32_t) * ((size_t)nc + 1)));
    if (st7) {
      k_agg1_7<<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, strong.as<uint8_t>(), state.as<uint8_t>(),
                                               id.as<int32_t>(), agg1.as<int32_t>(), cnt.as<int32_t>(), nc + 1);
      k_agg2_7<<<rs_grid(n), RS_BLOCK, 0, s>>>(g.nx, g.ny, g.nz, strong.as<uint8_t>(), ap7, state.as<uint8_t>(),
                                               agg1.as<int32_t>(), L->agg.as<int32_t>(), flag.as<int>());
    } else {
      k_agg1<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, rp, ci, strong.as<uint8_t>(), state.as<uint8_t>(), id.as<int32_t>(),
                                             agg1.as<int32_t>(), cnt.as<int32_t>(), nc + 1);
      k_agg2<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, rp, ci, strong.as<uint8_t>(), L->a.as<double>(), state.as<uint8_t>(),
                                             agg1.as<int32_t>(), L->agg.as<int32_t>(), flag.as<int>());
    }
    RS_HIP(hipGetLastError());
    L->nc = nc;
    // temporaries of the smoothed product, kept until the host read at the
    // end of the level (the RAS set-up allocates on a side stream meanwhile)
    dbuf rho, apoff, apcnt, apci, apv, tfill, trv, ident;
    int64_t ncand = 0;
    if (o.smooth) {
      // smoothed prolongator: on the CSR form (built here for the fine level)
      if (l == 0) RS_TRY(rs_amg_level0_csr(M, s));
      const int32_t *crp = L->rp.as<int32_t>(), *cci = L->ci.as<int32_t>();
      const double *ca = L->a.as<double>();
      const int64_t pcap = L->nnz + n + 1;
      RS_TRY(rho.alloc(sizeof(unsigned long long)));
      RS_HIP(hipMemsetAsync(rho.p, 0, sizeof(unsigned long long), s));
      k_sa_rho<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, crp, cci, ca, rho.as<unsigned long long>());
      RS_TRY(L->pcnt.alloc(sizeof(int32_t) * ((size_t)n + 1)));
      RS_TRY(L->pci.alloc(sizeof(int32_t) * pcap));
      RS_TRY(L->pv.alloc(sizeof(double) * pcap));
      k_sa_p<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, crp, cci, ca, L->agg.as<int32_t>(), rho.as<unsigned long long>(),
                                             o.trunc, L->pcnt.as<int32_t>(), L->pci.as<int32_t>(), L->pv.as<double>());
      RS_HIP(hipGetLastError());
      // AP, each row at the scan of its candidate count
      RS_TRY(apoff.alloc(sizeof(int32_t) * ((size_t)n + 1)));
      RS_TRY(apcnt.alloc(sizeof(int32_t) * ((size_t)n + 1)));
      k_sa_apcand<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, crp, cci, L->pcnt.as<int32_t>(), apcnt.as<int32_t>());
      RS_HIP(hipGetLastError());
      int64_t apt = 0;
      RS_TRY(scan_i32(apcnt.as<int32_t>(), apoff.as<int32_t>(), n, &apt, s, nullptr));
      if (apt < 0) return RS_E_NOMEM;             // more than 2^31 candidates
      RS_TRY(apci.alloc(sizeof(int32_t) * (apt + 1)));
      RS_TRY(apv.alloc(sizeof(double) * (apt + 1)));
      k_sa_ap<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, crp, cci, ca, L->pcnt.as<int32_t>(), L->pci.as<int32_t>(),
                                              L->pv.as<double>(), apoff.as<int32_t>(), apcnt.as<int32_t>(),
                                              apci.as<int32_t>(), apv.as<double>());
      RS_HIP(hipGetLastError());
      // P^T: fine rows of each coarse column, ascending
      RS_TRY(L->tptr.alloc(sizeof(int32_t) * ((size_t)nc + 1)));
      RS_TRY(tfill.alloc(sizeof(int32_t) * ((size_t)nc + 1)));
      RS_HIP(hipMemsetAsync(tfill.p, 0, sizeof(int32_t) * (nc + 1), s));
      k_sa_tcount<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, crp, L->pcnt.as<int32_t>(), L->pci.as<int32_t>(), cnt.as<int32_t>());
      RS_HIP(hipGetLastError());
      RS_TRY(scan_i32(cnt.as<int32_t>(), L->tptr.as<int32_t>(), nc + 1, nullptr, s, nullptr));
      RS_TRY(L->tri.alloc(sizeof(int32_t) * pcap));
      RS_TRY(trv.alloc(sizeof(double) * pcap));
      k_sa_tfill<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, crp, L->pcnt.as<int32_t>(), L->pci.as<int32_t>(), L->pv.as<double>(),
                                                 L->tptr.as<int32_t>(), tfill.as<int32_t>(), L->tri.as<int32_t>(),
                                                 trv.as<double>());
      k_sa_tsort<<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, L->tptr.as<int32_t>(), L->tri.as<int32_t>(), trv.as<double>());
      RS_TRY(ident.alloc(sizeof(int32_t) * pcap));
      k_iota<<<rs_grid(pcap), RS_BLOCK, 0, s>>>((int)pcap, ident.as<int32_t>());
      RS_HIP(hipGetLastError());
      // A_c = P^T (A P) by the Galerkin row builder, each "member" a P^T entry
      RS_TRY(off.alloc(sizeof(int32_t) * ((size_t)nc + 1)));
      k_sa_ccand<<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, L->tptr.as<int32_t>(), L->tri.as<int32_t>(), apcnt.as<int32_t>(),
                                                  cnt.as<int32_t>());
      RS_HIP(hipGetLastError());
      RS_TRY(scan_i32(cnt.as<int32_t>(), off.as<int32_t>(), nc, &ncand, s, nullptr));
      if (ncand < 0) return RS_E_NOMEM;
      RS_TRY(skey.alloc(sizeof(int32_t) * (ncand + 1)));
      RS_TRY(sval.alloc(sizeof(double) * (ncand + 1)));
      k_galerkin<rows_sa><<<rs_grid(nc, GAL_BLOCK), GAL_BLOCK, 0, s>>>(
          nc, L->tptr.as<int32_t>(), ident.as<int32_t>(),
          rows_sa{L->tri.as<int32_t>(), trv.as<double>(), apoff.as<int32_t>(), apcnt.as<int32_t>(), apci.as<int32_t>(),
                  apv.as<double>()},
          L->agg.as<int32_t>(), off.as<int32_t>(), skey.as<int32_t>(), sval.as<double>(), cnt.as<int32_t>());
      RS_HIP(hipGetLastError());
      // P and P^T values in the apply precision
      const size_t es = prec == 64 ? sizeof(double) : sizeof(float);
      RS_TRY(L->pvt.alloc(es * pcap));
      RS_TRY(L->trt.alloc(es * pcap));
      RS_TRY(L->z.alloc(es * ((size_t)n + 1)));
      if (prec == 64) {
        k_cast_t<double><<<rs_grid(pcap), RS_BLOCK, 0, s>>>(pcap, L->pv.as<double>(), L->pvt.as<double>());
        k_cast_t<double><<<rs_grid(pcap), RS_BLOCK, 0, s>>>(pcap, trv.as<double>(), L->trt.as<double>());
      } else {
        k_cast_t<float><<<rs_grid(pcap), RS_BLOCK, 0, s>>>(pcap, L->pv.as<double>(), L->pvt.as<float>());
        k_cast_t<float><<<rs_grid(pcap), RS_BLOCK, 0, s>>>(pcap, trv.as<double>(), L->trt.as<float>());
      }
      RS_HIP(hipGetLastError());
      L->sa = true;
    } else {
      // members of each aggregate, ascending
      RS_TRY(L->mptr.alloc(sizeof(int32_t) * (nc + 1)));
      RS_TRY(tfill.alloc(sizeof(int32_t) * ((size_t)nc + 1)));
      k_count_members<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, L->agg.as<int32_t>(), cnt.as<int32_t>(), tfill.as<int32_t>(),
                                                      nc + 1);
      RS_HIP(hipGetLastError());
      // members: at most n (no host read of the exact count)
      RS_TRY(scan_i32(cnt.as<int32_t>(), L->mptr.as<int32_t>(), nc + 1, nullptr, s, nullptr));
      RS_TRY(L->mem.alloc(sizeof(int32_t) * ((size_t)n + 1)));
      k_fill_members<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, L->agg.as<int32_t>(), L->mptr.as<int32_t>(), tfill.as<int32_t>(),
                                                     L->mem.as<int32_t>());
      k_sort_members<<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, L->mptr.as<int32_t>(), L->mem.as<int32_t>());
      RS_HIP(hipGetLastError());
      // Galerkin product
      RS_TRY(off.alloc(sizeof(int32_t) * (nc + 1)));
      if (st7) k_cand7<<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, g.nx, g.ny, g.nz, L->mptr.as<int32_t>(), L->mem.as<int32_t>(), cnt.as<int32_t>());
      else k_cand<<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, L->mptr.as<int32_t>(), L->mem.as<int32_t>(), rp, cnt.as<int32_t>());
      RS_HIP(hipGetLastError());
      // candidates: the members' row entries, at most this level's nnz
      RS_TRY(scan_i32(cnt.as<int32_t>(), off.as<int32_t>(), nc, nullptr, s, nullptr));
      ncand = L->nnz;
      RS_TRY(skey.alloc(sizeof(int32_t) * (ncand + 1)));
      RS_TRY(sval.alloc(sizeof(double) * (ncand + 1)));
      if (st7)
        k_galerkin<rows_7><<<rs_grid(nc, GAL_BLOCK), GAL_BLOCK, 0, s>>>(
            nc, L->mptr.as<int32_t>(), L->mem.as<int32_t>(), rows_7{g.nx, g.ny, g.nz, ap7}, L->agg.as<int32_t>(),
            off.as<int32_t>(), skey.as<int32_t>(), sval.as<double>(), cnt.as<int32_t>());
      else
        k_galerkin<rows_csr><<<rs_grid(nc, GAL_BLOCK), GAL_BLOCK, 0, s>>>(
            nc, L->mptr.as<int32_t>(), L->mem.as<int32_t>(), rows_csr{rp, ci, L->a.as<double>()}, L->agg.as<int32_t>(),
            off.as<int32_t>(), skey.as<int32_t>(), sval.as<double>(), cnt.as<int32_t>());
      RS_HIP(hipGetLastError());
    }
    amg_level *C = new amg_level();
    M->lev.push_back(C);
    C->n = nc;
    RS_TRY(C->rp.alloc(sizeof(int32_t) * (nc + 1)));
    // coarse nnz: on the device for rp[nc], read with the error flag below;
    // ci and a sized by the candidate bound
    RS_TRY(scan_i32(cnt.as<int32_t>(), C->rp.as<int32_t>(), nc, nullptr, s, flag.as<int32_t>() + 1));
    k_set_last<<<1, 1, 0, s>>>(C->rp.as<int32_t>(), nc, flag.as<int32_t>() + 1);
    RS_TRY(C->ci.alloc(sizeof(int32_t) * (ncand + 1)));
    RS_TRY(C->a.alloc(sizeof(double) * (ncand + 1)));
    RS_TRY(C->dl1.alloc((prec == 64 ? sizeof(double) : sizeof(float)) * ((size_t)nc + 1)));
    if (prec == 32) RS_TRY(C->ap.alloc(sizeof(float) * (ncand + 1)));
    if (prec == 64)
      k_galerkin_copy<double><<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, off.as<int32_t>(), skey.as<int32_t>(),
                                                               sval.as<double>(), C->rp.as<int32_t>(), C->ci.as<int32_t>(),
                                                               C->a.as<double>(), nullptr, C->dl1.as<double>());
    else
      k_galerkin_copy<float><<<rs_grid(nc), RS_BLOCK, 0, s>>>(nc, off.as<int32_t>(), skey.as<int32_t>(),
                                                              sval.as<double>(), C->rp.as<int32_t>(), C->ci.as<int32_t>(),
                                                              C->a.as<double>(), C->ap.as<float>(), C->dl1.as<float>());
    RS_HIP(hipGetLastError());
    int h[2] = {0, 0};
    RS_TRY(rs_wait_read(h, flag.p, sizeof(int) * 2, s));
    if (h[0]) return RS_E_HIP;
    C->nnz = h[1];
  }
  M->nlev = (int)M->lev.size();
  // coarsest level
  amg_level *C = M->lev.back();
  int nC = C->n;
  M->coarse_lu = nC <= o.lu_max;
  if (M->coarse_lu) {
    dbuf G;
    RS_TRY(G.alloc(sizeof(double) * 2 * (size_t)nC * nC + 8));
    RS_TRY(M->cinv.alloc(sizeof(double) * (size_t)nC * nC + 8));
    RS_TRY(M->cb.alloc(sizeof(double) * (nC + 1)));
    RS_TRY(M->cx.alloc(sizeof(double) * (nC + 1)));
    RS_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    k_densify<<<rs_grid(nC), RS_BLOCK, 0, s>>>(nC, C->rp.as<int32_t>(), C->ci.as<int32_t>(), C->a.as<double>(), G.as<double>());
    RS_TRY(dense_inverse_run(nC, G.as<double>(), M->cinv.as<double>(), flag.as<int>(), s));
    int h = 0;
    RS_TRY(rs_wait_read(&h, flag.p, sizeof(int), s));
    if (h) return RS_E_SINGULAR;
    return RS_OK;                 // the read waited for the stream
  }
  RS_TRY(rs_wait(s));
  return RS_OK;
}

template <class T>
static rs_status vcycle_t(rs_cpr_s *M, hipStream_t s) {
  int nl = M->nlev;
  // descend
  for (int l = 0; l < nl - 1; ++l) {
    amg_level *L = M->lev[l], *C = M->lev[l + 1];
    const T *a = (M->prec == 64) ? (const T *)L->a.p : (const T *)L->ap.p;
    if (l == 0 && L->s7.p) {
      const grid3 &g = M->A->g;
      k_vc_pre7<T><<<band_grid(g.nx, g.ny, g.nz), RS_BLOCK, 0, s>>>(L->n, g.nx, (int)g.nxy, L->s7.as<T>(), L->dl1.as<T>(),
                                                      L->b.as<T>(), L->y.as<T>(), L->r.as<T>());
    } else {
      k_vc_pre<T><<<rs_grid(L->n), RS_BLOCK, 0, s>>>(L->n, L->rp.as<int32_t>(), L->ci.as<int32_t>(), a,
                                                    L->dl1.as<T>(), L->b.as<T>(), L->r.as<T>());
    }
    if (L->sa)
      k_sa_restrict<T><<<rs_grid(L->nc), RS_BLOCK, 0, s>>>(L->nc, L->tptr.as<int32_t>(), L->tri.as<int32_t>(),
                                                           L->trt.as<T>(), L->r.as<T>(), C->b.as<T>());
    else
      k_vc_restrict<T><<<rs_grid(L->nc), RS_BLOCK, 0, s>>>(L->nc, L->mptr.as<int32_t>(), L->mem.as<int32_t>(),
                                                           L->r.as<T>(), C->b.as<T>());
  }
  // coarsest
  amg_level *C = M->lev[nl - 1];
  const T *ca = (M->prec == 64) ? (const T *)C->a.p : (const T *)C->ap.p;
  if (M->coarse_lu) {
    k_dense_mv<T><<<rs_grid(C->n, 4), 256, 0, s>>>(C->n, M->cinv.as<double>(), C->b.as<T>(), C->xp<T>());
  } else {
    T *xa = C->xp<T>(), *xb = C->r.as<T>();
    for (int sw = 0; sw < M->o.coarse_sweeps; ++sw) {
      k_vc_jacobi<T><<<rs_grid(C->n), RS_BLOCK, 0, s>>>(C->n, C->rp.as<int32_t>(), C->ci.as<int32_t>(), ca,
                                                        C->dl1.as<T>(), C->b.as<T>(), xb, xa, sw == 0);
      T *t = xa; xa = xb; xb = t;
    }
    if (xb != C->xp<T>())
      RS_HIP(hipMemcpyAsync(C->xp<T>(), xb, sizeof(T) * C->n, hipMemcpyDeviceToDevice, s));
  }
  // ascend
  for (int l = nl - 2; l >= 0; --l) {
    amg_level *L = M->lev[l], *Cl = M->lev[l + 1];
    const T *a = (M->prec == 64) ? (const T *)L->a.p : (const T *)L->ap.p;
    if (L->sa) {
      // z = y + P x_c, then the post-sweep from z
      const bool st = l == 0 && L->s7.p;
      k_sa_prolong<T><<<rs_grid(L->n), RS_BLOCK, 0, s>>>(L->n, L->rp.as<int32_t>(), L->pcnt.as<int32_t>(),
                                                         L->pci.as<int32_t>(), L->pvt.as<T>(),
                                                         st ? L->y.as<T>() : nullptr, L->b.as<T>(), L->dl1.as<T>(),
                                                         Cl->xp<T>(), L->z.as<T>());
      if (st) {
        const grid3 &g = M->A->g;
        k_vc_post7z<T><<<band_grid(g.nx, g.ny, g.nz), RS_BLOCK, 0, s>>>(L->n, g.nx, (int)g.nxy, L->s7.as<T>(), L->dl1.as<T>(),
                                                          L->b.as<T>(), L->z.as<T>(), L->xp<T>());
      } else {
        k_vc_postz<T><<<rs_grid(L->n), RS_BLOCK, 0, s>>>(L->n, L->rp.as<int32_t>(), L->ci.as<int32_t>(), a,
                                                         L->dl1.as<T>(), L->b.as<T>(), L->z.as<T>(), L->xp<T>());
      }
    } else if (l == 0 && L->s7.p) {
      const grid3 &g = M->A->g;
      k_vc_post7<T><<<band_grid(g.nx, g.ny, g.nz), RS_BLOCK, 0, s>>>(L->n, g.nx, (int)g.nxy, L->s7.as<T>(), L->dl1.as<T>(),
                                                       L->agg.as<int32_t>(), L->b.as<T>(), L->y.as<T>(),
                                                       Cl->xp<T>(), L->xp<T>());
    } else {
      k_vc_post<T><<<rs_grid(L->n), RS_BLOCK, 0, s>>>(L->n, L->rp.as<int32_t>(), L->ci.as<int32_t>(), a,
                                                     L->dl1.as<T>(), L->agg.as<int32_t>(), L->b.as<T>(),
                                                     Cl->xp<T>(), L->xp<T>());
    }
  }
  RS_HIP(hipGetLastError());
  return RS_OK;
}

rs_status rs_vcycle_run(rs_cpr_s *M, hipStream_t s) {
  return M->prec == 64 ? vcycle_t<double>(M, s) : vcycle_t<float>(M, s);
}

extern "C" int rs_cpr_nlevels(rs_cpr M) { return M ? M->nlev : 0; }

extern "C" rs_status rs_cpr_level(rs_cpr M, int l, int *h_n, int64_t *h_nnz, int32_t *h_rp,
                                  int32_t *h_ci, double *h_a, double *h_dl1, int32_t *h_agg) {
  if (!M || l < 0 || l >= M->nlev) return RS_E_ARG;
  RS_HIP(hipDeviceSynchronize());
  amg_level *L = M->lev[l];
  if (l == 0 && (h_rp || h_ci || h_a) && !L->a.p) {   // the fine level's CSR on demand
    RS_TRY(rs_amg_level0_csr(M, nullptr));
    RS_HIP(hipDeviceSynchronize());
  }
  if (h_n) *h_n = L->n;
  if (h_nnz) *h_nnz = L->nnz;
  if (h_rp) RS_HIP(hipMemcpy(h_rp, L->rp.p, sizeof(int32_t) * (L->n + 1), hipMemcpyDeviceToHost));
  if (h_ci) RS_HIP(hipMemcpy(h_ci, L->ci.p, sizeof(int32_t) * L->nnz, hipMemcpyDeviceToHost));
  if (h_a) RS_HIP(hipMemcpy(h_a, L->a.p, sizeof(double) * L->nnz, hipMemcpyDeviceToHost));
  if (h_agg) RS_HIP(hipMemcpy(h_agg, L->agg.p, sizeof(int32_t) * L->n, hipMemcpyDeviceToHost));
  if (h_dl1) {
    if (M->prec == 64) {
      RS_HIP(hipMemcpy(h_dl1, L->dl1.p, sizeof(double) * L->n, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> t(L->n);
      RS_HIP(hipMemcpy(t.data(), L->dl1.p, sizeof(float) * L->n, hipMemcpyDeviceToHost));
      for (int i = 0; i < L->n; ++i) h_dl1[i] = t[i];
    }
  }
  return RS_OK;
}

extern "C" rs_status rs_cpr_level_p(rs_cpr M, int l, int64_t *h_nnz, int32_t *h_rp, int32_t *h_ci, double *h_v) {
  if (!M || !h_nnz || l < 0 || l >= M->nlev - 1 || !M->lev[l]->sa) return RS_E_ARG;
  RS_HIP(hipDeviceSynchronize());
  amg_level *L = M->lev[l];
  const int n = L->n;
  std::vector<int32_t> rp(n + 1), cnt(n + 1);
  RS_HIP(hipMemcpy(rp.data(), L->rp.p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  RS_HIP(hipMemcpy(cnt.data(), L->pcnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  int64_t nnz = 0;
  for (int i = 0; i < n; ++i) nnz += cnt[i];
  *h_nnz = nnz;
  if (!h_rp && !h_ci && !h_v) return RS_OK;
  const int64_t cap = (int64_t)rp[n] + n;
  std::vector<int32_t> ci(cap > 0 ? cap : 1);
  std::vector<double> v(cap > 0 ? cap : 1);
  RS_HIP(hipMemcpy(ci.data(), L->pci.p, sizeof(int32_t) * cap, hipMemcpyDeviceToHost));
  RS_HIP(hipMemcpy(v.data(), L->pv.p, sizeof(double) * cap, hipMemcpyDeviceToHost));
  int64_t w = 0;
  for (int i = 0; i < n; ++i) {
    if (h_rp) h_rp[i] = (int32_t)w;
    for (int k = 0; k < cnt[i]; ++k, ++w) {
      if (h_ci) h_ci[w] = ci[(int64_t)rp[i] + i + k];
      if (h_v) h_v[w] = v[(int64_t)rp[i] + i + k];
    }
  }
  if (h_rp) h_rp[n] = (int32_t)w;
  return RS_OK;
}

extern "C" rs_status rs_dense_inverse(int n, const double *d_a, double *d_inv, void *stream) {
  if (n < 1 || !d_a || !d_inv) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  dbuf G, flag;
  RS_TRY(G.alloc(sizeof(double) * 2 * (size_t)n * n));
  RS_TRY(flag.alloc(sizeof(int)));
  RS_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  k_augment<<<rs_grid(2 * (int64_t)n * n), RS_BLOCK, 0, s>>>(n, d_a, G.as<double>());
  RS_TRY(dense_inverse_run(n, G.as<double>(), d_inv, flag.as<int>(), s));
  int h = 0;
  RS_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  RS_HIP(hipStreamSynchronize(s));
  return h ? RS_E_SINGULAR : RS_OK;
}

// ---- allocation-free dense inverse -----------------------------------------
// rs_dense_inverse_noalloc takes its scratch (the n x 2n augmented matrix and
// the singular flag) from this file-scope array instead of the pool: one copy
// per GPU, created with the code object and held until the process ends.  In
// host code `scratch` only names the symbol; its device address on each GPU
// comes from hipGetSymbolAddress, taken once per device at the first call
// there (with that device current) and kept in scratch_dev[].
constexpr size_t NOALLOC_G = 2 * (size_t)RS_DENSE_NOALLOC_MAX * RS_DENSE_NOALLOC_MAX;   // doubles
static __device__ __align__(256) double scratch[NOALLOC_G + 32];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_dev[NOALLOC_MAX_DEVICES];

rs_status scratch_ptr(double **out) {
  int dev = -1;
  RS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return RS_E_ARG;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    RS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RS_E_HIP;
    scratch_dev[dev] = (double *)p;
  }
  *out = scratch_dev[dev];
  return RS_OK;
}
}  // namespace

// k_augment that also clears the singular flag (a kernel rather than a
// memset node, so the flag starts at zero on every call)
__global__ void k_augment_clear(int n, const double *__restrict__ a, double *__restrict__ G, int *__restrict__ flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *flag = 0;
  if (t >= 2 * (int64_t)n * n) return;
  const int64_t r = t / (2 * n), c = t - r * 2 * n;
  G[t] = c < n ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
}

extern "C" rs_status rs_dense_inverse_noalloc(int n, const double *d_a, double *d_inv, void *stream) {
  if (n < 1 || n > RS_DENSE_NOALLOC_MAX || !d_a || !d_inv) return RS_E_ARG;
  double *G = nullptr;
  RS_TRY(scratch_ptr(&G));
  int *flag = (int *)(G + NOALLOC_G);
  hipStream_t s = rs_stream(stream);
  k_augment_clear<<<rs_grid(2 * (int64_t)n * n), RS_BLOCK, 0, s>>>(n, d_a, G, flag);
  RS_TRY(dense_inverse_run(n, G, d_inv, flag, s));
  int h = 0;
  RS_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  RS_HIP(hipStreamSynchronize(s));
  return h ? RS_E_SINGULAR : RS_OK;
}

extern "C" rs_status rs_cpr_vcycle(rs_cpr M, const double *d_b, double *d_x, void *stream) {
  if (!M || !d_b || !d_x) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  amg_level *L = M->lev[0];
  int n = L->n;
  if (M->prec == 64) {
    RS_HIP(hipMemcpyAsync(L->b.p, d_b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    RS_TRY(rs_vcycle_run(M, s));
    RS_HIP(hipMemcpyAsync(d_x, L->xp<double>(), sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  } else {
    k_from_f64<float><<<rs_grid(n), RS_BLOCK, 0, s>>>(n, d_b, L->b.as<float>());
    RS_TRY(rs_vcycle_run(M, s));
    k_to_f64<float><<<rs_grid(n), RS_BLOCK, 0, s>>>(n, L->xp<float>(), d_x);
    RS_HIP(hipGetLastError());
  }
  return RS_OK;
}

rs_status rs_amg_level0(rs_cpr_s *M, hipStream_t s) {
  (void)s;
  rs_bsr_s *A = M->A;
  amg_level *L = new amg_level();
  M->lev.push_back(L);
  L->n = (int)A->g.n;
  L->nnz = A->nnzb;
  return RS_OK;
}

// CSR arrays of the fine level (the validated 7-point pattern, values from
// the pressure entries by slot), for when it is the coarsest level or is
// inspected.
rs_status rs_amg_level0_csr(rs_cpr_s *M, hipStream_t s) {
  rs_bsr_s *A = M->A;
  amg_level *L = M->lev[0];
  if (L->a.p) return RS_OK;
  RS_TRY(L->rp.alloc(sizeof(int32_t) * (L->n + 1)));
  RS_TRY(L->ci.alloc(sizeof(int32_t) * L->nnz));
  RS_TRY(L->a.alloc(sizeof(double) * L->nnz));
  RS_HIP(hipMemcpyAsync(L->rp.p, A->rp.p, sizeof(int32_t) * (L->n + 1), hipMemcpyDeviceToDevice, s));
  RS_HIP(hipMemcpyAsync(L->ci.p, A->ci.p, sizeof(int32_t) * L->nnz, hipMemcpyDeviceToDevice, s));
  k_csr_from7<<<rs_grid(A->g.n), RS_BLOCK, 0, s>>>(A->g.nx, A->g.ny, A->g.nz, L->rp.as<int32_t>(),
                                                   M->D->ap7.as<double>(), L->a.as<double>());
  RS_HIP(hipGetLastError());
  return RS_OK;
}
