// cpr.hip -- CPR preconditioner: two-stage (pressure stage, then
// full-system stage) or three-stage CPR-FPF, and the full-system stage:
// block Jacobi or block ILU(0).
//
// Apply, for a residual r (FP64):
//   r~  = D^{-1} r                       decoupling (Eq. decoupled-eq)
//   x_p = Vcycle(A_p, r~[:,0])           pressure stage (Pi_r: unknown 0)
//   r~2 = r~ - A~[:,0] x_p               residual update (column 0 of A~)
//   z   = M2^{-1} r~2 + Pi_p x_p          second stage, then prolong x_p
// The paper's CPR-FPF (Section "Preconditioners", Algorithm pc-fpf) wraps
// the pressure stage between two full-system stages; its five steps, with
// f = r~:
//   y   = M2^{-1} f                       (the second stage with x_p = 0)
//   r~1 = f - A~ y                        k_fpf_resid, also b_p = r~1[:,0]
//   x_p = Vcycle(A_p, b_p)
//   z   = y + M2^{-1}(r~1 - A~[:,0] x_p) + Pi_p x_p
// where r~1 - A~[:,0] x_p is the residual of y + Pi_p x_p (step 4).
// In prec 32 every vector and stored operator of the preconditioner is FP32
// except the coarsest AMG solve (FP64).
//
// Block ILU(0) on the 7-point block pattern only modifies the diagonal
// blocks (no fill position lies on the pattern): D_i = A~_ii - sum over the
// lower neighbours k of A~_ik D_k^{-1} A~_ki.  Its factorisation and sweeps
// are the pipelined kernels of dilu.hip; the residual update r~2 is fused
// into the forward sweep and the prolongation Pi_p x_p into the backward
// sweep, so r~2 and the corrected z are never stored separately.
#include "rs_internal.h"
#include <math.h>
#include <mutex>

namespace {
#pragma clang fp contract(off)
#include "block4.h"
#pragma clang fp contract(fast)

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

template <class T>
__device__ __forceinline__ void ld16(const T *__restrict__ p, double (&M)[4][4]) {
#pragma unroll
  for (int e = 0; e < 16; ++e) M[e >> 2][e & 3] = (double)p[e];
}

// Block-Jacobi setup: invert A~_ii (FP64 arithmetic on the stored values).
template <class T>
__global__ void k_bj_setup(int64_t n, const T *__restrict__ t7, T *__restrict__ dinv2, int *__restrict__ flag) {
#pragma clang fp contract(off)
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double L[4][4], R[4][4];
  ld16<T>(t7 + (3 * n + c) * 16, L);
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) R[r][q] = (r == q) ? 1.0 : 0.0;
  int f = gje4<4>(L, R);
  if (f) atomicOr(flag, f);
#pragma unroll
  for (int e = 0; e < 16; ++e) dinv2[c * 16 + e] = (T)R[e >> 2][e & 3];
}

// ---- apply -------------------------------------------------------------------
template <class T> __device__ __forceinline__ T ldin(const double *p) { return (T)*p; }

// r~ = D^{-1} r; the pressure right-hand side b_p = r~[:,0].  Four lanes per cell.
// With `halt` set, the kernel does nothing when *halt is nonzero (a pass
// enqueued before the solver knew whether it would be needed).
template <class T>
__global__ __launch_bounds__(256) void k_cpr_in(int64_t n, const T *__restrict__ dinv,
                                                 const double *__restrict__ r, T *__restrict__ rt,
                                                 T *__restrict__ bp, const double *__restrict__ hs,
                                                 double *__restrict__ vout, const double *__restrict__ halt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  if (halt && *halt != 0.0) return;
  int64_t c = t >> 2;
  int row = (int)(t & 3);
  const T *d = dinv + c * 16 + 4 * row;
  // hs: the input is r / *hs (a Krylov vector before its normalisation),
  // which also goes to vout
  const double h = hs ? *hs : 1.0;
  T s = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double rv = hs ? r[4 * c + m] / h : r[4 * c + m];
    s = fma(d[m], (T)rv, s);
  }
  if (hs) vout[t] = r[t] / h;
  rt[t] = s;
  if (row == 0) bp[c] = s;
}

// r~2 for lane `row` of cell c: r~ - sum over the 7 slots of A~[:,0] x_p.
template <class T>
__device__ __forceinline__ T resid2(int64_t n, int64_t c, int row, int64_t nx, int64_t nxy,
                                    const T *__restrict__ rt, const T *__restrict__ col0,
                                    const T *__restrict__ xp) {
  T v = rt[4 * c + row];
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    int64_t q = nbr_of(c, s, nx, nxy);
    q = (q < 0 || q >= n) ? c : q;           // off-grid col0 entries are zero
    v = v - col0[c * 32 + 8 * row + s] * xp[q];
  }
  return v;
}

// 4x4 matvec across the four lanes of a cell: lane `row` returns (M v)[row]
// where v[m] lives in lane m of the group.
template <class T>
__device__ __forceinline__ T group_mv(const T *__restrict__ Mrow, T v) {
  int base = (threadIdx.x & 63) & ~3;
  T out = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) out = fma(Mrow[m], __shfl(v, base + m, 64), out);
  return out;
}

// Block Jacobi second stage, fused: z = D2^{-1} r~2 + Pi_p x_p.
template <class T>
__global__ __launch_bounds__(256) void k_bj_apply(int64_t n, int64_t nx, int64_t nxy,
                                                   const T *__restrict__ rt, const T *__restrict__ col0,
                                                   const T *__restrict__ xp, const T *__restrict__ dinv2,
                                                   T *__restrict__ z) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = t < 4 * n;
  int64_t c = ok ? (t >> 2) : 0;
  int row = (int)(t & 3);
  T v = resid2<T>(n, c, row, nx, nxy, rt, col0, xp);
  T o = group_mv<T>(dinv2 + c * 16 + 4 * row, v);
  if (row == 0) o = o + xp[c];
  if (ok) z[t] = o;
}

// CPR-FPF step 2: r~1 = r~ - A~ y in place of r~, and b_p = r~1[:,0].  Four
// lanes per cell, lane `row` owns block row `row` of the 7 decoupled blocks.
template <class T>
__global__ __launch_bounds__(256) void k_fpf_resid(int64_t n, int64_t nx, int64_t nxy, const T *__restrict__ t7,
                                                    const T *__restrict__ y, T *__restrict__ rt, T *__restrict__ bp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  const int64_t c = t >> 2;
  const int row = (int)(t & 3);
  T v = rt[t];
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    int64_t q = nbr_of(c, s, nx, nxy);
    q = (q < 0 || q >= n) ? c : q;           // off-grid blocks are zero
    const T *a = t7 + ((int64_t)s * n + c) * 16 + 4 * row;
#pragma unroll
    for (int m = 0; m < 4; ++m) v = v - a[m] * y[4 * q + m];
  }
  rt[t] = v;
  if (row == 0) bp[c] = v;
}

template <class T>
__global__ void k_fpf_add(int64_t m, const T *__restrict__ y, T *__restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) z[t] = z[t] + y[t];
}

template <class T>
__global__ void k_fill0(int64_t m, T *__restrict__ a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) a[t] = (T)0;
}

template <class T>
__global__ void k_vec_to_f64(int64_t m, const T *__restrict__ a, double *__restrict__ b) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) b[t] = (double)a[t];
}

}  // namespace

rs_status rs_amg_level0(rs_cpr_s *M, hipStream_t s);
rs_status rs_amg_build(rs_cpr_s *M, hipStream_t s);

extern "C" void rs_cpr_opts_default(rs_cpr_opts *o) {
  if (!o) return;
  o->smoother = RS_SM_DILU;
  o->theta = 0.5;
  o->max_row_sum = 0.9;
  o->coarse_n = 256;
  o->max_levels = 20;
  o->lu_max = 256;
  o->coarse_sweeps = 4;
  o->stages = 2;
  o->smooth = 0;
  o->trunc = 1e-2;
}

rs_cpr_s::~rs_cpr_s() {
  for (amg_level *L : lev) delete L;
  if (hpin) (void)hipHostFree(hpin);
  if (bpin) (void)hipHostFree(bpin);
}

extern "C" void rs_cpr_destroy(rs_cpr M) { delete M; }

// One non-blocking stream per device, at the default priority, for set-up
// work that does not depend on the AMG set-up (block Jacobi, layer RAS).
// nullptr if it cannot be created (the work then stays on the caller's stream).
static hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t ss[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!ss[dev] && hipStreamCreateWithFlags(&ss[dev], hipStreamNonBlocking) != hipSuccess) ss[dev] = nullptr;
  return ss[dev];
}

// The second-stage set-up (block Jacobi or layer RAS) reads only the
// decoupled blocks, the AMG set-up only the pressure matrix: the former runs
// on a side stream while the latter (many small launches and host reads)
// runs on the caller's stream.  The global DILU set-up stays on the
// caller's stream (its workgroups wait on each other).  Both streams are
// idle again when this returns, on every path.
extern "C" rs_status rs_cpr_setup(rs_bsr A, rs_dcpl D, const rs_cpr_opts *o, void *stream, rs_cpr *out) {
  if (!A || !D || !out || D->A != A) return RS_E_ARG;
  *out = nullptr;
  rs_cpr_opts opts;
  if (o) opts = *o; else rs_cpr_opts_default(&opts);
  const bool ras = opts.smoother == RS_SM_RAS || opts.smoother == RS_SM_RAS1;
  if ((opts.smoother != RS_SM_BJ && opts.smoother != RS_SM_DILU && !ras) ||
      (ras && rs_ras_check_shape(A->g, D->prec) != RS_OK) || opts.coarse_n < 1 ||
      opts.max_levels < 1 || opts.lu_max < 1 || opts.lu_max > 8192 || opts.coarse_sweeps < 1 ||
      (opts.stages != 2 && opts.stages != 3) || (opts.smooth != 0 && opts.smooth != 1) ||
      !(opts.trunc >= 0.0 && opts.trunc <= 1.0) || opts.theta != opts.theta ||
      opts.max_row_sum != opts.max_row_sum)
    return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  hipStream_t ss = opts.smoother == RS_SM_DILU ? nullptr : side_stream();
  hipEvent_t ev = nullptr;
  if (ss && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { ev = nullptr; ss = nullptr; }
  if (!ss) ss = s;
  const bool split = ss != s;
  rs_cpr_s *M = new rs_cpr_s();
  M->A = A; M->D = D; M->o = opts; M->prec = D->prec;
  int64_t n = A->g.n;
  size_t es = M->prec == 64 ? sizeof(double) : sizeof(float);
  rs_status st = RS_OK;
  dbuf flag;
  bool launched = false;
  do {
    if ((st = M->dinv2.alloc(es * 16 * n)) != RS_OK) break;
    if ((st = M->rt.alloc(es * 4 * n)) != RS_OK) break;
    if ((st = M->yv.alloc(es * 4 * n)) != RS_OK) break;
    if ((st = M->zt.alloc(es * 4 * n)) != RS_OK) break;
    if (opts.stages == 3) {
      const int64_t nz0 = n + 2 * A->g.nxy;     // x_p = 0 with the guards the second stage reads
      if ((st = M->fy.alloc(es * 4 * n)) != RS_OK) break;
      if ((st = M->fzero.alloc(es * nz0)) != RS_OK) break;
      if (M->prec == 64) k_fill0<double><<<rs_grid(nz0), RS_BLOCK, 0, s>>>(nz0, M->fzero.as<double>());
      else k_fill0<float><<<rs_grid(nz0), RS_BLOCK, 0, s>>>(nz0, M->fzero.as<float>());
    }
    if ((st = flag.alloc(sizeof(int))) != RS_OK) break;
    if (hipMemsetAsync(flag.p, 0, sizeof(int), s) != hipSuccess) { st = RS_E_HIP; break; }
    if (split) {
      if (hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(ss, ev, 0) != hipSuccess) { st = RS_E_HIP; break; }
    }
    launched = true;
    if (opts.smoother == RS_SM_BJ) {
      if (M->prec == 64) k_bj_setup<double><<<rs_grid(n), RS_BLOCK, 0, ss>>>(n, D->t7.as<double>(), M->dinv2.as<double>(), flag.as<int>());
      else k_bj_setup<float><<<rs_grid(n), RS_BLOCK, 0, ss>>>(n, D->t7.as<float>(), M->dinv2.as<float>(), flag.as<int>());
      if (hipGetLastError() != hipSuccess) { st = RS_E_HIP; break; }
    } else if (ras) {
      if ((st = rs_ras_setup_run(M, flag.as<int>(), ss)) != RS_OK) break;
    }
    if ((st = rs_amg_level0(M, s)) != RS_OK) break;
    if ((st = rs_amg_build(M, s)) != RS_OK) break;
    if (opts.smoother == RS_SM_DILU) {
      if ((st = rs_dilu_prepare(M)) != RS_OK) break;
      if ((st = rs_dilu_setup_run(M, flag.as<int>(), s)) != RS_OK) break;
    }
  } while (0);
  if (split && launched) {
    // join: the caller's stream waits for the side stream; the read of the
    // error word below waits for the caller's stream, hence for all the side
    // stream's work, before any buffer can go back to the pool
    if (hipEventRecord(ev, ss) != hipSuccess || hipStreamWaitEvent(s, ev, 0) != hipSuccess) {
      if (st == RS_OK) st = RS_E_HIP;
    }
  }
  if (st == RS_OK) {
    int h = 0;
    if (hipGetLastError() != hipSuccess || rs_wait_read(&h, flag.p, sizeof(int), s) != RS_OK) st = RS_E_HIP;
    else if (h & RSF_NONFINITE) st = RS_E_NONFINITE;
    else if (h & RSF_SINGULAR) st = RS_E_SINGULAR;
    else if (opts.smoother == RS_SM_DILU) st = rs_dilu_check(M, s);   // its set-up's bounded waits
  } else {
    (void)hipStreamSynchronize(s);
    if (split && launched) (void)hipStreamSynchronize(ss);
  }
  if (ev) (void)hipEventDestroy(ev);
  if (st != RS_OK) { delete M; return st; }
  *out = M;
  return RS_OK;
}

template <class T>
static rs_status second_stage(rs_cpr_s *M, const T *xp, T *z, hipStream_t s) {
  const grid3 &g = M->A->g;
  const int64_t n = g.n;
  if (M->o.smoother == RS_SM_BJ) {
    k_bj_apply<T><<<rs_grid(4 * n), RS_BLOCK, 0, s>>>(n, g.nx, g.nxy, M->rt.as<T>(), M->D->col0.as<T>(), xp,
                                                     M->dinv2.as<T>(), z);
  } else if (M->o.smoother == RS_SM_RAS || M->o.smoother == RS_SM_RAS1) {
    RS_TRY(rs_ras_apply_run<T>(M, xp, z, s));
  } else {
    RS_TRY(rs_dilu_apply_run<T>(M, xp, z, s));
  }
  RS_HIP(hipGetLastError());
  return RS_OK;
}

// The first pass of the CPR apply: r~ = D^{-1} r into M->rt and b_p.
template <class T>
static rs_status cpr_in_t(rs_cpr_s *M, const double *r, hipStream_t s, const double *hs, double *vout,
                          const double *halt) {
  int64_t n = M->A->g.n;
  k_cpr_in<T><<<rs_grid(4 * n), RS_BLOCK, 0, s>>>(n, M->D->dinv.as<T>(), r, M->rt.as<T>(), M->lev[0]->b.as<T>(),
                                                 hs, vout, halt);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

// The rest of the CPR apply, from M->rt and b_p to z.
template <class T>
static rs_status cpr_rest_t(rs_cpr_s *M, T *z, hipStream_t s) {
  const grid3 &g = M->A->g;
  int64_t n = g.n;
  amg_level *L0 = M->lev[0];
  if (M->o.stages == 3) {
    T *y = M->fy.as<T>();
    RS_TRY(second_stage<T>(M, M->fzero.as<T>() + g.nxy, y, s));
    k_fpf_resid<T><<<rs_grid(4 * n), RS_BLOCK, 0, s>>>(n, g.nx, g.nxy, M->D->t7.as<T>(), y, M->rt.as<T>(),
                                                      L0->b.as<T>());
    RS_HIP(hipGetLastError());
  }
  RS_TRY(rs_vcycle_run(M, s));
  RS_TRY(second_stage<T>(M, L0->xp<T>(), z, s));
  if (M->o.stages == 3) {
    k_fpf_add<T><<<rs_grid(4 * n), RS_BLOCK, 0, s>>>(4 * n, M->fy.as<T>(), z);
    RS_HIP(hipGetLastError());
  }
  return RS_OK;
}

template <class T>
static rs_status cpr_apply_t(rs_cpr_s *M, const double *r, T *z, hipStream_t s) {
  RS_TRY(cpr_in_t<T>(M, r, s, nullptr, nullptr, nullptr));
  return cpr_rest_t<T>(M, z, s);
}

rs_status rs_cpr_apply_any(rs_cpr_s *M, const double *r, void *z, int zprec, hipStream_t s) {
  if (zprec != M->prec) return RS_E_ARG;
  return M->prec == 64 ? cpr_apply_t<double>(M, r, (double *)z, s) : cpr_apply_t<float>(M, r, (float *)z, s);
}

rs_status rs_cpr_apply_in(rs_cpr_s *M, const double *w, const double *d_h, double *v, const double *d_halt,
                          hipStream_t s) {
  if (!d_h || !v) return RS_E_ARG;
  return M->prec == 64 ? cpr_in_t<double>(M, w, s, d_h, v, d_halt) : cpr_in_t<float>(M, w, s, d_h, v, d_halt);
}

rs_status rs_cpr_apply_rest(rs_cpr_s *M, void *z, int zprec, hipStream_t s) {
  if (zprec != M->prec) return RS_E_ARG;
  return M->prec == 64 ? cpr_rest_t<double>(M, (double *)z, s) : cpr_rest_t<float>(M, (float *)z, s);
}

extern "C" rs_status rs_cpr_apply(rs_cpr M, const double *d_r, double *d_z, void *stream) {
  if (!M || !d_r || !d_z || d_r == d_z) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  if (M->prec == 64) {
    RS_TRY(cpr_apply_t<double>(M, d_r, d_z, s));
    return rs_dilu_check(M, s);
  }
  int64_t m = 4 * M->A->g.n;
  dbuf tmp;
  RS_TRY(tmp.alloc(sizeof(float) * m));
  RS_TRY(cpr_apply_t<float>(M, d_r, tmp.as<float>(), s));
  k_vec_to_f64<float><<<rs_grid(m), RS_BLOCK, 0, s>>>(m, tmp.as<float>(), d_z);
  RS_HIP(hipGetLastError());
  RS_HIP(hipStreamSynchronize(s));   // tmp is freed on return
  return rs_dilu_check(M, s);
}

extern "C" rs_status rs_cpr_smoother_get(rs_cpr M, double *h_dinv2) {
  if (!M || !h_dinv2) return RS_E_ARG;
  RS_HIP(hipDeviceSynchronize());
  int64_t m = 16 * M->A->g.n;
  if (M->prec == 64) {
    RS_HIP(hipMemcpy(h_dinv2, M->dinv2.p, sizeof(double) * m, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> t(m);
    RS_HIP(hipMemcpy(t.data(), M->dinv2.p, sizeof(float) * m, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < m; ++e) h_dinv2[e] = t[e];
  }
  return RS_OK;
}
