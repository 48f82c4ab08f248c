// bicgstab.hip -- right-preconditioned BiCGSTAB with M = CPR, the Krylov
// method the paper's experiments use (Section "Linear Solver" names it beside
// GMRES).  Textbook recurrence (van der Vorst, 1992) with p^ = M^{-1} p and
// s^ = M^{-1} s, so the residual it updates is the original system's:
//   rho_i = (r^, r),  p = r + (rho_i / rho_{i-1})(alpha / omega)(p - omega v)
//   v = A p^,  alpha = rho_i / (r^, v),  s = r - alpha v
//   t = A s^,  omega = (t, s) / (t, t),  x += alpha p^ + omega s^,  r = s - omega t
// One iteration is five launches besides the two CPR applications:
//   k_bcg_p      p = r + beta (p - omega v)                       (beta from device scalars)
//   SpMV         v = A p^  with the epilogue dot (r^, v)
//   k_bcg_s      s = r - alpha v in place of r, ||s||^2
//   SpMV         t = A s^  with the epilogue dots (t, s), (t, t)
//   k_bcg_xr     x += alpha p^ + omega s^, r = s - omega t, (r^, r), ||r||^2
// Every dot is reduced in two fixed-order stages, so a solve is bitwise
// reproducible.  alpha, beta and omega are formed on the device from the
// reduced dots; the host reads a few doubles twice per iteration (after s and
// after r) to test convergence and breakdown.  p^ and s^ are stored in the
// preconditioner's precision and read as stored, so v = A p^ and t = A s^
// hold for the stored vectors.
#include "rs_internal.h"
#include <math.h>
#include <string.h>

namespace {

constexpr int NBLK = 1024;   // blocks of the vector kernels (partials per dot)

// Device scalar block (doubles).
enum {
  B_RHO = 0,     // rho_i = (r^, r)
  B_RHOP,        // rho_{i-1}
  B_ALPHA,
  B_OMEGA,
  B_RV,          // (r^, v)
  B_SN,          // ||s||^2
  B_TS,          // (t, s)
  B_TT,          // (t, t)
  B_RN,          // ||r||^2
  B_TOTAL
};

// Two partials per workgroup (dots d0, d1) into part[k * NBLK + blockIdx.x].
template <int ND>
__device__ __forceinline__ void store_partials(double d0, double d1, double *__restrict__ part) {
  __shared__ double sh[2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double d[2] = {d0, d1};
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    double v = d[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[k][wv] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < ND)
    part[(int64_t)threadIdx.x * NBLK + blockIdx.x] =
        ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}

// out[k] = sum of part[k * stride + b], b < nparts, in a fixed order (one
// workgroup per dot).
__global__ __launch_bounds__(1024) void k_bcg_reduce(int nparts, int stride, const double *__restrict__ part,
                                                     double *__restrict__ out) {
  __shared__ double sh[1024];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) s += part[(int64_t)k * stride + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = sh[0];
}

// First stage for long partial lists (one per SpMV workgroup): block
// (c, k) sums part[k * stride + b] over its contiguous chunk of b in a fixed
// order, into mid[k * gridDim.x + c].
__global__ __launch_bounds__(256) void k_bcg_reduce_chunks(int nparts, int stride, const double *__restrict__ part,
                                                           double *__restrict__ mid) {
  __shared__ double sh[256];
  const int k = blockIdx.y, nc = gridDim.x, c = blockIdx.x;
  const int chunk = (nparts + nc - 1) / nc, b0 = c * chunk, b1 = min(nparts, b0 + chunk);
  double s = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) s += part[(int64_t)k * stride + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) mid[k * nc + c] = sh[0];
}

// The vector kernels take two consecutive entries per thread and step
// (16-byte loads; N = 4n is even), which streams markedly faster than one.
template <class TZ> struct pair_of;
template <> struct pair_of<double> {
  __device__ static double2 ld(const double *p, int64_t t) { return ((const double2 *)p)[t]; }
};
template <> struct pair_of<float> {
  __device__ static double2 ld(const float *p, int64_t t) {
    const float2 f = ((const float2 *)p)[t];
    return make_double2((double)f.x, (double)f.y);
  }
};

// partial ||b||^2
__global__ __launch_bounds__(256) void k_bcg_norm2(int64_t N, const double *__restrict__ b, double *__restrict__ part) {
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (N >> 1); t += (int64_t)NBLK * blockDim.x) {
    const double2 v = pair_of<double>::ld(b, t);
    acc = fma(v.x, v.x, acc);
    acc = fma(v.y, v.y, acc);
  }
  store_partials<1>(acc, 0.0, part);
}

__global__ void k_bcg_zero(int64_t N, double *__restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) x[t] = 0.0;
}

// start of a cycle: p = v = 0, rho_{i-1} = alpha = omega = 1, rho = ||r||^2
// (the shadow r^ is a copy of r, so (r^, r) = ||r||^2)
__global__ void k_bcg_start(int64_t N, double *__restrict__ p, double *__restrict__ v, double *__restrict__ S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) { p[t] = 0.0; v[t] = 0.0; }
  if (t == 0) {
    S[B_RHO] = S[B_RN];
    S[B_RHOP] = 1.0;
    S[B_ALPHA] = 1.0;
    S[B_OMEGA] = 1.0;
  }
}

// p = r + beta (p - omega v), beta = (rho / rho_prev) (alpha / omega)
__global__ __launch_bounds__(256) void k_bcg_p(int64_t N, const double *__restrict__ r, const double *__restrict__ v,
                                               double *__restrict__ p, const double *__restrict__ S) {
  const double beta = (S[B_RHO] / S[B_RHOP]) * (S[B_ALPHA] / S[B_OMEGA]), omega = S[B_OMEGA];
  double2 *p2 = (double2 *)p;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (N >> 1); t += (int64_t)gridDim.x * blockDim.x) {
    const double2 rv = pair_of<double>::ld(r, t), vv = pair_of<double>::ld(v, t);
    double2 pv = p2[t];
    pv.x = rv.x + beta * (pv.x - omega * vv.x);
    pv.y = rv.y + beta * (pv.y - omega * vv.y);
    p2[t] = pv;
  }
}

// alpha = rho / (r^, v);  s = r - alpha v (in place);  partial ||s||^2
__global__ __launch_bounds__(256) void k_bcg_s(int64_t N, double *__restrict__ r, const double *__restrict__ v,
                                               double *__restrict__ S, double *__restrict__ part) {
  const double alpha = S[B_RHO] / S[B_RV];
  double acc = 0.0;
  double2 *r2 = (double2 *)r;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (N >> 1); t += (int64_t)NBLK * blockDim.x) {
    const double2 vv = pair_of<double>::ld(v, t);
    double2 sv = r2[t];
    sv.x = sv.x - alpha * vv.x;
    sv.y = sv.y - alpha * vv.y;
    r2[t] = sv;
    acc = fma(sv.x, sv.x, acc);
    acc = fma(sv.y, sv.y, acc);
  }
  store_partials<1>(acc, 0.0, part);
  if (blockIdx.x == 0 && threadIdx.x == 0) S[B_ALPHA] = alpha;
}

// x += alpha p^ (the iteration stopped at s)
template <class TZ>
__global__ void k_bcg_xa(int64_t N, const TZ *__restrict__ ph, const double *__restrict__ S, double *__restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) x[t] = x[t] + S[B_ALPHA] * (double)ph[t];
}

// omega = (t, s) / (t, t);  x += alpha p^ + omega s^;  r = s - omega t;
// partials (r^, r) and ||r||^2.  (t, t) == 0 (breakdown) takes omega = 0:
// x += alpha p^ and r = s.
template <class TZ>
__global__ __launch_bounds__(256) void k_bcg_xr(int64_t N, const TZ *__restrict__ ph, const TZ *__restrict__ sh,
                                                const double *__restrict__ tv, const double *__restrict__ rh,
                                                double *__restrict__ r, double *__restrict__ x,
                                                const double *__restrict__ S, double *__restrict__ part) {
  const double alpha = S[B_ALPHA], omega = S[B_TT] != 0.0 ? S[B_TS] / S[B_TT] : 0.0;
  double a0 = 0.0, a1 = 0.0;
  double2 *x2 = (double2 *)x, *r2 = (double2 *)r;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (N >> 1); t += (int64_t)NBLK * blockDim.x) {
    const double2 pp = pair_of<TZ>::ld(ph, t), ss = pair_of<TZ>::ld(sh, t);
    const double2 tt = pair_of<double>::ld(tv, t), hh = pair_of<double>::ld(rh, t);
    double2 xv = x2[t], rv = r2[t];
    xv.x = xv.x + alpha * pp.x + omega * ss.x;
    xv.y = xv.y + alpha * pp.y + omega * ss.y;
    rv.x = rv.x - omega * tt.x;
    rv.y = rv.y - omega * tt.y;
    x2[t] = xv;
    r2[t] = rv;
    a0 = fma(hh.x, rv.x, a0);
    a0 = fma(hh.y, rv.y, a0);
    a1 = fma(rv.x, rv.x, a1);
    a1 = fma(rv.y, rv.y, a1);
  }
  store_partials<2>(a0, a1, part);
}

// after k_bcg_xr's dots are reduced: omega stored, rho_prev = rho, rho = (r^, r)
__global__ void k_bcg_next(double *__restrict__ S, const double *__restrict__ d) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  S[B_OMEGA] = S[B_TT] != 0.0 ? S[B_TS] / S[B_TT] : 0.0;
  S[B_RHOP] = S[B_RHO];
  S[B_RHO] = d[0];
  S[B_RN] = d[1];
}

}  // namespace

extern "C" void rs_bicgstab_opts_default(rs_bicgstab_opts *o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->maxit = 300;
  o->zero_guess = 0;
}

// out[k] = sum over b < nparts of part[k * stride + b], k < K, deterministic:
// one workgroup per dot for short lists, two stages (64 chunks) for the
// SpMV's one-partial-per-workgroup lists.
constexpr int RED_CHUNKS = 64;
static void bcg_reduce(int K, int nparts, int stride, const double *part, double *mid, double *out, hipStream_t s) {
  if (nparts <= 4096) {
    k_bcg_reduce<<<K, 1024, 0, s>>>(nparts, stride, part, out);
  } else {
    k_bcg_reduce_chunks<<<dim3(RED_CHUNKS, K), 256, 0, s>>>(nparts, stride, part, mid);
    k_bcg_reduce<<<K, 1024, 0, s>>>(RED_CHUNKS, RED_CHUNKS, mid, out);
  }
}

static rs_status bcg_read(double *h, const double *d, int cnt, hipStream_t s) {
  RS_HIP(hipMemcpyAsync(h, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));   // h is pinned
  return rs_wait(s);
}

template <class TZ>
static rs_status bicgstab_t(rs_bsr_s *A, rs_cpr_s *M, const double *b, double *x, const rs_bicgstab_opts &o,
                            rs_solve_info *info, hipStream_t s) {
  const int64_t N = 4 * A->g.n;
  const unsigned nsp = rs_spmv_blocks(A);
  const int zp = sizeof(TZ) == 8 ? 64 : 32;
  if (M->bprec != zp || !M->bvec.p) {
    RS_TRY(M->bvec.alloc(sizeof(double) * N * 5 + sizeof(TZ) * N * 2));
    RS_TRY(M->bpart.alloc(sizeof(double) * (2 * ((size_t)nsp > NBLK ? nsp : NBLK) + 2 * RED_CHUNKS)));
    RS_TRY(M->bscal.alloc(sizeof(double) * (B_TOTAL + 4)));
    M->bprec = zp;
  }
  double *r = M->bvec.as<double>(), *rh = r + N, *p = rh + N, *v = p + N, *tv = v + N;
  TZ *ph = (TZ *)(tv + N), *shv = ph + N;
  double *part = M->bpart.as<double>(), *S = M->bscal.as<double>(), *D = S + B_TOTAL;
  double *mid = part + 2 * ((size_t)nsp > NBLK ? nsp : NBLK);
  if (!M->bpin) RS_HIP(hipHostMalloc((void **)&M->bpin, sizeof(double) * B_TOTAL, hipHostMallocDefault));
  double *hp = M->bpin;
  hipEvent_t e0, e1;
  RS_HIP(hipEventCreate(&e0));
  RS_HIP(hipEventCreate(&e1));
  RS_HIP(hipEventRecord(e0, s));
  rs_status st = RS_OK;
  int iters = 0, cycles = 0;
  double relres = 0.0, est = 0.0;
  const unsigned gN = rs_grid(N);
  // host copy of the scalar block, refreshed twice per iteration
  double *h = hp;
  auto read_scalars = [&]() -> rs_status { return bcg_read(h, S, B_TOTAL, s); };
  // r = b - A x and ||r||^2 into S[B_RN]
  auto residual = [&]() -> rs_status {
    RS_TRY(rs_spmv_dots(A, x, 64, r, b, 1, nullptr, part, s));
    bcg_reduce(1, nsp, nsp, part, mid, S + B_RN, s);
    RS_HIP(hipGetLastError());
    return read_scalars();
  };
  do {
    k_bcg_norm2<<<NBLK, 256, 0, s>>>(N, b, part);
    bcg_reduce(1, NBLK, NBLK, part, mid, D, s);
    if ((st = bcg_read(h, D, 1, s)) != RS_OK) break;
    const double bnorm = sqrt(h[0]);
    if (!isfinite(bnorm)) { st = RS_E_NONFINITE; break; }
    if (bnorm == 0.0) {
      k_bcg_zero<<<gN, RS_BLOCK, 0, s>>>(N, x);
      relres = 0.0;
      break;
    }
    bool zero_start = o.zero_guess != 0;
    for (;;) {
      if (zero_start) {
        // x0 = 0: r = b and ||r||^2 = ||b||^2 (already reduced into D[0])
        k_bcg_zero<<<gN, RS_BLOCK, 0, s>>>(N, x);
        if (hipMemcpyAsync(r, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(S + B_RN, D, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
          st = RS_E_HIP;
          break;
        }
        if ((st = read_scalars()) != RS_OK) break;
        zero_start = false;
      } else if ((st = residual()) != RS_OK) {
        break;
      }
      const double rn = sqrt(h[B_RN]);
      relres = rn / bnorm;
      if (!isfinite(rn)) { st = RS_E_NONFINITE; break; }
      if (rn <= o.rtol * bnorm) { st = RS_OK; break; }
      if (iters >= o.maxit) { st = RS_NOT_CONVERGED; break; }
      ++cycles;
      if (hipMemcpyAsync(rh, r, sizeof(double) * N, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        st = RS_E_HIP;
        break;
      }
      k_bcg_start<<<gN, RS_BLOCK, 0, s>>>(N, p, v, S);
      double rho = h[B_RN];                  // (r^, r) with r^ = r
      bool first = true, stop_early = false;
      while (iters < o.maxit) {
        if (rho == 0.0) { stop_early = first; break; }
        k_bcg_p<<<NBLK, 256, 0, s>>>(N, r, v, p, S);
        if ((st = rs_cpr_apply_any(M, p, ph, zp, s)) != RS_OK) break;
        if ((st = rs_spmv_dots(A, ph, zp, v, nullptr, 1, rh, part, s)) != RS_OK) break;
        bcg_reduce(1, nsp, nsp, part, mid, S + B_RV, s);
        k_bcg_s<<<NBLK, 256, 0, s>>>(N, r, v, S, part);
        bcg_reduce(1, NBLK, NBLK, part, mid, S + B_SN, s);
        if ((st = read_scalars()) != RS_OK) break;
        if (h[B_RV] == 0.0) { stop_early = first; break; }   // r now holds garbage; x is untouched
        ++iters;
        const double sn = sqrt(h[B_SN]);
        est = sn;
        if (!isfinite(sn)) { st = RS_E_NONFINITE; break; }
        if (sn <= o.rtol * bnorm) {
          k_bcg_xa<TZ><<<gN, RS_BLOCK, 0, s>>>(N, ph, S, x);
          break;
        }
        if ((st = rs_cpr_apply_any(M, r, shv, zp, s)) != RS_OK) break;
        if ((st = rs_spmv_dots(A, shv, zp, tv, nullptr, 2, r, part, s)) != RS_OK) break;
        bcg_reduce(2, nsp, nsp, part, mid, S + B_TS, s);
        k_bcg_xr<TZ><<<NBLK, 256, 0, s>>>(N, ph, shv, tv, rh, r, x, S, part);
        bcg_reduce(2, NBLK, NBLK, part, mid, D, s);
        k_bcg_next<<<1, 64, 0, s>>>(S, D);
        if (hipGetLastError() != hipSuccess) { st = RS_E_HIP; break; }
        if ((st = read_scalars()) != RS_OK) break;
        if (h[B_TT] == 0.0) { stop_early = first; break; }   // x += alpha p^ was applied
        const double rnn = sqrt(h[B_RN]);
        est = rnn;
        rho = h[B_RHO];
        first = false;
        if (!isfinite(rnn)) break;
        if (rnn <= o.rtol * bnorm || h[B_OMEGA] == 0.0) break;
      }
      if (st != RS_OK) break;
      if (stop_early) {
        if ((st = residual()) != RS_OK) break;
        relres = sqrt(h[B_RN]) / bnorm;
        st = relres <= o.rtol ? RS_OK : RS_NOT_CONVERGED;
        break;
      }
    }
    est = bnorm > 0.0 ? est / bnorm : 0.0;
  } while (0);
  if (st == RS_OK || st == RS_NOT_CONVERGED) {
    rs_status e = rs_dilu_check(M, s);
    if (e != RS_OK) st = e;
  }
  float ms = 0.f;
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (info) {
    info->iters = iters;
    info->cycles = cycles;
    info->status = st;
    info->relres = relres;
    info->est_relres = est;
    info->ms = ms;
  }
  return st;
}

extern "C" rs_status rs_bicgstab_solve(rs_bsr A, rs_cpr M, const double *d_b, double *d_x,
                                       const rs_bicgstab_opts *o, rs_solve_info *info, void *stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (!A || !M || !d_b || !d_x || d_b == d_x || M->A != A) return RS_E_ARG;
  if (((uintptr_t)d_b | (uintptr_t)d_x) & 15) return RS_E_ARG;     // read 16 bytes at a time
  rs_bicgstab_opts opts;
  if (o) opts = *o; else rs_bicgstab_opts_default(&opts);
  if (opts.maxit < 0 || !(opts.rtol >= 0.0)) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  return M->prec == 64 ? bicgstab_t<double>(A, M, d_b, d_x, opts, info, s)
                       : bicgstab_t<float>(A, M, d_b, d_x, opts, info, s);
}
