// gmres.hip -- restarted, right-preconditioned flexible GMRES (the Krylov
// solver of Section "Linear Solver"), Arnoldi by classical Gram-Schmidt
// applied twice (CGS2), Givens rotations on the device.
//
// One Arnoldi step j after z_j = M^{-1} v_j and w = A z_j makes three passes
// over the basis, each reading every v_i (i <= j) once:
//   pass 1  h1 = V^T w,  ||w||^2
//   pass 2  h2 = V^T (w - V h1)            (w - V h1 in registers only)
//   pass 3  w = (w - V h1) - V h2;  ||w||^2
// which is classical Gram-Schmidt applied twice, with the same operations
// per entry as updating w in place after each pass.
// followed by one single-thread kernel that forms h = h1 + h2, applies the
// previous rotations, builds the new one and updates g, and a normalisation
// v_{j+1} = w / h_{j+1,j} that reads h_{j+1,j} from device memory.  Every
// dot is reduced in two deterministic stages (fixed per-block partials, then
// a fixed-order sum), so a solve is bitwise reproducible.  The host reads
// one 3-double status word per step to decide whether to stop.
// Z (the preconditioned vectors of flexible GMRES) is stored in the
// preconditioner's precision; the SpMV and x += Z y read it as stored, so
// A Z = V H holds for the stored Z and x stays consistent in FP32 mode.
#include "rs_internal.h"
#include <math.h>
#include <string.h>

namespace {

constexpr int NBLK = 1024;     // blocks of the dot kernels (partials per dot)

template <int MK, class TV>
__device__ __forceinline__ void block_store_partials(double (&acc)[MK + 1], int K, bool norm,
                                                     double *__restrict__ part) {
  __shared__ double sh[4][MK + 1];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= MK; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wv][k] = v;
  }
  __syncthreads();
  int k = threadIdx.x;
  if (k < K || (norm && k == MK)) {
    double v = sh[0][k] + sh[1][k] + sh[2][k] + sh[3][k];
    int slot = (k == MK) ? K : k;
    part[(int64_t)slot * NBLK + blockIdx.x] = v;
  }
}

// pass 1: part[k] = V_k . w (k < K), part[K] = w . w.  Two consecutive
// entries per thread and step (16-byte loads; N = 4n is even): at 1024
// workgroups this streams about 1.5x faster than one entry per step.
template <int MK>
__global__ __launch_bounds__(256) void k_dots(int64_t N, int K, const double *__restrict__ V,
                                               const double *__restrict__ w, double *__restrict__ part) {
  double acc[MK + 1];
#pragma unroll
  for (int k = 0; k <= MK; ++k) acc[k] = 0.0;
  const int64_t N2 = N >> 1;
  const double2 *w2 = (const double2 *)w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N2; t += (int64_t)NBLK * blockDim.x) {
    const double2 wv = w2[t];
#pragma unroll
    for (int k = 0; k < MK; ++k)
      if (k < K) {
        const double2 v = ((const double2 *)(V + (int64_t)k * N))[t];
        acc[k] = fma(v.x, wv.x, acc[k]);
        acc[k] = fma(v.y, wv.y, acc[k]);
      }
    acc[MK] = fma(wv.x, wv.x, acc[MK]);
    acc[MK] = fma(wv.y, wv.y, acc[MK]);
  }
  block_store_partials<MK, double>(acc, K, true, part);
}

// pass 2 (PASS3 = false): w' = w - sum_k h1[k] V_k formed in registers only,
//   part[k] = V_k . w', part[K] = w' . w'  (read-only: w is not written)
// pass 3 (PASS3 = true): w' formed again with the same operations, then
//   w'' = w' - sum_k h2[k] V_k stored into w, part[0] = w'' . w''
// Keeping pass 2 read-only saves a vector write per Arnoldi step, and a
// kernel that both streams several vectors in and one out runs slower
// than a read-only one; the arithmetic is that of updating w in place.
template <int MK, bool PASS3>
__global__ __launch_bounds__(256) void k_axpy_dots(int64_t N, int K, const double *__restrict__ V,
                                                    const double *__restrict__ h1, const double *__restrict__ h2,
                                                    double *__restrict__ w, double *__restrict__ part) {
  double acc[MK + 1];
#pragma unroll
  for (int k = 0; k <= MK; ++k) acc[k] = 0.0;
  double g1[MK], g2[MK];
#pragma unroll
  for (int k = 0; k < MK; ++k) {
    g1[k] = (k < K) ? h1[k] : 0.0;
    g2[k] = (PASS3 && k < K) ? h2[k] : 0.0;
  }
  const int64_t N2 = N >> 1;
  double2 *w2 = (double2 *)w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N2; t += (int64_t)NBLK * blockDim.x) {
    double2 vk[MK];
    double2 wv = w2[t];
#pragma unroll
    for (int k = 0; k < MK; ++k) {
      vk[k] = (k < K) ? ((const double2 *)(V + (int64_t)k * N))[t] : make_double2(0.0, 0.0);
      wv.x = fma(-g1[k], vk[k].x, wv.x);
      wv.y = fma(-g1[k], vk[k].y, wv.y);
    }
    if (PASS3) {
#pragma unroll
      for (int k = 0; k < MK; ++k) {
        wv.x = fma(-g2[k], vk[k].x, wv.x);
        wv.y = fma(-g2[k], vk[k].y, wv.y);
      }
      w2[t] = wv;
    } else {
#pragma unroll
      for (int k = 0; k < MK; ++k)
        if (k < K) {
          acc[k] = fma(vk[k].x, wv.x, acc[k]);
          acc[k] = fma(vk[k].y, wv.y, acc[k]);
        }
    }
    acc[MK] = fma(wv.x, wv.x, acc[MK]);
    acc[MK] = fma(wv.y, wv.y, acc[MK]);
  }
  block_store_partials<MK, double>(acc, PASS3 ? 0 : K, true, part);
}

// out[k] = sum over blocks of part[k] in a fixed order, k < K
__global__ void k_reduce(int K, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double sh[256];
  int k = blockIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < NBLK; b += blockDim.x) s += part[(int64_t)k * NBLK + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = sh[0];
}

// Device scalar block layout (doubles):
enum {
  S_H1 = 0,            // 64: pass-1 dots, [j+1] = ||w||^2 before orthogonalisation
  S_H2 = 64,           // 64: pass-2 dots
  S_NRM = 128,         // ||w||^2 after pass 3
  S_HN = 129,          // h_{j+1,j}
  S_BETA = 130,        // norm of the residual at the cycle start
  S_STAT = 132,        // [0] |g_{j+1}|, [1] breakdown flag, [2] halt flag
  S_G = 136,           // 65: rotated rhs g
  S_CS = 208,          // 64
  S_SN = 272,          // 64
  S_Y = 336,           // 64
  S_H = 400,           // (m+1) x m Hessenberg, row-major with leading dim 64
  S_TOTAL = 400 + 65 * 64
};

// tol: the stopping bound on |g_{j+1}|; S_STAT[2] = 1 when the solve stops
// after this step (converged, broken down or not finite), else 0
__global__ void k_givens(int j, double *__restrict__ S, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double *H = S + S_H, *g = S + S_G, *cs = S + S_CS, *sn = S + S_SN;
  double wn0 = sqrt(S[S_H1 + j + 1]);
  double hn = sqrt(S[S_NRM]);
  for (int i = 0; i <= j; ++i) H[i * 64 + j] = (0.0 + S[S_H1 + i]) + S[S_H2 + i];
  H[(j + 1) * 64 + j] = hn;
  S[S_HN] = hn;
  for (int i = 0; i < j; ++i) {
    double a = H[i * 64 + j], c = H[(i + 1) * 64 + j];
    H[i * 64 + j] = cs[i] * a + sn[i] * c;
    H[(i + 1) * 64 + j] = -sn[i] * a + cs[i] * c;
  }
  double a = H[j * 64 + j], c = H[(j + 1) * 64 + j];
  double d = hypot(a, c);
  cs[j] = a / d;
  sn[j] = c / d;
  H[j * 64 + j] = d;
  H[(j + 1) * 64 + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  const double est = fabs(g[j + 1]);
  const bool brk = hn <= 1e-14 * wn0;
  S[S_STAT + 0] = est;
  S[S_STAT + 1] = brk ? 1.0 : 0.0;
  S[S_STAT + 2] = (brk || !(est > tol) || isinf(est)) ? 1.0 : 0.0;
}

__global__ void k_init_cycle(double *__restrict__ S, double beta) {
  int t = threadIdx.x;
  if (t < 65) S[S_G + t] = (t == 0) ? beta : 0.0;
  if (t == 0) S[S_BETA] = beta;
}

__global__ void k_backsolve(int k, double *__restrict__ S) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double *H = S + S_H, *g = S + S_G, *y = S + S_Y;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s = s - H[i * 64 + c] * y[c];
    y[i] = s / H[i * 64 + i];
  }
}

// v = w / S[idx] (device scalar) or w / beta (host scalar when idx < 0)
__global__ void k_scale(int64_t N, const double *w, const double *__restrict__ S, int idx,
                        double beta, double *v) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double d = idx >= 0 ? S[idx] : beta;
  v[t] = w[t] / d;
}

__global__ void k_zero(int64_t N, double *__restrict__ x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) x[t] = 0.0;
}

template <class TZ>
__global__ void k_update_x(int64_t N, int k, const TZ *__restrict__ Z, const double *__restrict__ S,
                           double *__restrict__ x, int x_zero) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double *y = S + S_Y;
  double v = x_zero ? 0.0 : x[t];                // x_zero: x = 0, not yet written
  for (int i = 0; i < k; ++i) v = fma(y[i], (double)Z[(int64_t)i * N + t], v);
  x[t] = v;
}

}  // namespace

extern "C" void rs_gmres_opts_default(rs_gmres_opts *o) {
  if (!o) return;
  o->restart = 30;
  o->rtol = 1e-8;
  o->maxit = 300;
  o->zero_guess = 0;
}

extern "C" const char *rs_status_string(int st) {
  switch (st) {
    case RS_OK: return "ok";
    case RS_NOT_CONVERGED: return "not converged (maximum iterations reached)";
    case RS_E_ARG: return "invalid argument";
    case RS_E_HIP: return "HIP runtime error";
    case RS_E_NOMEM: return "device memory allocation failed";
    case RS_E_SINGULAR: return "singular block or coarsest matrix";
    case RS_E_NONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

// dots of V_0..V_{K-1} (K may be 0) with w, plus ||w||^2 into S[off + K]
static rs_status run_dots(int64_t N, int K, const double *V, const double *w, double *part, double *S,
                          int off, hipStream_t s) {
  if (K <= 8) k_dots<8><<<NBLK, 256, 0, s>>>(N, K, V, w, part);
  else if (K <= 16) k_dots<16><<<NBLK, 256, 0, s>>>(N, K, V, w, part);
  else k_dots<32><<<NBLK, 256, 0, s>>>(N, K, V, w, part);
  k_reduce<<<K + 1, 256, 0, s>>>(K + 1, part, S + off);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

template <bool PASS3>
static rs_status run_axpy(int64_t N, int K, const double *V, const double *h1, const double *h2, double *w,
                          double *part, double *S, int off, hipStream_t s) {
  if (K <= 8) k_axpy_dots<8, PASS3><<<NBLK, 256, 0, s>>>(N, K, V, h1, h2, w, part);
  else if (K <= 16) k_axpy_dots<16, PASS3><<<NBLK, 256, 0, s>>>(N, K, V, h1, h2, w, part);
  else k_axpy_dots<32, PASS3><<<NBLK, 256, 0, s>>>(N, K, V, h1, h2, w, part);
  int nout = PASS3 ? 1 : K + 1;
  k_reduce<<<nout, 256, 0, s>>>(nout, part, S + off);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

static rs_status read_host(double *h, const double *d, int cnt, hipStream_t s) {
  RS_HIP(hipMemcpyAsync(h, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));   // h is pinned
  return rs_wait(s);
}

template <class TZ>
static rs_status gmres_t(rs_bsr_s *A, rs_cpr_s *M, const double *b, double *x, const rs_gmres_opts &o,
                         rs_solve_info *info, hipStream_t s) {
  int64_t N = 4 * A->g.n;
  int m = o.restart;
  if (M->m != m || !M->V.p) {
    RS_TRY(M->V.alloc(sizeof(double) * N * (m + 1)));
    RS_TRY(M->Z.alloc(sizeof(TZ) * N * m));
    RS_TRY(M->w.alloc(sizeof(double) * N));
    RS_TRY(M->part.alloc(sizeof(double) * NBLK * 66));
    RS_TRY(M->scal.alloc(sizeof(double) * S_TOTAL));
    M->m = m;
  }
  double *V = M->V.as<double>(), *w = M->w.as<double>(), *part = M->part.as<double>(), *S = M->scal.as<double>();
  TZ *Z = M->Z.as<TZ>();
  if (!M->hpin) RS_HIP(hipHostMalloc((void **)&M->hpin, sizeof(double) * 8, hipHostMallocDefault));
  struct { double *p; } hb = {M->hpin};
  hipEvent_t e0, e1, es;
  RS_HIP(hipEventCreate(&e0));
  RS_HIP(hipEventCreate(&e1));
  RS_HIP(hipEventCreateWithFlags(&es, hipEventDisableTiming));
  RS_HIP(hipEventRecord(e0, s));
  rs_status st = RS_OK;
  int iters = 0, cycles = 0;
  double relres = 0.0, est = 0.0;
  unsigned gN = rs_grid(N);
  do {
    // ||b||
    if ((st = run_dots(N, 0, V, b, part, S, S_NRM, s)) != RS_OK) break;
    if ((st = read_host(hb.p, S + S_NRM, 1, s)) != RS_OK) break;
    double bnorm = sqrt(hb.p[0]);
    if (!isfinite(bnorm)) { st = RS_E_NONFINITE; break; }
    if (bnorm == 0.0) {
      if (hipMemsetAsync(x, 0, sizeof(double) * N, s) != hipSuccess) st = RS_E_HIP;
      relres = 0.0;
      break;
    }
    bool zero_start = o.zero_guess != 0;
    bool x_zero = false;                         // x = 0 is implied, not stored
    for (;;) {
      double beta;
      if (zero_start) {
        // x0 = 0: r0 = b, ||r0|| = ||b||, V_0 = b / ||b|| (the k_scale below)
        x_zero = true;
        beta = bnorm;
      } else {
        // r = b - A x into V_0
        if ((st = rs_spmv_any(A, x, 64, V, b, s)) != RS_OK) break;
        if ((st = run_dots(N, 0, V, V, part, S, S_NRM, s)) != RS_OK) break;
        if ((st = read_host(hb.p, S + S_NRM, 1, s)) != RS_OK) break;
        beta = sqrt(hb.p[0]);
      }
      relres = beta / bnorm;
      if (!isfinite(beta)) { st = RS_E_NONFINITE; break; }
      if (beta <= o.rtol * bnorm) { st = RS_OK; break; }
      if (iters >= o.maxit) { st = RS_NOT_CONVERGED; break; }
      // V_0 = r0 / beta: from x0 = 0 (r0 = b) the preconditioner's first pass
      // forms it (with beta from S_BETA); a restart's residual is in V_0
      // itself and is scaled in place
      const bool v0_fused = zero_start;
      if (!v0_fused) k_scale<<<gN, RS_BLOCK, 0, s>>>(N, V, S, -1, beta, V);
      zero_start = false;
      k_init_cycle<<<1, 128, 0, s>>>(S, beta);
      ++cycles;
      const double tol = o.rtol * bnorm;
      const int zp = sizeof(TZ) == 8 ? 64 : 32;
      int k = 0;
      bool in_queued = false;                    // step j's first pass is already on the stream
      for (int j = 0; j < m; ++j) {
        double *vj = V + (int64_t)j * N;
        TZ *zj = Z + (int64_t)j * N;
        // V_j = w / h_{j,j-1} is formed by the preconditioner's first pass
        if (j == 0 && !v0_fused) {
          st = rs_cpr_apply_any(M, vj, zj, zp, s);
        } else {
          if (!in_queued) st = rs_cpr_apply_in(M, j > 0 ? w : b, S + (j > 0 ? S_HN : S_BETA), vj, nullptr, s);
          if (st == RS_OK) st = rs_cpr_apply_rest(M, zj, zp, s);
        }
        if (st != RS_OK) break;
        if ((st = rs_spmv_any(A, zj, zp, w, nullptr, s)) != RS_OK) break;
        if ((st = run_dots(N, j + 1, V, w, part, S, S_H1, s)) != RS_OK) break;
        if ((st = run_axpy<false>(N, j + 1, V, S + S_H1, nullptr, w, part, S, S_H2, s)) != RS_OK) break;
        if ((st = run_axpy<true>(N, j + 1, V, S + S_H1, S + S_H2, w, part, S, S_NRM, s)) != RS_OK) break;
        k_givens<<<1, 64, 0, s>>>(j, S, tol);
        if (hipGetLastError() != hipSuccess) { st = RS_E_HIP; break; }
        ++iters;
        k = j + 1;
        // the status goes to the host while the device already runs the next
        // step's first pass, which does nothing if k_givens set the halt flag
        // (the host stops on the same values)
        if (hipMemcpyAsync(hb.p, S + S_STAT, sizeof(double) * 2, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipEventRecord(es, s) != hipSuccess) { st = RS_E_HIP; break; }
        in_queued = j + 1 < m && iters < o.maxit;
        if (in_queued && (st = rs_cpr_apply_in(M, w, S + S_HN, vj + N, S + S_STAT + 2, s)) != RS_OK) break;
        if (hipEventSynchronize(es) != hipSuccess) { st = RS_E_HIP; break; }
        est = hb.p[0];
        if (!isfinite(est)) { st = RS_E_NONFINITE; break; }
        if (hb.p[1] != 0.0) break;                               // happy breakdown
        if (est <= tol || iters >= o.maxit) break;
      }
      if (st != RS_OK) break;
      k_backsolve<<<1, 64, 0, s>>>(k, S);
      k_update_x<TZ><<<gN, RS_BLOCK, 0, s>>>(N, k, Z, S, x, x_zero ? 1 : 0);
      x_zero = false;
      if (hipGetLastError() != hipSuccess) { st = RS_E_HIP; break; }
    }
    if (x_zero) k_zero<<<gN, RS_BLOCK, 0, s>>>(N, x);   // stopped before any update
    est = (bnorm > 0.0) ? est / bnorm : 0.0;
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
  (void)hipEventDestroy(es);
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

extern "C" rs_status rs_gmres_solve(rs_bsr A, rs_cpr M, const double *d_b, double *d_x,
                                    const rs_gmres_opts *o, rs_solve_info *info, void *stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (!A || !M || !d_b || !d_x || d_b == d_x || M->A != A) return RS_E_ARG;
  if (((uintptr_t)d_b | (uintptr_t)d_x) & 15) return RS_E_ARG;     // read 16 bytes at a time
  rs_gmres_opts opts;
  if (o) opts = *o; else rs_gmres_opts_default(&opts);
  if (opts.restart < 1 || opts.restart > 32 || opts.maxit < 0 || !(opts.rtol >= 0.0)) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  return M->prec == 64 ? gmres_t<double>(A, M, d_b, d_x, opts, info, s)
                       : gmres_t<float>(A, M, d_b, d_x, opts, info, s);
}

extern "C" rs_status rs_adjoint_solve(rs_bsr A, int method, int prec, const rs_cpr_opts *co,
                                      const double *d_w, double *d_lambda, const rs_gmres_opts *o,
                                      rs_solve_info *info, void *stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (!A || !d_w || !d_lambda || (((uintptr_t)d_w | (uintptr_t)d_lambda) & 15)) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  rs_cpr_opts opts;
  if (co) opts = *co; else rs_cpr_opts_default(&opts);
  bool same = A->at_m && A->at_method == method && A->at_prec == prec &&
              memcmp(&A->at_opts, &opts, sizeof(opts)) == 0;
  if (!same) {
    if (A->at_m) { rs_cpr_destroy(A->at_m); A->at_m = nullptr; }
    if (A->at_d) { rs_dcpl_destroy(A->at_d); A->at_d = nullptr; }
    if (!A->at) {
      A->at = new rs_bsr_s();
      rs_status st = rs_transpose7(A, A->at, s);
      if (st != RS_OK) { delete A->at; A->at = nullptr; return st; }
    }
    RS_TRY(rs_decouple(A->at, method, prec, stream, &A->at_d));
    rs_status st = rs_cpr_setup(A->at, A->at_d, &opts, stream, &A->at_m);
    if (st != RS_OK) { rs_dcpl_destroy(A->at_d); A->at_d = nullptr; return st; }
    A->at_method = method; A->at_prec = prec; A->at_opts = opts;
  }
  return rs_gmres_solve(A->at, A->at_m, d_w, d_lambda, o, info, stream);
}
