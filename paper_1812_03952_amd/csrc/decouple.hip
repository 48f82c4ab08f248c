// decouple.hip -- ABF / quasi-IMPES / FRS / FRS+ABF decoupling and
// pressure-matrix extraction.
//
// Decoupling is a left scaling (D^{-1} A) x = D^{-1} b (Eq. decoupled-eq)
// applied block row by block row with Gauss-Jordan elimination and row
// pivoting only (Section "Decoupling Methods").  Eight lanes work on one
// block row: lane s < 7 carries block column s of [A_ii | A_i,s] through the
// elimination, lane 7 carries the identity and so produces D_i^{-1}.  Lane 3
// loads A_ii as its own slot and the group takes it from there by shuffle;
// every lane then repeats the (cheap) pivot sequence on A_ii itself, which
// keeps the lanes independent and the per-lane state at 32 doubles.  Row
// exchanges are written as selects over compile-time indices so nothing
// spills.
//
// FMA contraction is off in this file: each update is one multiply and one
// subtract, in the same order as the FP64 reference, so the FP64 pressure
// matrix used by the AMG setup does not depend on the compiler's choices.
#pragma clang fp contract(off)
#include "rs_internal.h"
#include <math.h>
#include <type_traits>

namespace {
#include "block4.h"
#include "csr7.h"

// Where a decoupling kernel reads block (s, c) of A from.
//   src7:  the library's 7-slot copy a7 (after rs_bsr_create/rs_bsr_update);
//   srcu:  the caller's row-major blocks in CSR order through the slot map
//          pos7 (-1 off the grid: a zero block), for rs_bsr_update_decouple:
//          the lane that owns slot s also stores the block into a7 and flags
//          non-finite entries, so the update and the decoupling are one pass;
//   srcr:  attached values, the caller's layout read in place at the
//          closed-form positions; the lane that owns slot s flags non-finite
//          entries when asked, nothing is stored.
struct src7 {
  const double *a7;
  int64_t n;
  __device__ __forceinline__ void block(int s, int64_t c, bool, double (&M)[4][4], int &) const {
    load16(a7 + ((int64_t)s * n + c) * 16, M);
  }
  __device__ __forceinline__ void commit(int64_t) const {}
};
struct srcr {
  const double *vals;
  uint32_t nx, ny, nz;
  bool check;                // flag non-finite entries (values that just arrived)
  __device__ __forceinline__ csr7_row row(int64_t c) const { return csr7_of((uint32_t)c, nx, ny, nz); }
  __device__ __forceinline__ void block(int s, int64_t c, bool own, double (&M)[4][4], int &f) const {
    const csr7_row w = row(c);
    load16(vals + 16 * (int64_t)csr7_pos(w, s), M);
    if (!((w.mask >> s) & 1u)) {
#pragma unroll
      for (int e = 0; e < 16; ++e) M[e >> 2][e & 3] = 0.0;
    }
    if (check && own) {
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (!isfinite(M[e >> 2][e & 3])) f |= RSF_NONFINITE;
    }
  }
  __device__ __forceinline__ void commit(int64_t) const {}
};
// The 32 cells of a workgroup (8 lanes each) stage their blocks in LDS;
// commit() then writes each of the 7 slot planes as one contiguous 4 KB run
// (one 16-byte store per thread) instead of 16-byte pieces 128 bytes apart.
// Every thread of the workgroup must call commit().
struct srcu {
  const double *vals;
  const int64_t *pos7;
  double *a7;
  int64_t n;
  __device__ static double (&stage())[7][32][16] {
    __shared__ double sa[7][32][16];
    return sa;
  }
  __device__ __forceinline__ void block(int s, int64_t c, bool store, double (&M)[4][4], int &f) const {
    const int64_t p = pos7[(int64_t)s * n + c];
    if (p >= 0) {
      load16(vals + 16 * p, M);
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) M[e >> 2][e & 3] = 0.0;
    }
    if (store) {
      double(&sa)[7][32][16] = stage();
      const int cl = threadIdx.x >> 3;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        sa[s][cl][e] = M[e >> 2][e & 3];
        if (!isfinite(M[e >> 2][e & 3])) f |= RSF_NONFINITE;
      }
    }
  }
  __device__ __forceinline__ void commit(int64_t c0) const {
    __syncthreads();
    double(&sa)[7][32][16] = stage();
    const int cl = threadIdx.x >> 3, part = threadIdx.x & 7;   // 32 cells x 8 double2 per plane
    if (c0 + cl < n) {
#pragma unroll
      for (int s = 0; s < 7; ++s)
        *(double2 *)(a7 + ((int64_t)s * n + c0 + cl) * 16 + 2 * part) =
            make_double2(sa[s][cl][2 * part], sa[s][cl][2 * part + 1]);
    }
  }
};

template <class T>
__device__ __forceinline__ void store_block(T *__restrict__ t7, double *__restrict__ ap7, int s, int64_t n,
                                            int64_t c, const double (&R)[4][4]) {
  T *o = t7 + ((int64_t)s * n + c) * 16;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) o[4 * r + q] = (T)R[r][q];
  ap7[(int64_t)s * n + c] = R[0][0];
}

// Column 0 of every block of the row, per block row: col0[c][row][8] (the 7
// slots, then a zero pad).  The 32 cells of a workgroup (8 lanes each, lane =
// slot) stage their entries in LDS and write them out as contiguous 16-byte
// chunks.  Every thread of the workgroup must call this.
template <class T>
__device__ __forceinline__ void store_col0(T *__restrict__ col0, int64_t n, int64_t c0, bool valid, int lane,
                                           const double (&R)[4][4]) {
  __shared__ T sh[32][32];
  const int cl = threadIdx.x >> 3;
  if (valid) {
#pragma unroll
    for (int r = 0; r < 4; ++r) sh[cl][8 * r + lane] = lane < 7 ? (T)R[r][0] : (T)0;
  }
  __syncthreads();
  const int64_t c = c0 + cl;
  if (c < n) {
    const int q = threadIdx.x & 7;            // 4 consecutive entries of the cell's 32
    T *dst = col0 + c * 32 + 4 * q;
    if constexpr (sizeof(T) == 4) {
      *(float4 *)dst = make_float4(sh[cl][4 * q], sh[cl][4 * q + 1], sh[cl][4 * q + 2], sh[cl][4 * q + 3]);
    } else {
      ((double2 *)dst)[0] = make_double2(sh[cl][4 * q], sh[cl][4 * q + 1]);
      ((double2 *)dst)[1] = make_double2(sh[cl][4 * q + 2], sh[cl][4 * q + 3]);
    }
  }
}

// ABF, and the two-stage FRS+ABF when FRS is set: row 0 of A_ii and of every
// block the lane carries (the identity too, which becomes F) is first
// replaced by the sum of the four rows, in row order.  R holds the lane's
// block of cell c as loaded (slot `lane`; the identity on lane 7) and leaves
// with the decoupled block.
template <class T, bool FRS>
__device__ __forceinline__ void abf_cell(int64_t n, int64_t c, bool valid, int lane, double (&R)[4][4], int fsrc,
                                         T *__restrict__ t7, T *__restrict__ dinv, double *__restrict__ ap7,
                                         int *__restrict__ flag) {
  double L[4][4];
  // A_ii is slot 3's block: taken from lane 3 of the cell's group
#pragma unroll
  for (int e = 0; e < 16; ++e) L[e >> 2][e & 3] = __shfl(R[e >> 2][e & 3], 3, 8);
  if (FRS) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      L[0][q] = ((L[0][q] + L[1][q]) + L[2][q]) + L[3][q];
      R[0][q] = ((R[0][q] + R[1][q]) + R[2][q]) + R[3][q];
    }
  }
  int f = gje4<4>(L, R);
  if (valid && lane == 0 && f) atomicOr(flag, f);
  if (fsrc) atomicOr(flag, fsrc);
  if (lane == 3) {      // A~_ii = I exactly
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) R[r][q] = (r == q) ? 1.0 : 0.0;
  }
  if (valid) {
    if (lane == 7) {
      T *o = dinv + c * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) o[4 * r + q] = (T)R[r][q];
    } else {
      store_block<T>(t7, ap7, lane, n, c, R);
    }
  }
}

template <class SRC>
__device__ __forceinline__ void abf_load(const SRC &src, int lane, int64_t c, bool valid, double (&R)[4][4],
                                         int &fsrc) {
  if (lane < 7) {
    src.block(lane, c, valid, R, fsrc);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) R[r][q] = (r == q) ? 1.0 : 0.0;
  }
}

template <class T, bool FRS, class SRC>
__global__ __launch_bounds__(256) void k_decouple_abf(int64_t n, SRC src,
                                                       T *__restrict__ t7, T *__restrict__ dinv,
                                                       double *__restrict__ ap7, T *__restrict__ col0,
                                                       int *__restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < 8 * n;                 // all threads stay for the block-wide col0 store
  const int64_t c = valid ? t >> 3 : n - 1;
  const int lane = (int)(t & 7);
  double R[4][4];
  int fsrc = 0;
  abf_load(src, lane, c, valid, R, fsrc);
  abf_cell<T, FRS>(n, c, valid, lane, R, fsrc, t7, dinv, ap7, flag);
  src.commit(((int64_t)blockIdx.x * blockDim.x) >> 3);
  store_col0<T>(col0, n, ((int64_t)blockIdx.x * blockDim.x) >> 3, valid, lane, R);
}

// K cells per lane group (the workgroup's 32 K cells as K runs of 32): every
// cell's blocks are loaded before the first is decoupled, so a wave has the
// loads of K cells in flight (K = 2 measured fastest: 1.26 ms against 1.35
// for one cell at 200x200x100 in FP32).  Sources that stage through LDS
// (srcu) take k_decouple_abf.
template <class T, bool FRS, class SRC, int K>
__global__ __launch_bounds__(256) void k_decouple_abfk(int64_t n, SRC src,
                                                        T *__restrict__ t7, T *__restrict__ dinv,
                                                        double *__restrict__ ap7, T *__restrict__ col0,
                                                        int *__restrict__ flag) {
  const int64_t c0 = (int64_t)blockIdx.x * (32 * K);
  const int lane = (int)(threadIdx.x & 7), cl = (int)(threadIdx.x >> 3);
  double R[K][4][4];
  int f[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t c = c0 + 32 * k + cl;
    f[k] = 0;
    abf_load(src, lane, c < n ? c : n - 1, c < n, R[k], f[k]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t c = c0 + 32 * k + cl;
    abf_cell<T, FRS>(n, c < n ? c : n - 1, c < n, lane, R[k], f[k], t7, dinv, ap7, flag);
    if (k > 0) __syncthreads();                 // the col0 stage is reused
    store_col0<T>(col0, n, c0 + 32 * k, c < n, lane, R[k]);
  }
}

// Quasi-IMPES: w_i solves A_ii^T w_i = e_0; row 0 of each block in row i
// becomes w_i^T A_ij; rows 1-3 stay; D_i^{-1} = [w_i^T; e_1^T; e_2^T; e_3^T].
template <class T, class SRC>
__global__ __launch_bounds__(256) void k_decouple_qi(int64_t n, SRC src,
                                                      T *__restrict__ t7, T *__restrict__ dinv,
                                                      double *__restrict__ ap7, T *__restrict__ col0,
                                                      int *__restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < 8 * n;                 // all threads stay for the block-wide col0 store
  const int64_t c = valid ? t >> 3 : n - 1;
  const int lane = (int)(t & 7);
  double L[4][4], w[4][1], A[4][4];
  int fsrc = 0;
  if (lane < 7) {
    src.block(lane, c, valid, A, fsrc);
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) A[e >> 2][e & 3] = 0.0;
  }
  // A_ii is slot 3's block: taken from lane 3 of the cell's group, transposed
#pragma unroll
  for (int e = 0; e < 16; ++e) L[e & 3][e >> 2] = __shfl(A[e >> 2][e & 3], 3, 8);
#pragma unroll
  for (int r = 0; r < 4; ++r) w[r][0] = (r == 0) ? 1.0 : 0.0;
  int f = gje4<1>(L, w);
  double R[4][4];
  if (valid && lane == 0 && f) atomicOr(flag, f);
  if (lane < 7) {
    if (fsrc) atomicOr(flag, fsrc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) s = s + w[m][0] * A[m][q];
      R[0][q] = s;
    }
#pragma unroll
    for (int r = 1; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) R[r][q] = A[r][q];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) R[r][q] = 0.0;
  }
  if (valid) {
    if (lane == 7) {
      T *o = dinv + c * 16;
#pragma unroll
      for (int e = 0; e < 16; ++e) o[e] = (T)0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = (T)w[q][0];
      o[5] = o[10] = o[15] = (T)1.0;
    } else {
      store_block<T>(t7, ap7, lane, n, c, R);
    }
  }
  src.commit(((int64_t)blockIdx.x * blockDim.x) >> 3);
  store_col0<T>(col0, n, ((int64_t)blockIdx.x * blockDim.x) >> 3, valid, lane, R);
}

// FRS (Eq. decoupled-frs): D_i^{-1} = F (ones in row 0 and on the
// diagonal): row 0 of every block becomes the sum of its four rows, in row
// order; rows 1-3 stay.
template <class T, class SRC>
__global__ __launch_bounds__(256) void k_decouple_frs(int64_t n, SRC src,
                                                       T *__restrict__ t7, T *__restrict__ dinv,
                                                       double *__restrict__ ap7, T *__restrict__ col0,
                                                       int *__restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < 8 * n;                 // all threads stay for the block-wide col0 store
  const int64_t c = valid ? t >> 3 : n - 1;
  const int lane = (int)(t & 7);
  double R[4][4];
  if (lane < 7) {
    int fsrc = 0;
    src.block(lane, c, valid, R, fsrc);
    if (fsrc) atomicOr(flag, fsrc);
#pragma unroll
    for (int q = 0; q < 4; ++q) R[0][q] = ((R[0][q] + R[1][q]) + R[2][q]) + R[3][q];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) R[r][q] = (r == 0 || r == q) ? 1.0 : 0.0;
  }
  if (valid) {
    if (lane == 7) {
      T *o = dinv + c * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) o[4 * r + q] = (T)R[r][q];
    } else {
      store_block<T>(t7, ap7, lane, n, c, R);
    }
  }
  src.commit(((int64_t)blockIdx.x * blockDim.x) >> 3);
  store_col0<T>(col0, n, ((int64_t)blockIdx.x * blockDim.x) >> 3, valid, lane, R);
}

}  // namespace

template <class SRC>
static void launch_decouple(int method, int prec, int64_t n, SRC src, rs_dcpl_s *D, int *fl, hipStream_t s) {
  const unsigned grid = rs_grid(8 * n);
  double *ap7 = D->ap7.as<double>();
#define RS_DC(KERN, T) KERN<<<grid, RS_BLOCK, 0, s>>>(n, src, D->t7.as<T>(), D->dinv.as<T>(), ap7, D->col0.as<T>(), fl)
  constexpr bool staged = std::is_same<SRC, srcu>::value;   // stages its blocks through LDS
  if (method == RS_ABF || method == RS_FRS_ABF) {
    const bool frs = method == RS_FRS_ABF;
    if constexpr (!staged) {
      // two cells per lane group, both loaded before either is decoupled
      const unsigned g2 = (unsigned)((n + 63) / 64);
#define RS_DK(T, F) k_decouple_abfk<T, F, SRC, 2><<<g2, RS_BLOCK, 0, s>>>(n, src, D->t7.as<T>(), D->dinv.as<T>(), ap7, D->col0.as<T>(), fl)
      if (prec == 64) { if (frs) RS_DK(double, true); else RS_DK(double, false); }
      else { if (frs) RS_DK(float, true); else RS_DK(float, false); }
#undef RS_DK
    } else {
      if (prec == 64) { if (frs) RS_DC((k_decouple_abf<double, true, SRC>), double); else RS_DC((k_decouple_abf<double, false, SRC>), double); }
      else { if (frs) RS_DC((k_decouple_abf<float, true, SRC>), float); else RS_DC((k_decouple_abf<float, false, SRC>), float); }
    }
  } else if (method == RS_QIMPES) {
    if (prec == 64) RS_DC((k_decouple_qi<double, SRC>), double);
    else RS_DC((k_decouple_qi<float, SRC>), float);
  } else {
    if (prec == 64) RS_DC((k_decouple_frs<double, SRC>), double);
    else RS_DC((k_decouple_frs<float, SRC>), float);
  }
#undef RS_DC
}

// vals == nullptr: decouple A's current values; else store vals (caller
// layout) into A and decouple them in the same pass, or with attach, make A
// refer to vals in place and decouple them.
static rs_status decouple_impl(rs_bsr_s *A, const double *vals, bool attach, int method, int prec, hipStream_t s,
                               rs_dcpl *out) {
  if (!A || !out || method < RS_ABF || method > RS_FRS_ABF || (prec != 32 && prec != 64))
    return RS_E_ARG;
  if (vals && ((uintptr_t)vals & 15)) return RS_E_ARG;     // block rows are read 16 bytes at a time
  *out = nullptr;
  int64_t n = A->g.n;
  size_t es = prec == 64 ? sizeof(double) : sizeof(float);
  rs_dcpl_s *D = new rs_dcpl_s();
  D->A = A; D->method = method; D->prec = prec;
  rs_status st = RS_OK;
  int h = 0;
  do {
    if ((st = D->t7.alloc(es * 7 * n * 16)) != RS_OK) break;
    if ((st = D->dinv.alloc(es * n * 16)) != RS_OK) break;
    if ((st = D->ap7.alloc(sizeof(double) * 7 * n)) != RS_OK) break;
    if ((st = D->col0.alloc(es * 32 * n)) != RS_OK) break;
    dbuf flag;
    if ((st = flag.alloc(sizeof(int))) != RS_OK) break;
    if (hipMemsetAsync(flag.p, 0, sizeof(int), s) != hipSuccess) { st = RS_E_HIP; break; }
    const grid3 &g = A->g;
    if (vals && attach) A->ref = vals;
    if (vals && !attach) {
      launch_decouple(method, prec, n, srcu{vals, A->pos7.as<int64_t>(), A->a7.as<double>(), n}, D, flag.as<int>(), s);
      A->ref = nullptr;
    } else if (A->ref) {
      // attached values are checked for finiteness when they arrive
      const srcr src{A->ref, (uint32_t)g.nx, (uint32_t)g.ny, (uint32_t)g.nz, vals != nullptr};
      launch_decouple(method, prec, n, src, D, flag.as<int>(), s);
    } else {
      launch_decouple(method, prec, n, src7{A->a7.as<double>(), n}, D, flag.as<int>(), s);
    }
    if (hipGetLastError() != hipSuccess || rs_wait_read(&h, flag.p, sizeof(int), s) != RS_OK) {
      st = RS_E_HIP;
      break;
    }
    if (h & RSF_NONFINITE) st = RS_E_NONFINITE;
    else if (h & RSF_SINGULAR) st = RS_E_SINGULAR;
  } while (0);
  if (st != RS_OK) { delete D; return st; }
  *out = D;
  return RS_OK;
}

extern "C" rs_status rs_decouple(rs_bsr A, int method, int prec, void *stream, rs_dcpl *out) {
  return decouple_impl(A, nullptr, false, method, prec, rs_stream(stream), out);
}

extern "C" rs_status rs_bsr_update_decouple(rs_bsr A, const double *d_vals, int method, int prec, void *stream,
                                            rs_dcpl *out) {
  if (!A || !d_vals || !out) return RS_E_ARG;
  rs_bsr_drop_adjoint(A);
  return decouple_impl(A, d_vals, false, method, prec, rs_stream(stream), out);
}

extern "C" rs_status rs_bsr_attach_decouple(rs_bsr A, const double *d_vals, int method, int prec, void *stream,
                                            rs_dcpl *out) {
  if (!A || !d_vals || !out) return RS_E_ARG;
  rs_bsr_drop_adjoint(A);
  return decouple_impl(A, d_vals, true, method, prec, rs_stream(stream), out);
}

extern "C" void rs_dcpl_destroy(rs_dcpl D) { delete D; }

rs_status rs_from7_host(const rs_bsr_s *A, const void *a7, int prec, double *h_vals);

extern "C" rs_status rs_dcpl_get(rs_dcpl D, double *h_vals, double *h_dinv) {
  if (!D) return RS_E_ARG;
  RS_HIP(hipDeviceSynchronize());
  if (h_vals) RS_TRY(rs_from7_host(D->A, D->t7.p, D->prec, h_vals));
  if (h_dinv) {
    int64_t n = D->A->g.n;
    if (D->prec == 64) {
      RS_HIP(hipMemcpy(h_dinv, D->dinv.p, sizeof(double) * 16 * n, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp(16 * n);
      RS_HIP(hipMemcpy(tmp.data(), D->dinv.p, sizeof(float) * 16 * n, hipMemcpyDeviceToHost));
      for (int64_t e = 0; e < 16 * n; ++e) h_dinv[e] = tmp[e];
    }
  }
  return RS_OK;
}
