// bsr.hip -- block matrix ingestion, 7-slot device layout, SpMV, transpose.
//
// Device layout of A: seven planes of 4x4 blocks, one per stencil slot in
// ascending column order (-z, -y, -x, self, +x, +y, +z), each plane [n][16]
// doubles.  Blocks that would couple across the grid boundary are stored as
// zeros, so every kernel walks the same fixed stencil with no column
// indices: the SpMV reads 7*128 B of matrix per cell in fully coalesced
// 32-byte pieces (four lanes per cell, one block row each) and never reads a
// column index.  The padding costs (7n - nnzb)/nnzb, 0.6% at 200x200x100.
//
// Attached values (rs_bsr_attach_decouple) stay in the caller's CSR layout;
// the SpMV then finds each block from the closed-form row start of csr7.h,
// with the same 32-byte row pieces and the same arithmetic.
#include "rs_internal.h"
#include <algorithm>
#include <math.h>

namespace {
#include "csr7.h"

__device__ __forceinline__ int64_t slot_nbr(int64_t c, int s, int64_t nx, int64_t nxy) {
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

// Does slot s of cell (i,j,k) lie inside the grid?
__device__ __forceinline__ bool slot_in(int s, int i, int j, int k, int nx, int ny, int nz) {
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

// Validate the caller pattern row by row and record, for each (slot, cell),
// the caller block index (or -1 off-grid).
__global__ void k_validate(int nx, int ny, int nz, int64_t nnzb, const int32_t *__restrict__ rp,
                           const int32_t *__restrict__ ci, int64_t *__restrict__ pos7,
                           int *__restrict__ bad) {
  int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
  int64_t p = rp[c], end = rp[c + 1];
  int err = 0;
  if (c == 0 && p != 0) err = 1;
  if (c == n - 1 && end != nnzb) err = 1;
  if (p < 0 || end < p || end > nnzb) err = 1;      // no column index is read outside [0, nnzb)
  for (int s = 0; s < 7; ++s) {
    int64_t q = -1;
    if (slot_in(s, i, j, k, nx, ny, nz)) {
      if (err == 0 && p < end && ci[p] == (int32_t)slot_nbr(c, s, nx, nxy)) q = p++;
      else err = 1;
    }
    pos7[s * n + c] = q;
  }
  if (p != end) err = 1;
  // the closed-form row start the kernels on attached values rely on
  if (rp[c] != (int32_t)csr7_of((uint32_t)c, (uint32_t)nx, (uint32_t)ny, (uint32_t)nz).start) err = 1;
  if (err) atomicOr(bad, 1);
}

// Scatter caller-layout block values into the 7-slot layout (zeros off-grid),
// one block row (32 bytes) per thread.
__global__ __launch_bounds__(256) void k_to7(int64_t n, const int64_t *__restrict__ pos7,
                                             const double *__restrict__ vals, double *__restrict__ a7,
                                             int *__restrict__ bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 7 * n * 4) return;
  int64_t sc = t >> 2;
  int r = (int)(t & 3);
  int64_t p = pos7[sc];
  double2 v0 = make_double2(0.0, 0.0), v1 = v0;
  if (p >= 0) {
    const double2 *src = (const double2 *)(vals + 16 * p + 4 * r);
    v0 = src[0]; v1 = src[1];
    if (!(isfinite(v0.x) && isfinite(v0.y) && isfinite(v1.x) && isfinite(v1.y))) atomicOr(bad, 2);
  }
  double2 *dst = (double2 *)(a7 + 4 * t);
  dst[0] = v0; dst[1] = v1;
}

typedef double v2d __attribute__((ext_vector_type(2)));

template <class T> struct vec4_of;
template <> struct vec4_of<double> {
  __device__ static void load(const double *p, double v[4]) {
    const double2 *q = (const double2 *)p;
    double2 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};
template <> struct vec4_of<float> {
  __device__ static void load(const float *p, double v[4]) {
    float4 a = *(const float4 *)p;
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
};

// y = A x  or  y = b - A x.  Four lanes per cell, lane r owns block row r:
// for each of the 7 slots it loads 32 contiguous bytes of A (the 4 entries of
// row r) and the 4 unknowns of the neighbour (shared by the 4 lanes, served
// by the L1/L2).  FP64 accumulation; x may be FP64 or FP32.
// ND > 0 adds dot products of the result as an epilogue, one deterministic
// partial per workgroup in part[d * gridDim.x + blockIdx.x]:
//   ND = 1:  d0 = y . u   (u == nullptr: y . y)
//   ND = 2:  d0 = y . u,  d1 = y . y
// so a Krylov step gets (r^, v) or (t, s) and (t, t) without re-reading y.
// CSR: a7 is the caller's row-major blocks in CSR order (attached values);
// an off-grid slot reads the row's diagonal block and zeroes it, so both
// layouts give the same products in the same order.
// Without dot products (ND = 0) the cells are handed out in row bands, one
// per XCD: workgroup i runs on XCD i % 8 (round-robin dispatch) and takes the
// (i / 8)-th run of 64 cells of band i % 8, the rows j in
// [x ny / 8, (x + 1) ny / 8) of every plane.  A cell's +-x, +-y and +-z
// neighbours are then mostly in the same band, so x is fetched into one L2
// instead of several (the results do not depend on the mapping; the grid is
// spmv_band_grid).  With dot products the natural order keeps each
// workgroup's partial over the same cells as before.
__host__ __device__ inline int64_t spmv_band_rows(int ny, int b) { return (int64_t)(b + 1) * ny / 8 - (int64_t)b * ny / 8; }

template <class TX, bool RES, int ND, bool CSR>
__global__ __launch_bounds__(256) void k_spmv7(int64_t n, int ny, int nz, int64_t nx, int64_t nxy,
                                                const double *__restrict__ a7,
                                                const TX *__restrict__ x,
                                                const double *__restrict__ b,
                                                double *__restrict__ y,
                                                const double *__restrict__ u,
                                                double *__restrict__ part) {
  int64_t t;
  bool valid;
  if constexpr (ND == 0) {
    const int xb = (int)(blockIdx.x & 7u);
    const uint32_t m = (blockIdx.x >> 3) * 64u + (threadIdx.x >> 2);        // cell within the band
    const uint32_t j0 = (uint32_t)((int64_t)xb * ny / 8);
    const uint32_t band = (uint32_t)(spmv_band_rows(ny, xb) * nx);          // cells of the band per plane
    valid = band > 0 && m < band * (uint32_t)nz;                              // n < 2^31
    const uint32_t k = valid ? m / band : 0, in = valid ? m - k * band : 0;
    t = 4 * ((int64_t)k * nxy + (int64_t)j0 * nx + in) + (threadIdx.x & 3);
  } else {
    t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    valid = t < 4 * n;
  }
  double yv = 0.0;
  if (valid) {
    int64_t c = t >> 2;
    int r = (int)(t & 3);
    double acc = 0.0;
    csr7_row w = {0, 0};
    if (CSR) w = csr7_of((uint32_t)c, (uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      int64_t q = slot_nbr(c, s, nx, nxy);
      q = (q < 0 || q >= n) ? c : q;           // off-grid blocks are zero
      const int64_t blk = CSR ? (int64_t)csr7_pos(w, s) : (int64_t)s * n + c;
      const v2d *ap = (const v2d *)(a7 + blk * 16 + 4 * r);
      // plain loads: the non-temporal hint measured about 8 points of HBM
      // bandwidth slower here
      v2d a01 = ap[0];
      v2d a23 = ap[1];
      if (CSR && !((w.mask >> s) & 1u)) { a01 = v2d{0.0, 0.0}; a23 = a01; }
      double xv[4];
      vec4_of<TX>::load(x + 4 * q, xv);
      acc = fma(a01.x, xv[0], acc);
      acc = fma(a01.y, xv[1], acc);
      acc = fma(a23.x, xv[2], acc);
      acc = fma(a23.y, xv[3], acc);
    }
    yv = RES ? b[t] - acc : acc;
    // non-temporal: y is not read again by this kernel, and the store leaves
    // the L2 to the streamed A (1 to 2 % faster at 0.5M to 32M cells)
    __builtin_nontemporal_store(yv, y + t);
  }
  if (ND > 0) {
    __shared__ double sh[2][4];
    double d[2];
    d[0] = valid ? yv * (u ? u[t] : yv) : 0.0;
    d[1] = yv * yv;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      double v = d[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) sh[k][wv] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < ND)
      part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
          ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
  }
}

// A^T in the 7-slot layout: slot s of cell c holds the transpose of the
// opposite slot (6-s) of the neighbour.  vals (attached values, caller
// layout) replaces a7 as the source when given.
__global__ void k_transpose7(int64_t n, int64_t nx, int64_t nxy, const int64_t *__restrict__ pos7,
                             const double *__restrict__ a7, const double *__restrict__ vals,
                             double *__restrict__ t7) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 7 * n * 16) return;
  int64_t sc = t >> 4;
  int e = (int)(t & 15);
  int s = (int)(sc / n);
  int64_t c = sc - (int64_t)s * n;
  double v = 0.0;
  if (pos7[sc] >= 0) {
    int64_t q = slot_nbr(c, s, nx, nxy);
    int r = e >> 2, col = e & 3;
    v = vals ? vals[16 * pos7[(int64_t)(6 - s) * n + q] + 4 * col + r]
             : a7[((int64_t)(6 - s) * n + q) * 16 + 4 * col + r];
  }
  t7[t] = v;
}

// Gather the 7-slot layout back to caller layout (used for inspection).
template <class T>
__global__ void k_from7(int64_t n, const int64_t *__restrict__ pos7, const T *__restrict__ a7,
                        double *__restrict__ vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 7 * n * 16) return;
  int64_t p = pos7[t >> 4];
  if (p >= 0) vals[16 * p + (t & 15)] = (double)a7[t];
}

__global__ void k_pattern(int nx, int ny, int nz, int32_t *__restrict__ rp, int32_t *__restrict__ ci) {
  int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / nxy);
  // blocks stored before row c: one diagonal per earlier cell plus one per
  // face direction per earlier cell that has that neighbour
  int64_t before = c;
  // -x/+x faces: each interior x-face contributes one block to each side
  int64_t rows_full = c / nx;                    // complete x-lines before c
  before += 2 * (rows_full * (nx - 1)) + (i > 0 ? 2 * i - 1 : 0);
  // -y/+y
  int64_t planes_full = k;                       // complete z-planes before c
  int64_t in_plane = c - planes_full * nxy;      // cells before c in its plane
  int64_t ylinks_plane = (int64_t)nx * (ny - 1);
  // cells in its plane before c that have a +y neighbour / a -y neighbour
  int64_t py = in_plane < ylinks_plane ? in_plane : ylinks_plane;
  int64_t my = in_plane > nx ? in_plane - nx : 0;
  before += planes_full * 2 * ylinks_plane + py + my;
  // -z/+z
  int64_t zlinks = nxy * (nz - 1);
  int64_t pz = c < zlinks ? c : zlinks;
  int64_t mz = c > nxy ? c - nxy : 0;
  before += pz + mz;
  rp[c] = (int32_t)before;
  int64_t p = before;
  for (int s = 0; s < 7; ++s)
    if (slot_in(s, i, j, k, nx, ny, nz)) ci[p++] = (int32_t)slot_nbr(c, s, nx, nxy);
  if (c == n - 1) rp[n] = (int32_t)p;
}

}  // namespace

// ---------------------------------------------------------------------------
rs_bsr_s::~rs_bsr_s() {
  if (at_m) rs_cpr_destroy(at_m);
  if (at_d) rs_dcpl_destroy(at_d);
  if (at) delete at;
}

static int64_t grid_nnzb(int nx, int ny, int nz) {
  int64_t n = (int64_t)nx * ny * nz;
  return n + 2 * ((int64_t)(nx - 1) * ny * nz + (int64_t)nx * (ny - 1) * nz + (int64_t)nx * ny * (nz - 1));
}

static rs_status load_values(rs_bsr_s *A, const double *d_vals, hipStream_t s) {
  if ((uintptr_t)d_vals & 15) return RS_E_ARG;         // block rows are read 16 bytes at a time
  int64_t n = A->g.n;
  dbuf flag;
  RS_TRY(flag.alloc(sizeof(int)));
  RS_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  k_to7<<<rs_grid(7 * n * 4), RS_BLOCK, 0, s>>>(n, A->pos7.as<int64_t>(), d_vals, A->a7.as<double>(),
                                                  flag.as<int>());
  RS_HIP(hipGetLastError());
  int h = 0;
  A->ref = nullptr;                     // A holds its own copy again
  RS_TRY(rs_wait_read(&h, flag.p, sizeof(int), s));
  return h ? RS_E_NONFINITE : RS_OK;
}

extern "C" rs_status rs_bsr_create(int nx, int ny, int nz, int bs, int64_t nnzb,
                                   const int32_t *d_row_ptr, const int32_t *d_col_idx,
                                   const double *d_vals, void *stream, rs_bsr *out) {
  if (!out) return RS_E_ARG;
  *out = nullptr;
  if (bs != 4 || !rs_grid_dims_ok(nx, ny, nz) || !d_row_ptr || !d_col_idx || !d_vals) return RS_E_ARG;
  int64_t n = (int64_t)nx * ny * nz;
  if (nnzb != grid_nnzb(nx, ny, nz) || nnzb > INT32_MAX) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  rs_bsr_s *A = new rs_bsr_s();
  A->g = {nx, ny, nz, n, (int64_t)nx * ny};
  A->nnzb = nnzb;
  rs_status st = RS_OK;
  do {
    if ((st = A->rp.alloc(sizeof(int32_t) * (n + 1))) != RS_OK) break;
    if ((st = A->ci.alloc(sizeof(int32_t) * nnzb)) != RS_OK) break;
    if ((st = A->pos7.alloc(sizeof(int64_t) * 7 * n)) != RS_OK) break;
    if ((st = A->a7.alloc(sizeof(double) * 7 * n * 16)) != RS_OK) break;
    if (hipMemcpyAsync(A->rp.p, d_row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(A->ci.p, d_col_idx, sizeof(int32_t) * nnzb, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      st = RS_E_HIP; break;
    }
    dbuf flag;
    if ((st = flag.alloc(sizeof(int))) != RS_OK) break;
    if (hipMemsetAsync(flag.p, 0, sizeof(int), s) != hipSuccess) { st = RS_E_HIP; break; }
    k_validate<<<rs_grid(n), RS_BLOCK, 0, s>>>(nx, ny, nz, nnzb, A->rp.as<int32_t>(), A->ci.as<int32_t>(),
                                               A->pos7.as<int64_t>(), flag.as<int>());
    int h = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = RS_E_HIP; break; }
    if (h) { st = RS_E_ARG; break; }
    st = load_values(A, d_vals, s);
  } while (0);
  if (st != RS_OK) { delete A; return st; }
  *out = A;
  return RS_OK;
}

// New values make the cached transpose, its decoupling and CPR stale.
void rs_bsr_drop_adjoint(rs_bsr_s *A) {
  if (A->at_m) { rs_cpr_destroy(A->at_m); A->at_m = nullptr; }
  if (A->at_d) { rs_dcpl_destroy(A->at_d); A->at_d = nullptr; }
  if (A->at) { delete A->at; A->at = nullptr; }
}

extern "C" rs_status rs_bsr_update(rs_bsr A, const double *d_vals, void *stream) {
  if (!A || !d_vals) return RS_E_ARG;
  rs_bsr_drop_adjoint(A);
  return load_values(A, d_vals, rs_stream(stream));
}

extern "C" void rs_bsr_destroy(rs_bsr A) { delete A; }

rs_status rs_spmv_any(const rs_bsr_s *A, const void *x, int xprec, double *y, const double *b_minus,
                      hipStream_t s) {
  return rs_spmv_dots(A, x, xprec, y, b_minus, 0, nullptr, nullptr, s);
}

unsigned rs_spmv_blocks(const rs_bsr_s *A) { return rs_grid(4 * A->g.n); }

// grid of the banded SpMV (ND = 0): 8 x the workgroups of the largest band
static unsigned spmv_band_grid(const grid3 &g) {
  int64_t most = 0;
  for (int b = 0; b < 8; ++b) most = std::max(most, spmv_band_rows(g.ny, b) * g.nx * g.nz);
  return (unsigned)(8 * ((most + 63) / 64));
}

// LDS reserved by every SpMV launch, unused by the kernel: it caps the SpMV at
// three workgroups (12 waves) per CU.  Fewer requests in flight at once
// stream A faster on this part (measured 4 to 6 % at 0.5M to 32M cells
// against the 8 workgroups the registers would allow).
static constexpr size_t SPMV_LDS_CAP = 160 * 1024 / 3 - 1024;

rs_status rs_spmv_dots(const rs_bsr_s *A, const void *x, int xprec, double *y, const double *b_minus,
                       int nd, const double *u, double *part, hipStream_t s) {
  int64_t n = A->g.n;
  const unsigned grid = nd == 0 ? spmv_band_grid(A->g) : rs_grid(4 * n);
  const double *a7 = A->ref ? A->ref : A->a7.as<double>();
  const int64_t nx = A->g.nx, nxy = A->g.nxy;
  const int ny = A->g.ny, nz = A->g.nz;
#define RS_SPMV(TX, RES, ND)                                                                                   \
  do {                                                                                                        \
    if (A->ref)                                                                                               \
      k_spmv7<TX, RES, ND, true><<<grid, RS_BLOCK, SPMV_LDS_CAP, s>>>(n, ny, nz, nx, nxy, a7, (const TX *)x, b_minus, y, u, \
                                                           part);                                             \
    else                                                                                                      \
      k_spmv7<TX, RES, ND, false><<<grid, RS_BLOCK, SPMV_LDS_CAP, s>>>(n, ny, nz, nx, nxy, a7, (const TX *)x, b_minus, y, \
                                                            u, part);                                         \
  } while (0)
  if (nd < 0 || nd > 2 || (nd > 0 && !part)) return RS_E_ARG;
  if (xprec == 64) {
    if (b_minus) {
      if (nd == 0) RS_SPMV(double, true, 0);
      else if (nd == 1) RS_SPMV(double, true, 1);
      else RS_SPMV(double, true, 2);
    } else {
      if (nd == 0) RS_SPMV(double, false, 0);
      else if (nd == 1) RS_SPMV(double, false, 1);
      else RS_SPMV(double, false, 2);
    }
  } else {
    if (b_minus) {
      if (nd == 0) RS_SPMV(float, true, 0);
      else if (nd == 1) RS_SPMV(float, true, 1);
      else RS_SPMV(float, true, 2);
    } else {
      if (nd == 0) RS_SPMV(float, false, 0);
      else if (nd == 1) RS_SPMV(float, false, 1);
      else RS_SPMV(float, false, 2);
    }
  }
#undef RS_SPMV
  RS_HIP(hipGetLastError());
  return RS_OK;
}

extern "C" rs_status rs_spmv(rs_bsr A, const double *d_x, double *d_y, void *stream) {
  if (!A || !d_x || !d_y || d_x == d_y || (((uintptr_t)d_x | (uintptr_t)d_y) & 15)) return RS_E_ARG;
  return rs_spmv_any(A, d_x, 64, d_y, nullptr, rs_stream(stream));
}

rs_status rs_transpose7(const rs_bsr_s *A, rs_bsr_s *At, hipStream_t s) {
  int64_t n = A->g.n;
  At->g = A->g;
  At->nnzb = A->nnzb;
  RS_TRY(At->rp.alloc(sizeof(int32_t) * (n + 1)));
  RS_TRY(At->ci.alloc(sizeof(int32_t) * A->nnzb));
  RS_TRY(At->pos7.alloc(sizeof(int64_t) * 7 * n));
  RS_TRY(At->a7.alloc(sizeof(double) * 7 * n * 16));
  RS_HIP(hipMemcpyAsync(At->rp.p, A->rp.p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  RS_HIP(hipMemcpyAsync(At->ci.p, A->ci.p, sizeof(int32_t) * A->nnzb, hipMemcpyDeviceToDevice, s));
  RS_HIP(hipMemcpyAsync(At->pos7.p, A->pos7.p, sizeof(int64_t) * 7 * n, hipMemcpyDeviceToDevice, s));
  k_transpose7<<<rs_grid(7 * n * 16), RS_BLOCK, 0, s>>>(n, A->g.nx, A->g.nxy, A->pos7.as<int64_t>(),
                                                        A->a7.as<double>(), A->ref, At->a7.as<double>());
  RS_HIP(hipGetLastError());
  return RS_OK;
}

rs_status rs_from7_host(const rs_bsr_s *A, const void *a7, int prec, double *h_vals) {
  int64_t n = A->g.n;
  dbuf tmp;
  RS_TRY(tmp.alloc(sizeof(double) * 16 * A->nnzb));
  if (prec == 64)
    k_from7<double><<<rs_grid(7 * n * 16), RS_BLOCK>>>(n, A->pos7.as<int64_t>(), (const double *)a7, tmp.as<double>());
  else
    k_from7<float><<<rs_grid(7 * n * 16), RS_BLOCK>>>(n, A->pos7.as<int64_t>(), (const float *)a7, tmp.as<double>());
  RS_HIP(hipGetLastError());
  RS_HIP(hipMemcpy(h_vals, tmp.p, sizeof(double) * 16 * A->nnzb, hipMemcpyDeviceToHost));
  return RS_OK;
}

extern "C" rs_status rs_pattern(int nx, int ny, int nz, int32_t *d_row_ptr, int32_t *d_col_idx,
                                int64_t *h_nnzb, void *stream) {
  if (!rs_grid_dims_ok(nx, ny, nz) || !d_row_ptr || !d_col_idx) return RS_E_ARG;
  int64_t n = (int64_t)nx * ny * nz;
  if (grid_nnzb(nx, ny, nz) > INT32_MAX) return RS_E_ARG;
  k_pattern<<<rs_grid(n), RS_BLOCK, 0, rs_stream(stream)>>>(nx, ny, nz, d_row_ptr, d_col_idx);
  RS_HIP(hipGetLastError());
  if (h_nnzb) *h_nnzb = grid_nnzb(nx, ny, nz);
  return RS_OK;
}
