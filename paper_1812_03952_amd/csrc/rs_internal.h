// rs_internal.h -- shared declarations of librsolve (HIP, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>
#include "../../include/rsolve.h"

#define RS_BLOCK 256

// ---- error handling: every HIP call is checked and mapped to rs_status ----
#define RS_HIP(call)                                                   \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) return (e_ == hipErrorOutOfMemory) ? RS_E_NOMEM : RS_E_HIP; \
  } while (0)
#define RS_TRY(expr)                        \
  do {                                      \
    rs_status s_ = (expr);                  \
    if (s_ != RS_OK) return s_;             \
  } while (0)

static inline hipStream_t rs_stream(void *s) { return (hipStream_t)s; }

// Device memory comes from the library's pool (pool.hip): a freed block is
// cached and reused by later requests of a similar size.
void *rs_pool_get(size_t bytes, size_t *got);   // nullptr when out of memory
void rs_pool_put(void *p, size_t bytes);
// Wait for the work queued on s (rs_wait), or copy bytes (at most 256) from
// device memory to h and wait for them (rs_wait_read), polling an event.
rs_status rs_wait(hipStream_t s);
rs_status rs_wait_read(void *h, const void *d, size_t bytes, hipStream_t s);

// A device allocation owned by a handle.  `bytes` is the size of the block
// actually held (at least what was asked for).
struct dbuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~dbuf() { release(); }
  dbuf() = default;
  dbuf(const dbuf &) = delete;
  dbuf &operator=(const dbuf &) = delete;
  rs_status alloc(size_t b) {
    if (p && bytes >= b) return RS_OK;
    release();
    if (b == 0) b = 16;
    size_t got = 0;
    p = rs_pool_get(b, &got);
    if (!p) return RS_E_NOMEM;
    bytes = got;
    return RS_OK;
  }
  void release() { if (p) rs_pool_put(p, bytes); p = nullptr; bytes = 0; }
  template <class T> T *as() const { return (T *)p; }
};

static inline unsigned rs_grid(int64_t work, int block = RS_BLOCK) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// ---- grid geometry --------------------------------------------------------
// The 7 stencil slots in ascending column order: -z -y -x self +x +y +z.
struct grid3 {
  int nx, ny, nz;
  int64_t n, nxy;
};

// grid extents the library takes: each at least 1 and at most 2^30 cells in
// all (cell and block indices stay in int32), the product formed without
// overflow
static inline bool rs_grid_dims_ok(int nx, int ny, int nz) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  const int64_t nxy = (int64_t)nx * ny;
  return nxy <= INT32_MAX / 2 && nxy * nz <= INT32_MAX / 2;
}

// ---- handles --------------------------------------------------------------
struct rs_bsr_s {
  grid3 g;
  int64_t nnzb;
  dbuf rp, ci;       // caller pattern (copy), int32
  dbuf pos7;         // int64 per (slot, cell): caller block index or -1
  dbuf a7;           // double [7][n][16]: blocks by stencil slot (zeros off-grid)
  // attached values (caller layout, rs_bsr_attach_decouple): when set, the
  // values of A are read there and a7 is stale
  const double *ref = nullptr;
  // adjoint cache
  rs_bsr_s *at = nullptr;
  rs_dcpl_s *at_d = nullptr;
  rs_cpr_s *at_m = nullptr;
  int at_method = -1, at_prec = -1;
  rs_cpr_opts at_opts;
  ~rs_bsr_s();
};

struct rs_dcpl_s {
  rs_bsr_s *A;
  int method, prec;
  dbuf t7;      // decoupled blocks [7][n][16], prec
  dbuf dinv;    // D^{-1} [n][16], prec
  dbuf ap7;     // pressure entries [7][n], double
  dbuf col0;    // column 0 of the decoupled blocks, [n][4 rows][8] (slots 0-6, pad), prec
};

struct amg_level {
  int n = 0, nc = 0;
  int64_t nnz = 0;
  dbuf rp, ci;        // int32 CSR
  dbuf a;             // double values (setup precision)
  dbuf ap;            // values in apply precision (alias of a when prec 64)
  dbuf dl1;           // l1 diagonal, apply precision
  dbuf agg;           // int32 aggregate per row (-1 none)
  dbuf mptr, mem;     // members of each aggregate (ascending), for restriction
  dbuf b, x, r;       // cycle work vectors, apply precision
  int64_t xoff = 0;   // x starts xoff elements into its buffer (zero guard planes at level 0)
  // level 0 only: values by stencil slot [7][n] (zero off the grid) and
  // y = b ./ d, apply precision, for the structured cycle kernels
  dbuf s7, y;
  // smoothed prolongator (rs_cpr_opts.smooth): row i of P at rp[i] + i,
  // pcnt[i] entries (coarse columns pci, FP64 values pv, apply-precision
  // values pvt); P^T by coarse row (tptr, fine rows tri ascending, values
  // trt in apply precision); z = y + P x_c in the cycle
  bool sa = false;
  dbuf pcnt, pci, pv, pvt, tptr, tri, trt, z;
  template <class T> T *xp() const { return x.as<T>() + xoff; }
};

struct rs_cpr_s {
  rs_bsr_s *A;
  rs_dcpl_s *D;
  rs_cpr_opts o;
  int prec;
  int nlev = 0;
  std::vector<amg_level *> lev;
  int coarse_lu = 0;
  dbuf cinv;          // dense inverse of the coarsest level (double)
  dbuf cb, cx;        // coarsest rhs / solution in double
  dbuf dinv2;         // second-stage block inverses [n][16], prec
  // pipelined DILU sweeps: brick size, brick grid, ticket order, progress
  int pb = 0, pnj = 0, pnk = 0;
  uint32_t pepoch = 0;       // tag of the last pipelined sweep
  dbuf pord, pdone, pctl, pxch;
  // RAS sweeps: scaled blocks and x_p in wavefront order; strips per layer,
  // their boundary exchange words, [fwd ticket, bwd ticket, error] and the
  // tag of the last sweep
  dbuf rblk, rxp, rxw, rctl;
  int rs_strips = 1, rs_h = 0;
  // RAS with overlap 1: layer factors P0 (dinv2 holds P1, the owned ones),
  // P2, scaled blocks of P1 and P2, the middle and top sweeps' vectors and a
  // zero x_p for the top layer's backward sweep
  dbuf rdv0, rdv2, rblk1, rblk2, ry1, rz2, rzero;
  uint32_t repoch = 0;
  // CPR work
  dbuf rt, bp, xp, yv, zt;   // prec vectors
  dbuf fy, fzero;             // CPR-FPF: first-stage result, zero x_p with guards
  // GMRES work (allocated on first solve)
  int m = 0;
  dbuf V, Z, w, part, scal;
  double *hpin = nullptr;     // pinned host status word
  // BiCGSTAB work vectors (r, r^, p, v, t in FP64; p^, s^ in the
  // preconditioner's precision), partials and scalars
  dbuf bvec, bpart, bscal;
  int bprec = 0;
  double *bpin = nullptr;     // pinned host copy of the scalar block
  ~rs_cpr_s();
};

// ---- internal entry points shared between translation units ---------------
rs_status rs_spmv_any(const rs_bsr_s *A, const void *x, int xprec, double *y,
                      const double *b_minus, hipStream_t s);
// The SpMV with ND epilogue dots (see k_spmv7): partials in
// part[d * rs_spmv_blocks(A) + block].
rs_status rs_spmv_dots(const rs_bsr_s *A, const void *x, int xprec, double *y, const double *b_minus,
                       int nd, const double *u, double *part, hipStream_t s);
unsigned rs_spmv_blocks(const rs_bsr_s *A);
void rs_bsr_drop_adjoint(rs_bsr_s *A);
rs_status rs_cpr_apply_any(rs_cpr_s *M, const double *r, void *z, int zprec,
                           hipStream_t s);
// z = M^{-1} (w / *d_h) in two calls, with v = w / *d_h written by the first
// (d_h on the device): the normalisation of a Krylov vector fused into the
// first stage.  rs_cpr_apply_in does nothing on the device when d_halt is
// given and *d_halt is nonzero at the time it runs; rs_cpr_apply_rest takes
// the first call's output and must follow it on the same stream.
rs_status rs_cpr_apply_in(rs_cpr_s *M, const double *w, const double *d_h, double *v, const double *d_halt,
                          hipStream_t s);
rs_status rs_cpr_apply_rest(rs_cpr_s *M, void *z, int zprec, hipStream_t s);
rs_status rs_vcycle_run(rs_cpr_s *M, hipStream_t s);
rs_status rs_transpose7(const rs_bsr_s *A, rs_bsr_s *At, hipStream_t s);
rs_status rs_dilu_prepare(rs_cpr_s *M);
rs_status rs_dilu_setup_run(rs_cpr_s *M, int *flag, hipStream_t s);
template <class T> rs_status rs_dilu_apply_run(rs_cpr_s *M, const T *xp, T *out, hipStream_t s);
rs_status rs_dilu_check(rs_cpr_s *M, hipStream_t s);
rs_status rs_ras_check_shape(const grid3 &g, int prec);
rs_status rs_ras_setup_run(rs_cpr_s *M, int *flag, hipStream_t s);
template <class T> rs_status rs_ras_apply_run(rs_cpr_s *M, const T *xp, T *out, hipStream_t s);
