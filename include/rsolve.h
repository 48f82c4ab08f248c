/* rsolve.h -- C-ABI of librsolve.so: the linear solve inside each Newton step
 * of a fully implicit thermal reservoir simulator (Liu & Chen, "A Scalable
 * Thermal Reservoir Simulator for Giant Models on Parallel Computers",
 * arXiv 1812.03952), on one AMD Instinct MI355X (gfx950).
 *
 * The system is A x = b with A the block Jacobian of Eq. mat-ja (Section
 * "Linear Solver"): unknowns numbered grid block by grid block, 4x4 blocks
 * (unknowns p, N_w, N_o, T), 7-point pattern of a 3-D Cartesian grid.  The
 * library decouples it (Section "Decoupling Methods"), builds a two-stage
 * CPR preconditioner from the pressure sub-matrix and an aggregation AMG
 * (Section "Preconditioners", Fig. fig-ds-amg-par), and solves with
 * restarted flexible GMRES.
 *
 * Conventions for every call
 *   - Pointers named d_* are device pointers (any allocator: hipMalloc,
 *     torch); h_* are host pointers.  Buffers passed in are borrowed for the
 *     duration of the call only; the library keeps no reference to them,
 *     with one exception: rs_bsr_attach_decouple keeps d_vals as the
 *     matrix's values until the handle's next update or its destruction
 *     (the caller keeps that buffer alive and unchanged meanwhile).
 *   - Handles (rs_bsr, rs_dcpl, rs_cpr) are opaque and owned by the library;
 *     free them with the matching *_destroy.  A handle may be used by one
 *     host thread at a time.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream).  All
 *     device work is enqueued on it.  Calls that return scalars to the host
 *     (setup status, solve info) synchronise that stream before returning.
 *   - Grids: nx, ny, nz >= 1 and nx*ny*nz < 2^30 cells (RS_E_ARG otherwise).
 *   - Cell c = i + nx*(j + ny*k), 0-based, i fastest.  Block rows follow the
 *     cell order; in a row the stored columns are ascending:
 *     c-nx*ny, c-nx, c-1, c, c+1, c+nx, c+nx*ny (those inside the grid).
 *     Block values are row-major 4x4, vals[16*p + 4*r + s].
 *   - Vectors hold 4 doubles per cell (unknown 0 is pressure), length 4*n.
 *   - Errors are returned, never raised or aborted on; rs_status_string()
 *     names them.  RS_NOT_CONVERGED is not fatal: x holds the last iterate.
 *   - Device memory of handles comes from the library's pool: a destroyed
 *     handle's blocks are kept and reused by later calls (see rs_pool_trim).
 *     Reuse on the same stream is ordered by the stream; before destroying a
 *     handle whose work may still be pending on another stream, synchronise.
 */
#ifndef RSOLVE_H
#define RSOLVE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_bsr_s *rs_bsr;
typedef struct rs_dcpl_s *rs_dcpl;
typedef struct rs_cpr_s *rs_cpr;

typedef enum {
  RS_OK = 0,
  RS_NOT_CONVERGED = 1,
  RS_E_ARG = -1,        /* invalid argument or pattern                  */
  RS_E_HIP = -2,        /* a HIP runtime call failed                    */
  RS_E_NOMEM = -3,      /* device allocation failed                     */
  RS_E_SINGULAR = -4,   /* a 4x4 block or the coarsest matrix is singular */
  RS_E_NONFINITE = -5   /* NaN/Inf in the input or during the iteration */
} rs_status;

#define RS_ABF 0        /* alternate block factorisation, Eq. decoupled-abf */
#define RS_QIMPES 1     /* quasi-IMPES: pressure row of A_ii^{-1} only      */
#define RS_FRS 2        /* full row sum, Eq. decoupled-frs: row 0 of each block
                           becomes the sum of its four rows                 */
#define RS_FRS_ABF 3    /* two-stage FRS then ABF (same section); equals ABF
                           in exact arithmetic                               */
#define RS_SM_BJ 0      /* second stage: block Jacobi over cells (RAS, overlap 0, one cell each) */
#define RS_SM_DILU 1    /* second stage: block ILU(0) of the whole matrix, natural order        */
#define RS_SM_RAS 2     /* second stage: RAS, overlap 0, one xy-layer per subdomain, block
                           ILU(0) in each (Section "Preconditioners"); needs ny <= 480 with
                           FP64 storage, ny <= 960 with FP32, else RS_E_ARG               */
#define RS_SM_RAS1 3    /* second stage: RAS with overlap 1, the paper's default overlap
                           (Section "Preconditioners"): each xy-layer extended by the
                           layers below and above, block ILU(0) of the restricted matrix of
                           that extension in natural order, each cell taking the value of
                           its own layer's extension (restricted prolongation); limits as
                           for RS_SM_RAS                                                   */

typedef struct {
  int smoother;        /* RS_SM_BJ, RS_SM_DILU, RS_SM_RAS or RS_SM_RAS1 (default DILU) */
  double theta;        /* AMG strength threshold (default 0.5, Fig. fig-ds-amg-par) */
  double max_row_sum;  /* AMG weak-row threshold (default 0.9, same figure)       */
  int coarse_n;        /* stop coarsening at <= this many rows (default 256)     */
  int max_levels;      /* AMG depth limit (default 20)                           */
  int lu_max;          /* largest coarsest level inverted densely (default 256; a
                          larger coarsest level, one on which no aggregate forms,
                          is relaxed by coarse_sweeps l1-Jacobi sweeps; at most
                          8192)                                                 */
  int coarse_sweeps;   /* l1-Jacobi sweeps if the coarsest is larger (default 4) */
  int stages;          /* 2: pressure then full (default); 3: CPR-FPF, full,
                          pressure, full (Algorithm pc-fpf)                       */
  int smooth;          /* AMG prolongator: 0 piecewise constant over the
                          aggregates (default); 1 smoothed by one damped Jacobi
                          step, P = (I - omega D^{-1} A) P_t with omega = 4/(3 rho),
                          rho = max_i sum_j |a_ij| / |a_ii|, then truncated      */
  double trunc;        /* smoothed P: weights below trunc times the row's largest
                          are dropped and the rest scaled to the row's former sum
                          (default 1e-2, "trunc error" of Fig. fig-ds-amg-par)   */
} rs_cpr_opts;

typedef struct {
  int restart;         /* Krylov dimension per cycle (default 30, max 32)        */
  double rtol;         /* stop at ||b - A x|| <= rtol ||b|| (default 1e-8)       */
  int maxit;           /* Arnoldi steps in total (default 300)                   */
  int zero_guess;      /* 1: start from x0 = 0 whatever d_x holds (r0 = b, no
                          product with A); 0: d_x is the initial guess (default) */
} rs_gmres_opts;

typedef struct {
  double rtol;         /* stop at ||b - A x|| <= rtol ||b|| (default 1e-8)       */
  int maxit;           /* iterations in total (default 300); each applies A and
                          M twice (once if it stops half-way)                    */
  int zero_guess;      /* as in rs_gmres_opts                                    */
} rs_bicgstab_opts;

typedef struct {
  int iters;           /* Arnoldi steps (GMRES) or iterations (BiCGSTAB) run      */
  int cycles;          /* restart cycles run                                     */
  int status;          /* rs_status of the solve                                 */
  double relres;       /* true FP64 ||b - A x|| / ||b|| at exit                  */
  double est_relres;   /* last residual estimate / ||b||: |g_{j+1}| (GMRES), the
                          updated ||r|| or ||s|| (BiCGSTAB)                      */
  double ms;           /* wall time of the solve on the stream (hipEvents)       */
} rs_solve_info;

void rs_cpr_opts_default(rs_cpr_opts *o);
void rs_gmres_opts_default(rs_gmres_opts *o);
void rs_bicgstab_opts_default(rs_bicgstab_opts *o);
const char *rs_status_string(int status);

/* ---- the five calls of the solve ---------------------------------------- */

/* Ingest a 4x4-block BSR Jacobian (Eq. mat-ja).  bs must be 4 and
 * nx*ny*nz*... must match: the pattern (d_row_ptr[n+1], d_col_idx[nnzb]) is
 * validated against the 7-point pattern of the nx x ny x nz grid described
 * above (RS_E_ARG otherwise).  Values (d_vals, 16*nnzb doubles) are copied
 * into the library's own device layout; the caller may free its buffers
 * afterwards.  d_vals must be 16-byte aligned (RS_E_ARG otherwise).
 * Non-finite values give RS_E_NONFINITE. */
rs_status rs_bsr_create(int nx, int ny, int nz, int bs, int64_t nnzb,
                        const int32_t *d_row_ptr, const int32_t *d_col_idx,
                        const double *d_vals, void *stream, rs_bsr *out);

/* Replace the values of A (same pattern, caller layout), e.g. at the next
 * Newton step.  Invalidates the cached transpose used by rs_adjoint_solve;
 * decouplings and preconditioners built from the old values are not
 * updated (rebuild them). */
rs_status rs_bsr_update(rs_bsr A, const double *d_vals, void *stream);

/* rs_bsr_update followed by rs_decouple, in one pass over the values: the
 * new values (caller layout, 16-byte aligned) are read once, stored into A
 * and decoupled; the results equal those of the two calls.  For the Newton
 * loop, where every step brings a new Jacobian to decouple.  Errors as for
 * the two calls; after RS_E_SINGULAR A holds the new values. */
rs_status rs_bsr_update_decouple(rs_bsr A, const double *d_vals, int method, int prec, void *stream,
                                 rs_dcpl *out);

/* As rs_bsr_update_decouple, but without a copy: A refers to d_vals (caller
 * layout, 16-byte aligned) in place, and every later use of A's values (the
 * SpMV inside the solvers, rs_decouple, the transpose of rs_adjoint_solve)
 * reads them there, with results bitwise equal to those of the copying call.
 * The caller keeps d_vals allocated and unchanged until A no longer refers to
 * it: until the next rs_bsr_update, rs_bsr_update_decouple or
 * rs_bsr_attach_decouple on A, or rs_bsr_destroy.  For the Newton loop, where
 * the Jacobian is assembled in device memory the caller owns anyway: it
 * saves writing the library's copy (16 * 7 * n doubles) on every step.
 * Errors as for rs_bsr_update_decouple; after RS_E_NONFINITE or
 * RS_E_SINGULAR A refers to d_vals, after RS_E_ARG nothing has changed. */
rs_status rs_bsr_attach_decouple(rs_bsr A, const double *d_vals, int method, int prec, void *stream,
                                 rs_dcpl *out);

/* Decoupling (D^{-1} A) x = D^{-1} b, Eq. decoupled-eq, computed block row by
 * block row with Gauss-Jordan elimination and row pivoting (Section
 * "Decoupling Methods").  method: RS_ABF (D = diag(A_11..A_nn), Eq.
 * decoupled-abf), RS_QIMPES (only the pressure row is replaced, by row 0
 * of A_ii^{-1} A_ij), RS_FRS (Eq. decoupled-frs: D^{-1} = F, ones in row 0
 * and on the diagonal, so row 0 becomes the sum of the four rows), or
 * RS_FRS_ABF (FRS, then ABF on the result).  prec: 64 or 32, the storage and arithmetic precision
 * of the decoupled blocks used by the preconditioner; the pressure matrix
 * used by the AMG setup is always kept in FP64.  A singular diagonal block
 * (pivot <= 1e-300 or <= 1e-14 max|A_ii|) gives RS_E_SINGULAR. */
rs_status rs_decouple(rs_bsr A, int method, int prec, void *stream, rs_dcpl *out);

/* CPR setup (Section "Preconditioners"): pressure sub-matrix
 * A_p[i][j] = A~_ij[0][0] ("getting sub-matrix (for CPR)", Section "Linear
 * Solver"), aggregation-AMG hierarchy on A_p built on the device, and the
 * second stage (block Jacobi or block ILU(0)) on the decoupled matrix.
 * With o->stages == 3 the apply is CPR-FPF (Algorithm pc-fpf, read as its
 * five described steps): y = M2^{-1} f, the pressure correction of the
 * residual f - A~ y, then M2^{-1} of the new residual added to y.
 * o == NULL takes the defaults.  The handle keeps references to A and D:
 * destroy it before them. */
rs_status rs_cpr_setup(rs_bsr A, rs_dcpl D, const rs_cpr_opts *o, void *stream,
                       rs_cpr *out);

/* Solve A x = b with restarted flexible GMRES right-preconditioned by M
 * (Section "Linear Solver").  d_x holds the initial guess on entry and the
 * iterate on exit.  o == NULL takes the defaults.  info (host, may be NULL)
 * receives iterations, cycles and the true FP64 relative residual.  d_b and
 * d_x must be 16-byte aligned (RS_E_ARG otherwise).  Returns RS_OK when the
 * true residual meets rtol, RS_NOT_CONVERGED at maxit. */
rs_status rs_gmres_solve(rs_bsr A, rs_cpr M, const double *d_b, double *d_x,
                         const rs_gmres_opts *o, rs_solve_info *info, void *stream);

/* Solve A x = b with BiCGSTAB right-preconditioned by M, the Krylov method
 * of the paper's experiments (Section "Linear Solver" names it).  The
 * textbook recurrence with p^ = M^{-1} p, s^ = M^{-1} s; it stops when the
 * updated residual (||s|| half-way, ||r|| at the end of an iteration) meets
 * rtol, then recomputes the true residual and starts again from it (shadow
 * r^ = r) if that misses rtol.  A breakdown ((r^, r), (r^, v) or (t, t)
 * zero) restarts likewise, and ends the solve when it comes in the first
 * iteration after a start.  d_x holds the initial guess on entry.  o == NULL
 * takes the defaults.  The work vectors (7 of 4n entries) live in M.  d_b and
 * d_x must be 16-byte aligned (RS_E_ARG otherwise).  Returns RS_OK when the
 * true residual meets rtol, RS_NOT_CONVERGED otherwise. */
rs_status rs_bicgstab_solve(rs_bsr A, rs_cpr M, const double *d_b, double *d_x,
                            const rs_bicgstab_opts *o, rs_solve_info *info, void *stream);

/* Adjoint solve A^T lambda = w (not in the paper; gives dJ/dA = -lambda x^T
 * for J = w^T x).  Builds on first use and caches, inside A, the block
 * transpose, its decoupling (method, prec) and its CPR (co); the cache is
 * dropped by rs_bsr_update.  d_lambda holds the initial guess on entry;
 * d_w and d_lambda must be 16-byte aligned (RS_E_ARG otherwise). */
rs_status rs_adjoint_solve(rs_bsr A, int method, int prec, const rs_cpr_opts *co,
                           const double *d_w, double *d_lambda,
                           const rs_gmres_opts *o, rs_solve_info *info, void *stream);

void rs_bsr_destroy(rs_bsr A);
void rs_dcpl_destroy(rs_dcpl D);
void rs_cpr_destroy(rs_cpr M);

/* ---- building blocks of the path, exposed for tests and measurement ----- */

/* y = A x (Fig. fig-mv).  d_x, d_y: 4n doubles, 16-byte aligned, must not alias. */
rs_status rs_spmv(rs_bsr A, const double *d_x, double *d_y, void *stream);

/* One application of the CPR preconditioner, z = M^{-1} r (FP64 in/out). */
rs_status rs_cpr_apply(rs_cpr M, const double *d_r, double *d_z, void *stream);

/* Assemble the synthetic Jacobian on the device into caller-layout BSR
 * values (16*nnzb doubles; pattern as described above), from the seeded
 * draws: log-permeability d_logk[n], vertical ratio kvkh, transmissibility
 * constant tscale, face blocks d_Mf, d_Mb [3][n][16], accumulation d_B
 * [n][16], time step dt, wells d_wcell[nw] (ascending cell ids) with
 * coefficients d_wu[nw]; d_row_ptr is the pattern's row pointer array.  Face transmissibility is tscale times the
 * harmonic mean of the directional permeabilities (Section "Numerical
 * Methods"); A[c][c+e_d] = -T Mf[d][c], A[c+e_d][c] = -T Mb[d][c], and each
 * diagonal block is B/dt plus the row's T*M terms plus u*k*I at wells. */
rs_status rs_assemble(int nx, int ny, int nz, const double *d_logk, double kvkh,
                      double tscale, const double *d_Mf, const double *d_Mb,
                      const double *d_B, double dt, int nw, const int32_t *d_wcell,
                      const double *d_wu, const int32_t *d_row_ptr, double *d_vals,
                      void *stream);

/* ---- the system of one Newton step of the thermal model ------------------ */

/* Constants of the water / oil / energy subset of the paper's thermal model
 * (units: psi, deg F, ft, day, md, cp, lbmole, Btu).  The defaults hold the
 * values the paper prints, and readings where it prints none:
 *   printed: the heavy-oil example's cell sizes (29.17, 29.17, 10 ft),
 *     porosity 0.3 and its coefficient 5e-4 1/psi, producers' bottom-hole
 *     pressure 17 psi and injection temperature 450 F; the light-oil
 *     component's density (0.2092 lbmole/ft^3, 5e-6 1/psi, 3.8e-4 1/F) and
 *     viscosity (avisc 0.287352 cp, bvisc 3728.2, T absolute); the water
 *     enthalpy constants (gas-based, cpg1..5, hvr 4820, ev 0.38, J/gmol, C);
 *     the oil's liquid heat capacity (0.5 Btu/(lb F), M = 250 lb/lbmole);
 *     the relative-permeability tables (Figs. rela-swt, rela-slt) and the
 *     water viscosity table (Fig. fig-wat-vis), compiled in;
 *   readings: water density 3.4605 lbmole/ft^3 at 14.696 psi and 60 F with
 *     3e-6 1/psi and 1e-4 1/F; water T_crit 374.15 C; rock heat capacity
 *     35 Btu/(ft^3 F); conductivities water 8.6, oil 1.8, rock 24
 *     Btu/(ft day F); Darcy constant 1.127e-3 bbl/(day psi cp md ft) and
 *     5.614583 ft^3/bbl. */
typedef struct {
  double dx, dy, dz, dt;                  /* cell sizes (ft), time step (day)            */
  double ctrans;                          /* Darcy constant, ft^3 cp / (day psi md ft)   */
  double p_ref, t_ref;                    /* reference pressure (psi) and temperature (F) */
  double rhow_ref, cpw, ct1w, ct2w, cptw; /* water density correlation                   */
  double rhoo_ref, cpo, ct1o, ct2o, cpto; /* oil component density correlation           */
  double avisc_o, bvisc_o;                /* oil viscosity avisc exp(bvisc / (T + 459.67)) */
  double cpl_o;                           /* oil heat capacity, Btu/(lbmole F)           */
  double cpg[5], hvr_w, ev_w, tcrit_w;    /* water gas-based enthalpy, J/gmol and deg C  */
  double por_ref, cpor;                   /* porosity phi_ref (1 + cpor (p - p_ref))     */
  double cp_rock;                         /* rock heat capacity, Btu/(ft^3 F)            */
  double kw, ko, kr;                      /* thermal conductivities, Btu/(ft day F)      */
  double pv_btu, jmol_btu;                /* psi ft^3 in Btu; J/gmol in Btu/lbmole       */
  double p_bh, t_inj;                     /* producers' bottom-hole pressure, injection T */
  double bbl_ft3;                         /* ft^3 per bbl                                */
} rs_thermal_params;

void rs_thermal_params_default(rs_thermal_params *q);

/* Residual R(u) and Jacobian dR/du of one backward-Euler Newton step
 * (Section "Numerical Methods") of a water / oil / energy subset of the
 * thermal model (Section "Mathematical Model", Eqs. eq4.1-eq4.3): water
 * with the water component only, oil with one oil component only, no gas
 * (S_g = 0, the switched constraint of the gas-free state), no capillary
 * pressure, no gravity, no heat loss.
 *   Unknowns per cell u = (p, N_w, N_o, T): pressure, moles of water and of
 *   oil per unit bulk volume (S = N / (phi rho)), temperature.
 *   Equations per cell, in this order: water and oil mole balance
 *   V/dt (N - N_old) - sum of face flows in - wells; energy balance
 *   V/dt (E - E_old) - ... with E = N_w U_w + N_o U_o + (1 - phi_ref) U_r;
 *   the saturation constraint V/dt (phi - N_w/rho_w - N_o/rho_o).
 *   Face flow of phase a into a cell: G lambda_a,up (p_nbr - p_cell), G the
 *   Darcy constant times area/length times the harmonic mean of the two
 *   cells' permeabilities along the face (zero on the boundary), lambda =
 *   k_r rho / mu upstream (higher pressure; the lower-numbered cell on a
 *   tie); energy flow sum_a F_a H_a,up plus conduction with the harmonic
 *   mean of K_T = phi (S_w K_w + S_o K_o) + (1 - phi) K_r; k_ro by Stone's
 *   model II; Peaceman wells: producers Q_a = -ctrans WI lambda_a
 *   (p - p_bh) when p > p_bh, injectors a fixed water rate at t_inj.
 * Arguments (device pointers, 16-byte aligned where vectors): per-cell
 * permeabilities d_kx, d_ky, d_kz (md, n each); the iterate d_u and the
 * previous time step's state d_uold (4n each, 4 unknowns per cell as
 * above); nw well perforations: d_wcell (ascending, unique cells, else
 * RS_E_ARG), d_wkind (+1 injector, -1 producer), d_wval (injector: water
 * rate in bbl/day of cold water; producer: well index in md ft).
 * Outputs: d_vals (16*nnzb doubles, the caller layout of the 7-point
 * pattern described above: block (i,j) = dR_i/du_j, rows = equations,
 * columns = unknowns; may be NULL) and d_res (4n, may be NULL; not both).
 * The Newton step solves J du = -R. */
rs_status rs_thermal_assemble(int nx, int ny, int nz, const rs_thermal_params *q, const double *d_kx,
                              const double *d_ky, const double *d_kz, const double *d_u,
                              const double *d_uold, int nw, const int32_t *d_wcell,
                              const int32_t *d_wkind, const double *d_wval, double *d_vals,
                              double *d_res, void *stream);

/* u = (p, N_w, N_o, T) per cell from p, S_w, S_o, T (n each, device): N = phi
 * rho S with the densities and porosity of rs_thermal_assemble, for states
 * given in saturations. */
rs_status rs_thermal_state(int64_t n, const rs_thermal_params *q, const double *d_p, const double *d_sw,
                           const double *d_so, const double *d_t, double *d_u, void *stream);

/* Write the 7-point block pattern of an nx x ny x nz grid (row pointers
 * n+1, column indices nnzb) into device buffers; *h_nnzb (host, may be NULL)
 * receives the number of stored blocks. */
rs_status rs_pattern(int nx, int ny, int nz, int32_t *d_row_ptr, int32_t *d_col_idx,
                     int64_t *h_nnzb, void *stream);

/* d_G[16*nnzb] (caller layout) = -lambda_i x_j^T for every stored block
 * (i,j): the gradient of J = w^T x with respect to the values of A when
 * A^T lambda = w. */
rs_status rs_grad_vals(rs_bsr A, const double *d_lambda, const double *d_x,
                       double *d_G, void *stream);

/* Chain rule of rs_assemble: d_g[n] = sum over blocks of G : dA/dlogk_c
 * given d_G = dJ/dA in caller layout (arguments as for rs_assemble). */
rs_status rs_grad_logk(int nx, int ny, int nz, const double *d_logk, double kvkh,
                       double tscale, const double *d_Mf, const double *d_Mb,
                       int nw, const int32_t *d_wcell, const double *d_wu,
                       const int32_t *d_row_ptr, const double *d_G, double *d_g,
                       void *stream);

/* ---- device memory pool -------------------------------------------------- */

/* Return every cached (unused) pool block to the HIP runtime.  Blocks held
 * by live handles are not affected.  Call it when another allocator needs
 * the memory; no stream work may still use a destroyed handle's memory. */
void rs_pool_trim(void);
/* Bytes held by live handles and bytes cached for reuse (either may be NULL). */
void rs_pool_usage(size_t *live_bytes, size_t *cached_bytes);

/* ---- inspection (copies to host; synchronise the stream) --------------- */

/* Decoupled blocks in caller layout (16*nnzb doubles, upcast if FP32) and
 * D^{-1} (16*n doubles); either pointer may be NULL. */
rs_status rs_dcpl_get(rs_dcpl D, double *h_vals, double *h_dinv);
/* Number of AMG levels. */
int rs_cpr_nlevels(rs_cpr M);
/* Level l of the hierarchy: rows, stored entries, and (any may be NULL)
 * CSR arrays, FP64 values, l1 diagonal, aggregate of each row (-1 = not
 * aggregated; the coarsest level has none). */
rs_status rs_cpr_level(rs_cpr M, int l, int *h_n, int64_t *h_nnz, int32_t *h_rp,
                       int32_t *h_ci, double *h_a, double *h_dl1, int32_t *h_agg);
/* Smoothed prolongator of level l (to level l+1) as CSR on the host:
 * *h_nnz entries (always filled), then, when the arrays are given, row
 * pointers h_rp[n+1], coarse columns h_ci (ascending in each row) and FP64
 * values h_v.  RS_E_ARG when level l has the piecewise-constant prolongator
 * (rs_cpr_opts.smooth = 0) or is the coarsest. */
rs_status rs_cpr_level_p(rs_cpr M, int l, int64_t *h_nnz, int32_t *h_rp, int32_t *h_ci, double *h_v);
/* Second-stage block inverses (16*n doubles, upcast if FP32). */
rs_status rs_cpr_smoother_get(rs_cpr M, double *h_dinv2);
/* Inverse of a dense n x n FP64 matrix (row-major, device) by the kernels
 * that invert the coarsest AMG level (Gauss-Jordan with partial pivoting:
 * register tiles up to n = 156, one workgroup up to 256, one launch pair per
 * column beyond); 16 n^2 bytes of scratch.  A zero pivot gives
 * RS_E_SINGULAR. */
rs_status rs_dense_inverse(int n, const double *d_a, double *d_inv, void *stream);
/* rs_dense_inverse without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels and result as rs_dense_inverse (bitwise).
 * n <= RS_DENSE_NOALLOC_MAX, else RS_E_ARG.  The scratch (the n x 2n
 * augmented matrix and the singular flag, 16 MiB + 256 B) is a static device
 * array of the library: one copy per GPU, held until the process ends, and
 * shared by every call on that GPU.  Calls that overlap on one GPU (several
 * streams or host threads) race on it and must be serialised by the caller.
 * d_a and d_inv (n*n doubles, device) may alias.  The call synchronises the
 * stream to read the singular flag; a zero pivot gives RS_E_SINGULAR. */
#define RS_DENSE_NOALLOC_MAX 1024
rs_status rs_dense_inverse_noalloc(int n, const double *d_a, double *d_inv, void *stream);
/* One V-cycle on the pressure hierarchy, b -> x (n doubles each, device). */
rs_status rs_cpr_vcycle(rs_cpr M, const double *d_b, double *d_x, void *stream);

#ifdef __cplusplus
}
#endif
#endif
