/* oracle.h -- plain, slow FP64 CPU reference for the CPR-GMRES linear solve
 * of Liu & Chen, "A Scalable Thermal Reservoir Simulator for Giant Models on
 * Parallel Computers" (arXiv 1812.03952).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library
 * against the paper's definitions.  It is called by the test suite, by the
 * smoke check in __graft_entry__.py and by the CPU-baseline leg of the
 * benchmark, and by nothing else.  It shares no code, header, table or
 * constant generator with the HIP library and must never be linked into it.
 *
 * Conventions
 *   - Grid cells are numbered c = i + nx*(j + ny*k), 0-based, i fastest
 *     (the paper numbers unknowns grid block by grid block, Eq. mat-ja).
 *   - A block-sparse matrix is CSR over 4x4 blocks: rp[n+1], ci[nnzb]
 *     (columns ascending within a row), v[16*nnzb] (block k is row-major at
 *     v + 16*k).  Vectors hold 4 unknowns per cell, unknown 0 = pressure.
 *   - Every routine works in IEEE double, one operation at a time, in the
 *     order written; build with -ffp-contract=off so no FMA is formed.
 *   - Return codes: 0 ok, -1 bad argument, -4 singular block, -5 non-finite.
 *
 * Parity status per function is stated at its definition in the .c files.
 */
#ifndef RS_ORACLE_H
#define RS_ORACLE_H
#include <stdint.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_SINGULAR (-4)
#define OR_E_NONFINITE (-5)

/* ---- grid pattern and assembly (Section "Numerical Methods": transmissibility) */
int64_t or_nnzb(int nx, int ny, int nz);
int or_pattern(int nx, int ny, int nz, int *rp, int *ci);
int or_assemble(int nx, int ny, int nz, const double *logk, double kvkh, double tscale,
                const double *Mf, const double *Mb, const double *B, double dt,
                int nw, const int *wcell, const double *wu,
                const int *rp, const int *ci, double *v);

/* ---- block matrix operations (Section "Linear System", Fig. fig-mv) */
void or_spmv(int n, const int *rp, const int *ci, const double *v,
             const double *x, double *y);
int or_transpose(int n, const int *rp, const int *ci, const double *v, double *vt);

/* ---- decoupling (Section "Decoupling Methods", Eqs. decoupled-eq, decoupled-abf) */
#define OR_ABF 0
#define OR_QIMPES 1
#define OR_FRS 2        /* full row sum, Eq. decoupled-frs */
#define OR_FRS_ABF 3    /* two-stage: FRS, then ABF */
int or_decouple(int n, const int *rp, const int *ci, const double *v, int method,
                double *vt, double *dinv);
void or_extract_pressure(int64_t nnzb, const double *vt, double *ap);

/* ---- second stage: block-Jacobi (RAS with zero overlap) and block ILU(0) */
int or_bj_setup(int n, const int *rp, const int *ci, const double *vt, double *dinv2);
int or_dilu_setup(int n, const int *rp, const int *ci, const double *vt, double *dinv2);
void or_bj_apply(int n, const double *dinv2, const double *r, double *z);
void or_dilu_apply(int n, const int *rp, const int *ci, const double *vt,
                   const double *dinv2, const double *r, double *z);
int or_ras_restrict(int n, int64_t sub, const int *rp, const int *ci, const double *vt,
                    int **rp2, int **ci2, double **vt2);
void or_free(void *p);

/* ---- restricted additive Schwarz with overlap (ras.c) */
typedef struct or_rasov or_rasov;
or_rasov *or_rasov_setup(int n, const int *rp, const int *ci, const double *vt, int64_t sub, int ov,
                         int *status);
void or_rasov_apply(const or_rasov *R, const double *vt, const double *r, double *z);
void or_rasov_owned_dinv(const or_rasov *R, double *dinv2);
int or_rasov_ext(const or_rasov *R, int m, int *ext);
void or_rasov_ext_dinv(const or_rasov *R, int m, double *dinv);
void or_rasov_free(or_rasov *R);

/* ---- aggregation AMG on the pressure matrix (Fig. fig-ds-amg-par parameters) */
typedef struct or_amg or_amg;
typedef struct {
  double theta;         /* strength threshold                         */
  double max_row_sum;   /* rows with |row sum| > this*|a_ii| are weak  */
  int coarse_n;         /* stop coarsening at or below this many rows  */
  int max_levels;       /* hierarchy depth limit                       */
  int lu_max;           /* largest coarsest level solved by dense LU   */
  int coarse_sweeps;    /* l1-Jacobi sweeps when the coarsest is larger */
  int smooth;           /* 0: piecewise-constant P; 1: smoothed P        */
  double trunc;         /* smoothed P: interpolation truncation factor   */
} or_amg_opts;
void or_amg_defaults(or_amg_opts *o);
or_amg *or_amg_setup(int n, const int *rp, const int *ci, const double *a,
                     const or_amg_opts *o, int *status);
int or_amg_nlevels(const or_amg *h);
int or_amg_level_n(const or_amg *h, int l);
int64_t or_amg_level_nnz(const or_amg *h, int l);
void or_amg_level_get(const or_amg *h, int l, int *rp, int *ci, double *a,
                      double *dl1, int *agg, int *strong);
int or_amg_coarsest_is_lu(const or_amg *h);
/* smoothed prolongator of level l (to level l+1): returns its number of
 * entries; fills prp[n+1], pci, pv when they are not NULL.  -1 when level l
 * has the piecewise-constant P (its agg array) or is the coarsest. */
int64_t or_amg_level_p(const or_amg *h, int l, int *prp, int *pci, double *pv);
void or_amg_vcycle(const or_amg *h, const double *b, double *x);
void or_amg_free(or_amg *h);

/* ---- two-stage CPR preconditioner (Section "Preconditioners") */
#define OR_SM_BJ 0
#define OR_SM_DILU 1
#define OR_SM_RAS 2     /* zero-overlap RAS, DILU in each subdomain of sub cells */
#define OR_SM_RAS1 3    /* RAS with overlap 1 (ras.c), DILU in each extended subdomain */
typedef struct or_cpr or_cpr;
or_cpr *or_cpr_setup(int n, const int *rp, const int *ci, const double *v,
                     int method, int smoother, int64_t sub, int stages,
                     const or_amg_opts *ao, int *status);
void or_cpr_apply(const or_cpr *M, const double *r, double *z);
const double *or_cpr_decoupled(const or_cpr *M);
const double *or_cpr_dinv(const or_cpr *M);
const double *or_cpr_dinv2(const or_cpr *M);
const double *or_cpr_pressure(const or_cpr *M);
const or_amg *or_cpr_amg(const or_cpr *M);
void or_cpr_free(or_cpr *M);

/* ---- restarted flexible GMRES (Section "Linear Solver") */
typedef struct {
  int iters, cycles, status;
  double relres;        /* true ||b-Ax||/||b|| at exit */
} or_info;
int or_gmres(int n, const int *rp, const int *ci, const double *v, const or_cpr *M,
             const double *b, double *x, int restart, double rtol, int maxit,
             or_info *info, double *hist, int hist_len);

/* ---- right-preconditioned BiCGSTAB (Section "Linear Solver") */
int or_bicgstab(int n, const int *rp, const int *ci, const double *v, const or_cpr *M,
                const double *b, double *x, double rtol, int maxit, or_info *info,
                double *hist, int hist_len);

/* ---- thermal model subset: residual and Jacobian of one Newton step (thermal.c) */
typedef struct {
  double dx, dy, dz, dt;                  /* cell sizes (ft), time step (day)           */
  double ctrans;                          /* transmissibility constant                  */
  double p_ref, t_ref;                    /* reference pressure (psi), temperature (F)  */
  double rhow_ref, cpw, ct1w, ct2w, cptw; /* water density correlation                  */
  double rhoo_ref, cpo, ct1o, ct2o, cpto; /* oil component density correlation          */
  double avisc_o, bvisc_o;                /* oil viscosity avisc exp(bvisc / T_abs)     */
  double cpl_o;                           /* oil liquid heat capacity, Btu/(lbmole F)   */
  double cpg[5], hvr_w, ev_w, tcrit_w;    /* water gas-based enthalpy (J/gmol, deg C)   */
  double por_ref, cpor;                   /* linear porosity                            */
  double cp_rock;                         /* rock heat capacity, Btu/(ft^3 F)           */
  double kw, ko, kr;                      /* thermal conductivities, Btu/(ft day F)     */
  double pv_btu, jmol_btu;                /* unit factors: psi ft^3 and J/gmol in Btu   */
  double p_bh, t_inj;                     /* producer bottom-hole pressure, injection T */
  double bbl_ft3;                         /* bbl -> ft^3                                */
} or_thermal_params;
void or_thermal_defaults(or_thermal_params *q);
int or_thermal_assemble(int nx, int ny, int nz, const or_thermal_params *q, const double *kx,
                        const double *ky, const double *kz, const double *u, const double *uold, int nw,
                        const int *wcell, const int *wkind, const double *wval, const int *rp, const int *ci,
                        double *vals, double *res);
void or_thermal_props(const or_thermal_params *q, const double *u, double *out);
double or_relperm(int which, double s, double *slope);
double or_stone2(double sw, double sg, double *d_sw, double *d_sg);
double or_water_visc(double t, double *dmu_dt);
double or_water_enthalpy(const or_thermal_params *q, double t, double *dh_dt);
void or_thermal_state(const or_thermal_params *q, int n, const double *p, const double *sw, const double *so,
                      const double *t, double *u);

/* ---- adjoint gradient with respect to log-permeability */
int or_grad_logk(int nx, int ny, int nz, const double *logk, double kvkh, double tscale,
                 const double *Mf, const double *Mb, int nw, const int *wcell,
                 const double *wu, const double *lam, const double *x, double *g);

#endif
