/* thermal.c -- residual and Jacobian of one backward-Euler Newton step of a
 * water / heavy-oil / energy subset of the paper's thermal model: the block
 * system the linear solver receives.  FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Model (Section "Mathematical Model" and Section "Numerical Methods"):
 *   - phases water (water component only) and oil (one oil component only);
 *     the gas phase is absent, so the switched constraint is S_g = 0 and the
 *     saturation constraint reads S_w + S_o = 1;
 *   - unknowns per cell, in this order: p (psi), N_w and N_o (moles of
 *     water and oil per unit bulk volume, lbmole/ft^3), T (deg F), with
 *     S_w = N_w/(phi rho_w) and S_o = N_o/(phi rho_o);
 *   - equations per cell, in this order: water and oil mole conservation
 *     (Eq. eq4.2), energy conservation (Eq. eq4.3, without heat loss), and the
 *     saturation constraint in volume form (the "one additional equation"
 *     that keeps p and T independent):
 *       R_w = V/dt (N_w - N_w^n) - sum_faces F_w - Q_w
 *       R_o = V/dt (N_o - N_o^n) - sum_faces F_o - Q_o
 *       R_E = V/dt (E - E^n)     - sum_faces F_E - Q_E
 *       R_v = V/dt (phi - N_w/rho_w - N_o/rho_o)
 *     with E = N_w U_w + N_o U_o + (1 - phi_ref) U_r (rock volume constant,
 *     the paper's default) and F the flow into the cell across a face;
 *   - Darcy's law (Eq. eq4.1) without capillary pressure (the paper's tables
 *     give none) and without gravity (the synthetic grid has no depth);
 *   - face flow of phase a: F_a = G lambda_a,up (p_nbr - p_cell), with G the
 *     geometric transmissibility (harmonic mean of the two cells'
 *     permeabilities, zero on the boundary) and the mole mobility
 *     lambda_a = k_ra rho_a / mu_a taken upstream (the cell of higher
 *     pressure; on a tie the lower-numbered cell of the face);
 *   - energy flow: sum_a F_a H_a,up plus conduction Gc K_h (T_nbr - T_cell),
 *     K_h the harmonic mean of the two cells' K_T = phi (S_w K_w + S_o K_o)
 *     + (1 - phi) K_r (the paper's linear mixing rule);
 *   - densities: the paper's exponential correlation in p and T; the oil
 *     phase has one component, so rho_o is that component's density;
 *   - viscosities: oil mu = avisc exp(bvisc / T_abs); water from the paper's
 *     viscosity table (Fig. fig-wat-vis) by linear interpolation in deg C;
 *   - relative permeabilities: the paper's swt and slt tables (Figs.
 *     rela-swt, rela-slt) by linear interpolation, Stone's model II for
 *     k_ro with S_g = 0;
 *   - enthalpies: water by the gas-based method with the paper's constants
 *     (H_w = H_g,W - H_v,W, J/gmol with t in deg C), oil by the liquid-based
 *     method with cpl1 = 0.5 Btu/(lb F) and M = 250; U = H - p/rho; rock
 *     U_r = cp_r (T - T_ref);
 *   - porosity: linear, phi = phi_ref (1 + cpor (p - p_ref));
 *   - wells (Peaceman, Eq. well-model): producers at a bottom-hole pressure
 *     with the cell's phase mobilities, Q_a = -WI lambda_a (p - p_bh) when
 *     p > p_bh (no back-flow), WI in md ft as the paper's inputs give it;
 *     injectors at a fixed water rate (bbl/day of cold water, converted with
 *     rho_w,ref) and injection temperature, Q_w = q, Q_E = q H_w(T_inj).
 * The Jacobian block (a, b) is dR_a/du_b, written in caller layout (4x4
 * row-major, rows = equations, columns = unknowns).
 * Pinned by: central finite differences of the residual (every entry of the
 * Jacobian on small grids), conservation (the face flows of a pair cancel,
 * so the flow part of every block column sums to zero), the printed table
 * values at their nodes, Stone II reducing to k_row at S_g = 0 and to k_rog
 * at connate water, and closed forms of the enthalpy integral. */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* Fig. rela-swt: S_w, k_rw, k_row */
static const double SWT[12][3] = {
  {0.45, 0.0, 0.4},         {0.47, 0.000056, 0.361}, {0.50, 0.000552, 0.30625},
  {0.55, 0.00312, 0.225},   {0.60, 0.00861, 0.15625}, {0.65, 0.01768, 0.1},
  {0.70, 0.03088, 0.05625}, {0.75, 0.04871, 0.025},  {0.77, 0.05724, 0.016},
  {0.80, 0.07162, 0.00625}, {0.82, 0.08229, 0.00225}, {0.85, 0.1, 0.0}};
/* Fig. rela-slt: S_l, k_rg, k_rog */
static const double SLT[19][3] = {
  {0.45, 0.2, 0.0},         {0.55, 0.14202, 0.0},     {0.57, 0.13123, 0.00079},
  {0.60, 0.11560, 0.00494}, {0.62, 0.10555, 0.00968}, {0.65, 0.09106, 0.01975},
  {0.67, 0.08181, 0.02844}, {0.70, 0.06856, 0.04444}, {0.72, 0.06017, 0.05709},
  {0.75, 0.04829, 0.07901}, {0.77, 0.04087, 0.09560}, {0.80, 0.03054, 0.12346},
  {0.83, 0.02127, 0.15486}, {0.85, 0.01574, 0.17778}, {0.87, 0.01080, 0.20227},
  {0.90, 0.00467, 0.24198}, {0.92, 0.00165, 0.27042}, {0.94, 0.0, 0.30044},
  {1.0, 0.0, 0.4}};
/* Fig. fig-wat-vis: temperature (deg C), water viscosity (cp) */
static const double WVIS[28][2] = {
  {5.0, 1.5182},    {8.0, 1.386},     {10.0, 1.311},    {20.0, 1.005},    {30.0, 0.8004},
  {40.0, 0.6543},   {50.0, 0.5518},   {60.0, 0.4714},   {70.0, 0.4066},   {80.0, 0.3570},
  {90.0, 0.3182},   {100.0, 0.2828},  {125.0, 0.2227},  {150.0, 0.1848},  {175.0, 0.1586},
  {200.0, 0.1394},  {225.0, 0.1238},  {250.0, 0.1117},  {275.0, 0.1005},  {300.0, 9.9125e-2},
  {325.0, 8.4075e-2}, {350.0, 7.7437e-2}, {375.0, 7.2818e-2}, {400.0, 7.2818e-2},
  {500.0, 7.2818e-2}, {600.0, 7.2818e-2}, {700.0, 7.2818e-2}, {800.0, 7.2818e-2}};

void or_thermal_defaults(or_thermal_params *q) {
  memset(q, 0, sizeof(*q));
  q->dx = 29.17; q->dy = 29.17; q->dz = 10.0;   /* the heavy-oil example's cells (ft) */
  q->dt = 1.0;                                   /* day */
  q->ctrans = 1.127e-3 * 5.614583;               /* md ft -> ft^3 cp/(day psi) */
  q->p_ref = 14.696; q->t_ref = 60.0;
  q->rhow_ref = 3.4605; q->cpw = 3.0e-6; q->ct1w = 1.0e-4; q->ct2w = 0.0; q->cptw = 0.0;
  q->rhoo_ref = 0.2092; q->cpo = 5.0e-6; q->ct1o = 3.8e-4; q->ct2o = 0.0; q->cpto = 0.0;  /* LO */
  q->avisc_o = 0.287352; q->bvisc_o = 3728.2;    /* LO, cp and deg R */
  q->cpl_o = 0.5 * 250.0;                         /* Btu/(lbmole F) */
  q->cpg[0] = 34.49885; q->cpg[1] = -0.01426; q->cpg[2] = 4.7356e-5;
  q->cpg[3] = -3.56759e-8; q->cpg[4] = 9.35531e-12;   /* water, J/gmol with t in C */
  q->hvr_w = 4820.0; q->ev_w = 0.38; q->tcrit_w = 374.15;
  q->por_ref = 0.3; q->cpor = 5.0e-4;
  q->cp_rock = 35.0;                              /* Btu/(ft^3 F) */
  q->kw = 8.6; q->ko = 1.8; q->kr = 24.0;         /* Btu/(ft day F) */
  q->pv_btu = 144.0 / 778.169;                    /* psi ft^3 -> Btu */
  q->jmol_btu = 453.59237 / 1055.05585;           /* J/gmol -> Btu/lbmole */
  q->p_bh = 17.0; q->t_inj = 450.0;               /* the heavy-oil example's wells */
  q->bbl_ft3 = 5.614583;
}

/* linear interpolation in column col of a table, constant outside */
static double interp(const double *tab, int stride, int n, int col, double x, double *slope) {
  if (x <= tab[0]) { *slope = 0.0; return tab[col]; }
  if (x >= tab[(n - 1) * stride]) { *slope = 0.0; return tab[(n - 1) * stride + col]; }
  int i = 0;
  while (!(x < tab[(i + 1) * stride])) ++i;
  double x0 = tab[i * stride], x1 = tab[(i + 1) * stride];
  double y0 = tab[i * stride + col], y1 = tab[(i + 1) * stride + col];
  *slope = (y1 - y0) / (x1 - x0);
  return y0 + (y1 - y0) * (x - x0) / (x1 - x0);
}

double or_relperm(int which, double s, double *slope) {
  double d = 0.0, v = 0.0;
  switch (which) {
    case 0: v = interp(&SWT[0][0], 3, 12, 1, s, &d); break;   /* k_rw(S_w)  */
    case 1: v = interp(&SWT[0][0], 3, 12, 2, s, &d); break;   /* k_row(S_w) */
    case 2: v = interp(&SLT[0][0], 3, 19, 1, s, &d); break;   /* k_rg(S_l)  */
    case 3: v = interp(&SLT[0][0], 3, 19, 2, s, &d); break;   /* k_rog(S_l) */
    default: break;
  }
  if (slope) *slope = d;
  return v;
}

/* Stone's model II; derivatives with respect to S_w and S_g */
double or_stone2(double sw, double sg, double *d_sw, double *d_sg) {
  double drw, drow, drg, drog;
  double krw = or_relperm(0, sw, &drw), krow = or_relperm(1, sw, &drow);
  double krg = or_relperm(2, 1.0 - sg, &drg), krog = or_relperm(3, 1.0 - sg, &drog);
  drg = -drg; drog = -drog;                       /* d/dS_g of functions of S_l = 1 - S_g */
  double dtmp;
  double krocw = or_relperm(1, SWT[0][0], &dtmp); /* k_row at connate water */
  double a = krow / krocw + krw, b = krog / krocw + krg;
  double kro = krocw * (a * b - krw - krg);
  double dsw = krocw * ((drow / krocw + drw) * b - drw);
  double dsg = krocw * (a * (drog / krocw + drg) - drg);
  if (kro < 0.0) { kro = 0.0; dsw = 0.0; dsg = 0.0; }
  if (d_sw) *d_sw = dsw;
  if (d_sg) *d_sg = dsg;
  return kro;
}

/* water viscosity (cp) at T (deg F) and its T derivative */
double or_water_visc(double t, double *dmu_dt) {
  double d;
  double mu = interp(&WVIS[0][0], 2, 28, 1, (t - 32.0) / 1.8, &d);
  if (dmu_dt) *dmu_dt = d / 1.8;
  return mu;
}

/* water enthalpy (Btu/lbmole) at T (deg F): gas-based, H_w = H_g,W - H_v,W */
double or_water_enthalpy(const or_thermal_params *q, double t, double *dh_dt) {
  double tc = (t - 32.0) / 1.8, trc = (q->t_ref - 32.0) / 1.8;
  double hg = 0.0, cpv = 0.0, tk = tc, trk = trc, tcp = 1.0;
  for (int k = 0; k < 5; ++k) {                   /* integral of sum c_k t^k from T_ref */
    hg = hg + q->cpg[k] * (tk - trk) / (double)(k + 1);
    cpv = cpv + q->cpg[k] * tcp;
    tcp = tcp * tc; tk = tk * tc; trk = trk * trc;
  }
  double hv = 0.0, dhv = 0.0;
  if (tc < q->tcrit_w) {
    hv = q->hvr_w * pow(q->tcrit_w - tc, q->ev_w);
    dhv = -q->hvr_w * q->ev_w * pow(q->tcrit_w - tc, q->ev_w - 1.0);
  }
  if (dh_dt) *dh_dt = (cpv - dhv) * q->jmol_btu / 1.8;
  return (hg - hv) * q->jmol_btu;
}

typedef struct {
  double p, nw, no, t;
  double phi, phi_p;
  double rw, rw_p, rw_t, ro, ro_p, ro_t;
  double sw, sw_u[4], so, so_u[4];
  double lw, lw_u[4], lo, lo_u[4];               /* mole mobilities */
  double hw, hw_t, ho, ho_t;
  double e, e_u[4];                               /* energy per bulk volume */
  double kt, kt_u[4];                             /* thermal conductivity */
  double vol, vol_u[4];                           /* phi - N_w/rho_w - N_o/rho_o */
} cellp;

static void props(const or_thermal_params *q, const double *u, cellp *c) {
  memset(c, 0, sizeof(*c));
  c->p = u[0]; c->nw = u[1]; c->no = u[2]; c->t = u[3];
  double dp = c->p - q->p_ref, dT = c->t - q->t_ref;
  c->phi = q->por_ref * (1.0 + q->cpor * dp);
  c->phi_p = q->por_ref * q->cpor;
  c->rw = q->rhow_ref * exp(q->cpw * dp - q->ct1w * dT - 0.5 * q->ct2w * dT * dT + q->cptw * dp * dT);
  c->rw_p = c->rw * (q->cpw + q->cptw * dT);
  c->rw_t = c->rw * (-q->ct1w - q->ct2w * dT + q->cptw * dp);
  c->ro = q->rhoo_ref * exp(q->cpo * dp - q->ct1o * dT - 0.5 * q->ct2o * dT * dT + q->cpto * dp * dT);
  c->ro_p = c->ro * (q->cpo + q->cpto * dT);
  c->ro_t = c->ro * (-q->ct1o - q->ct2o * dT + q->cpto * dp);
  /* saturations S = N / (phi rho) */
  double fw = c->phi * c->rw, fo = c->phi * c->ro;
  c->sw = c->nw / fw;
  c->sw_u[0] = -c->nw * (c->phi_p * c->rw + c->phi * c->rw_p) / (fw * fw);
  c->sw_u[1] = 1.0 / fw;
  c->sw_u[3] = -c->nw * c->phi * c->rw_t / (fw * fw);
  c->so = c->no / fo;
  c->so_u[0] = -c->no * (c->phi_p * c->ro + c->phi * c->ro_p) / (fo * fo);
  c->so_u[2] = 1.0 / fo;
  c->so_u[3] = -c->no * c->phi * c->ro_t / (fo * fo);
  /* relative permeabilities: k_rw(S_w), Stone II k_ro(S_w, S_g = 0) */
  double dkrw, dkro;
  double krw = or_relperm(0, c->sw, &dkrw);
  double kro = or_stone2(c->sw, 0.0, &dkro, NULL);
  /* viscosities */
  double dmw;
  double mw = or_water_visc(c->t, &dmw);
  double tabs = c->t + 459.67;
  double mo = q->avisc_o * exp(q->bvisc_o / tabs);
  double dmo = -mo * q->bvisc_o / (tabs * tabs);
  /* mole mobilities lambda = k_r rho / mu */
  c->lw = krw * c->rw / mw;
  c->lo = kro * c->ro / mo;
  for (int k = 0; k < 4; ++k) {
    double rwk = k == 0 ? c->rw_p : (k == 3 ? c->rw_t : 0.0);
    double rok = k == 0 ? c->ro_p : (k == 3 ? c->ro_t : 0.0);
    double mwk = k == 3 ? dmw : 0.0, mok = k == 3 ? dmo : 0.0;
    c->lw_u[k] = (dkrw * c->sw_u[k] * c->rw + krw * rwk) / mw - krw * c->rw * mwk / (mw * mw);
    c->lo_u[k] = (dkro * c->sw_u[k] * c->ro + kro * rok) / mo - kro * c->ro * mok / (mo * mo);
  }
  /* enthalpies and internal energies */
  c->hw = or_water_enthalpy(q, c->t, &c->hw_t);
  c->ho = q->cpl_o * dT;
  c->ho_t = q->cpl_o;
  double uw = c->hw - q->pv_btu * c->p / c->rw, uo = c->ho - q->pv_btu * c->p / c->ro;
  double uw_p = -q->pv_btu * (1.0 / c->rw - c->p * c->rw_p / (c->rw * c->rw));
  double uw_t = c->hw_t + q->pv_btu * c->p * c->rw_t / (c->rw * c->rw);
  double uo_p = -q->pv_btu * (1.0 / c->ro - c->p * c->ro_p / (c->ro * c->ro));
  double uo_t = c->ho_t + q->pv_btu * c->p * c->ro_t / (c->ro * c->ro);
  double ur = q->cp_rock * dT;
  c->e = c->nw * uw + c->no * uo + (1.0 - q->por_ref) * ur;
  c->e_u[0] = c->nw * uw_p + c->no * uo_p;
  c->e_u[1] = uw;
  c->e_u[2] = uo;
  c->e_u[3] = c->nw * uw_t + c->no * uo_t + (1.0 - q->por_ref) * q->cp_rock;
  /* conductivity, linear mixing */
  c->kt = c->phi * (c->sw * q->kw + c->so * q->ko) + (1.0 - c->phi) * q->kr;
  for (int k = 0; k < 4; ++k) {
    double phk = k == 0 ? c->phi_p : 0.0;
    c->kt_u[k] = phk * (c->sw * q->kw + c->so * q->ko) + c->phi * (c->sw_u[k] * q->kw + c->so_u[k] * q->ko)
                 - phk * q->kr;
  }
  /* saturation constraint in volume form */
  c->vol = c->phi - c->nw / c->rw - c->no / c->ro;
  c->vol_u[0] = c->phi_p + c->nw * c->rw_p / (c->rw * c->rw) + c->no * c->ro_p / (c->ro * c->ro);
  c->vol_u[1] = -1.0 / c->rw;
  c->vol_u[2] = -1.0 / c->ro;
  c->vol_u[3] = c->nw * c->rw_t / (c->rw * c->rw) + c->no * c->ro_t / (c->ro * c->ro);
}

/* block (row-major 4x4) of stored block index pos */
static double *blk(double *vals, int64_t pos) { return vals + 16 * pos; }

static int64_t find_pos(const int *rp, const int *ci, int row, int col) {
  for (int64_t p = rp[row]; p < rp[row + 1]; ++p)
    if (ci[p] == col) return p;
  return -1;
}

int or_thermal_assemble(int nx, int ny, int nz, const or_thermal_params *q, const double *kx,
                        const double *ky, const double *kz, const double *u, const double *uold, int nw,
                        const int *wcell, const int *wkind, const double *wval, const int *rp, const int *ci,
                        double *vals, double *res) {
  int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
  if (n < 1) return OR_E_ARG;
  cellp *cp = (cellp *)malloc(sizeof(cellp) * (size_t)n);
  for (int64_t c = 0; c < n; ++c) props(q, &u[4 * c], &cp[c]);
  const double vb = q->dx * q->dy * q->dz, acc = vb / q->dt;
  if (vals) memset(vals, 0, sizeof(double) * 16 * (size_t)rp[n]);
  if (res) memset(res, 0, sizeof(double) * 4 * (size_t)n);
  int status = OR_OK;
  /* accumulation and the constraint */
  for (int64_t c = 0; c < n && status == OR_OK; ++c) {
    cellp o;
    props(q, &uold[4 * c], &o);
    if (res) {
      res[4 * c + 0] = acc * (cp[c].nw - o.nw);
      res[4 * c + 1] = acc * (cp[c].no - o.no);
      res[4 * c + 2] = acc * (cp[c].e - o.e);
      res[4 * c + 3] = acc * cp[c].vol;
    }
    if (vals) {
      int64_t pd = find_pos(rp, ci, (int)c, (int)c);
      if (pd < 0) { status = OR_E_ARG; break; }
      double *D = blk(vals, pd);
      D[4 * 0 + 1] += acc;
      D[4 * 1 + 2] += acc;
      for (int k = 0; k < 4; ++k) {
        D[4 * 2 + k] += acc * cp[c].e_u[k];
        D[4 * 3 + k] += acc * cp[c].vol_u[k];
      }
    }
  }
  /* faces: each interior face once, its flows added to both cells */
  for (int64_t a = 0; a < n && status == OR_OK; ++a) {
    int i = (int)(a % nx), j = (int)((a / nx) % ny), k = (int)(a / nxy);
    for (int d = 0; d < 3; ++d) {
      int64_t b;
      double area, len, ka, kb;
      if (d == 0) { if (i + 1 >= nx) continue; b = a + 1; area = q->dy * q->dz; len = q->dx; ka = kx[a]; kb = kx[b]; }
      else if (d == 1) { if (j + 1 >= ny) continue; b = a + nx; area = q->dx * q->dz; len = q->dy; ka = ky[a]; kb = ky[b]; }
      else { if (k + 1 >= nz) continue; b = a + nxy; area = q->dx * q->dy; len = q->dz; ka = kz[a]; kb = kz[b]; }
      double kh = (ka + kb > 0.0) ? 2.0 * ka * kb / (ka + kb) : 0.0;
      double G = q->ctrans * area / len * kh, Gc = area / len;
      const cellp *A = &cp[a], *B = &cp[b];
      double dp = B->p - A->p;
      const cellp *U = dp > 0.0 ? B : A;         /* upstream: higher pressure, ties to a (< b) */
      int up_b = dp > 0.0;
      /* flows into a (the flow into b is their negative) */
      double fw = G * U->lw * dp, fo = G * U->lo * dp;
      double fe_c = G * (U->lw * U->hw + U->lo * U->ho) * dp;
      double ks = A->kt + B->kt;
      double kth = ks > 0.0 ? 2.0 * A->kt * B->kt / ks : 0.0;
      double fe = fe_c + Gc * kth * (B->t - A->t);
      if (res) {
        res[4 * a + 0] -= fw; res[4 * a + 1] -= fo; res[4 * a + 2] -= fe;
        res[4 * b + 0] += fw; res[4 * b + 1] += fo; res[4 * b + 2] += fe;
      }
      if (!vals) continue;
      /* derivatives of (fw, fo, fe) with respect to u_a (s = 0) and u_b (s = 1) */
      double dfw[2][4], dfo[2][4], dfe[2][4];
      for (int s = 0; s < 2; ++s) {
        const cellp *X = s ? B : A;
        int is_up = (s == 1) == up_b;
        double sgn = s ? 1.0 : -1.0;               /* d dp / d p_x */
        for (int m = 0; m < 4; ++m) {
          double ddp = m == 0 ? sgn : 0.0;
          double lw_m = is_up ? U->lw_u[m] : 0.0, lo_m = is_up ? U->lo_u[m] : 0.0;
          double hw_m = (is_up && m == 3) ? U->hw_t : 0.0, ho_m = (is_up && m == 3) ? U->ho_t : 0.0;
          dfw[s][m] = G * (lw_m * dp + U->lw * ddp);
          dfo[s][m] = G * (lo_m * dp + U->lo * ddp);
          double conv = G * ((lw_m * U->hw + U->lw * hw_m + lo_m * U->ho + U->lo * ho_m) * dp +
                             (U->lw * U->hw + U->lo * U->ho) * ddp);
          /* d kth / d K_x = 2 K_other^2 / (K_a + K_b)^2 */
          double ko_ = s ? A->kt : B->kt;
          double dkth = ks > 0.0 ? 2.0 * ko_ * ko_ / (ks * ks) * X->kt_u[m] : 0.0;
          double dT = m == 3 ? sgn : 0.0;
          dfe[s][m] = conv + Gc * (dkth * (B->t - A->t) + kth * dT);
        }
      }
      int64_t paa = find_pos(rp, ci, (int)a, (int)a), pab = find_pos(rp, ci, (int)a, (int)b);
      int64_t pba = find_pos(rp, ci, (int)b, (int)a), pbb = find_pos(rp, ci, (int)b, (int)b);
      if (paa < 0 || pab < 0 || pba < 0 || pbb < 0) { status = OR_E_ARG; break; }
      for (int m = 0; m < 4; ++m) {
        /* R_a -= f:  dR_a/du_a -= df/du_a,  dR_a/du_b -= df/du_b */
        blk(vals, paa)[0 * 4 + m] -= dfw[0][m]; blk(vals, pab)[0 * 4 + m] -= dfw[1][m];
        blk(vals, paa)[1 * 4 + m] -= dfo[0][m]; blk(vals, pab)[1 * 4 + m] -= dfo[1][m];
        blk(vals, paa)[2 * 4 + m] -= dfe[0][m]; blk(vals, pab)[2 * 4 + m] -= dfe[1][m];
        /* R_b += f */
        blk(vals, pba)[0 * 4 + m] += dfw[0][m]; blk(vals, pbb)[0 * 4 + m] += dfw[1][m];
        blk(vals, pba)[1 * 4 + m] += dfo[0][m]; blk(vals, pbb)[1 * 4 + m] += dfo[1][m];
        blk(vals, pba)[2 * 4 + m] += dfe[0][m]; blk(vals, pbb)[2 * 4 + m] += dfe[1][m];
      }
    }
  }
  /* wells */
  for (int w = 0; w < nw && status == OR_OK; ++w) {
    int64_t c = wcell[w];
    if (c < 0 || c >= n) { status = OR_E_ARG; break; }
    const cellp *C = &cp[c];
    double qw = 0.0, qo = 0.0, qe = 0.0, dqw[4] = {0, 0, 0, 0}, dqo[4] = {0, 0, 0, 0}, dqe[4] = {0, 0, 0, 0};
    if (wkind[w] > 0) {                           /* injector: water rate in bbl/day (cold water) */
      double dh;
      qw = wval[w] * q->bbl_ft3 * q->rhow_ref;
      qe = qw * or_water_enthalpy(q, q->t_inj, &dh);
    } else if (C->p > q->p_bh) {                   /* producer at bottom-hole pressure, WI in md ft */
      double wi = q->ctrans * wval[w], drive = C->p - q->p_bh;
      qw = -wi * C->lw * drive;
      qo = -wi * C->lo * drive;
      qe = qw * C->hw + qo * C->ho;
      for (int m = 0; m < 4; ++m) {
        double ddr = m == 0 ? 1.0 : 0.0;
        dqw[m] = -wi * (C->lw_u[m] * drive + C->lw * ddr);
        dqo[m] = -wi * (C->lo_u[m] * drive + C->lo * ddr);
        dqe[m] = dqw[m] * C->hw + qw * (m == 3 ? C->hw_t : 0.0) + dqo[m] * C->ho + qo * (m == 3 ? C->ho_t : 0.0);
      }
    }
    if (res) { res[4 * c + 0] -= qw; res[4 * c + 1] -= qo; res[4 * c + 2] -= qe; }
    if (vals) {
      int64_t pd = find_pos(rp, ci, (int)c, (int)c);
      for (int m = 0; m < 4; ++m) {
        blk(vals, pd)[0 * 4 + m] -= dqw[m];
        blk(vals, pd)[1 * 4 + m] -= dqo[m];
        blk(vals, pd)[2 * 4 + m] -= dqe[m];
      }
    }
  }
  free(cp);
  return status;
}

/* properties of one state, for tests: S_w, S_o, lambda_w, lambda_o, H_w, H_o,
 * E, K_T, vol (9 values) */
void or_thermal_props(const or_thermal_params *q, const double *u, double *out) {
  cellp c;
  props(q, u, &c);
  out[0] = c.sw; out[1] = c.so; out[2] = c.lw; out[3] = c.lo; out[4] = c.hw; out[5] = c.ho;
  out[6] = c.e; out[7] = c.kt; out[8] = c.vol;
}

/* Unknowns (p, N_w, N_o, T) of n cells from pressures, saturations and
 * temperatures: N = phi(p) rho(p, T) S, for building test states. */
void or_thermal_state(const or_thermal_params *q, int n, const double *p, const double *sw, const double *so,
                      const double *t, double *u) {
  for (int64_t c = 0; c < n; ++c) {
    double u0[4] = {p[c], 0.0, 0.0, t[c]};
    cellp cc;
    props(q, u0, &cc);
    u[4 * c + 0] = p[c];
    u[4 * c + 1] = cc.phi * cc.rw * sw[c];
    u[4 * c + 2] = cc.phi * cc.ro * so[c];
    u[4 * c + 3] = t[c];
  }
}
