// thermal.hip -- the linear system of one Newton step of a water / oil /
// energy subset of the paper's thermal model, assembled on the device: the
// residual R(u) and the Jacobian dR/du as 4x4 blocks in the caller's CSR
// layout of the 7-point pattern, ready for rs_bsr_attach_decouple.
//
// Per cell, unknowns (p, N_w, N_o, T) and equations (water, oil, energy,
// saturation constraint in volume form), with Eqs. eq4.1-eq4.3 of Section
// "Mathematical Model" discretised as in Section "Numerical Methods"
// (backward Euler; face transmissibility = harmonic geometric part times the
// upstream fluid part); the model, its constants and their sources are
// listed with rs_thermal_assemble in rsolve.h.
//
// One thread per cell: it evaluates its own properties and those of each
// neighbour across its six faces, and writes its whole block row (diagonal,
// up to six off-diagonal blocks) and its residual, so no two threads write
// the same place.  The face flow seen from either side is the same number
// (up to sign): the upstream cell is the one of higher pressure, on a tie
// the lower-numbered one, whichever cell computes it.
#include "rs_internal.h"
#include <math.h>

namespace {
#include "csr7.h"

// Fig. rela-swt of the paper: S_w, k_rw, k_row
__constant__ double kSwt[12][3] = {
    {0.45, 0.0, 0.4},       {0.47, 0.000056, 0.361},    {0.50, 0.000552, 0.30625},  {0.55, 0.00312, 0.225},
    {0.60, 0.00861, 0.15625}, {0.65, 0.01768, 0.1},     {0.70, 0.03088, 0.05625},   {0.75, 0.04871, 0.025},
    {0.77, 0.05724, 0.016}, {0.80, 0.07162, 0.00625},   {0.82, 0.08229, 0.00225},   {0.85, 0.1, 0.0}};
// Fig. rela-slt: S_l, k_rg, k_rog
__constant__ double kSlt[19][3] = {
    {0.45, 0.2, 0.0},         {0.55, 0.14202, 0.0},     {0.57, 0.13123, 0.00079}, {0.60, 0.11560, 0.00494},
    {0.62, 0.10555, 0.00968}, {0.65, 0.09106, 0.01975}, {0.67, 0.08181, 0.02844}, {0.70, 0.06856, 0.04444},
    {0.72, 0.06017, 0.05709}, {0.75, 0.04829, 0.07901}, {0.77, 0.04087, 0.09560}, {0.80, 0.03054, 0.12346},
    {0.83, 0.02127, 0.15486}, {0.85, 0.01574, 0.17778}, {0.87, 0.01080, 0.20227}, {0.90, 0.00467, 0.24198},
    {0.92, 0.00165, 0.27042}, {0.94, 0.0, 0.30044},     {1.0, 0.0, 0.4}};
// Fig. fig-wat-vis: deg C, cp
__constant__ double kWvis[28][2] = {
    {5.0, 1.5182},       {8.0, 1.386},       {10.0, 1.311},      {20.0, 1.005},      {30.0, 0.8004},
    {40.0, 0.6543},      {50.0, 0.5518},     {60.0, 0.4714},     {70.0, 0.4066},     {80.0, 0.3570},
    {90.0, 0.3182},      {100.0, 0.2828},    {125.0, 0.2227},    {150.0, 0.1848},    {175.0, 0.1586},
    {200.0, 0.1394},     {225.0, 0.1238},    {250.0, 0.1117},    {275.0, 0.1005},    {300.0, 9.9125e-2},
    {325.0, 8.4075e-2},  {350.0, 7.7437e-2}, {375.0, 7.2818e-2}, {400.0, 7.2818e-2}, {500.0, 7.2818e-2},
    {600.0, 7.2818e-2},  {700.0, 7.2818e-2}, {800.0, 7.2818e-2}};

// piecewise-linear table value and slope at x (columns of a row-major table
// of `cols` columns; constant beyond the first and last abscissa)
template <int ROWS, int COLS>
__device__ double table_lin(const double (&tab)[ROWS][COLS], int col, double x, double &slope) {
  if (x <= tab[0][0]) { slope = 0.0; return tab[0][col]; }
  if (x >= tab[ROWS - 1][0]) { slope = 0.0; return tab[ROWS - 1][col]; }
  int lo = 0, hi = ROWS - 1;                 // tab[lo][0] <= x < tab[hi][0]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x < tab[mid][0]) hi = mid; else lo = mid;
  }
  const double x0 = tab[lo][0], x1 = tab[hi][0], y0 = tab[lo][col], y1 = tab[hi][col];
  slope = (y1 - y0) / (x1 - x0);
  return y0 + (y1 - y0) * (x - x0) / (x1 - x0);
}

// everything the flows, the accumulation and the constraint need of a cell
struct tcell {
  double p, t;
  double lw, lo, lw_u[4], lo_u[4];   // mole mobilities k_r rho / mu and their u-gradients
  double hw, hw_t, ho;               // enthalpies (Btu/lbmole); dH_o/dT = cpl_o
  double kt, kt_u[4];                // thermal conductivity
  double e, e_u[4];                  // energy per bulk volume
  double vol, vol_u[4];              // phi - N_w/rho_w - N_o/rho_o
};

__device__ double water_h(const rs_thermal_params &q, double t, double &dh) {
  const double tc = (t - 32.0) / 1.8, tr = (q.t_ref - 32.0) / 1.8;
  // integral of c0 + c1 s + ... + c4 s^4 from tr to tc, and the integrand at tc
  double h = 0.0, cp = 0.0;
  double pc = tc, pr = tr, pw = 1.0;
  for (int k = 0; k < 5; ++k) {
    h += q.cpg[k] * (pc - pr) / (k + 1);
    cp += q.cpg[k] * pw;
    pc *= tc; pr *= tr; pw *= tc;
  }
  double hv = 0.0, dhv = 0.0;              // heat of vaporisation, zero above T_crit
  if (tc < q.tcrit_w) {
    const double g = pow(q.tcrit_w - tc, q.ev_w - 1.0);
    hv = q.hvr_w * g * (q.tcrit_w - tc);
    dhv = -q.hvr_w * q.ev_w * g;
  }
  dh = (cp - dhv) * q.jmol_btu / 1.8;
  return (h - hv) * q.jmol_btu;
}

__device__ void cell_eval(const rs_thermal_params &q, const double *__restrict__ u4, tcell &c) {
  const double p = u4[0], nw = u4[1], no = u4[2], t = u4[3];
  const double dp = p - q.p_ref, dT = t - q.t_ref;
  c.p = p; c.t = t;
  const double phi = q.por_ref * (1.0 + q.cpor * dp), phi_p = q.por_ref * q.cpor;
  const double rw = q.rhow_ref * exp(q.cpw * dp - q.ct1w * dT - 0.5 * q.ct2w * dT * dT + q.cptw * dp * dT);
  const double rw_p = rw * (q.cpw + q.cptw * dT), rw_t = rw * (q.cptw * dp - q.ct1w - q.ct2w * dT);
  const double ro = q.rhoo_ref * exp(q.cpo * dp - q.ct1o * dT - 0.5 * q.ct2o * dT * dT + q.cpto * dp * dT);
  const double ro_p = ro * (q.cpo + q.cpto * dT), ro_t = ro * (q.cpto * dp - q.ct1o - q.ct2o * dT);
  // S = N / (phi rho): gradients in (p, N_w, N_o, T)
  const double aw = phi * rw, ao = phi * ro;
  const double sw = nw / aw, so = no / ao;
  const double sw_u[4] = {-sw * (phi_p * rw + phi * rw_p) / aw, 1.0 / aw, 0.0, -sw * phi * rw_t / aw};
  const double so_u[4] = {-so * (phi_p * ro + phi * ro_p) / ao, 0.0, 1.0 / ao, -so * phi * ro_t / ao};
  // relative permeabilities: k_rw, and Stone II with no gas (S_l = 1)
  double dkrw, dkrow, dkrg, dkrog, d0;
  const double krw = table_lin(kSwt, 1, sw, dkrw), krow = table_lin(kSwt, 2, sw, dkrow);
  const double krg = table_lin(kSlt, 1, 1.0, dkrg), krog = table_lin(kSlt, 2, 1.0, dkrog);
  const double krocw = table_lin(kSwt, 2, kSwt[0][0], d0);
  double kro = krocw * ((krow / krocw + krw) * (krog / krocw + krg) - krw - krg);
  double dkro = krocw * ((dkrow / krocw + dkrw) * (krog / krocw + krg) - dkrw);
  if (kro < 0.0) { kro = 0.0; dkro = 0.0; }
  // viscosities
  double dmw;
  const double mw = table_lin(kWvis, 1, (t - 32.0) / 1.8, dmw);
  dmw /= 1.8;
  const double ta = t + 459.67;
  const double mo = q.avisc_o * exp(q.bvisc_o / ta), dmo = -mo * q.bvisc_o / (ta * ta);
  c.lw = krw * rw / mw;
  c.lo = kro * ro / mo;
  for (int m = 0; m < 4; ++m) {
    const double drw = m == 0 ? rw_p : (m == 3 ? rw_t : 0.0), dro = m == 0 ? ro_p : (m == 3 ? ro_t : 0.0);
    const double dmuw = m == 3 ? dmw : 0.0, dmuo = m == 3 ? dmo : 0.0;
    c.lw_u[m] = (dkrw * sw_u[m] * rw + krw * drw) / mw - krw * rw * dmuw / (mw * mw);
    c.lo_u[m] = (dkro * sw_u[m] * ro + kro * dro) / mo - kro * ro * dmuo / (mo * mo);
  }
  // enthalpies, internal energies U = H - p/rho, energy per bulk volume
  c.hw = water_h(q, t, c.hw_t);
  c.ho = q.cpl_o * dT;
  const double uw = c.hw - q.pv_btu * p / rw, uo = c.ho - q.pv_btu * p / ro;
  const double uw_p = -q.pv_btu * (1.0 / rw - p * rw_p / (rw * rw)), uw_t = c.hw_t + q.pv_btu * p * rw_t / (rw * rw);
  const double uo_p = -q.pv_btu * (1.0 / ro - p * ro_p / (ro * ro)), uo_t = q.cpl_o + q.pv_btu * p * ro_t / (ro * ro);
  c.e = nw * uw + no * uo + (1.0 - q.por_ref) * q.cp_rock * dT;
  c.e_u[0] = nw * uw_p + no * uo_p;
  c.e_u[1] = uw;
  c.e_u[2] = uo;
  c.e_u[3] = nw * uw_t + no * uo_t + (1.0 - q.por_ref) * q.cp_rock;
  // conductivity (linear mixing) and the saturation constraint
  const double mix = sw * q.kw + so * q.ko;
  c.kt = phi * mix + (1.0 - phi) * q.kr;
  for (int m = 0; m < 4; ++m) {
    const double dphi = m == 0 ? phi_p : 0.0;
    c.kt_u[m] = dphi * (mix - q.kr) + phi * (sw_u[m] * q.kw + so_u[m] * q.ko);
  }
  c.vol = phi - nw / rw - no / ro;
  c.vol_u[0] = phi_p + nw * rw_p / (rw * rw) + no * ro_p / (ro * ro);
  c.vol_u[1] = -1.0 / rw;
  c.vol_u[2] = -1.0 / ro;
  c.vol_u[3] = nw * rw_t / (rw * rw) + no * ro_t / (ro * ro);
}

// energy per bulk volume only (the previous time step's state)
__device__ double cell_energy(const rs_thermal_params &q, const double *__restrict__ u4) {
  const double p = u4[0], nw = u4[1], no = u4[2], t = u4[3];
  const double dp = p - q.p_ref, dT = t - q.t_ref;
  const double rw = q.rhow_ref * exp(q.cpw * dp - q.ct1w * dT - 0.5 * q.ct2w * dT * dT + q.cptw * dp * dT);
  const double ro = q.rhoo_ref * exp(q.cpo * dp - q.ct1o * dT - 0.5 * q.ct2o * dT * dT + q.cpto * dp * dT);
  double dh;
  const double hw = water_h(q, t, dh), ho = q.cpl_o * dT;
  return nw * (hw - q.pv_btu * p / rw) + no * (ho - q.pv_btu * p / ro) + (1.0 - q.por_ref) * q.cp_rock * dT;
}

__global__ __launch_bounds__(128) void k_thermal(int nx, int ny, int nz, rs_thermal_params q,
                                                 const double *__restrict__ kx, const double *__restrict__ ky,
                                                 const double *__restrict__ kz, const double *__restrict__ u,
                                                 const double *__restrict__ uold, int nw,
                                                 const int32_t *__restrict__ wcell, const int32_t *__restrict__ wkind,
                                                 const double *__restrict__ wval, double *__restrict__ vals,
                                                 double *__restrict__ res) {
  const int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  tcell A;
  cell_eval(q, u + 4 * c, A);
  const double acc = q.dx * q.dy * q.dz / q.dt;
  double D[16], R[4];
  for (int e = 0; e < 16; ++e) D[e] = 0.0;
  R[0] = acc * (u[4 * c + 1] - uold[4 * c + 1]);
  R[1] = acc * (u[4 * c + 2] - uold[4 * c + 2]);
  R[2] = acc * (A.e - cell_energy(q, uold + 4 * c));
  R[3] = acc * A.vol;
  D[1] = acc;                                  // row 0, column N_w
  D[6] = acc;                                  // row 1, column N_o
  for (int m = 0; m < 4; ++m) { D[8 + m] = acc * A.e_u[m]; D[12 + m] = acc * A.vol_u[m]; }
  const csr7_row w = csr7_of((uint32_t)c, (uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
  const int64_t off[7] = {-nxy, -(int64_t)nx, -1, 0, 1, (int64_t)nx, nxy};
  for (int s = 0; s < 7; ++s) {
    if (s == 3 || !((w.mask >> s) & 1u)) continue;
    const int64_t b = c + off[s];
    tcell B;
    cell_eval(q, u + 4 * b, B);
    const int ax = s == 2 || s == 4 ? 0 : (s == 1 || s == 5 ? 1 : 2);
    const double *kk = ax == 0 ? kx : (ax == 1 ? ky : kz);
    const double area = ax == 0 ? q.dy * q.dz : (ax == 1 ? q.dx * q.dz : q.dx * q.dy);
    const double len = ax == 0 ? q.dx : (ax == 1 ? q.dy : q.dz);
    const double k1 = kk[c], k2 = kk[b];
    const double G = q.ctrans * area / len * ((k1 + k2 > 0.0) ? 2.0 * k1 * k2 / (k1 + k2) : 0.0);
    const double Gc = area / len;
    // upstream: the higher pressure, on a tie the lower-numbered cell
    const bool up_b = c < b ? (B.p > A.p) : !(A.p > B.p);
    const tcell &U = up_b ? B : A;
    const double dp = B.p - A.p;                // flow into c is positive for dp > 0
    const double fw = G * U.lw * dp, fo = G * U.lo * dp;
    const double hflux = U.lw * U.hw + U.lo * U.ho;
    const double ksum = A.kt + B.kt;
    const double kh = ksum > 0.0 ? 2.0 * A.kt * B.kt / ksum : 0.0;
    const double fe = G * hflux * dp + Gc * kh * (B.t - A.t);
    R[0] -= fw; R[1] -= fo; R[2] -= fe;
    double O[16];                                // -dF/du_b, this face's off-diagonal block
    for (int side = 0; side < 2; ++side) {      // 0: derivatives in u_c, 1: in u_b
      const tcell &X = side ? B : A;
      const bool up = side ? up_b : !up_b;
      const double sg = side ? 1.0 : -1.0;
      const double kother = side ? A.kt : B.kt;
      const double dkh_dk = ksum > 0.0 ? 2.0 * kother * kother / (ksum * ksum) : 0.0;
      for (int m = 0; m < 4; ++m) {
        const double ddp = m == 0 ? sg : 0.0;
        const double lwm = up ? U.lw_u[m] : 0.0, lom = up ? U.lo_u[m] : 0.0;
        const double hwm = (up && m == 3) ? U.hw_t : 0.0, hom = (up && m == 3) ? q.cpl_o : 0.0;
        const double dfw = G * (lwm * dp + U.lw * ddp);
        const double dfo = G * (lom * dp + U.lo * ddp);
        const double dfe = G * ((lwm * U.hw + U.lw * hwm + lom * U.ho + U.lo * hom) * dp + hflux * ddp) +
                           Gc * (dkh_dk * X.kt_u[m] * (B.t - A.t) + kh * (m == 3 ? sg : 0.0));
        if (side == 0) {
          D[m] -= dfw; D[4 + m] -= dfo; D[8 + m] -= dfe;
        } else {
          O[m] = -dfw; O[4 + m] = -dfo; O[8 + m] = -dfe; O[12 + m] = 0.0;
        }
      }
    }
    if (vals) {
      double2 *ob = (double2 *)(vals + 16 * (int64_t)csr7_pos(w, s));
      for (int e = 0; e < 8; ++e) ob[e] = make_double2(O[2 * e], O[2 * e + 1]);
    }
  }
  // wells (cells ascending and unique): binary search for this cell
  int lo = 0, hi = nw;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (wcell[mid] < c) lo = mid + 1; else hi = mid;
  }
  if (lo < nw && wcell[lo] == c) {
    if (wkind[lo] > 0) {                         // injector: water rate (bbl/day of cold water)
      double dh;
      const double qw = wval[lo] * q.bbl_ft3 * q.rhow_ref;
      R[0] -= qw;
      R[2] -= qw * water_h(q, q.t_inj, dh);
    } else if (A.p > q.p_bh) {                   // producer at bottom-hole pressure
      const double wi = q.ctrans * wval[lo], drive = A.p - q.p_bh;
      const double qw = -wi * A.lw * drive, qo = -wi * A.lo * drive;
      R[0] -= qw; R[1] -= qo; R[2] -= qw * A.hw + qo * A.ho;
      for (int m = 0; m < 4; ++m) {
        const double dd = m == 0 ? 1.0 : 0.0;
        const double dqw = -wi * (A.lw_u[m] * drive + A.lw * dd), dqo = -wi * (A.lo_u[m] * drive + A.lo * dd);
        D[m] -= dqw;
        D[4 + m] -= dqo;
        D[8 + m] -= dqw * A.hw + qw * (m == 3 ? A.hw_t : 0.0) + dqo * A.ho + qo * (m == 3 ? q.cpl_o : 0.0);
      }
    }
  }
  if (vals) {
    double2 *db = (double2 *)(vals + 16 * (int64_t)csr7_pos(w, 3));
    for (int e = 0; e < 8; ++e) db[e] = make_double2(D[2 * e], D[2 * e + 1]);
  }
  if (res) {
    double2 *rr = (double2 *)(res + 4 * c);
    rr[0] = make_double2(R[0], R[1]);
    rr[1] = make_double2(R[2], R[3]);
  }
}

// wells must be ascending and unique, inside the grid
__global__ void k_thermal_wells_check(int64_t n, int nw, const int32_t *__restrict__ wcell, int *__restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nw) return;
  if (wcell[t] < 0 || wcell[t] >= n || (t > 0 && wcell[t - 1] >= wcell[t])) atomicOr(bad, 1);
}

// (p, N_w, N_o, T) from (p, S_w, S_o, T): N = phi rho S
__global__ void k_thermal_state(int64_t n, rs_thermal_params q, const double *__restrict__ p,
                                const double *__restrict__ sw, const double *__restrict__ so,
                                const double *__restrict__ t, double *__restrict__ u) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double dp = p[c] - q.p_ref, dT = t[c] - q.t_ref;
  const double phi = q.por_ref * (1.0 + q.cpor * dp);
  const double rw = q.rhow_ref * exp(q.cpw * dp - q.ct1w * dT - 0.5 * q.ct2w * dT * dT + q.cptw * dp * dT);
  const double ro = q.rhoo_ref * exp(q.cpo * dp - q.ct1o * dT - 0.5 * q.ct2o * dT * dT + q.cpto * dp * dT);
  double2 *o = (double2 *)(u + 4 * c);
  o[0] = make_double2(p[c], phi * rw * sw[c]);
  o[1] = make_double2(phi * ro * so[c], t[c]);
}

}  // namespace

extern "C" void rs_thermal_params_default(rs_thermal_params *q) {
  if (!q) return;
  *q = rs_thermal_params{};
  q->dx = 29.17; q->dy = 29.17; q->dz = 10.0;
  q->dt = 1.0;
  q->ctrans = 1.127e-3 * 5.614583;
  q->p_ref = 14.696; q->t_ref = 60.0;
  q->rhow_ref = 3.4605; q->cpw = 3.0e-6; q->ct1w = 1.0e-4; q->ct2w = 0.0; q->cptw = 0.0;
  q->rhoo_ref = 0.2092; q->cpo = 5.0e-6; q->ct1o = 3.8e-4; q->ct2o = 0.0; q->cpto = 0.0;
  q->avisc_o = 0.287352; q->bvisc_o = 3728.2;
  q->cpl_o = 125.0;
  q->cpg[0] = 34.49885; q->cpg[1] = -0.01426; q->cpg[2] = 4.7356e-5; q->cpg[3] = -3.56759e-8;
  q->cpg[4] = 9.35531e-12;
  q->hvr_w = 4820.0; q->ev_w = 0.38; q->tcrit_w = 374.15;
  q->por_ref = 0.3; q->cpor = 5.0e-4;
  q->cp_rock = 35.0;
  q->kw = 8.6; q->ko = 1.8; q->kr = 24.0;
  q->pv_btu = 144.0 / 778.169;
  q->jmol_btu = 453.59237 / 1055.05585;
  q->p_bh = 17.0; q->t_inj = 450.0;
  q->bbl_ft3 = 5.614583;
}

extern "C" rs_status rs_thermal_assemble(int nx, int ny, int nz, const rs_thermal_params *q, const double *d_kx,
                                         const double *d_ky, const double *d_kz, const double *d_u,
                                         const double *d_uold, int nw, const int32_t *d_wcell,
                                         const int32_t *d_wkind, const double *d_wval, double *d_vals,
                                         double *d_res, void *stream) {
  if (!rs_grid_dims_ok(nx, ny, nz) || !q || !d_kx || !d_ky || !d_kz || !d_u || !d_uold || nw < 0 ||
      (nw > 0 && (!d_wcell || !d_wkind || !d_wval)) || (!d_vals && !d_res))
    return RS_E_ARG;
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t nnzb = n + 2 * ((int64_t)(nx - 1) * ny * nz + (int64_t)nx * (ny - 1) * nz + (int64_t)nx * ny * (nz - 1));
  if (n > INT32_MAX / 2 || nnzb > INT32_MAX) return RS_E_ARG;
  if (((uintptr_t)d_u | (uintptr_t)d_uold | (uintptr_t)d_vals | (uintptr_t)d_res) & 15) return RS_E_ARG;
  if (!(q->dt > 0.0) || !(q->dx > 0.0) || !(q->dy > 0.0) || !(q->dz > 0.0)) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  if (nw > 0) {
    dbuf flag;
    RS_TRY(flag.alloc(sizeof(int)));
    RS_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    k_thermal_wells_check<<<rs_grid(nw), RS_BLOCK, 0, s>>>(n, nw, d_wcell, flag.as<int>());
    int h = 0;
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    if (h) return RS_E_ARG;
  }
  k_thermal<<<rs_grid(n, 128), 128, 0, s>>>(nx, ny, nz, *q, d_kx, d_ky, d_kz, d_u, d_uold, nw, d_wcell, d_wkind,
                                           d_wval, d_vals, d_res);
  RS_HIP(hipGetLastError());
  return RS_OK;
}

extern "C" rs_status rs_thermal_state(int64_t n, const rs_thermal_params *q, const double *d_p, const double *d_sw,
                                      const double *d_so, const double *d_t, double *d_u, void *stream) {
  if (n < 1 || !q || !d_p || !d_sw || !d_so || !d_t || !d_u || ((uintptr_t)d_u & 15)) return RS_E_ARG;
  hipStream_t s = rs_stream(stream);
  k_thermal_state<<<rs_grid(n), RS_BLOCK, 0, s>>>(n, *q, d_p, d_sw, d_so, d_t, d_u);
  RS_HIP(hipGetLastError());
  return RS_OK;
}
