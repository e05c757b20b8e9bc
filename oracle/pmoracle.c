/*
 * pmoracle.c -- FP64 CPU reference ("oracle") for the MRT lattice Boltzmann
 * model of arXiv:2011.15073: D2Q9 MRT flow with Boussinesq buoyancy and a
 * porous (Brinkman-Forchheimer) force, a local modified power-law viscosity,
 * and a D2Q5 MRT thermal field in a square cavity.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg to check the HIP path.  Never on the product
 * path.  It shares no code with the GPU library.
 *
 * Plain and slow on purpose: every node is collided with explicit 9x9 and
 * 5x5 matrix products (moments m = M f, equilibria m_eq = M f_eq, forcing
 * F_m = M F_i, back-transform with a numerically inverted M), then streamed
 * from a separate post-collision copy.  Compile with -O2 -fno-fast-math
 * -ffp-contract=off.
 *
 * Citations are to the paper's sections and equations:
 *   Sec. "Multiple-Relaxation-Time Lattice Boltzmann Method": Eq. (12) the MRT
 *     LBE with forcing, Eq. (13) S, Eq. (14) the D2Q9 velocities, Eq. (15)
 *     nu = c_s^2 (tau - 1/2), Eqs. (16)-(17) rho and u.
 *   Sec. "Multiple-Relaxation-Time Thermal Lattice Boltzmann Method":
 *     Eq. (18) the D2Q5 MRT LBE, Eq. (19) D2Q5 velocities, Eq. (20) T.
 *   Sec. "Power-law Viscosity Model": Eq. (21) the modified power law,
 *     Eq. (22) the strain-rate tensor from non-equilibrium moments,
 *     Eq. (23) its Frobenius magnitude.
 *   Sec. "Average Rate of Heat Transfer": Eq. (24) the average Nusselt number.
 *   Sec. "Mathematical Formulations": Eq. (5) boundary conditions, Eq. (6)
 *     nondimensional groups, Eqs. (8)-(9) nondimensional momentum (Darcy
 *     term -U D/Da, buoyancy +Pr*theta), Eq. (10) energy, Eq. (11) the
 *     power-law factor D.
 * Equation numbers count the paper's displayed equations in order.
 * Where the paper is silent the reading used is stated at the point of use.
 *
 * Parity unpinned (nothing outside this file fixes them; the tests pin only
 * their self-consistency and the limits that hold for any choice):
 *   - the D2Q5 higher-moment rates sT_e, sT_nu (every thermal pin holds for
 *     any value);
 *   - the choice of the provisional velocity inside the strain rate (Eq. 22);
 *   - the Mach number of the lattice mapping.
 */
#include "pmoracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[256];
const char* orc_last_error(void) { return g_err; }
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }

/* ---- D2Q9 lattice, Eq. (14): 0 rest; 1-4 E, N, W, S; 5-8 NE, NW, SW, SE ---- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* weights of the rest-state equilibrium, c_s^2 = 1/3 (Eq. 15) */
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Moment basis (rho, e, epsilon, jx, qx, jy, qy, pxx, pxy).  The paper does
 * not print M; this order is the one in which the rates of Eq. (13) pair up
 * as printed: s0 = s3 = s5 on the conserved rho, jx, jy; s1, s2 on e and
 * epsilon; s4 = s6 on the energy fluxes qx, qy; s7 = s8 = 1/tau on the
 * stresses pxx, pxy. */
static const double M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* ---- D2Q5 lattice, Eq. (19): 0 rest; 1-4 E, N, W, S ---- */
static const int EX5[5] = {0, 1, 0, -1, 0};
static const int EY5[5] = {0, 0, 1, 0, -1};
static const int OPP5[5] = {0, 3, 4, 1, 2};
/* D2Q5 weights (reading: w0 = 1/3 so that c_s^2 = 1/3 as in the flow part) */
static const double W5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
/* D2Q5 moment basis (T, jx, jy, e, nu) -- not printed in the paper. */
static const double N5[5][5] = {{1, 1, 1, 1, 1},
                                {0, 1, 0, -1, 0},
                                {0, 0, 1, 0, -1},
                                {-4, 1, 1, 1, 1},
                                {0, 1, -1, 1, -1}};

static double M9inv[9][9];
static double N5inv[5][5];
static int g_inv_ready = 0;

/* Gauss-Jordan inversion with partial pivoting (n <= 9). */
static void invert(int n, const double* A, double* Ainv) {
  double a[9][18];
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) a[r][c] = A[r * n + c];
    for (int c = 0; c < n; ++c) a[r][n + c] = (r == c) ? 1.0 : 0.0;
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = a[col][c];
        a[col][c] = a[piv][c];
        a[piv][c] = t;
      }
    double d = a[col][col];
    for (int c = 0; c < 2 * n; ++c) a[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double fct = a[r][col];
      if (fct != 0.0)
        for (int c = 0; c < 2 * n; ++c) a[r][c] -= fct * a[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ainv[r * n + c] = a[r][n + c];
}

static void ensure_inverses(void) {
  if (g_inv_ready) return;
  invert(9, &M9[0][0], &M9inv[0][0]);
  invert(5, &N5[0][0], &N5inv[0][0]);
  g_inv_ready = 1;
}

void orc_matrices(double* M, double* Minv, double* N, double* Ninv) {
  ensure_inverses();
  if (M) memcpy(M, M9, sizeof M9);
  if (Minv) memcpy(Minv, M9inv, sizeof M9inv);
  if (N) memcpy(N, N5, sizeof N5);
  if (Ninv) memcpy(Ninv, N5inv, sizeof N5inv);
}

static void matvec9(const double A[9][9], const double* x, double* y) {
  for (int r = 0; r < 9; ++r) {
    double s = 0.0;
    for (int c = 0; c < 9; ++c) s += A[r][c] * x[c];
    y[r] = s;
  }
}
static void matvec5(const double A[5][5], const double* x, double* y) {
  for (int r = 0; r < 5; ++r) {
    double s = 0.0;
    for (int c = 0; c < 5; ++c) s += A[r][c] * x[c];
    y[r] = s;
  }
}

/* ---- Step 0: physical groups -> lattice parameters (Eq. 6, Eq. 21) ----
 * The paper gives no lattice mapping (reading): U_lb = Ma * c_s; L = N;
 *   nu0_lb   = nu0 * U_lb * N with nu0 = Pr / sqrt(Ra)^(2-n)      (Eq. 21)
 *   alpha_lb = U_lb * N / sqrt(Ra)                                (Eq. 10)
 *   gbeta_lb = Pr * U_lb^2 / N                                    (Eq. 9)
 *   K        = Da * N^2                                           (Eq. 6)
 *   F_eps    = 1.75 / sqrt(150 eps^3)    (Ergun; porous reading)
 * so that the nondimensional coefficients of Eqs. (8)-(10) are reproduced. */
int orc_map_physics(const orc_physics* p, orc_lattice* L) {
  if (p->nx < 2 || p->ny < 2) {
    set_err("grid must be at least 2x2");
    return -1;
  }
  if (!(p->n > 0.0) || !(p->Ra > 0.0) || !(p->Pr > 0.0) || !(p->mach > 0.0) ||
      !(p->eps > 0.0 && p->eps <= 1.0) || !(p->Da > 0.0)) {
    set_err("n, Ra, Pr, mach, Da must be > 0 and eps in (0, 1]");
    return -1;
  }
  memset(L, 0, sizeof *L);
  const double N = (double)p->nx;
  const double U = p->mach / sqrt(3.0);
  L->nx = p->nx;
  L->ny = p->ny;
  L->periodic_x = p->periodic_x;
  L->periodic_y = p->periodic_y;
  L->U_lb = U;
  L->npow = p->n;
  L->nu0 = p->Pr / pow(sqrt(p->Ra), 2.0 - p->n) * U * N;
  L->gamma_scale = N / U;
  if (p->clamp_mode == 0) {
    L->nu_min = p->nu_lo * L->nu0;
    L->nu_max = p->nu_hi * L->nu0;
  } else {
    /* shear-rate thresholds gamma1 <= |gamma*| <= gamma2 (Eq. 21, made
     * continuous): nu = nu0 * clamp(gamma*, g1, g2)^(n-1) */
    double a = L->nu0 * pow(p->nu_lo, p->n - 1.0);
    double b = L->nu0 * pow(p->nu_hi, p->n - 1.0);
    L->nu_min = a < b ? a : b;
    L->nu_max = a < b ? b : a;
  }
  L->eps = p->eps;
  L->K_scale = N * N;
  L->K = isinf(p->Da) ? INFINITY : p->Da * N * N;
  L->Feps = p->forchheimer ? 1.75 / sqrt(150.0 * p->eps * p->eps * p->eps) : 0.0;
  L->gbeta = p->Pr * U * U / N;
  L->T_m = 0.5;
  L->gx = p->gx;
  L->gy = p->gy;
  L->alpha = U * N / sqrt(p->Ra);
  L->s_e = p->s_e > 0 ? p->s_e : 1.4;
  L->s_eps = p->s_eps > 0 ? p->s_eps : 1.4;
  L->s_q = p->s_q > 0 ? p->s_q : 1.2;
  L->sT_e = p->sT_e > 0 ? p->sT_e : 1.0;
  L->sT_nu = p->sT_nu > 0 ? p->sT_nu : 1.0;
  L->T_hot = 1.0;
  L->T_cold = 0.0;
  L->T_init = p->T_init;
  return 0;
}

/* ---- equilibria and forcing populations ----
 * The paper does not print f_eq, m_eq or F (reading): the generalised
 * porous-medium model of Guo & Zhao (2002), which reduces to the standard
 * incompressible-limit MRT forms at eps = 1. */
void orc_feq(double eps, double rho, double ux, double uy, double* feq) {
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    const double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = W9[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu / eps - 1.5 * uu / eps);
  }
}

void orc_forcing(double eps, double rho, double ux, double uy, double Fx,
                 double Fy, double* Fi) {
  const double uF = ux * Fx + uy * Fy;
  for (int i = 0; i < 9; ++i) {
    const double eu = EX[i] * ux + EY[i] * uy;
    const double eF = EX[i] * Fx + EY[i] * Fy;
    Fi[i] = W9[i] * rho * (3.0 * eF + 9.0 * eu * eF / eps - 3.0 * uF / eps);
  }
}

void orc_geq(double T, double ux, double uy, double* geq) {
  for (int i = 0; i < 5; ++i) {
    const double eu = EX5[i] * ux + EY5[i] * uy;
    geq[i] = W5[i] * T * (1.0 + 3.0 * eu);
  }
}

/* ---- Eqs. (22)-(23): strain-rate magnitude from non-equilibrium moments ----
 * gamma_ab = -3/(2 rho c^2) sum_i e_ia e_ib sum_j (M^-1 S M)_ij (f_j - f_j^eq)
 * |gamma|  = sqrt(2 gamma_ab gamma_ab), c = 1.  f_eq is taken at the
 * provisional velocity v (reading: the porous velocity itself depends on nu,
 * so the viscosity-independent v is used inside the strain rate). */
double orc_shear_sq(const orc_lattice* L, const double* f, double rho,
                    double vx, double vy, double s_nu) {
  ensure_inverses();
  double feq[9], fneq[9], m[9], x[9], y[9];
  orc_feq(L->eps, rho, vx, vy, feq);
  for (int i = 0; i < 9; ++i) fneq[i] = f[i] - feq[i];
  matvec9(M9, fneq, m);
  const double S[9] = {1.0, L->s_e, L->s_eps, 1.0, L->s_q, 1.0, L->s_q, s_nu, s_nu};
  for (int k = 0; k < 9; ++k) x[k] = S[k] * m[k];
  matvec9((const double(*)[9])M9inv, x, y);
  double pxx = 0, pyy = 0, pxy = 0;
  for (int i = 0; i < 9; ++i) {
    pxx += EX[i] * EX[i] * y[i];
    pyy += EY[i] * EY[i] * y[i];
    pxy += EX[i] * EY[i] * y[i];
  }
  const double c = -3.0 / (2.0 * rho);
  const double gxx = c * pxx, gyy = c * pyy, gxy = c * pxy;
  return 2.0 * (gxx * gxx + gyy * gyy + 2.0 * gxy * gxy);
}

/* ---- Eq. (21) with Eqs. (15), (22), (23): the local viscosity ----
 * The strain rate of Eq. (22) contains s_nu = 1/tau, and tau depends on nu
 * through nu = (tau - 1/2)/3 (Eq. 15; the printed "tau = (3 nu + 1)/2" is
 * read as tau = 3 nu + 1/2).  The viscosity is therefore the fixed point of
 *   nu = clamp(nu0 * (gamma_scale * |gamma(s_nu(nu))|)^(n-1), nu_min, nu_max).
 * |gamma|^2 is a quadratic in s_nu; its coefficients are obtained by
 * evaluating the literal formula at s_nu = -1, 0, 1.  The fixed point is
 * unique: G(x) = x - ln h(e^x), with h the unclamped power law, is strictly
 * increasing in x = ln nu, and the clamped fixed point is clamp(root of G).
 * Solved by Newton's method on G, safeguarded by bisection. */
static double solve_nu(const orc_lattice* L, double a, double b, double c) {
  const double n = L->npow;
  if (n == 1.0) {
    double nu = L->nu0;
    if (nu < L->nu_min) nu = L->nu_min;
    if (nu > L->nu_max) nu = L->nu_max;
    return nu;
  }
  const double lnnu0 = log(L->nu0), lnsc = log(L->gamma_scale);
#define G_OF(xv, Gv, dGv)                                                  \
  do {                                                                     \
    double nu_ = exp(xv);                                                  \
    double s_ = 1.0 / (3.0 * nu_ + 0.5);                                   \
    double g2_ = a + b * s_ + c * s_ * s_;                                 \
    if (g2_ < 0.0) g2_ = 0.0;                                              \
    Gv = (xv) - lnnu0 - (n - 1.0) * (lnsc + 0.5 * log(g2_));               \
    double dg2_ = (b + 2.0 * c * s_) * (-3.0 * nu_ * s_ * s_);             \
    dGv = 1.0 - (n - 1.0) * 0.5 * dg2_ / g2_;                              \
  } while (0)
  double lo = log(L->nu_min), hi = log(L->nu_max), Glo, Ghi, dG;
  G_OF(lo, Glo, dG);
  if (Glo >= 0.0) return L->nu_min;
  G_OF(hi, Ghi, dG);
  if (Ghi <= 0.0) return L->nu_max;
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double Gx;
    G_OF(x, Gx, dG);
    if (Gx == 0.0) break;
    if (Gx < 0.0)
      lo = x;
    else
      hi = x;
    double xn = x - Gx / dG;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const double dx = fabs(xn - x);
    x = xn;
    if (dx <= 2e-15 || hi - lo <= 2e-15) break;
  }
#undef G_OF
  return exp(x);
}

double orc_viscosity(const orc_lattice* L, const double* f, double rho,
                     double vx, double vy) {
  if (L->npow == 1.0) return solve_nu(L, 0, 0, 0);
  const double gm = orc_shear_sq(L, f, rho, vx, vy, -1.0);
  const double g0 = orc_shear_sq(L, f, rho, vx, vy, 0.0);
  const double gp = orc_shear_sq(L, f, rho, vx, vy, 1.0);
  const double a = g0;
  const double b = 0.5 * (gp - gm);
  const double c = 0.5 * (gp + gm) - g0;
  return solve_nu(L, a, b, c);
}

/* ---- one node: Steps 2-9 of the update ---- */
void orc_collide_node(const orc_lattice* L, double K, const double* f,
                      const double* g, double* fo, double* go, double* rho_o,
                      double* ux_o, double* uy_o, double* T_o, double* nu_o) {
  ensure_inverses();
  /* Step 2: macroscopic moments, Eqs. (16), (17), (20) */
  double rho = 0, jx = 0, jy = 0, T = 0;
  for (int i = 0; i < 9; ++i) {
    rho += f[i];
    jx += EX[i] * f[i];
    jy += EY[i] * f[i];
  }
  for (int i = 0; i < 5; ++i) T += g[i];
  /* Step 3: body force G: Boussinesq buoyancy g*beta*(T - T_m) along +y
   * (Eq. 17's G; Eq. 9's +Pr*theta) plus any extra uniform body force. */
  const double Gx = L->gx;
  const double Gy = L->gy + L->gbeta * (T - L->T_m);
  /* Step 4: provisional velocity v = j/rho + eps*G/2 (Eq. 17, porous form) */
  const double vx = jx / rho + 0.5 * L->eps * Gx;
  const double vy = jy / rho + 0.5 * L->eps * Gy;
  /* Step 5: local power-law viscosity (Eqs. 21-23) */
  const double nu = orc_viscosity(L, f, rho, vx, vy);
  /* Step 6: porous velocity -- u solves u = v - (eps nu/(2K)) u
   * - (eps F_eps/(2 sqrt K)) |u| u, i.e. u = v / (c0 + sqrt(c0^2 + c1 |v|)) */
  const double invK = isinf(K) ? 0.0 : 1.0 / K;
  const double invsK = sqrt(invK);
  const double c0 = 0.5 * (1.0 + 0.5 * L->eps * nu * invK);
  const double c1 = 0.5 * L->eps * L->Feps * invsK;
  const double vmag = sqrt(vx * vx + vy * vy);
  const double den = c0 + sqrt(c0 * c0 + c1 * vmag);
  const double ux = vx / den, uy = vy / den;
  /* Step 7: total force per unit mass: Darcy (Eq. 8's -U D/Da, with the
   * local power-law viscosity), Forchheimer, and eps*G. */
  const double umag = sqrt(ux * ux + uy * uy);
  const double Fx = -L->eps * nu * invK * ux - L->eps * L->Feps * invsK * umag * ux + L->eps * Gx;
  const double Fy = -L->eps * nu * invK * uy - L->eps * L->Feps * invsK * umag * uy + L->eps * Gy;
  /* Step 8: D2Q9 MRT collision in moment space, Eq. (12), rates Eq. (13);
   * s7 = s8 = 1/tau with tau = 3 nu + 1/2 (Eq. 15) */
  double feq[9], Fi[9], m[9], meq[9], Fm[9], ms[9];
  orc_feq(L->eps, rho, ux, uy, feq);
  orc_forcing(L->eps, rho, ux, uy, Fx, Fy, Fi);
  matvec9(M9, f, m);
  matvec9(M9, feq, meq);
  matvec9(M9, Fi, Fm);
  const double snu = 1.0 / (3.0 * nu + 0.5);
  const double S[9] = {1.0, L->s_e, L->s_eps, 1.0, L->s_q, 1.0, L->s_q, snu, snu};
  for (int k = 0; k < 9; ++k) ms[k] = m[k] - S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * S[k]) * Fm[k];
  matvec9((const double(*)[9])M9inv, ms, fo);
  /* Step 9: D2Q5 MRT thermal collision, Eq. (18), advected by u;
   * flux moments relax at 1/tau_g with alpha = (tau_g - 1/2)/3. */
  double geq[5], n5[5], neq[5], ns[5];
  orc_geq(T, ux, uy, geq);
  matvec5(N5, g, n5);
  matvec5(N5, geq, neq);
  const double sg = 1.0 / (3.0 * L->alpha + 0.5);
  const double ST[5] = {1.0, sg, sg, L->sT_e, L->sT_nu};
  for (int k = 0; k < 5; ++k) ns[k] = n5[k] - ST[k] * (n5[k] - neq[k]);
  matvec5((const double(*)[5])N5inv, ns, go);
  if (rho_o) *rho_o = rho;
  if (ux_o) *ux_o = ux;
  if (uy_o) *uy_o = uy;
  if (T_o) *T_o = T;
  if (nu_o) *nu_o = nu;
}

/* ---- state ---- */
struct orc_state {
  orc_lattice L;
  size_t nn;       /* nodes */
  double* f;       /* [9][nn] pre-collision */
  double* g;       /* [5][nn] */
  double* fp;      /* post-collision copies */
  double* gp;
  double* logda;   /* optional [nn] */
  int64_t steps;
};

static int lattice_ok(const orc_lattice* L) {
  if (L->nx < 2 || L->ny < 2) return 0;
  if (!(L->nu0 > 0) || !(L->nu_min > 0) || !(L->nu_max >= L->nu_min)) return 0;
  if (!(L->alpha > 0) || !(L->eps > 0) || !(L->U_lb > 0)) return 0;
  return 1;
}

orc_state* orc_new(const orc_lattice* L) {
  if (!lattice_ok(L)) {
    set_err("invalid lattice parameters");
    return NULL;
  }
  orc_state* s = (orc_state*)calloc(1, sizeof *s);
  s->L = *L;
  s->nn = (size_t)L->nx * (size_t)L->ny;
  s->f = (double*)malloc(9 * s->nn * sizeof(double));
  s->fp = (double*)malloc(9 * s->nn * sizeof(double));
  s->g = (double*)malloc(5 * s->nn * sizeof(double));
  s->gp = (double*)malloc(5 * s->nn * sizeof(double));
  if (!s->f || !s->fp || !s->g || !s->gp) {
    orc_free(s);
    set_err("out of memory");
    return NULL;
  }
  /* Step 1: uniform rest equilibrium rho = 1, u = 0, T = T_init */
  for (int q = 0; q < 9; ++q)
    for (size_t k = 0; k < s->nn; ++k) s->f[q * s->nn + k] = W9[q];
  for (int q = 0; q < 5; ++q)
    for (size_t k = 0; k < s->nn; ++k) s->g[q * s->nn + k] = W5[q] * L->T_init;
  return s;
}

void orc_free(orc_state* s) {
  if (!s) return;
  free(s->f);
  free(s->fp);
  free(s->g);
  free(s->gp);
  free(s->logda);
  free(s);
}

int orc_set_logda(orc_state* s, const double* logda) {
  if (!logda) {
    free(s->logda);
    s->logda = NULL;
    return 0;
  }
  if (!s->logda) s->logda = (double*)malloc(s->nn * sizeof(double));
  memcpy(s->logda, logda, s->nn * sizeof(double));
  return 0;
}

void orc_get_state(const orc_state* s, double* f, double* g) {
  if (f) memcpy(f, s->f, 9 * s->nn * sizeof(double));
  if (g) memcpy(g, s->g, 5 * s->nn * sizeof(double));
}
void orc_set_state(orc_state* s, const double* f, const double* g) {
  if (f) memcpy(s->f, f, 9 * s->nn * sizeof(double));
  if (g) memcpy(s->g, g, 5 * s->nn * sizeof(double));
}
int64_t orc_steps_done(const orc_state* s) { return s->steps; }

static double node_K(const orc_state* s, size_t k) {
  if (s->logda) return pow(10.0, s->logda[k]) * s->L.K_scale;
  return s->L.K;
}

static void collide_all(orc_state* s) {
  const orc_lattice* L = &s->L;
  const size_t nn = s->nn;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < L->ny; ++j) {
    for (int i = 0; i < L->nx; ++i) {
      const size_t k = (size_t)j * L->nx + i;
      double f[9], g[5], fo[9], go[5];
      for (int q = 0; q < 9; ++q) f[q] = s->f[q * nn + k];
      for (int q = 0; q < 5; ++q) g[q] = s->g[q * nn + k];
      orc_collide_node(L, node_K(s, k), f, g, fo, go, NULL, NULL, NULL, NULL, NULL);
      for (int q = 0; q < 9; ++q) s->fp[q * nn + k] = fo[q];
      for (int q = 0; q < 5; ++q) s->gp[q * nn + k] = go[q];
    }
  }
}

/* Streaming with the boundary conditions (Eq. 12 / Eq. 18 left-hand sides).
 * Flow: halfway bounce-back on every wall (no-slip, corners included).
 * Thermal (reading of the garbled BC list against the text: left wall hot,
 * right wall cold, top/bottom adiabatic): anti-bounce-back at x = 0 (T_hot)
 * and x = nx (T_cold), bounce-back (zero flux) at y = 0 and y = ny. */
static void stream_all(orc_state* s) {
  const orc_lattice* L = &s->L;
  const size_t nn = s->nn;
  const int nx = L->nx, ny = L->ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const size_t k = (size_t)j * nx + i;
      for (int q = 0; q < 9; ++q) {
        int si = i - EX[q], sj = j - EY[q];
        if (L->periodic_x) si = (si + nx) % nx;
        if (L->periodic_y) sj = (sj + ny) % ny;
        if (si >= 0 && si < nx && sj >= 0 && sj < ny)
          s->f[q * nn + k] = s->fp[q * nn + (size_t)sj * nx + si];
        else
          s->f[q * nn + k] = s->fp[OPP[q] * nn + k];
      }
      for (int q = 0; q < 5; ++q) {
        int si = i - EX5[q], sj = j - EY5[q];
        if (L->periodic_x) si = (si + nx) % nx;
        if (L->periodic_y) sj = (sj + ny) % ny;
        if (si >= 0 && si < nx && sj >= 0 && sj < ny)
          s->g[q * nn + k] = s->gp[q * nn + (size_t)sj * nx + si];
        else if (si < 0)
          s->g[q * nn + k] = -s->gp[OPP5[q] * nn + k] + 2.0 * W5[q] * L->T_hot;
        else if (si >= nx)
          s->g[q * nn + k] = -s->gp[OPP5[q] * nn + k] + 2.0 * W5[q] * L->T_cold;
        else
          s->g[q * nn + k] = s->gp[OPP5[q] * nn + k];
      }
    }
  }
}

void orc_step(orc_state* s, int64_t k) {
  for (int64_t t = 0; t < k; ++t) {
    collide_all(s);
    stream_all(s);
    s->steps++;
  }
}

void orc_macros(const orc_state* s, double* rho, double* ux, double* uy,
                double* T, double* nu) {
  const orc_lattice* L = &s->L;
  const size_t nn = s->nn;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < L->ny; ++j) {
    for (int i = 0; i < L->nx; ++i) {
      const size_t k = (size_t)j * L->nx + i;
      double f[9], g[5], fo[9], go[5], r, a, b, t, v;
      for (int q = 0; q < 9; ++q) f[q] = s->f[q * nn + k];
      for (int q = 0; q < 5; ++q) g[q] = s->g[q * nn + k];
      orc_collide_node(L, node_K(s, k), f, g, fo, go, &r, &a, &b, &t, &v);
      if (rho) rho[k] = r;
      if (ux) ux[k] = a;
      if (uy) uy[k] = b;
      if (T) T[k] = t;
      if (nu) nu[k] = v;
    }
  }
}

/* Eq. (24): Nu_bar = (1/L) int_0^L -dtheta/dX|_{X=0} dY.  Reading: the wall
 * gradient is the one-sided quadratic through the wall value (x = 0) and the
 * first two node values (x = 1/2, 3/2): -dtheta/dx = (8 th_w - 9 th_0 + th_1)/3;
 * X = x / L with L = nx; the Y integral is the midpoint rule over the ny
 * wall-adjacent nodes.  theta = (T - T_cold)/(T_hot - T_cold). */
double orc_nu_bar(const orc_state* s) {
  const orc_lattice* L = &s->L;
  const size_t nn = s->nn;
  const double dT = L->T_hot - L->T_cold;
  double sum = 0.0;
  for (int j = 0; j < L->ny; ++j) {
    double t0 = 0, t1 = 0;
    for (int q = 0; q < 5; ++q) {
      t0 += s->g[q * nn + (size_t)j * L->nx + 0];
      t1 += s->g[q * nn + (size_t)j * L->nx + 1];
    }
    const double th0 = (t0 - L->T_cold) / dT, th1 = (t1 - L->T_cold) / dT;
    sum += (double)L->nx * (8.0 * 1.0 - 9.0 * th0 + th1) / 3.0;
  }
  return sum / (double)L->ny;
}

double orc_run_to_steady(orc_state* s, double tol, int64_t check_every,
                         int64_t max_steps, int64_t* steps_out) {
  const size_t nn = s->nn;
  double* prev = (double*)malloc(nn * sizeof(double));
  double* cur = (double*)malloc(nn * sizeof(double));
  orc_macros(s, NULL, NULL, NULL, prev, NULL);
  double r = INFINITY;
  int64_t done = 0;
  while (done < max_steps) {
    int64_t chunk = check_every;
    if (done + chunk > max_steps) chunk = max_steps - done;
    orc_step(s, chunk);
    done += chunk;
    orc_macros(s, NULL, NULL, NULL, cur, NULL);
    r = 0.0;
    int bad = 0;
    for (size_t k = 0; k < nn; ++k) {
      double d = fabs(cur[k] - prev[k]);
      if (isnan(d)) bad = 1;
      else if (d > r) r = d;
      prev[k] = cur[k];
    }
    if (bad) r = NAN; /* a NaN anywhere is reported as the residual */
    if (r < tol || bad) break;
  }
  free(prev);
  free(cur);
  if (steps_out) *steps_out = done;
  return r;
}
