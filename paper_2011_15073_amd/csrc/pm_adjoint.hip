// pm_adjoint.hip -- discrete adjoint of one time step of the update, for
// gradients of the hot-wall Nusselt number (Eq. 24) with respect to the
// per-cell log10(Da) field, the power-law index n and the Rayleigh number.
//
// One step maps the pre-collision state S_k to S_{k+1} = Stream(Collide(S_k)).
// Given lambda_{k+1} = dJ/dS_{k+1} (FP64, natural layout [14][ny][nx]):
//   1. mu* = Stream^T lambda_{k+1}: for each node x and direction q,
//      mu*_q(x) = lambda_q(x + e_q) when x + e_q is inside, otherwise
//      lambda_opp(q)(x) (bounce-back) -- with a minus sign for the thermal
//      populations leaving through the Dirichlet walls (anti-bounce-back);
//   2. lambda_k(x) = (dCollide/dS)^T mu*(x): the forward node update is
//      recomputed in FP64 from the stored state and differentiated in
//      reverse order, line by line;
//   3. the parameter derivatives (dCollide/dtheta)^T mu*(x) are accumulated
//      in FP64: per cell for log10(Da), per workgroup (fixed slot, fixed
//      order) for ln nu0, n (direct) and the thermal rate s_g.
// The local viscosity is an implicit function (the fixed point of Eq. (21)
// with Eqs. (15), (22), (23)); its derivative is taken with the implicit
// function theorem on G(y; A, B, log2 nu0, n) = 0, y = log2 nu, or on the
// clamp (nu = bound * nu0) when the bound is active.
#include "pm_device.h"

namespace pm {
namespace {

using namespace pm::dev;

constexpr double LN2 = 0.693147180559945309417232121458176568;
constexpr double LN10 = 2.302585092994045684017991454684364208;

// Viscosity of one node in FP64 with the data the adjoint needs.
struct NuSol {
  double nu, y, s, g2, Gp;
  int branch;  // 0: power law (root of G), 1: at nu_min, 2: at nu_max
};

__device__ __forceinline__ NuSol nu_fp64(const AdjParams& a, double A, double B) {
  NuSol r;
  if (!a.pow) {  // Newtonian: nu = nu0 (the bounds bracket 1), G = y - log2 nu0
    r.y = a.log2nu0;
    r.nu = a.nu0;
    r.s = 1.0 / (3.0 * r.nu + 0.5);
    r.g2 = A + B * r.s * r.s;
    r.Gp = 1.0;
    r.branch = 0;
    return r;
  }
  const double hn = 0.5 * a.nm1;
  // Start: the closed-form root for A << B s^2, 3 nu >> 1/2, refined by a few
  // FP32 Newton steps on the hardware exp2 / log2 / reciprocal (about 1e-6 in
  // y), so that the FP64 Newton steps below converge in two or three.
  float yf;
  {
    const float lo = (float)a.y_lo, hi = (float)a.y_hi, lc0 = (float)a.lc0, nm1 = (float)a.nm1;
    const float Af = (float)A, Bf = (float)B;
    // log2(0) = -inf (no shear, or B below the FP32 range) lands on a bound
    yf = (lc0 + nm1 * (0.5f * __builtin_amdgcn_logf(Bf) - 1.5849625007f)) * (float)a.inv_n;
    yf = fminf(fmaxf(yf, lo), hi);
    for (int it = 0; it < 6; ++it) {
      const float nu = __builtin_amdgcn_exp2f(yf);
      const float sf = __builtin_amdgcn_rcpf(3.0f * nu + 0.5f);
      const float g2 = Af + Bf * sf * sf;
      if (!(g2 > 0.0f)) break;  // no shear in FP32: leave it to the FP64 steps
      const float G = (yf - lc0) - 0.5f * nm1 * __builtin_amdgcn_logf(g2);
      const float dG = 1.0f + 3.0f * nm1 * Bf * sf * sf * sf * nu * __builtin_amdgcn_rcpf(g2);
      yf = fminf(fmaxf(yf - G * __builtin_amdgcn_rcpf(dG), lo), hi);
    }
  }
  double y = fmin(fmax((double)yf, a.y_lo), a.y_hi);
  if (!(y == y)) y = a.y_hi;  // NaN start (no shear at all): the FP64 steps decide
  // Newton converges quadratically here: G' lies between min(n, 1) and
  // max(n, 1) and G'' is of order |n - 1|, so a step of size d leaves an
  // error of order d^2.  A step below 1e-9 therefore ends the iteration
  // (the error left is below 1e-17) without a further step to confirm it;
  // from the FP32 start that is two FP64 steps.  nu at the last iterate is
  // then 2^y of the one before times 2^d = 1 + t + t^2/2 (t = d ln 2, the
  // next term below 1e-28): no further exp2.
  double nu_last = 0.0, d_last = 0.0;
  bool conv = false;
  for (int it = 0; it < 60; ++it) {
    const double nu = exp2(y);
    const double s = 1.0 / (3.0 * nu + 0.5);
    const double g2 = A + B * s * s;
    const double G = (y - a.lc0) - hn * log2(g2);
    const double dG = 1.0 + 3.0 * a.nm1 * B * s * s * s * nu / g2;
    double yn = y - G / dG;
    if (!(g2 > 0.0)) yn = G < 0.0 ? a.y_hi : a.y_lo;
    yn = fmin(fmax(yn, a.y_lo), a.y_hi);
    d_last = yn - y;
    nu_last = nu;
    y = yn;
    if (fabs(d_last) <= 1e-9) {
      conv = true;
      break;
    }
  }
  r.y = y;
  if (conv) {
    const double t = d_last * LN2;
    r.nu = nu_last * (1.0 + t * (1.0 + 0.5 * t));
  } else {
    r.nu = exp2(y);
  }
  r.s = 1.0 / (3.0 * r.nu + 0.5);
  r.g2 = A + B * r.s * r.s;
  r.Gp = 1.0 + 3.0 * a.nm1 * B * r.s * r.s * r.s * r.nu / r.g2;
  r.branch = (y <= a.y_lo) ? 1 : ((y >= a.y_hi) ? 2 : 0);
  return r;
}

// Reverse-mode derivative of the node update (Steps 2-9) at the state
// (df, dg) (shifted populations, FP64), seeded with mu = dJ/d(post-collision).
__device__ __forceinline__ void vjp_node(const AdjParams& a, const double df[9], const double dg[5],
                                         double logda, const double mf[9], const double mg[5],
                                         double lf[9], double lg[5], double& g_ld, double& g_lnnu0,
                                         double& g_n, double& g_sg) {
  const double eps = a.eps, ie = a.inv_eps;
  // ---------------- forward recompute ----------------
  const double drho = (df[0] + ((df[1] + df[2]) + (df[3] + df[4]))) + ((df[5] + df[6]) + (df[7] + df[8]));
  const double rho = 1.0 + drho;
  const double jx = ((df[1] - df[3]) + (df[5] - df[6])) - (df[7] - df[8]);
  const double jy = ((df[2] - df[4]) + (df[5] + df[6])) - (df[7] + df[8]);
  const double dT = dg[0] + ((dg[1] + dg[2]) + (dg[3] + dg[4]));
  const double Gx = a.gx;
  const double Gy = a.gy + a.gbeta * (dT - a.dTm);
  const double irho = 1.0 / rho;
  const double vx = jx * irho + 0.5 * eps * Gx;
  const double vy = jy * irho + 0.5 * eps * Gy;
  const double s14 = (df[1] + df[2]) + (df[3] + df[4]);
  const double s58 = (df[5] + df[6]) + (df[7] + df[8]);
  const double m1 = (-4.0 * df[0] - s14) + 2.0 * s58;
  const double m7 = (df[1] - df[2]) + (df[3] - df[4]);
  const double m8 = (df[5] - df[6]) + (df[7] - df[8]);
  const double vxx = vx * vx, vyy = vy * vy;
  const double en = (m1 + 2.0 * drho) - 3.0 * rho * (vxx + vyy) * ie;
  const double pn = m7 - rho * (vxx - vyy) * ie;
  const double qn = m8 - rho * vx * vy * ie;
  const double irho2 = irho * irho;
  const double A = 0.25 * a.s_e * a.s_e * en * en * irho2;
  const double B = 2.25 * (pn * pn + 4.0 * qn * qn) * irho2;
  const NuSol ns = nu_fp64(a, A, B);
  const double nu = ns.nu;
  double invK, invsK;
  if (a.has_logda) {
    invK = exp2(-3.321928094887362347870319429489390175864831 * logda) * a.inv_Kscale;
    invsK = sqrt(invK);
  } else {
    invK = a.invK;
    invsK = a.invsK;
  }
  const double c0 = 0.5 * (1.0 + 0.5 * eps * nu * invK);
  const double c1 = 0.5 * eps * a.Feps * invsK;
  const double vm = sqrt(vx * vx + vy * vy);
  const double sq = sqrt(c0 * c0 + c1 * vm);
  const double den = c0 + sq;
  const double iden = 1.0 / den;
  const double ux = vx * iden, uy = vy * iden;
  const double um = sqrt(ux * ux + uy * uy);
  const double drag = eps * nu * invK + eps * a.Feps * invsK * um;
  const double Fx = eps * Gx - drag * ux;
  const double Fy = eps * Gy - drag * uy;
  const double uu = ux * ux + uy * uy;
  const double uF = ux * Fx + uy * Fy;
  const double snu = 1.0 / (3.0 * nu + 0.5);
  const double hnu = 1.0 - 0.5 * snu;
  // (m2, m4, m6 enter the collision linearly: only their adjoints are needed)
  const double P7 = rho * (ux * ux - uy * uy) * ie, Q7 = 2.0 * rho * (ux * Fx - uy * Fy) * ie;
  const double P8 = rho * ux * uy * ie, Q8 = rho * (ux * Fy + uy * Fx) * ie;
  const double Tabs = a.T_ref + dT;
  const double n1 = dg[1] - dg[3], n2 = dg[2] - dg[4];

  // ---------------- reverse sweep ----------------
  // Step 9: g* = N^-1 (dT, ns1..ns4)
  const double bn0 = (mg[0] + mg[1] + mg[2] + mg[3] + mg[4]) * 0.2;
  const double bn1 = (mg[1] - mg[3]) * 0.5;
  const double bn2 = (mg[2] - mg[4]) * 0.5;
  const double bn3 = (-4.0 * mg[0] + mg[1] + mg[2] + mg[3] + mg[4]) * 0.05;
  const double bn4 = (mg[1] - mg[2] + mg[3] - mg[4]) * 0.25;
  double b_ux = 0.0, b_uy = 0.0, b_dT = 0.0, b_Tabs = 0.0, b_sg = 0.0;
  const double b_n1 = (1.0 - a.s_g) * bn1;
  b_ux += a.s_g * Tabs * bn1;
  b_Tabs += a.s_g * ux * bn1;
  b_sg += (ux * Tabs - n1) * bn1;
  const double b_n2 = (1.0 - a.s_g) * bn2;
  b_uy += a.s_g * Tabs * bn2;
  b_Tabs += a.s_g * uy * bn2;
  b_sg += (uy * Tabs - n2) * bn2;
  const double b_n3 = (1.0 - a.sT_e) * bn3;
  b_dT += -a.sT_e * (2.0 / 3.0) * bn3;
  const double b_n4 = (1.0 - a.sT_nu) * bn4;
  b_dT += bn0;
  b_dT += b_Tabs;

  // Step 8: f* = M^-1 ms
  const double sm58 = (mf[5] + mf[6]) + (mf[7] + mf[8]);
  const double sm14 = (mf[1] + mf[2]) + (mf[3] + mf[4]);
  // (the row norms 9, 36, 6, 12 of M as multiplications: FP64 division is a
  // long instruction sequence on this path)
  constexpr double i9 = 1.0 / 9.0, i36 = 1.0 / 36.0, i6 = 1.0 / 6.0, i12 = 1.0 / 12.0;
  const double bm0 = (mf[0] + sm14 + sm58) * i9;
  const double bm1 = (-4.0 * mf[0] - sm14 + 2.0 * sm58) * i36;
  const double bm2 = (4.0 * mf[0] - 2.0 * sm14 + sm58) * i36;
  const double bm3 = ((mf[1] - mf[3]) + (mf[5] - mf[6]) - (mf[7] - mf[8])) * i6;
  const double bm4 = (-2.0 * (mf[1] - mf[3]) + (mf[5] - mf[6]) - (mf[7] - mf[8])) * i12;
  const double bm5 = ((mf[2] - mf[4]) + (mf[5] + mf[6]) - (mf[7] + mf[8])) * i6;
  const double bm6 = (-2.0 * (mf[2] - mf[4]) + (mf[5] + mf[6]) - (mf[7] + mf[8])) * i12;
  const double bm7 = ((mf[1] - mf[2]) + (mf[3] - mf[4])) * 0.25;
  const double bm8 = ((mf[5] - mf[6]) + (mf[7] - mf[8])) * 0.25;
  double b_drho = bm0, b_rho = 0.0, b_Fx = 0.0, b_Fy = 0.0, b_snu = 0.0, b_hnu = 0.0;
  double b_m1 = 0.0, b_m7 = 0.0, b_m8 = 0.0;
  double b_ruu = 0.0, b_Fm1 = 0.0, b_rux = 0.0, b_ruy = 0.0;
  // ms1 = (1 - se) m1 + se (-2 drho + ruu) + (1 - se/2) Fm1
  b_m1 += (1.0 - a.s_e) * bm1;
  b_drho += -2.0 * a.s_e * bm1;
  b_ruu += a.s_e * bm1;
  b_Fm1 += (1.0 - 0.5 * a.s_e) * bm1;
  // ms2 = (1 - seps) m2 + seps (drho - ruu) - (1 - seps/2) Fm1
  const double b_m2 = (1.0 - a.s_eps) * bm2;
  b_drho += a.s_eps * bm2;
  b_ruu += -a.s_eps * bm2;
  b_Fm1 += -(1.0 - 0.5 * a.s_eps) * bm2;
  // ms3 = rux + rho Fx / 2
  b_rux += bm3;
  b_rho += 0.5 * Fx * bm3;
  b_Fx += 0.5 * rho * bm3;
  // ms4 = (1 - sq) m4 - sq rux - (1 - sq/2) rho Fx
  const double b_m4 = (1.0 - a.s_q) * bm4;
  b_rux += -a.s_q * bm4;
  b_rho += -(1.0 - 0.5 * a.s_q) * Fx * bm4;
  b_Fx += -(1.0 - 0.5 * a.s_q) * rho * bm4;
  // ms5, ms6
  b_ruy += bm5;
  b_rho += 0.5 * Fy * bm5;
  b_Fy += 0.5 * rho * bm5;
  const double b_m6 = (1.0 - a.s_q) * bm6;
  b_ruy += -a.s_q * bm6;
  b_rho += -(1.0 - 0.5 * a.s_q) * Fy * bm6;
  b_Fy += -(1.0 - 0.5 * a.s_q) * rho * bm6;
  // ms7 = (1 - snu) m7 + snu P7 + hnu Q7
  b_m7 += (1.0 - snu) * bm7;
  b_snu += (P7 - m7) * bm7;
  b_hnu += Q7 * bm7;
  double b_ux2 = 0.0, b_uy2 = 0.0;  // collected below into b_ux, b_uy
  {
    const double bP = snu * bm7, bQ = hnu * bm7;
    b_rho += (ux * ux - uy * uy) * ie * bP + 2.0 * (ux * Fx - uy * Fy) * ie * bQ;
    b_ux2 += 2.0 * rho * ux * ie * bP + 2.0 * rho * Fx * ie * bQ;
    b_uy2 += -2.0 * rho * uy * ie * bP - 2.0 * rho * Fy * ie * bQ;
    b_Fx += 2.0 * rho * ux * ie * bQ;
    b_Fy += -2.0 * rho * uy * ie * bQ;
  }
  // ms8 = (1 - snu) m8 + snu P8 + hnu Q8
  b_m8 += (1.0 - snu) * bm8;
  b_snu += (P8 - m8) * bm8;
  b_hnu += Q8 * bm8;
  {
    const double bP = snu * bm8, bQ = hnu * bm8;
    b_rho += ux * uy * ie * bP + (ux * Fy + uy * Fx) * ie * bQ;
    b_ux2 += rho * uy * ie * bP + rho * Fy * ie * bQ;
    b_uy2 += rho * ux * ie * bP + rho * Fx * ie * bQ;
    b_Fy += rho * ux * ie * bQ;
    b_Fx += rho * uy * ie * bQ;
  }
  b_ux += b_ux2;
  b_uy += b_uy2;
  b_snu += -0.5 * b_hnu;
  double b_nu = b_snu * (-3.0 * snu * snu);
  // Fm1 = 6 rho uF / eps
  b_rho += 6.0 * uF * ie * b_Fm1;
  const double b_uF = 6.0 * rho * ie * b_Fm1;
  b_ux += Fx * b_uF;
  b_uy += Fy * b_uF;
  b_Fx += ux * b_uF;
  b_Fy += uy * b_uF;
  // ruu = 3 rho uu / eps
  b_rho += 3.0 * uu * ie * b_ruu;
  const double b_uu = 3.0 * rho * ie * b_ruu;
  b_ux += 2.0 * ux * b_uu;
  b_uy += 2.0 * uy * b_uu;
  // rux = rho ux, ruy = rho uy
  b_rho += ux * b_rux + uy * b_ruy;
  b_ux += rho * b_rux;
  b_uy += rho * b_ruy;

  // Step 7: F = eps G - drag u, drag = eps nu invK + eps Feps invsK |u|
  double b_Gx = eps * b_Fx, b_Gy = eps * b_Fy;
  const double b_drag = -(ux * b_Fx + uy * b_Fy);
  b_ux += -drag * b_Fx;
  b_uy += -drag * b_Fy;
  b_nu += eps * invK * b_drag;
  double b_invK = eps * nu * b_drag;
  double b_invsK = eps * a.Feps * um * b_drag;
  const double b_um = eps * a.Feps * invsK * b_drag;
  if (um > 0.0) {
    const double ium = 1.0 / um;
    b_ux += ux * ium * b_um;
    b_uy += uy * ium * b_um;
  }

  // Step 6: u = v / (c0 + sqrt(c0^2 + c1 |v|))
  double b_vx = iden * b_ux, b_vy = iden * b_uy;
  const double b_iden = vx * b_ux + vy * b_uy;
  const double b_den = -iden * iden * b_iden;
  double b_c0 = b_den;
  const double b_sq = b_den;
  double b_c1 = 0.0;
  if (sq > 0.0) {
    const double isq = 1.0 / sq;
    b_c0 += c0 * isq * b_sq;
    b_c1 += 0.5 * vm * isq * b_sq;
    const double b_vm = 0.5 * c1 * isq * b_sq;
    if (vm > 0.0) {
      const double ivm = 1.0 / vm;
      b_vx += vx * ivm * b_vm;
      b_vy += vy * ivm * b_vm;
    }
  }
  b_nu += 0.25 * eps * invK * b_c0;
  b_invK += 0.25 * eps * nu * b_c0;
  b_invsK += 0.5 * eps * a.Feps * b_c1;
  // invK = 10^-logDa / N^2, invsK = sqrt(invK)
  g_ld = a.has_logda ? (-LN10 * invK * b_invK - 0.5 * LN10 * invsK * b_invsK) : 0.0;

  // Step 5: nu from (A, B, log2 nu0, n) -- implicit function / clamp
  double b_A = 0.0, b_B = 0.0;
  g_lnnu0 = 0.0;
  g_n = 0.0;
  if (ns.branch != 0) {
    g_lnnu0 += nu * b_nu;  // nu = bound * nu0
  } else {
    const double b_y = b_nu * nu * LN2;  // nu = 2^y
    const double w = b_y / ns.Gp;
    // dy = -(G_A dA + G_B dB + G_L0 dL0 + G_n dn) / G'
    constexpr double ILN2 = 1.0 / LN2;
    g_lnnu0 += w * ILN2;  // L0 = log2 nu0, G_L0 = -1
    // At zero shear (possible only with n = 1, where no clamp is active) the
    // power law is singular in n and its one-sided limits sit on a clamp,
    // which does not depend on n at fixed nu0: no n or shear terms.
    if (ns.g2 > 0.0) {
      // G_n = -log2(gamma*).  At the root G = 0 gives log2(g2) = (y - lc0) / hn
      // (to the root's error over hn; the log is taken where hn is small).
      const double hn = 0.5 * a.nm1;
      const double l2g2 = fabs(hn) >= 1e-3 ? (ns.y - a.lc0) / hn : log2(ns.g2);
      g_n += w * (a.log2c + 0.5 * l2g2);
      if (ns.g2 > a.g2_floor) {
        const double wg = w * 0.5 * a.nm1 * ILN2 / ns.g2;
        b_A += wg;
        b_B += wg * ns.s * ns.s;
      }
    }
  }
  // A = se^2 en^2 irho2 / 4, B = 9 (pn^2 + 4 qn^2) irho2 / 4
  const double b_en = 0.5 * a.s_e * a.s_e * en * irho2 * b_A;
  const double b_pn = 4.5 * pn * irho2 * b_B;
  const double b_qn = 18.0 * qn * irho2 * b_B;
  const double b_irho2 = 0.25 * a.s_e * a.s_e * en * en * b_A + 2.25 * (pn * pn + 4.0 * qn * qn) * b_B;
  double b_irho = 2.0 * irho * b_irho2;
  // en, pn, qn
  b_m1 += b_en;
  b_drho += 2.0 * b_en;
  b_rho += -3.0 * (vxx + vyy) * ie * b_en - (vxx - vyy) * ie * b_pn - vx * vy * ie * b_qn;
  const double b_vxx = -3.0 * rho * ie * b_en - rho * ie * b_pn;
  const double b_vyy = -3.0 * rho * ie * b_en + rho * ie * b_pn;
  b_m7 += b_pn;
  b_m8 += b_qn;
  b_vx += 2.0 * vx * b_vxx - rho * vy * ie * b_qn;
  b_vy += 2.0 * vy * b_vyy - rho * vx * ie * b_qn;

  // Step 4: v = j / rho + eps G / 2
  const double b_jx = irho * b_vx, b_jy = irho * b_vy;
  b_irho += jx * b_vx + jy * b_vy;
  b_Gx += 0.5 * eps * b_vx;
  b_Gy += 0.5 * eps * b_vy;
  b_rho += -irho * irho * b_irho;
  // Step 3: Gy = gy + gbeta (dT - dTm)
  b_dT += a.gbeta * b_Gy;
  (void)b_Gx;
  // Step 2
  b_drho += b_rho;
  // populations: drho, jx, jy and the moments m1, m2, m4, m6, m7, m8 are
  // linear in df (rows of M)
  lf[0] = b_drho - 4.0 * b_m1 + 4.0 * b_m2;
  lf[1] = b_drho + b_jx - b_m1 - 2.0 * b_m2 - 2.0 * b_m4 + b_m7;
  lf[2] = b_drho + b_jy - b_m1 - 2.0 * b_m2 - 2.0 * b_m6 - b_m7;
  lf[3] = b_drho - b_jx - b_m1 - 2.0 * b_m2 + 2.0 * b_m4 + b_m7;
  lf[4] = b_drho - b_jy - b_m1 - 2.0 * b_m2 + 2.0 * b_m6 - b_m7;
  lf[5] = b_drho + b_jx + b_jy + 2.0 * b_m1 + b_m2 + b_m4 + b_m6 + b_m8;
  lf[6] = b_drho - b_jx + b_jy + 2.0 * b_m1 + b_m2 - b_m4 + b_m6 - b_m8;
  lf[7] = b_drho - b_jx - b_jy + 2.0 * b_m1 + b_m2 - b_m4 - b_m6 + b_m8;
  lf[8] = b_drho + b_jx - b_jy + 2.0 * b_m1 + b_m2 + b_m4 - b_m6 - b_m8;
  // thermal: dT, n1..n4 are linear in dg (rows of N)
  lg[0] = b_dT - 4.0 * b_n3;
  lg[1] = b_dT + b_n1 + b_n3 + b_n4;
  lg[2] = b_dT + b_n2 + b_n3 - b_n4;
  lg[3] = b_dT - b_n1 + b_n3 + b_n4;
  lg[4] = b_dT - b_n2 + b_n3 - b_n4;
  g_sg = b_sg;
}

// Adjoint of the streaming step: mu*_q(x) from lambda_{k+1} (natural layout).
// Each lambda value is read by at most two nodes of a launch (its pull
// neighbour, and the node itself at a wall) and written once, so the loads
// here and the stores in k_adjoint are non-temporal; measured 2-8% faster per
// launch from 256^2 to 4096^2 than cached accesses.
// The adjoint state is stored as L: double, or float for FP32 forward states
// (the arithmetic stays FP64; only the values kept between steps are
// rounded, to nearest).  gather_mu only loads; mu_signs then applies the
// anti-bounce-back sign of the Dirichlet walls, so that no arithmetic on a
// loaded value (and no wait for it) sits between the node's loads.
// Every address below is a select between two indices whose row parts are
// wave-uniform (j is the workgroup's row) and whose column part is the lane's,
// with the inside test as a bitwise and: no branches between the loads.
template <typename L>
__device__ __forceinline__ void gather_mu(const AdjParams& a, const L* __restrict__ lam, int i, int j,
                                          L rf[9], L rg[5]) {
  const int nx = a.nx, ny = a.ny;
  const int64_t nn = (int64_t)nx * ny, k = (int64_t)j * nx + i;
  const bool in_ip = i + 1 < nx, in_im = i >= 1, in_jp = j + 1 < ny, in_jm = j >= 1;
  const int64_t r0 = (int64_t)j * nx;
#pragma unroll
  for (int q = 0; q < 14; ++q) {
    const int d = q < 9 ? q : q - 9;  // direction within D2Q9 / D2Q5
    const int od = OPP[d] + (q < 9 ? 0 : 9);
    const bool in = (EXv[d] > 0 ? in_ip : (EXv[d] < 0 ? in_im : true)) &
                    (EYv[d] > 0 ? in_jp : (EYv[d] < 0 ? in_jm : true));
    const int64_t idx = in ? q * nn + r0 + EYv[d] * (int64_t)nx + (i + EXv[d]) : od * nn + k;
    const L v = __builtin_nontemporal_load(&lam[idx]);
    if (q < 9) rf[q] = v;
    else rg[q - 9] = v;
  }
}

template <typename L>
__device__ __forceinline__ void mu_signs(const AdjParams& a, int i, const L rf[9], const L rg[5], double mf[9],
                                         double mg[5]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) mf[q] = (double)rf[q];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double v = (double)rg[q];
    const bool wall = (EXv[q] == 1 && i + 1 >= a.nx) || (EXv[q] == -1 && i == 0);
    mg[q] = wall ? -v : v;  // anti-bounce-back at the hot and cold walls
  }
}

// ODD: the parity of the step whose state is read (a template parameter, so
// that each variant's loads are one straight-line sequence).
template <typename S, typename L, bool ODD>
__global__ __launch_bounds__(TILE) void k_adjoint(KParams<S> st, AdjParams a,
                                                  const L* __restrict__ lam_next,
                                                  L* __restrict__ lam, double* __restrict__ g_logda,
                                                  double* __restrict__ partial) {
  static_assert(TILE % 64 == 0, "whole waves per workgroup");
  constexpr int NW = TILE / 64;  // waves per workgroup
  __shared__ double red[ADJ_PART][NW];
  const int tiles_x = (a.nx + TILE - 1) / TILE;
  const int j = blockIdx.x / tiles_x;
  const int i = (blockIdx.x - j * tiles_x) * TILE + threadIdx.x;
  double c_lnnu0 = 0.0, c_n = 0.0, c_sg = 0.0, lmax = 0.0;
  // The workgroup's partials and the node's gradient are read, updated and
  // written back; their reads are issued with the node's loads, so that the
  // end of the wave does not wait on a load.
  double p_old = 0.0;
  if (threadIdx.x < ADJ_PART) p_old = partial[ADJ_PART * blockIdx.x + threadIdx.x];
  if (i < a.nx) {
    // Loads in this order: lambda_{k+1}, the old gradient, the state (whose
    // wall conditions need their values), log10 Da.  Each wait then covers
    // loads that are all in flight already: one memory round trip.
    const int64_t k = (int64_t)j * a.nx + i, nn = (int64_t)a.nx * a.ny;
    L rf[9], rg[5];
    gather_mu(a, lam_next, i, j, rf, rg);
    const double gl_old = a.has_logda ? g_logda[k] : 0.0;
    S sf[9], sg[5];
    load_node_raw<S, ODD>(st, i, j, sf, sg);
    const double ld = a.has_logda ? (double)st.logda[k] : 0.0;
    if (ODD) pull_walls(st, i, sg);
    double df[9], dg[5], mf[9], mg[5], lf[9], lg[5];
#pragma unroll
    for (int q = 0; q < 9; ++q) df[q] = (double)sf[q];
#pragma unroll
    for (int q = 0; q < 5; ++q) dg[q] = (double)sg[q];
    mu_signs(a, i, rf, rg, mf, mg);
    double g_ld;
    vjp_node(a, df, dg, ld, mf, mg, lf, lg, g_ld, c_lnnu0, c_n, c_sg);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      __builtin_nontemporal_store((L)lf[q], &lam[q * nn + k]);
      lmax = fmax(lmax, fabs(lf[q]));
      if (lf[q] != lf[q]) lmax = INFINITY;  // NaN counts as unbounded
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      __builtin_nontemporal_store((L)lg[q], &lam[(9 + q) * nn + k]);
      lmax = fmax(lmax, fabs(lg[q]));
      if (lg[q] != lg[q]) lmax = INFINITY;
    }
    if (a.has_logda) g_logda[k] = gl_old + g_ld;
  }
  // Workgroup sums (and the max): a butterfly over the 64 lanes of each
  // wave, then the NW wave results in wave order, in one fixed order.
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c_lnnu0 += __shfl_xor(c_lnnu0, off);
    c_n += __shfl_xor(c_n, off);
    c_sg += __shfl_xor(c_sg, off);
    lmax = fmax(lmax, __shfl_xor(lmax, off));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = c_lnnu0;
    red[1][wv] = c_n;
    red[2][wv] = c_sg;
    red[3][wv] = lmax;
  }
  __syncthreads();
  if (threadIdx.x < ADJ_PART) {
    const int q = threadIdx.x;
    double v = red[q][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) v = q < 3 ? v + red[q][w] : fmax(v, red[q][w]);
    partial[ADJ_PART * blockIdx.x + q] = q < 3 ? p_old + v : fmax(p_old, v);
  }
}

// lambda_T = dJ/dS_T for J = Nu_bar (Eq. 24): only the thermal populations of
// the two hot-wall columns contribute.
template <typename L>
__global__ void k_adjoint_seed(int nx, int ny, double seed, L* __restrict__ lam) {
  const int64_t nn = (int64_t)nx * ny;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 14 * nn;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(t / nn);
    const int64_t k = t - q * nn;
    const int i = (int)(k % nx);
    double v = 0.0;
    if (q >= 9) {
      if (i == 0) v = -3.0 * nx / (double)ny;
      else if (i == 1) v = nx / (3.0 * ny);
    }
    lam[t] = (L)(seed * v);
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ a, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    a[t] = 0.0;
}

// The per-workgroup adjoint partials reduced in workgroup order, as the host
// reduces them: out[q] = sum_b partial[b][q] for q < 3, out[3] = max_b
// partial[b][3] with a NaN turning it to +inf.  One thread per component, so
// the sums are added in exactly that order.
__global__ void k_adj_reduce(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  const int q = threadIdx.x;
  if (q >= ADJ_PART) return;
  double acc = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const double m = partial[ADJ_PART * (int64_t)b + q];
    if (q < 3) acc += m;
    else acc = (m != m) ? INFINITY : (acc < m ? m : acc);
  }
  out[q] = acc;
}

}  // namespace

hipError_t launch_fill_zero(double* a, int64_t n, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)b), dim3(256), 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const double* partial, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(64), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

template <typename S, typename L>
hipError_t launch_adjoint(const KParams<S>& st, const AdjParams& a, int parity, const L* lam_next, L* lam,
                          double* g_logda, double* partial, hipStream_t s) {
  const int tiles_x = (a.nx + TILE - 1) / TILE;
  if (parity)
    hipLaunchKernelGGL((k_adjoint<S, L, true>), dim3(tiles_x * a.ny), dim3(TILE), 0, s, st, a, lam_next, lam,
                       g_logda, partial);
  else
    hipLaunchKernelGGL((k_adjoint<S, L, false>), dim3(tiles_x * a.ny), dim3(TILE), 0, s, st, a, lam_next, lam,
                       g_logda, partial);
  return hipGetLastError();
}

template <typename L>
hipError_t launch_adjoint_seed(int nx, int ny, double seed, L* lam, hipStream_t s) {
  const int64_t n = 14 * (int64_t)nx * ny;
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL((k_adjoint_seed<L>), dim3((unsigned)b), dim3(256), 0, s, nx, ny, seed, lam);
  return hipGetLastError();
}

template hipError_t launch_adjoint<float, double>(const KParams<float>&, const AdjParams&, int, const double*,
                                                  double*, double*, double*, hipStream_t);
template hipError_t launch_adjoint<float, float>(const KParams<float>&, const AdjParams&, int, const float*,
                                                 float*, double*, double*, hipStream_t);
template hipError_t launch_adjoint<double, double>(const KParams<double>&, const AdjParams&, int, const double*,
                                                   double*, double*, double*, hipStream_t);
template hipError_t launch_adjoint_seed<double>(int, int, double, double*, hipStream_t);
template hipError_t launch_adjoint_seed<float>(int, int, double, float*, hipStream_t);

}  // namespace pm
