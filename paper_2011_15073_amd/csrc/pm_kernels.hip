// pm_kernels.hip -- gfx950 kernels of the MRT lattice Boltzmann update for
// power-law natural convection in a porous cavity (arXiv:2011.15073).
//
// One time step is one fused kernel over all nodes: gather the 9 + 5
// populations, collide (D2Q9 MRT with buoyancy and porous drag, Eq. 12;
// local power-law viscosity, Eqs. 21-23; D2Q5 MRT, Eq. 18) and scatter.
// Memory follows the AA pattern: a single copy of the populations, updated in
// place.
//   even step: node x reads its own slots f_q(x), writes f*_q to slot opp(q)
//              of the same node (no streaming);
//   odd step:  node x pulls f_q from slot opp(q) of node x - e_q and pushes
//              f*_q to slot q of node x + e_q, which completes the streaming
//              of both steps.
// Each node reads and writes exactly the same 14 addresses in a step, so the
// update is race-free without a second buffer; the walls (halfway
// bounce-back, thermal anti-bounce-back) are applied on the odd step's pull
// and push.  Every population is read once and written once per step: the
// algorithmic traffic is 14 * 2 * sizeof(T) bytes per node update.
//
// Planes are SoA [q][ny][nx] with x fastest; one workgroup of 256 threads
// covers a 256-node row segment, so every load and store of a wave is a
// contiguous 256 B (FP32) run; workgroups run in row-major tile order.  The
// streaming hint is used on every access that is not shifted along x (those
// lines are touched exactly once per step); the x-shifted accesses of the odd
// step straddle lines that the neighbouring wave also touches, so they keep
// the default caching.
#include "pm_internal.h"

#include <cmath>

namespace pm {
namespace {

// D2Q9 velocities, Eq. (14): 0 rest; 1-4 E, N, W, S; 5-8 NE, NW, SW, SE.
// D2Q5 (Eq. 19) uses the first five.
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int EXv[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EYv[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Workgroup b handles row tile b in row-major order.  Dispatch deals
// consecutive workgroups round-robin to the 8 XCDs, so at any moment all XCDs
// stream through one narrow band of each plane; that keeps the HBM accesses
// of the whole chip within few DRAM pages.  (Giving each XCD its own
// contiguous band of rows measured 5% slower at 4096^2: eight bands far apart
// in every plane.)
__device__ __forceinline__ int tile_of_block(int b, int) { return b; }

// Arithmetic helpers.  FP32 uses the hardware approximations directly
// (v_rcp_f32, v_exp_f32, v_log_f32, v_sqrt_f32, about 1 ulp): the FP32 path is
// held to 1e-4 against the FP64 oracle.  FP64 keeps IEEE division and the
// library exp2 / log2 / sqrt.
#ifndef PM_FAST_MATH
#define PM_FAST_MATH 1
#endif
template <typename T> __device__ __forceinline__ T frcp(T x);
template <typename T> __device__ __forceinline__ T flog2(T x);
template <typename T> __device__ __forceinline__ T fexp2(T x);
template <typename T> __device__ __forceinline__ T fsqrt(T x);
#if PM_FAST_MATH
template <> __device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ float flog2<float>(float x) { return __builtin_amdgcn_logf(x); }
template <> __device__ __forceinline__ float fexp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
#else
template <> __device__ __forceinline__ float frcp<float>(float x) { return 1.0f / x; }
template <> __device__ __forceinline__ float flog2<float>(float x) { return log2f(x); }
template <> __device__ __forceinline__ float fexp2<float>(float x) { return exp2f(x); }
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return sqrtf(x); }
#endif
template <> __device__ __forceinline__ double frcp<double>(double x) { return 1.0 / x; }
template <> __device__ __forceinline__ double flog2<double>(double x) { return log2(x); }
template <> __device__ __forceinline__ double fexp2<double>(double x) { return exp2(x); }
template <> __device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }

// Global loads and stores; NT = streaming (non-temporal) hint, used for the
// aligned population accesses of the step (each value is touched once per
// step, so keeping it in L2/MALL only evicts useful lines).
template <typename T, bool NT>
__device__ __forceinline__ T ldg(const T* a) {
  if constexpr (NT) return __builtin_nontemporal_load(a);
  else return *a;
}
template <typename T, bool NT>
__device__ __forceinline__ void stg(T* a, T v) {
#ifdef PM_EMULATE_FP32_STORAGE
  v = (T)(float)v;
#endif
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// ---- neighbour addressing for the odd (streaming) step ----
// Source of the pull of direction Q into node (i, j): node (i, j) - e_Q, or
// the node itself when that crosses a wall.  Returns whether it is inside.
template <int Q>
__device__ __forceinline__ bool nbr(int nx, int ny, int px, int py, int i, int j, int sx, int sy,
                                    int& idx) {
  // (sx, sy) = +-e_Q direction sign applied by the caller
  int si = i + sx * EXv[Q], sj = j + sy * EYv[Q];
  bool in = true;
  if (EXv[Q] != 0) {
    if (px) {
      si = si < 0 ? si + nx : si;
      si = si >= nx ? si - nx : si;
    } else {
      in = in && (si >= 0) && (si < nx);
    }
  }
  if (EYv[Q] != 0) {
    if (py) {
      sj = sj < 0 ? sj + ny : sj;
      sj = sj >= ny ? sj - ny : sj;
    } else {
      in = in && (sj >= 0) && (sj < ny);
    }
  }
  idx = sj * nx + si;
  return in;
}

template <typename T, int Q>
__device__ __forceinline__ T pull_f(const KParams<T>& p, int i, int j, int k) {
  int s;
  const bool in = nbr<Q>(p.nx, p.ny, p.px, p.py, i, j, -1, -1, s);
  const T* a = in ? (p.f + OPP[Q] * p.P + s) : (p.f + Q * p.P + k);
  return ldg<T, EXv[Q] == 0>(a);
}

template <typename T, int Q>
__device__ __forceinline__ void push_f(const KParams<T>& p, int i, int j, int k, T v) {
  int d;
  const bool in = nbr<Q>(p.nx, p.ny, p.px, p.py, i, j, 1, 1, d);
  T* a = in ? (p.f + Q * p.P + d) : (p.f + OPP[Q] * p.P + k);
  stg<T, EXv[Q] == 0>(a, v);
}

// Thermal pull: across x = 0 the incoming dg_1 is -dg*_3 + hotc (anti-bounce-
// back, hot wall), across x = nx the incoming dg_3 is -dg*_1 + coldc (cold
// wall), across y = 0, ny plain bounce-back (adiabatic).
template <typename T, int Q>
__device__ __forceinline__ T pull_g(const KParams<T>& p, int i, int j, int k) {
  int s;
  const bool in = nbr<Q>(p.nx, p.ny, p.px, p.py, i, j, -1, -1, s);
  const T* a = in ? (p.g + OPP[Q] * p.P + s) : (p.g + Q * p.P + k);
  T v = ldg<T, EXv[Q] == 0>(a);
  if (EXv[Q] == 1) v = in ? v : p.hotc - v;
  if (EXv[Q] == -1) v = in ? v : p.coldc - v;
  return v;
}

template <typename T, int Q>
__device__ __forceinline__ void push_g(const KParams<T>& p, int i, int j, int k, T v) {
  int d;
  const bool in = nbr<Q>(p.nx, p.ny, p.px, p.py, i, j, 1, 1, d);
  T* a = in ? (p.g + Q * p.P + d) : (p.g + OPP[Q] * p.P + k);
  T w = v;
  if (EXv[Q] == -1) w = in ? v : p.hotc - v;  // leaves through x = 0
  if (EXv[Q] == 1) w = in ? v : p.coldc - v;  // leaves through x = nx
  stg<T, EXv[Q] == 0>(a, w);
}

// Interior fast path of the odd step: every neighbour is inside the grid, so
// the source / destination of direction Q is node k -/+ (e_Qx + e_Qy nx),
// addressed as a uniform plane base plus a 32-bit offset.
template <typename T, int Q>
__device__ __forceinline__ T pull_f_in(const KParams<T>& p, int k) {
  const T* plane = p.f + OPP[Q] * p.P;
  return ldg<T, EXv[Q] == 0>(plane + (unsigned)(k - EXv[Q] - EYv[Q] * p.nx));
}
template <typename T, int Q>
__device__ __forceinline__ void push_f_in(const KParams<T>& p, int k, T v) {
  T* plane = p.f + Q * p.P;
  stg<T, EXv[Q] == 0>(plane + (unsigned)(k + EXv[Q] + EYv[Q] * p.nx), v);
}
template <typename T, int Q>
__device__ __forceinline__ T pull_g_in(const KParams<T>& p, int k) {
  const T* plane = p.g + OPP[Q] * p.P;
  return ldg<T, EXv[Q] == 0>(plane + (unsigned)(k - EXv[Q] - EYv[Q] * p.nx));
}
template <typename T, int Q>
__device__ __forceinline__ void push_g_in(const KParams<T>& p, int k, T v) {
  T* plane = p.g + Q * p.P;
  stg<T, EXv[Q] == 0>(plane + (unsigned)(k + EXv[Q] + EYv[Q] * p.nx), v);
}

template <typename T>
__device__ __forceinline__ void load_interior_odd(const KParams<T>& p, int k, T df[9], T dg[5]) {
  df[0] = ldg<T, true>(p.f + (unsigned)k);
  df[1] = pull_f_in<T, 1>(p, k);
  df[2] = pull_f_in<T, 2>(p, k);
  df[3] = pull_f_in<T, 3>(p, k);
  df[4] = pull_f_in<T, 4>(p, k);
  df[5] = pull_f_in<T, 5>(p, k);
  df[6] = pull_f_in<T, 6>(p, k);
  df[7] = pull_f_in<T, 7>(p, k);
  df[8] = pull_f_in<T, 8>(p, k);
  dg[0] = ldg<T, true>(p.g + (unsigned)k);
  dg[1] = pull_g_in<T, 1>(p, k);
  dg[2] = pull_g_in<T, 2>(p, k);
  dg[3] = pull_g_in<T, 3>(p, k);
  dg[4] = pull_g_in<T, 4>(p, k);
}

template <typename T>
__device__ __forceinline__ void store_interior_odd(const KParams<T>& p, int k, const T df[9],
                                                   const T dg[5]) {
  stg<T, true>(p.f + (unsigned)k, df[0]);
  push_f_in<T, 1>(p, k, df[1]);
  push_f_in<T, 2>(p, k, df[2]);
  push_f_in<T, 3>(p, k, df[3]);
  push_f_in<T, 4>(p, k, df[4]);
  push_f_in<T, 5>(p, k, df[5]);
  push_f_in<T, 6>(p, k, df[6]);
  push_f_in<T, 7>(p, k, df[7]);
  push_f_in<T, 8>(p, k, df[8]);
  stg<T, true>(p.g + (unsigned)k, dg[0]);
  push_g_in<T, 1>(p, k, dg[1]);
  push_g_in<T, 2>(p, k, dg[2]);
  push_g_in<T, 3>(p, k, dg[3]);
  push_g_in<T, 4>(p, k, dg[4]);
}

// Pre-collision populations of node (i, j) for a state of the given parity.
template <typename T, bool ODD>
__device__ __forceinline__ void load_node(const KParams<T>& p, int i, int j, T df[9], T dg[5]) {
  const int k = j * p.nx + i;
  if (!ODD) {
#pragma unroll
    for (int q = 0; q < 9; ++q) df[q] = ldg<T, true>(p.f + q * p.P + k);
#pragma unroll
    for (int q = 0; q < 5; ++q) dg[q] = ldg<T, true>(p.g + q * p.P + k);
  } else {
    df[0] = ldg<T, true>(p.f + k);
    df[1] = pull_f<T, 1>(p, i, j, k);
    df[2] = pull_f<T, 2>(p, i, j, k);
    df[3] = pull_f<T, 3>(p, i, j, k);
    df[4] = pull_f<T, 4>(p, i, j, k);
    df[5] = pull_f<T, 5>(p, i, j, k);
    df[6] = pull_f<T, 6>(p, i, j, k);
    df[7] = pull_f<T, 7>(p, i, j, k);
    df[8] = pull_f<T, 8>(p, i, j, k);
    dg[0] = ldg<T, true>(p.g + k);
    dg[1] = pull_g<T, 1>(p, i, j, k);
    dg[2] = pull_g<T, 2>(p, i, j, k);
    dg[3] = pull_g<T, 3>(p, i, j, k);
    dg[4] = pull_g<T, 4>(p, i, j, k);
  }
}

template <typename T, bool ODD>
__device__ __forceinline__ void load_g(const KParams<T>& p, int i, int j, T dg[5]) {
  const int k = j * p.nx + i;
  if (!ODD) {
#pragma unroll
    for (int q = 0; q < 5; ++q) dg[q] = p.g[q * p.P + k];
  } else {
    dg[0] = p.g[k];
    dg[1] = pull_g<T, 1>(p, i, j, k);
    dg[2] = pull_g<T, 2>(p, i, j, k);
    dg[3] = pull_g<T, 3>(p, i, j, k);
    dg[4] = pull_g<T, 4>(p, i, j, k);
  }
}

template <typename T, bool ODD>
__device__ __forceinline__ void store_node(const KParams<T>& p, int i, int j, const T df[9],
                                           const T dg[5]) {
  const int k = j * p.nx + i;
  if (!ODD) {
#pragma unroll
    for (int q = 0; q < 9; ++q) stg<T, true>(p.f + OPP[q] * p.P + k, df[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) stg<T, true>(p.g + OPP[q] * p.P + k, dg[q]);
  } else {
    stg<T, true>(p.f + k, df[0]);
    push_f<T, 1>(p, i, j, k, df[1]);
    push_f<T, 2>(p, i, j, k, df[2]);
    push_f<T, 3>(p, i, j, k, df[3]);
    push_f<T, 4>(p, i, j, k, df[4]);
    push_f<T, 5>(p, i, j, k, df[5]);
    push_f<T, 6>(p, i, j, k, df[6]);
    push_f<T, 7>(p, i, j, k, df[7]);
    push_f<T, 8>(p, i, j, k, df[8]);
    stg<T, true>(p.g + k, dg[0]);
    push_g<T, 1>(p, i, j, k, dg[1]);
    push_g<T, 2>(p, i, j, k, dg[2]);
    push_g<T, 3>(p, i, j, k, dg[3]);
    push_g<T, 4>(p, i, j, k, dg[4]);
  }
}

// ---- local viscosity, Eq. (21) with Eqs. (15), (22), (23) ----
// |gamma|^2 = A + B s^2 with s = 1/(3 nu + 1/2); nu is the unique fixed point
// of nu = clamp(nu0 (gamma_scale |gamma|)^(n-1), nu_min, nu_max).  With
// y = log2(nu),
//   G(y) = y - log2 nu0 - (n-1) (log2 gamma_scale + log2(A + B s^2)/2)
// is strictly increasing (slope between min(n,1) and max(n,1)), and the
// clamped fixed point is the unclamped root clamped to [y_lo, y_hi].
// Start: the root for A << B s^2 and 3 nu >> 1/2, where G is linear in y:
//   n y0 = log2 nu0 + (n-1) (log2 gamma_scale + log2(B)/2 - log2 3).
// Then Newton steps, each clamped to [y_lo, y_hi] (iterates that leave the
// range stay on the bound the root lies beyond).  All lanes of a wave step
// together until every lane has converged.
template <typename T>
__device__ __forceinline__ T solve_nu(const KParams<T>& p, T A, T B) {
  const T half = T(0.5);
  const T hn = half * p.nm1;
  T y = (p.lc0 + p.nm1 * (half * flog2<T>(B) - T(1.584962500721156181453738943947816508))) * p.inv_n;
  y = fmin(fmax(y, p.y_lo), p.y_hi);  // log2(B = 0) = -inf: lands on a bound
  for (int it = 0; it < p.max_it; ++it) {
    const T nu = fexp2<T>(y);
    const T s = frcp<T>(T(3) * nu + half);
    const T s2 = s * s;
    const T g2 = A + B * s2;
    const T G = (y - p.lc0) - hn * flog2<T>(g2);
    const T dG = T(1) + T(3) * p.nm1 * B * s2 * s * nu * frcp<T>(g2);
    T yn = y - G * frcp<T>(dG);
    // no shear at all (g2 = 0): G = -inf (n < 1) or +inf (n > 1)
    if (!(g2 > T(0))) yn = G < T(0) ? p.y_hi : p.y_lo;
    yn = fmin(fmax(yn, p.y_lo), p.y_hi);
    const bool done = fabs(yn - y) <= p.tol;
    y = yn;
    if (__all(done)) break;
  }
  return fexp2<T>(y);
}

template <typename T>
struct Macro {
  T rho, ux, uy, T_abs, nu;
};

// Steps 2-6 of the update for one node (shifted populations in registers):
// moments, buoyancy, provisional velocity, viscosity, porous velocity.
template <typename T, bool POW, bool LOGDA>
__device__ __forceinline__ void node_macros(const KParams<T>& p, int k, const T df[9],
                                            const T dg[5], T& drho, T& rho, T& jx, T& jy,
                                            T& dT, T& Gx, T& Gy, T& nu, T& ux, T& uy, T& invK,
                                            T& invsK, T& m1, T& m7, T& m8) {
  drho = (df[0] + ((df[1] + df[2]) + (df[3] + df[4]))) + ((df[5] + df[6]) + (df[7] + df[8]));
  rho = T(1) + drho;
  jx = ((df[1] - df[3]) + (df[5] - df[6])) - (df[7] - df[8]);
  jy = ((df[2] - df[4]) + (df[5] + df[6])) - (df[7] + df[8]);
  dT = dg[0] + ((dg[1] + dg[2]) + (dg[3] + dg[4]));
  // Step 3: G = (gx, gy + g beta (T - T_m)), T - T_m = dT - (T_m - T_ref)
  Gx = p.gx;
  Gy = p.gy + p.gbeta * (dT - p.dTm);
  // Step 4: provisional velocity v = j/rho + eps G / 2
  const T irho = frcp<T>(rho);
  const T vx = jx * irho + T(0.5) * p.eps * Gx;
  const T vy = jy * irho + T(0.5) * p.eps * Gy;
  // moments e, pxx, pxy of the shifted populations (rest moments removed)
  const T s14 = (df[1] + df[2]) + (df[3] + df[4]);
  const T s58 = (df[5] + df[6]) + (df[7] + df[8]);
  m1 = (T(-4) * df[0] - s14) + T(2) * s58;
  m7 = (df[1] - df[2]) + (df[3] - df[4]);
  m8 = (df[5] - df[6]) + (df[7] - df[8]);
  // Step 5: viscosity
  if (POW) {
    const T vxx = vx * vx, vyy = vy * vy;
    const T en = (m1 + T(2) * drho) - T(3) * rho * (vxx + vyy) * p.inv_eps;
    const T pn = m7 - rho * (vxx - vyy) * p.inv_eps;
    const T qn = m8 - rho * vx * vy * p.inv_eps;
    const T irho2 = irho * irho;
    const T A = T(0.25) * p.s_e * p.s_e * en * en * irho2;
    const T B = T(2.25) * (pn * pn + T(4) * qn * qn) * irho2;
    nu = solve_nu<T>(p, A, B);
  } else {
    nu = p.nu_newt;
  }
  // Step 6: porous velocity u = v / (c0 + sqrt(c0^2 + c1 |v|))
  if (LOGDA) {
    // K = 10^logDa N^2
    invK = fexp2<T>(T(-3.321928094887362347870319) * p.logda[k]) * p.inv_Kscale;
    invsK = fsqrt<T>(invK);
  } else {
    invK = p.invK;
    invsK = p.invsK;
  }
  const T c0 = T(0.5) * (T(1) + T(0.5) * p.eps * nu * invK);
  const T c1 = T(0.5) * p.eps * p.Feps * invsK;
  const T vm = fsqrt<T>(vx * vx + vy * vy);
  const T iden = frcp<T>(c0 + fsqrt<T>(c0 * c0 + c1 * vm));
  ux = vx * iden;
  uy = vy * iden;
}

// The full local update: Steps 2-9 on shifted populations, in place.
template <typename T, bool POW, bool LOGDA>
__device__ __forceinline__ void collide(const KParams<T>& p, int k, T df[9], T dg[5]) {
  T drho, rho, jx, jy, dT, Gx, Gy, nu, ux, uy, invK, invsK, m1, m7, m8;
  node_macros<T, POW, LOGDA>(p, k, df, dg, drho, rho, jx, jy, dT, Gx, Gy, nu, ux, uy, invK,
                             invsK, m1, m7, m8);
  // Step 7: force per unit mass (Darcy + Forchheimer drag, eps G)
  const T um = fsqrt<T>(ux * ux + uy * uy);
  const T drag = p.eps * nu * invK + p.eps * p.Feps * invsK * um;
  const T Fx = p.eps * Gx - drag * ux;
  const T Fy = p.eps * Gy - drag * uy;
  // Step 8: D2Q9 MRT collision in moment space (shifted moments)
  const T ie = p.inv_eps;
  const T uu = ux * ux + uy * uy;
  const T ruu = T(3) * rho * uu * ie;
  const T uF = ux * Fx + uy * Fy;
  const T snu = frcp<T>(T(3) * nu + T(0.5));
  const T m2 = (T(4) * df[0] - T(2) * ((df[1] + df[2]) + (df[3] + df[4]))) +
               ((df[5] + df[6]) + (df[7] + df[8]));
  const T m4 = T(-2) * (df[1] - df[3]) + ((df[5] - df[6]) - (df[7] - df[8]));
  const T m6 = T(-2) * (df[2] - df[4]) + ((df[5] + df[6]) - (df[7] + df[8]));
  const T rux = rho * ux, ruy = rho * uy;
  const T Fm1 = T(6) * rho * uF * ie;
  const T ms1 = m1 - p.s_e * (m1 - (T(-2) * drho + ruu)) + (T(1) - T(0.5) * p.s_e) * Fm1;
  const T ms2 = m2 - p.s_eps * (m2 - (drho - ruu)) - (T(1) - T(0.5) * p.s_eps) * Fm1;
  const T ms3 = rux + T(0.5) * rho * Fx;
  const T ms4 = m4 - p.s_q * (m4 + rux) - (T(1) - T(0.5) * p.s_q) * rho * Fx;
  const T ms5 = ruy + T(0.5) * rho * Fy;
  const T ms6 = m6 - p.s_q * (m6 + ruy) - (T(1) - T(0.5) * p.s_q) * rho * Fy;
  const T hnu = T(1) - T(0.5) * snu;
  const T ms7 = m7 - snu * (m7 - rho * (ux * ux - uy * uy) * ie) +
                hnu * T(2) * rho * (ux * Fx - uy * Fy) * ie;
  const T ms8 = m8 - snu * (m8 - rho * ux * uy * ie) + hnu * rho * (ux * Fy + uy * Fx) * ie;
  // back to populations: M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
  const T a0 = drho * T(1.0 / 9.0);
  const T a1 = ms1 * T(1.0 / 36.0), a2 = ms2 * T(1.0 / 36.0);
  const T a3 = ms3 * T(1.0 / 6.0), a4 = ms4 * T(1.0 / 12.0);
  const T a5 = ms5 * T(1.0 / 6.0), a6 = ms6 * T(1.0 / 12.0);
  const T a7 = ms7 * T(0.25), a8 = ms8 * T(0.25);
  const T b14 = (a0 - a1) - T(2) * a2;
  const T b58 = (a0 + T(2) * a1) + a2;
  const T x1 = a3 - T(2) * a4, y1 = a5 - T(2) * a6;
  const T x5 = a3 + a4, y5 = a5 + a6;
  df[0] = (a0 - T(4) * a1) + T(4) * a2;
  df[1] = (b14 + x1) + a7;
  df[2] = (b14 + y1) - a7;
  df[3] = (b14 - x1) + a7;
  df[4] = (b14 - y1) - a7;
  df[5] = (b58 + x5) + (y5 + a8);
  df[6] = (b58 - x5) + (y5 - a8);
  df[7] = (b58 - x5) - (y5 - a8);
  df[8] = (b58 + x5) - (y5 + a8);
  // Step 9: D2Q5 MRT thermal collision (flux moments relax to u T)
  const T Tabs = p.T_ref + dT;
  const T n1 = dg[1] - dg[3], n2 = dg[2] - dg[4];
  const T n3 = T(-4) * dg[0] + ((dg[1] + dg[2]) + (dg[3] + dg[4]));
  const T n4 = (dg[1] - dg[2]) + (dg[3] - dg[4]);
  const T ns1 = n1 - p.s_g * (n1 - ux * Tabs);
  const T ns2 = n2 - p.s_g * (n2 - uy * Tabs);
  const T ns3 = n3 - p.sT_e * (n3 + T(2.0 / 3.0) * dT);
  const T ns4 = n4 - p.sT_nu * n4;
  const T c0 = dT * T(0.2), c1 = ns1 * T(0.5), c2 = ns2 * T(0.5);
  const T c3 = ns3 * T(0.05), c4 = ns4 * T(0.25);
  const T c03 = c0 + c3;
  dg[0] = c0 - T(4) * c3;
  dg[1] = (c03 + c1) + c4;
  dg[2] = (c03 + c2) - c4;
  dg[3] = (c03 - c1) + c4;
  dg[4] = (c03 - c2) - c4;
}

// One row tile [i0, i0 + TILE) of row j: gather, collide, scatter.
template <typename T, bool ODD, bool POW, bool LOGDA>
__device__ __forceinline__ void step_tile(const KParams<T>& p, int i0, int j) {
  const int i = i0 + threadIdx.x;
  T df[9], dg[5];
  if (ODD) {
    // Waves whose 64 nodes all have their 8 neighbours inside the grid take
    // the branch-free interior path (wave-uniform test).
    const int w0 = i0 + (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63);
    const bool interior = w0 >= 1 && w0 + 63 <= p.nx - 2 && j >= 1 && j <= p.ny - 2;
    if (interior) {
      const int k = j * p.nx + i;
      load_interior_odd<T>(p, k, df, dg);
      collide<T, POW, LOGDA>(p, k, df, dg);
      store_interior_odd<T>(p, k, df, dg);
      return;
    }
  }
  if (i >= p.nx) return;
  load_node<T, ODD>(p, i, j, df, dg);
  collide<T, POW, LOGDA>(p, j * p.nx + i, df, dg);
  store_node<T, ODD>(p, i, j, df, dg);
}

template <typename T, bool ODD, bool POW, bool LOGDA>
__global__ __launch_bounds__(TILE) void k_step(KParams<T> p, int tiles_x, int ntiles) {
  const int tile = tile_of_block(blockIdx.x, ntiles);
  const int j = tile / tiles_x;
  step_tile<T, ODD, POW, LOGDA>(p, (tile - j * tiles_x) * TILE, j);
}

// ---- batched parameter sweep: one launch steps every live case ----
// Workgroup b takes the (case, tile) pair of entry b of the schedule; cases
// that have met their stopping test are skipped.  Each case runs the same
// tile body as the single-case kernel, so a case advanced here is bitwise
// identical to the same case advanced alone.
template <typename T, bool ODD>
__global__ __launch_bounds__(TILE) void k_step_multi(const SweepCase<T>* __restrict__ cases,
                                                     const int2* __restrict__ sched,
                                                     const int* __restrict__ live) {
  const int2 e = sched[blockIdx.x];  // (case, tile within the case)
  if (!live[e.x]) return;
  const SweepCase<T>& c = cases[e.x];
  const int j = e.y / c.tiles_x;
  const int i0 = (e.y - j * c.tiles_x) * TILE;
  if (c.pow) step_tile<T, ODD, true, false>(c.p, i0, j);
  else step_tile<T, ODD, false, false>(c.p, i0, j);
}

// Rest state: df = 0, dg_q = w_q (T_init - T_ref).
template <typename T>
__global__ void k_init(KParams<T> p, T dg_init) {
  const int64_t n = (int64_t)p.nx * p.ny;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int q = 0; q < 9; ++q) p.f[q * p.P + k] = T(0);
    p.g[k] = dg_init * T(2);  // w_0 = 1/3 = 2 w_1
#pragma unroll
    for (int q = 1; q < 5; ++q) p.g[q * p.P + k] = dg_init;
  }
}

// Eq. (24): one workgroup, fixed summation order (deterministic).
template <typename T>
__global__ __launch_bounds__(256) void k_nu(KParams<T> p, int parity, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < p.ny; j += 256) {
    T g0[5], g1[5];
    if (parity) {
      load_g<T, true>(p, 0, j, g0);
      load_g<T, true>(p, 1, j, g1);
    } else {
      load_g<T, false>(p, 0, j, g0);
      load_g<T, false>(p, 1, j, g1);
    }
    const double t0 = (double)p.T_ref + (double)(g0[0] + ((g0[1] + g0[2]) + (g0[3] + g0[4])));
    const double t1 = (double)p.T_ref + (double)(g1[0] + ((g1[1] + g1[2]) + (g1[3] + g1[4])));
    acc += (double)p.nx * (8.0 - 9.0 * t0 + t1) / 3.0;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (double)p.ny;
}

// Residual: per-block max |theta - snapshot|, snapshot := theta.
template <typename T>
__global__ __launch_bounds__(256) void k_resid(KParams<T> p, int parity, T* snap,
                                               double* partial, int snapshot_only) {
  __shared__ double red[256];
  double mx = 0.0;
  const int64_t n = (int64_t)p.nx * p.ny;
  for (int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const int j = (int)(k / p.nx), i = (int)(k - (int64_t)j * p.nx);
    T g[5];
    if (parity) load_g<T, true>(p, i, j, g); else load_g<T, false>(p, i, j, g);
    const T dT = g[0] + ((g[1] + g[2]) + (g[3] + g[4]));
    double d = fabs((double)dT - (double)snap[k]);
    if (!(d <= 1.7976931348623157e308)) d = INFINITY;  // NaN / Inf -> +Inf
    mx = d > mx ? d : mx;
    snap[k] = dT;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = red[threadIdx.x + s];
      red[threadIdx.x] = o > red[threadIdx.x] ? o : red[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = snapshot_only ? 0.0 : red[0];
}

__global__ __launch_bounds__(256) void k_max_final(const double* partial, int n, double* out) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) mx = partial[b] > mx ? partial[b] : mx;
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = red[threadIdx.x + s];
      red[threadIdx.x] = o > red[threadIdx.x] ? o : red[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Sweep residual: one workgroup per schedule entry (a row tile of a live
// case) -> max |theta - snapshot| over the tile into the tile's slot of the
// case-major partial array, snapshot := theta.
template <typename T>
__global__ __launch_bounds__(TILE) void k_resid_multi(const SweepCase<T>* __restrict__ cases,
                                                      const int2* __restrict__ sched,
                                                      const int* __restrict__ live, int parity,
                                                      double* __restrict__ partial) {
  __shared__ double red[TILE];
  const int2 e = sched[blockIdx.x];
  if (!live[e.x]) return;  // uniform over the workgroup
  const SweepCase<T>& c = cases[e.x];
  const int j = e.y / c.tiles_x;
  const int i = (e.y - j * c.tiles_x) * TILE + threadIdx.x;
  double mx = 0.0;
  if (i < c.p.nx) {
    T g[5];
    if (parity) load_g<T, true>(c.p, i, j, g); else load_g<T, false>(c.p, i, j, g);
    const T dT = g[0] + ((g[1] + g[2]) + (g[3] + g[4]));
    const int64_t k = (int64_t)j * c.p.nx + i;
    double d = fabs((double)dT - (double)c.snap[k]);
    if (!(d <= 1.7976931348623157e308)) d = INFINITY;  // NaN / Inf -> +Inf
    mx = d;
    c.snap[k] = dT;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = TILE / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = red[threadIdx.x + s];
      red[threadIdx.x] = o > red[threadIdx.x] ? o : red[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[c.tile_base + e.y] = red[0];
}

// Stopping test of every live case after a chunk of steps: r = max over the
// case's tiles; the case stops when r < tol, when r is not finite, or when
// it has reached max_steps.  One workgroup, one thread per case.
template <typename T>
__global__ void k_retire(const SweepCase<T>* __restrict__ cases, int ncases,
                         const double* __restrict__ partial, int* __restrict__ live,
                         SweepStatus* __restrict__ st, int64_t chunk, double tol,
                         int64_t max_steps) {
  for (int c = threadIdx.x; c < ncases; c += blockDim.x) {
    if (!live[c]) continue;
    const SweepCase<T>& cs = cases[c];
    double r = 0.0;
    for (int b = 0; b < cs.ntiles; ++b) {
      const double v = partial[cs.tile_base + b];
      r = v > r ? v : r;
    }
    st[c].steps += chunk;
    st[c].residual = r;
    const bool finite = r <= 1.7976931348623157e308;
    if (r < tol || !finite || st[c].steps >= max_steps) live[c] = 0;
  }
}

template <typename T, bool ODD, bool POW, bool LOGDA, typename O>
__global__ __launch_bounds__(TILE) void k_fields(KParams<T> p, O* U, O* V, O* th, O* nuo) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= p.nx) return;
  T df[9], dg[5];
  load_node<T, ODD>(p, i, j, df, dg);
  T drho, rho, jx, jy, dT, Gx, Gy, nu, ux, uy, invK, invsK, m1, m7, m8;
  const int k = j * p.nx + i;
  node_macros<T, POW, LOGDA>(p, k, df, dg, drho, rho, jx, jy, dT, Gx, Gy, nu, ux, uy, invK,
                             invsK, m1, m7, m8);
  if (U) U[k] = (O)(ux * p.inv_U);
  if (V) V[k] = (O)(uy * p.inv_U);
  if (th) th[k] = (O)(p.T_ref + dT);
  if (nuo) nuo[k] = (O)nu;
}

// D2Q9 / D2Q5 rest weights for the absolute <-> shifted conversions.
template <typename T>
__device__ __forceinline__ T w9(int q) {
  return q == 0 ? T(4.0 / 9.0) : (q < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}
template <typename T>
__device__ __forceinline__ T w5(int q) {
  return q == 0 ? T(1.0 / 3.0) : T(1.0 / 6.0);
}

template <typename T, bool ODD, typename O>
__global__ __launch_bounds__(TILE) void k_get_pop(KParams<T> p, O* f, O* g) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= p.nx) return;
  T df[9], dg[5];
  load_node<T, ODD>(p, i, j, df, dg);
  const int64_t k = (int64_t)j * p.nx + i, n = (int64_t)p.nx * p.ny;
#pragma unroll
  for (int q = 0; q < 9; ++q) f[q * n + k] = (O)((double)df[q] + (double)w9<T>(q));
#pragma unroll
  for (int q = 0; q < 5; ++q) g[q * n + k] = (O)((double)dg[q] + (double)w5<T>(q) * (double)p.T_ref);
}

template <typename T, typename I>
__global__ __launch_bounds__(TILE) void k_set_pop(KParams<T> p, const I* f, const I* g) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= p.nx) return;
  const int64_t k = (int64_t)j * p.nx + i, n = (int64_t)p.nx * p.ny;
#pragma unroll
  for (int q = 0; q < 9; ++q) p.f[q * p.P + k] = (T)((double)f[q * n + k] - (double)w9<T>(q));
#pragma unroll
  for (int q = 0; q < 5; ++q)
    p.g[q * p.P + k] = (T)((double)g[q * n + k] - (double)w5<T>(q) * (double)p.T_ref);
}

template <typename T, typename I>
__global__ void k_convert(T* dst, const I* src, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = (T)src[k];
}

__global__ void k_header(int64_t* dst, int64_t steps, uint64_t tag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = (int64_t)tag;
    dst[1] = steps;
  }
}

typedef float v4f __attribute__((ext_vector_type(4)));

// One 16-byte vector per thread, streaming (non-temporal) load and store.
__global__ __launch_bounds__(256) void k_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                              int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (k < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

inline int grid_for(int64_t n, int per = 256, int cap = 65536) {
  int64_t b = (n + per - 1) / per;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

template <typename T>
hipError_t launch_step(const KParams<T>& p, const Launch& L, int parity, bool pow, bool logda) {
  dim3 grid(L.ntiles), block(TILE);
#define PM_STEP(ODD, POW, LOG) \
  hipLaunchKernelGGL((k_step<T, ODD, POW, LOG>), grid, block, 0, L.stream, p, L.tiles_x, L.ntiles)
  if (parity) {
    if (pow) { if (logda) PM_STEP(true, true, true); else PM_STEP(true, true, false); }
    else { if (logda) PM_STEP(true, false, true); else PM_STEP(true, false, false); }
  } else {
    if (pow) { if (logda) PM_STEP(false, true, true); else PM_STEP(false, true, false); }
    else { if (logda) PM_STEP(false, false, true); else PM_STEP(false, false, false); }
  }
#undef PM_STEP
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_multi(const SweepCase<T>* cases, const int2* sched, const int* live,
                             int nsched, int parity, hipStream_t s) {
  if (parity)
    hipLaunchKernelGGL((k_step_multi<T, true>), dim3(nsched), dim3(TILE), 0, s, cases, sched, live);
  else
    hipLaunchKernelGGL((k_step_multi<T, false>), dim3(nsched), dim3(TILE), 0, s, cases, sched, live);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_multi(const SweepCase<T>* cases, int ncases, const int2* sched, int* live,
                              int nsched, int parity, double* partial, SweepStatus* st,
                              int64_t chunk, double tol, int64_t max_steps, hipStream_t s) {
  hipLaunchKernelGGL((k_resid_multi<T>), dim3(nsched), dim3(TILE), 0, s, cases, sched,
                     (const int*)live, parity, partial);
  hipLaunchKernelGGL((k_retire<T>), dim3(1), dim3(64), 0, s, cases, ncases, (const double*)partial,
                     live, st, chunk, tol, max_steps);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const KParams<T>& p, const Launch& L, T dg_init) {
  hipLaunchKernelGGL((k_init<T>), dim3(grid_for((int64_t)p.nx * p.ny)), dim3(256), 0, L.stream,
                     p, dg_init);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_nu(const KParams<T>& p, const Launch& L, int parity, double* out) {
  hipLaunchKernelGGL((k_nu<T>), dim3(1), dim3(256), 0, L.stream, p, parity, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const KParams<T>& p, const Launch& L, int parity, T* snap,
                           double* partial, double* out, int snapshot_only) {
  const int nb = grid_for((int64_t)p.nx * p.ny, 256, RED_BLOCKS);
  hipLaunchKernelGGL((k_resid<T>), dim3(nb), dim3(256), 0, L.stream, p, parity, snap, partial,
                     snapshot_only);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, L.stream, (const double*)partial, nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fields(const KParams<T>& p, const Launch& L, int parity, bool pow, bool logda,
                         void* U, void* V, void* th, void* nu, int out_fp64) {
  dim3 grid(L.tiles_x, p.ny), block(TILE);
#define PM_F(ODD, POW, LOG, O)                                                              \
  hipLaunchKernelGGL((k_fields<T, ODD, POW, LOG, O>), grid, block, 0, L.stream, p, (O*)U, \
                     (O*)V, (O*)th, (O*)nu)
#define PM_F2(ODD, POW, LOG) \
  do { if (out_fp64) PM_F(ODD, POW, LOG, double); else PM_F(ODD, POW, LOG, float); } while (0)
#define PM_F3(ODD, POW) \
  do { if (logda) PM_F2(ODD, POW, true); else PM_F2(ODD, POW, false); } while (0)
#define PM_F4(ODD) do { if (pow) PM_F3(ODD, true); else PM_F3(ODD, false); } while (0)
  if (parity) PM_F4(true); else PM_F4(false);
#undef PM_F4
#undef PM_F3
#undef PM_F2
#undef PM_F
  return hipGetLastError();
}

template <typename T>
hipError_t launch_get_pop(const KParams<T>& p, const Launch& L, int parity, void* f, void* g,
                          int out_fp64) {
  dim3 grid(L.tiles_x, p.ny), block(TILE);
  if (parity) {
    if (out_fp64) hipLaunchKernelGGL((k_get_pop<T, true, double>), grid, block, 0, L.stream, p, (double*)f, (double*)g);
    else hipLaunchKernelGGL((k_get_pop<T, true, float>), grid, block, 0, L.stream, p, (float*)f, (float*)g);
  } else {
    if (out_fp64) hipLaunchKernelGGL((k_get_pop<T, false, double>), grid, block, 0, L.stream, p, (double*)f, (double*)g);
    else hipLaunchKernelGGL((k_get_pop<T, false, float>), grid, block, 0, L.stream, p, (float*)f, (float*)g);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_set_pop(const KParams<T>& p, const Launch& L, const void* f, const void* g,
                          int in_fp64) {
  dim3 grid(L.tiles_x, p.ny), block(TILE);
  if (in_fp64)
    hipLaunchKernelGGL((k_set_pop<T, double>), grid, block, 0, L.stream, p, (const double*)f, (const double*)g);
  else
    hipLaunchKernelGGL((k_set_pop<T, float>), grid, block, 0, L.stream, p, (const float*)f, (const float*)g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_set_logda(const KParams<T>& p, const Launch& L, T* dst, const void* src,
                            int in_fp64) {
  const int64_t n = (int64_t)p.nx * p.ny;
  if (in_fp64)
    hipLaunchKernelGGL((k_convert<T, double>), dim3(grid_for(n)), dim3(256), 0, L.stream, dst, (const double*)src, n);
  else
    hipLaunchKernelGGL((k_convert<T, float>), dim3(grid_for(n)), dim3(256), 0, L.stream, dst, (const float*)src, n);
  return hipGetLastError();
}

hipError_t launch_write_header(void* dst, int64_t steps, uint64_t tag, hipStream_t s) {
  hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, (int64_t*)dst, steps, tag);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const v4f*)src, (v4f*)dst, n);
  return hipGetLastError();
}

#define PM_INST(T)                                                                              \
  template hipError_t launch_step<T>(const KParams<T>&, const Launch&, int, bool, bool);        \
  template hipError_t launch_init<T>(const KParams<T>&, const Launch&, T);                      \
  template hipError_t launch_nu<T>(const KParams<T>&, const Launch&, int, double*);             \
  template hipError_t launch_residual<T>(const KParams<T>&, const Launch&, int, T*, double*,    \
                                         double*, int);                                         \
  template hipError_t launch_fields<T>(const KParams<T>&, const Launch&, int, bool, bool, void*, \
                                       void*, void*, void*, int);                               \
  template hipError_t launch_get_pop<T>(const KParams<T>&, const Launch&, int, void*, void*, int); \
  template hipError_t launch_set_pop<T>(const KParams<T>&, const Launch&, const void*,          \
                                        const void*, int);                                      \
  template hipError_t launch_set_logda<T>(const KParams<T>&, const Launch&, T*, const void*, int); \
  template hipError_t launch_step_multi<T>(const SweepCase<T>*, const int2*, const int*, int, int, \
                                           hipStream_t);                                          \
  template hipError_t launch_resid_multi<T>(const SweepCase<T>*, int, const int2*, int*, int, int, \
                                            double*, SweepStatus*, int64_t, double, int64_t,      \
                                            hipStream_t);
PM_INST(float)
PM_INST(double)
#undef PM_INST

}  // namespace pm
