// pm_device.h -- device-side building blocks of the gfx950 lattice Boltzmann
// update shared by the forward, sweep and adjoint kernels: population
// addressing (AA pattern), the local viscosity solve, the node update.
#pragma once

#include "pm_internal.h"

#include <cmath>
#include <type_traits>

namespace pm {
namespace dev {


// D2Q9 velocities, Eq. (14): 0 rest; 1-4 E, N, W, S; 5-8 NE, NW, SW, SE.
// D2Q5 (Eq. 19) uses the first five.
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int EXv[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EYv[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Workgroup b handles row tile b in row-major order.  Dispatch deals
// consecutive workgroups round-robin to the 8 XCDs, so at any moment all XCDs
// stream through one narrow band of rows, within few DRAM pages.  (Giving
// each XCD its own contiguous band of rows, or groups of 2-64 consecutive
// tiles, measured no faster.)
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

// Global loads and stores of stored populations (type S), converted from and
// to the compute type T (a store to _Float16 rounds to nearest); NT =
// streaming (non-temporal) hint, used for the aligned population accesses of
// the step (each value is touched once per step, so keeping it in L2/MALL
// only evicts useful lines).
template <typename T, bool NT, typename S>
__device__ __forceinline__ T ldg(const S* a) {
  S v;
  if constexpr (NT) v = __builtin_nontemporal_load(a);
  else v = *a;
  return (T)v;
}
// Store v as S.  HSR (FP32 value, half storage): the conversion rounds
// stochastically with the hardware's FP32 -> FP16 conversion, r the random
// word (its high bits decide; every r rounds to one of the two halves that
// bracket v, and a uniformly random r rounds without bias).
template <typename T, bool NT, bool HSR = false, typename S>
__device__ __forceinline__ void stg(S* a, T v, unsigned r = 0) {
#ifdef PM_EMULATE_FP32_STORAGE
  v = (T)(float)v;
#endif
  S w;
  if constexpr (HSR) {
    static_assert(std::is_same<S, _Float16>::value && std::is_same<T, float>::value,
                  "hardware stochastic rounding: FP32 values into half storage");
    typedef short short2_t __attribute__((ext_vector_type(2)));
    const short2_t h = __builtin_amdgcn_cvt_sr_f16_f32(short2_t{0, 0}, v, r, false);
    w = __builtin_bit_cast(_Float16, (short)h.x);
  } else {
    w = (S)v;
  }
  if constexpr (NT) __builtin_nontemporal_store(w, a);
  else *a = w;
}

// The stochastic conversion of population q (f0..f8, g0..g4 as q = 0..13)
// takes the node's word rotated by SR_ROT[q] bits, so that the populations'
// rounding decisions are not all taken at the same threshold (opposite
// directions sit 14-16 bits apart).
constexpr int SR_ROT[14] = {0, 2, 4, 16, 18, 6, 8, 20, 22, 10, 12, 14, 26, 24};
__device__ __forceinline__ unsigned rot_word(unsigned r, int q) {
  return SR_ROT[q] ? __builtin_amdgcn_alignbit(r, r, SR_ROT[q]) : r;
}

// ---- population addressing ----
// Population q of node (i, j) lives at f[q * qs + j * rs + i] (g likewise);
// see KParams.  pop_off gives the node part j * rs + i.
template <typename T, typename S>
__device__ __forceinline__ int64_t pop_off(const KParams<T, S>& p, int i, int j) {
  return (int64_t)j * p.rs + i;
}

// ---- neighbour addressing for the odd (streaming) step ----
// Source of the pull of direction Q into node (i, j): node (i, j) - e_Q, or
// the node itself when that crosses a wall.  Returns whether it is inside.
template <int Q>
__device__ __forceinline__ bool nbr(int nx, int ny, int px, int py, int i, int j, int sx, int sy,
                                    int& si, int& sj) {
  // (sx, sy) = +-e_Q direction sign applied by the caller
  si = i + sx * EXv[Q];
  sj = j + sy * EYv[Q];
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
  return in;
}

// Thermal pull (o = pop_off(p, i, j) of the node itself): across x = 0 the
// incoming dg_1 is -dg*_3 + hotc (anti-bounce-back, hot wall), across x = nx
// the incoming dg_3 is -dg*_1 + coldc (cold wall), across y = 0, ny plain
// bounce-back (adiabatic).  load_g uses it; the step kernels use
// load_node_raw and pull_walls, which compute the same.
template <typename T, int Q, typename S>
__device__ __forceinline__ T pull_g(const KParams<T, S>& p, int i, int j, int64_t o) {
  int si, sj;
  const bool in = nbr<Q>(p.nx, p.ny, p.px, p.py, i, j, -1, -1, si, sj);
  const S* a = in ? (p.g + OPP[Q] * p.qs + pop_off(p, si, sj)) : (p.g + Q * p.qs + o);
  T v = ldg<T, EXv[Q] == 0>(a);
  if (EXv[Q] == 1) v = in ? v : p.hotc - v;
  if (EXv[Q] == -1) v = in ? v : p.coldc - v;
  return v;
}

// Interior fast path of the odd step: every neighbour is inside the grid.
// Rows j - 1, j, j + 1 are addressed from one wave-uniform base (row j - 1)
// plus a non-negative 32-bit lane offset.
template <typename S>
struct RowBase {
  S* f;  // p.f + (j - 1) rs
  S* g;
};
template <typename T, typename S>
__device__ __forceinline__ RowBase<S> row_base(const KParams<T, S>& p, int j) {
  const int64_t o = (int64_t)(j - 1) * p.rs;
  return RowBase<S>{p.f + o, p.g + o};
}
// offset of population q of node (i + dx, j + dy) from row j - 1
template <typename T, typename S>
__device__ __forceinline__ unsigned in_off(const KParams<T, S>& p, int q, int i, int dx, int dy) {
  return (unsigned)(q * p.qs + (1 + dy) * p.rs + (i + dx));
}

template <typename T, typename S>
__device__ __forceinline__ void load_interior_odd(const KParams<T, S>& p, const RowBase<S>& b, int i,
                                                  T df[9], T dg[5]) {
  df[0] = ldg<T, true>(b.f + in_off(p, 0, i, 0, 0));
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    const S* a = b.f + in_off(p, OPP[q], i, -EXv[q], -EYv[q]);
    df[q] = EXv[q] == 0 ? ldg<T, true>(a) : ldg<T, false>(a);
  }
  dg[0] = ldg<T, true>(b.g + in_off(p, 0, i, 0, 0));
#pragma unroll
  for (int q = 1; q < 5; ++q) {
    const S* a = b.g + in_off(p, OPP[q], i, -EXv[q], -EYv[q]);
    dg[q] = EXv[q] == 0 ? ldg<T, true>(a) : ldg<T, false>(a);
  }
}

template <typename T, bool HSR = false, typename S>
__device__ __forceinline__ void store_interior_odd(const KParams<T, S>& p, const RowBase<S>& b, int i,
                                                   const T df[9], const T dg[5], unsigned r = 0) {
  stg<T, true, HSR>(b.f + in_off(p, 0, i, 0, 0), df[0], r);
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    S* a = b.f + in_off(p, q, i, EXv[q], EYv[q]);
    if (EXv[q] == 0) stg<T, true, HSR>(a, df[q], rot_word(r, q));
    else stg<T, false, HSR>(a, df[q], rot_word(r, q));
  }
  stg<T, true, HSR>(b.g + in_off(p, 0, i, 0, 0), dg[0], rot_word(r, 9));
#pragma unroll
  for (int q = 1; q < 5; ++q) {
    S* a = b.g + in_off(p, q, i, EXv[q], EYv[q]);
    if (EXv[q] == 0) stg<T, true, HSR>(a, dg[q], rot_word(r, 9 + q));
    else stg<T, false, HSR>(a, dg[q], rot_word(r, 9 + q));
  }
}

// Pre-collision populations of node (i, j) for a state of the given parity,
// before the odd step's thermal wall conditions (pull_walls).
template <typename T, bool ODD, typename S>
__device__ __forceinline__ void load_node_raw(const KParams<T, S>& p, int i, int j, T df[9], T dg[5]) {
  const int64_t o = pop_off(p, i, j);
  if (!ODD) {
#pragma unroll
    for (int q = 0; q < 9; ++q) df[q] = ldg<T, true>(p.f + q * p.qs + o);
#pragma unroll
    for (int q = 0; q < 5; ++q) dg[q] = ldg<T, true>(p.g + q * p.qs + o);
    return;
  }
  // Odd step: the pull of direction q into (i, j) reads population OPP[q] of
  // node (i, j) - e_q, or the node's own population q where that crosses a
  // wall (bounce-back; the thermal walls' constants are pull_walls').  The source column (i - 1, i or i + 1, wrapped on a
  // periodic axis) and row (j - 1, j or j + 1: wave-uniform) and whether
  // each is inside are worked out once; each address is then a select
  // between two indices, so no branch separates the 14 loads and all of
  // them are in flight before any value is used.
  const int nx = p.nx, ny = p.ny;
  const int im = p.px && i == 0 ? nx - 1 : i - 1;       // source column of e_x = +1
  const int ip = p.px && i == nx - 1 ? 0 : i + 1;       // of e_x = -1
  const bool in_im = p.px || i >= 1, in_ip = p.px || i + 1 < nx;
  const int jm = p.py && j == 0 ? ny - 1 : j - 1;       // source row of e_y = +1
  const int jp = p.py && j == ny - 1 ? 0 : j + 1;       // of e_y = -1
  const bool in_jm = p.py || j >= 1, in_jp = p.py || j + 1 < ny;
  const int64_t rm = (int64_t)jm * p.rs, r0 = (int64_t)j * p.rs, rp = (int64_t)jp * p.rs;
#pragma unroll
  for (int q = 0; q < 14; ++q) {
    const int d = q < 9 ? q : q - 9;  // direction within D2Q9 / D2Q5
    const S* base = q < 9 ? p.f : p.g;
    const int si = EXv[d] > 0 ? im : (EXv[d] < 0 ? ip : i);
    const int64_t rs = EYv[d] > 0 ? rm : (EYv[d] < 0 ? rp : r0);
    const bool in = (EXv[d] > 0 ? in_im : (EXv[d] < 0 ? in_ip : true)) &
                    (EYv[d] > 0 ? in_jm : (EYv[d] < 0 ? in_jp : true));
    const int64_t idx = in ? OPP[d] * p.qs + rs + si : d * p.qs + o;
    const T v = EXv[d] == 0 ? ldg<T, true>(base + idx) : ldg<T, false>(base + idx);
    if (q < 9) df[q] = v;
    else dg[q - 9] = v;
  }
}

// The thermal conditions of the odd step's pull, as in pull_g: at the hot
// wall (x = 0) the pulled dg_1 is hotc - dg_1 as loaded, at the cold wall
// (x = nx - 1) the pulled dg_3 is coldc - dg_3 (anti-bounce-back).
template <typename T, typename S>
__device__ __forceinline__ void pull_walls(const KParams<T, S>& p, int i, T dg[5]) {
  const bool hot = !p.px & (i == 0), cold = !p.px & (i == p.nx - 1);  // selects, no branch
  dg[1] = hot ? p.hotc - dg[1] : dg[1];
  dg[3] = cold ? p.coldc - dg[3] : dg[3];
}

// Pre-collision populations of node (i, j) for a state of the given parity.
template <typename T, bool ODD, typename S>
__device__ __forceinline__ void load_node(const KParams<T, S>& p, int i, int j, T df[9], T dg[5]) {
  load_node_raw<T, ODD>(p, i, j, df, dg);
  if (ODD) pull_walls(p, i, dg);
}

template <typename T, bool ODD, typename S>
__device__ __forceinline__ void load_g(const KParams<T, S>& p, int i, int j, T dg[5]) {
  const int64_t o = pop_off(p, i, j);
  if (!ODD) {
#pragma unroll
    for (int q = 0; q < 5; ++q) dg[q] = (T)p.g[q * p.qs + o];
  } else {
    dg[0] = (T)p.g[o];
    dg[1] = pull_g<T, 1>(p, i, j, o);
    dg[2] = pull_g<T, 2>(p, i, j, o);
    dg[3] = pull_g<T, 3>(p, i, j, o);
    dg[4] = pull_g<T, 4>(p, i, j, o);
  }
}

template <typename T, bool ODD, bool HSR = false, typename S>
__device__ __forceinline__ void store_node(const KParams<T, S>& p, int i, int j, const T df[9],
                                           const T dg[5], unsigned r = 0) {
  const int64_t o = pop_off(p, i, j);
  if (!ODD) {
#pragma unroll
    for (int q = 0; q < 9; ++q) stg<T, true, HSR>(p.f + OPP[q] * p.qs + o, df[q], rot_word(r, q));
#pragma unroll
    for (int q = 0; q < 5; ++q) stg<T, true, HSR>(p.g + OPP[q] * p.qs + o, dg[q], rot_word(r, 9 + q));
  } else {
    // Odd step: post-collision population q goes to slot q of node (i, j) +
    // e_q, or back into the node's own slot OPP[q] where that crosses a wall;
    // the destination column (i + 1, i or i - 1, wrapped on a periodic axis),
    // row (wave-uniform) and inside tests are worked out once and each
    // address is a select between two indices.
    const int nx = p.nx, ny = p.ny;
    const int ip = p.px && i == nx - 1 ? 0 : i + 1;  // destination column of e_x = +1
    const int im = p.px && i == 0 ? nx - 1 : i - 1;  // of e_x = -1
    const bool in_ip = p.px || i + 1 < nx, in_im = p.px || i >= 1;
    const int jp = p.py && j == ny - 1 ? 0 : j + 1;  // destination row of e_y = +1
    const int jm = p.py && j == 0 ? ny - 1 : j - 1;  // of e_y = -1
    const bool in_jp = p.py || j + 1 < ny, in_jm = p.py || j >= 1;
    const int64_t rp = (int64_t)jp * p.rs, r0 = (int64_t)j * p.rs, rm = (int64_t)jm * p.rs;
#pragma unroll
    for (int q = 0; q < 14; ++q) {
      const int d = q < 9 ? q : q - 9;  // direction within D2Q9 / D2Q5
      S* base = q < 9 ? p.f : p.g;
      const int di = EXv[d] > 0 ? ip : (EXv[d] < 0 ? im : i);
      const int64_t rs = EYv[d] > 0 ? rp : (EYv[d] < 0 ? rm : r0);
      const bool in = (EXv[d] > 0 ? in_ip : (EXv[d] < 0 ? in_im : true)) &
                      (EYv[d] > 0 ? in_jp : (EYv[d] < 0 ? in_jm : true));
      const int64_t idx = in ? d * p.qs + rs + di : OPP[d] * p.qs + o;
      T w = q < 9 ? df[d] : dg[d];
      // thermal populations leaving through the hot (x = 0) or cold (x = nx)
      // wall come back anti-bounced: hotc - v or coldc - v
      if (q >= 9 && EXv[d] == -1) w = in ? w : p.hotc - w;
      if (q >= 9 && EXv[d] == 1) w = in ? w : p.coldc - w;
      if (EXv[d] == 0) stg<T, true, HSR>(base + idx, w, rot_word(r, q));
      else stg<T, false, HSR>(base + idx, w, rot_word(r, q));
    }
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
// range stay on the bound the root lies beyond).  The lanes of a wave loop
// together until every lane has converged; a converged lane stops updating.
// FP64 first takes the start and four Newton steps in FP32 on the hardware
// exp2 / log2 / reciprocal (cheap, ~1e-6 in y), so that its own Newton steps,
// whose library exp2 and log2 cost about 170 instructions each, converge in
// two instead of four or five.
constexpr int NU_FP32_STEPS = 4;

template <typename T, typename S>
__device__ __forceinline__ T nu_start(const KParams<T, S>& p, T A, T B) {
  if constexpr (std::is_same<T, double>::value) {
    const float lo = (float)p.y_lo, hi = (float)p.y_hi, lc0 = (float)p.lc0, nm1 = (float)p.nm1;
    const float Af = (float)A, Bf = (float)B;
    float y = (lc0 + nm1 * (0.5f * __builtin_amdgcn_logf(Bf) - 1.5849625007f)) * (float)p.inv_n;
    y = fminf(fmaxf(y, lo), hi);
    for (int it = 0; it < NU_FP32_STEPS; ++it) {  // a fixed count: no lane depends on another
      const float nu = __builtin_amdgcn_exp2f(y);
      const float s = __builtin_amdgcn_rcpf(3.0f * nu + 0.5f);
      const float g2 = Af + Bf * s * s;
      const float G = (y - lc0) - 0.5f * nm1 * __builtin_amdgcn_logf(g2);
      const float dG = 1.0f + 3.0f * nm1 * Bf * s * s * s * nu * __builtin_amdgcn_rcpf(g2);
      const float yn = y - G * __builtin_amdgcn_rcpf(dG);
      if (g2 > 0.0f && yn == yn) y = fminf(fmaxf(yn, lo), hi);  // no shear in FP32: the FP64 steps decide
    }
    return fmin(fmax((double)y, p.y_lo), p.y_hi);
  } else {
    const T y = (p.lc0 + p.nm1 * (T(0.5) * flog2<T>(B) - T(1.584962500721156181453738943947816508))) * p.inv_n;
    return fmin(fmax(y, p.y_lo), p.y_hi);  // log2(B = 0) = -inf: lands on a bound
  }
}

template <typename T, typename S>
__device__ __forceinline__ T solve_nu(const KParams<T, S>& p, T A, T B) {
  const T half = T(0.5);
  const T hn = half * p.nm1;
  T y = nu_start<T>(p, A, B);
  bool conv = false;
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
    // each lane keeps the first iterate whose step is within the tolerance,
    // so a node's viscosity does not depend on which nodes share its wave
    if (!conv) {
      conv = fabs(yn - y) <= p.tol;
      y = yn;
    }
    if (__all(conv)) break;
  }
  return fexp2<T>(y);
}

template <typename T>
struct Macro {
  T rho, ux, uy, T_abs, nu;
};

// Steps 2-6 of the update for one node (shifted populations in registers):
// moments, buoyancy, provisional velocity, viscosity, porous velocity.
template <typename T, bool POW, bool LOGDA, typename S>
__device__ __forceinline__ void node_macros(const KParams<T, S>& p, int k, const T df[9],
                                            const T dg[5], T& drho, T& rho, T& jx, T& jy,
                                            T& dT, T& Gx, T& Gy, T& nu, T& ux, T& uy, T& invK,
                                            T& invsK, T& m1, T& m7, T& m8) {
  // read first, so that the load is in flight with the node's populations
  const T ldk = LOGDA ? (T)p.logda[k] : T(0);
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
    nu = solve_nu(p, A, B);
  } else {
    nu = p.nu_newt;
  }
  // Step 6: porous velocity u = v / (c0 + sqrt(c0^2 + c1 |v|))
  if (LOGDA) {
    // K = 10^logDa N^2
    invK = fexp2<T>(T(-3.321928094887362347870319) * ldk) * p.inv_Kscale;
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

// ---- stochastic rounding of the population updates (PM_ROUND_STOCHASTIC) ----
// With round-to-nearest, a state near a steady flow rounds the same way step
// after step, and the slowly decaying modes of the cavity accumulate that
// fixed rounding pattern into a bias far above one rounding.  The update is
// therefore written as f* = a + b (a the stored population, b its change from
// the moment changes) and rounded to the storage type without bias:
//   * FP32 storage: added as a + (b + xi), xi uniform on (-ulp(a), ulp(a)),
//     then rounded to nearest by the FP32 add.  A uniform dither whose width
//     is a whole number of grid spacings leaves rounding to nearest unbiased,
//     and 2 ulp(a) is one, two or four spacings at a + b (a + b one binade
//     above a, in a's binade, or one below).
//   * half storage: a + b in FP32, then the hardware's stochastically
//     rounding FP32 -> FP16 conversion at the store (it rounds up with the
//     probability of the fraction of a half spacing cut off, subnormal halves
//     included).
// One random word per node update serves all 14 populations (each is still
// rounded without bias); it comes from one round of the "lowbias32" integer
// hash (Chris Wellons, hash prospector, public domain) of the node index and
// three of the node's incoming populations, so it is deterministic, changes
// from step to step as the state does, and is the same in every kernel that
// updates the node.
__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// The node's random word.
__device__ __forceinline__ unsigned node_word(int k, float a0, float a1, float a2) {
  return mix32((unsigned)k * 0x9e3779b1u ^ __float_as_uint(a0) ^
               __builtin_amdgcn_alignbit(__float_as_uint(a1), __float_as_uint(a1), 11) ^
               __builtin_amdgcn_alignbit(__float_as_uint(a2), __float_as_uint(a2), 22));
}

// The FP32 dither scale: u 2^-22 with u uniform on (-1/2, 1/2) (24 bits of
// the word), so that us * 2^e(a) = u * 2 ulp(a).
__device__ __forceinline__ float dither_scale(unsigned h) {
  constexpr float sc = 0x1p-22f;
  return __builtin_fmaf((float)(h >> 8), 0x1p-24f * sc, (0x1p-25f - 0.5f) * sc);
}

// a + b with the node's FP32 dither (2^e(a) is 0 for a zero or subnormal a:
// no dither there).
__device__ __forceinline__ float dither_add(float a, float b, float us) {
  const unsigned e = __float_as_uint(a) & 0x7f800000u;
  return a + __builtin_fmaf(us, __uint_as_float(e), b);
}

// f* = a + b ahead of its rounding to the storage type S (see above).
template <typename S>
__device__ __forceinline__ float sr_add(float a, float b, float us) {
  if constexpr (std::is_same<S, _Float16>::value) return a + b;
  else return dither_add(a, b, us);
}

// The full local update: Steps 2-9 on shifted populations, in place.
// With SR and half storage, *rw receives the node's random word for the
// stores' stochastic conversion (the caller passes rw then).
template <typename T, bool POW, bool LOGDA, bool SR = false, typename S>
__device__ __forceinline__ void collide(const KParams<T, S>& p, int k, T df[9], T dg[5],
                                        unsigned* rw = nullptr) {
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
  float us = 0.0f;  // the node's dither scale (SR)
  if constexpr (SR) {
    static_assert(sizeof(T) == 4, "stochastic rounding is for FP32 compute (FP32 or FP16 storage)");
    const unsigned h = node_word(k, df[0], dg[0], df[5]);
    if constexpr (std::is_same<S, _Float16>::value) *rw = h;
    else us = dither_scale(h);
    // the same back-transform applied to the moment changes ms - m (the
    // density is conserved), added to the incoming populations
    const T d1 = (ms1 - m1) * T(1.0 / 36.0), d2 = (ms2 - m2) * T(1.0 / 36.0);
    const T d3 = (ms3 - jx) * T(1.0 / 6.0), d4 = (ms4 - m4) * T(1.0 / 12.0);
    const T d5 = (ms5 - jy) * T(1.0 / 6.0), d6 = (ms6 - m6) * T(1.0 / 12.0);
    const T d7 = (ms7 - m7) * T(0.25), d8 = (ms8 - m8) * T(0.25);
    const T e14 = -d1 - T(2) * d2, e58 = T(2) * d1 + d2;
    const T u1 = d3 - T(2) * d4, v1 = d5 - T(2) * d6;
    const T u5 = d3 + d4, v5 = d5 + d6;
    df[0] = sr_add<S>(df[0], T(4) * (d2 - d1), us);
    df[1] = sr_add<S>(df[1], (e14 + u1) + d7, us);
    df[2] = sr_add<S>(df[2], (e14 + v1) - d7, us);
    df[3] = sr_add<S>(df[3], (e14 - u1) + d7, us);
    df[4] = sr_add<S>(df[4], (e14 - v1) - d7, us);
    df[5] = sr_add<S>(df[5], (e58 + u5) + (v5 + d8), us);
    df[6] = sr_add<S>(df[6], (e58 - u5) + (v5 - d8), us);
    df[7] = sr_add<S>(df[7], (e58 - u5) - (v5 - d8), us);
    df[8] = sr_add<S>(df[8], (e58 + u5) - (v5 + d8), us);
  } else {
    df[0] = (a0 - T(4) * a1) + T(4) * a2;
    df[1] = (b14 + x1) + a7;
    df[2] = (b14 + y1) - a7;
    df[3] = (b14 - x1) + a7;
    df[4] = (b14 - y1) - a7;
    df[5] = (b58 + x5) + (y5 + a8);
    df[6] = (b58 - x5) + (y5 - a8);
    df[7] = (b58 - x5) - (y5 - a8);
    df[8] = (b58 + x5) - (y5 + a8);
  }
  // Step 9: D2Q5 MRT thermal collision (flux moments relax to u T)
  const T Tabs = p.T_ref + dT;
  const T n1 = dg[1] - dg[3], n2 = dg[2] - dg[4];
  const T n3 = T(-4) * dg[0] + ((dg[1] + dg[2]) + (dg[3] + dg[4]));
  const T n4 = (dg[1] - dg[2]) + (dg[3] - dg[4]);
  const T ns1 = n1 - p.s_g * (n1 - ux * Tabs);
  const T ns2 = n2 - p.s_g * (n2 - uy * Tabs);
  const T ns3 = n3 - p.sT_e * (n3 + T(2.0 / 3.0) * dT);
  const T ns4 = n4 - p.sT_nu * n4;
  if constexpr (SR) {
    const T e1 = (ns1 - n1) * T(0.5), e2 = (ns2 - n2) * T(0.5);
    const T e3 = (ns3 - n3) * T(0.05), e4 = (ns4 - n4) * T(0.25);  // T is conserved
    dg[0] = sr_add<S>(dg[0], T(-4) * e3, us);
    dg[1] = sr_add<S>(dg[1], (e3 + e1) + e4, us);
    dg[2] = sr_add<S>(dg[2], (e3 + e2) - e4, us);
    dg[3] = sr_add<S>(dg[3], (e3 - e1) + e4, us);
    dg[4] = sr_add<S>(dg[4], (e3 - e2) - e4, us);
  } else {
    const T c0 = dT * T(0.2), c1 = ns1 * T(0.5), c2 = ns2 * T(0.5);
    const T c3 = ns3 * T(0.05), c4 = ns4 * T(0.25);
    const T c03 = c0 + c3;
    dg[0] = c0 - T(4) * c3;
    dg[1] = (c03 + c1) + c4;
    dg[2] = (c03 + c2) - c4;
    dg[3] = (c03 - c1) + c4;
    dg[4] = (c03 - c2) - c4;
  }
}

// One row tile [i0, i0 + TILE) of row j: gather from the state p, collide,
// scatter into the state d (d == p: the in-place AA update; d != p: the same
// update written to another buffer, which then holds the complete next
// state because every slot is written exactly once per step).
template <typename T, bool ODD, bool POW, bool LOGDA, bool SR = false, typename S>
__device__ __forceinline__ void step_tile(const KParams<T, S>& p, const KParams<T, S>& d, int i0, int j, int lx) {
  const int i = i0 + lx;
  T df[9], dg[5];
  constexpr bool HSR = SR && std::is_same<S, _Float16>::value;  // stochastic conversion at the stores
  unsigned rw = 0;
  if (ODD) {
    // Waves whose 64 nodes all have their 8 neighbours inside the grid take
    // the branch-free interior path (wave-uniform test; a wave covers 64
    // consecutive columns of row j starting at a multiple of 64 in lx).
    const int w0 = i0 + (__builtin_amdgcn_readfirstlane(lx) & ~63);
    const bool interior = w0 >= 1 && w0 + 63 <= p.nx - 2 && j >= 1 && j <= p.ny - 2;
    if (interior) {
      load_interior_odd<T>(p, row_base(p, j), i, df, dg);
      collide<T, POW, LOGDA, SR>(p, j * p.nx + i, df, dg, &rw);
      store_interior_odd<T, HSR>(d, row_base(d, j), i, df, dg, rw);
      return;
    }
  }
  if (i >= p.nx) return;
  load_node<T, ODD>(p, i, j, df, dg);
  collide<T, POW, LOGDA, SR>(p, j * p.nx + i, df, dg, &rw);
  store_node<T, ODD, HSR>(d, i, j, df, dg, rw);
}

}  // namespace dev
}  // namespace pm
