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
// Each grid row stores its 9 + 5 population rows one after the other (x
// fastest, rows padded to 64 elements), so a node update touches one
// contiguous block per grid row; one workgroup covers a row segment of 64,
// 128 or 256 nodes (chosen by the host from the grid size and dtype), one
// lane per node, so every load and store of a wave is a contiguous 256 B
// (FP32) run; workgroups run in row-major tile order.  The
// streaming hint is used on every access that is not shifted along x (those
// lines are touched exactly once per step); the x-shifted accesses of the odd
// step straddle lines that the neighbouring wave also touches, so they keep
// the default caching.
#include "pm_device.h"

#include <algorithm>
#include <type_traits>

namespace pm {
namespace {

using namespace pm::dev;

// One workgroup per row segment of blockDim.x nodes (64, 128 or 256).
template <typename T, bool ODD, bool POW, bool LOGDA, bool SR, typename S>
__global__ __launch_bounds__(TILE) void k_step(KParams<T, S> p, int tiles_x, int ntiles) {
  const int tile = tile_of_block(blockIdx.x, ntiles);
  const int j = tile / tiles_x;
  step_tile<T, ODD, POW, LOGDA, SR>(p, p, (tile - j * tiles_x) * (int)blockDim.x, j, threadIdx.x);
}

// The same step, read from state src and written to state dst (another
// buffer of the same layout).
template <typename T, bool ODD, bool POW, bool LOGDA, bool SR>
__global__ __launch_bounds__(TILE) void k_step_oop(KParams<T> src, KParams<T> dst, int tiles_x) {
  const int j = blockIdx.x / tiles_x;
  step_tile<T, ODD, POW, LOGDA, SR>(src, dst, (blockIdx.x - j * tiles_x) * (int)blockDim.x, j, threadIdx.x);
}

// ---- two time steps in one pass (FP32, cavity walls) ----
// Reads the state S_k in its natural layout (k even) from src and writes
// S_{k+2}, also natural, to dst (another buffer: neighbouring workgroups read
// the halo of src that this one's outputs cover).  Each workgroup owns a strip
// of PAIR_W output columns and PAIR_R output rows and marches up its rows:
//   A. row a: gather S_k, collide (step k) -> post-collision f*;
//   B. row a - 1: pull f* from rows a - 2 .. a (walls: bounce-back, thermal
//      anti-bounce-back), collide (step k + 1) -> f**;
//   C. row a - 2: pull f** from rows a - 3 .. a - 1 -> S_{k+2}, store.
// The number of rows per workgroup is chosen by the host (around 24: fewer
// rows recompute more halo rows, more rows give fewer, longer workgroups).
// Thread t works on column x0 - 2 + t, so step k covers two halo columns on
// each side and step k + 1 one.  The populations that move along x go
// through LDS rings of the last three rows; those that do not stay in the
// thread's registers.  The per-node arithmetic is the single-step kernels'
// (collide), so two passes of this kernel equal four single steps bit for
// bit.  (Rings of two rows, with the row below carried in registers, allow
// five workgroups per CU instead of three but measured 3% slower.)
// populations that move along x, in LDS order: f1 f3 f5 f6 f7 f8 g1 g3
constexpr int NXS = 8;

struct Still {  // the populations with e_x = 0 of one node: f0 f2 f4 g0 g2 g4
  float f0, f2, f4, g0, g2, g4;
};

__device__ __forceinline__ void put_row(float (*ring)[NXS][TILE], int slot, int t, const float df[9],
                                        const float dg[5], Still& st) {
  ring[slot][0][t] = df[1];
  ring[slot][1][t] = df[3];
  ring[slot][2][t] = df[5];
  ring[slot][3][t] = df[6];
  ring[slot][4][t] = df[7];
  ring[slot][5][t] = df[8];
  ring[slot][6][t] = dg[1];
  ring[slot][7][t] = dg[3];
  st = Still{df[0], df[2], df[4], dg[0], dg[2], dg[4]};
}

// Pre-collision populations of node (c, b) one step after the post-collision
// rows held in ring (slots sm, s0, sp = rows b - 1, b, b + 1) and in the
// registers lo, mid, hi (same rows, this column).
__device__ __forceinline__ void pull_pair(const KParams<float>& p, float (*ring)[NXS][TILE], int sm, int s0,
                                          int sp, int t, int c, int b, const Still& lo, const Still& mid,
                                          const Still& hi, float df[9], float dg[5]) {
  const bool xl = c - 1 >= 0, xr = c + 1 < p.nx, yb = b - 1 >= 0, yt = b + 1 < p.ny;
  df[0] = mid.f0;
  df[1] = xl ? ring[s0][0][t - 1] : ring[s0][1][t];          // from (c-1, b) or own f*3
  df[2] = yb ? lo.f2 : mid.f4;                                // from (c, b-1) or own f*4
  df[3] = xr ? ring[s0][1][t + 1] : ring[s0][0][t];          // from (c+1, b) or own f*1
  df[4] = yt ? hi.f4 : mid.f2;                                // from (c, b+1) or own f*2
  df[5] = (xl && yb) ? ring[sm][2][t - 1] : ring[s0][4][t];  // from (c-1, b-1) or own f*7
  df[6] = (xr && yb) ? ring[sm][3][t + 1] : ring[s0][5][t];  // from (c+1, b-1) or own f*8
  df[7] = (xr && yt) ? ring[sp][4][t + 1] : ring[s0][2][t];  // from (c+1, b+1) or own f*5
  df[8] = (xl && yt) ? ring[sp][5][t - 1] : ring[s0][3][t];  // from (c-1, b+1) or own f*6
  dg[0] = mid.g0;
  dg[1] = xl ? ring[s0][6][t - 1] : p.hotc - ring[s0][7][t];   // hot wall: anti-bounce-back
  dg[2] = yb ? lo.g2 : mid.g4;
  dg[3] = xr ? ring[s0][7][t + 1] : p.coldc - ring[s0][6][t];  // cold wall: anti-bounce-back
  dg[4] = yt ? hi.g4 : mid.g2;
}

template <bool POW, bool LOGDA, bool SR>
__global__ __launch_bounds__(TILE) void k_step2(KParams<float> src, KParams<float> dst, int rows) {
  __shared__ float ring1[3][NXS][TILE];  // f* of rows a - 2 .. a
  __shared__ float ring2[3][NXS][TILE];  // f** of rows a - 3 .. a - 1
  const int t = threadIdx.x;
  // Tile of this workgroup.  The dispatcher deals consecutive workgroups to
  // the 8 XCDs in turn; tiles (row group major, strip minor) are dealt to
  // them in blocks of XCD_BLOCK adjacent strips instead, so that a strip's
  // halo columns, which its neighbours also read, are mostly fetched into
  // the same XCD's L2, while all XCDs still advance through the same rows.
  // The last G mod (8 XCD_BLOCK) workgroups keep their own tile (the map is
  // a bijection on the tiles).
  constexpr int XCD_BLOCK = 8;
  const int G = gridDim.x * gridDim.y;
  const int L = blockIdx.y * gridDim.x + blockIdx.x;
  const int Gf = G / (8 * XCD_BLOCK) * (8 * XCD_BLOCK);
  int tl = L;
  if (L < Gf) {
    const int xcd = L & 7, q = L >> 3;
    tl = ((q / XCD_BLOCK) * 8 + xcd) * XCD_BLOCK + q % XCD_BLOCK;
  }
  const int sy = tl / (int)gridDim.x, sx = tl - sy * (int)gridDim.x;
  const int x0 = sx * PAIR_W, y0 = sy * rows;
  const int c = x0 - 2 + t;
  const bool col = c >= 0 && c < src.nx;
  const int y_end = min(y0 + rows, src.ny);  // output rows [y0, y_end)
  Still r1m{}, r10{}, r1p{};  // f* of rows a - 2, a - 1, a (this column)
  Still r2m{}, r20{}, r2p{};  // f** of rows a - 3, a - 2, a - 1
  int s1 = 0;                 // slot of row a; rows a - 1, a - 2 in s1 - 1, s1 - 2 (mod 3)
  // S_k of the row A gathers next, loaded one row ahead: the loads of row
  // a + 1 are issued once row a has been collided, and are in flight while
  // rows a - 1 and a - 2 are finished (src is only read by this kernel).
  float nf[9] = {}, ng[5] = {};
  if (col && y0 - 2 >= 0) load_node<float, false>(src, c, y0 - 2, nf, ng);
  for (int a = y0 - 2; a <= y_end + 1; ++a, s1 = s1 == 2 ? 0 : s1 + 1) {
    const int s1m = s1 == 0 ? 2 : s1 - 1, s1mm = s1m == 0 ? 2 : s1m - 1;
    // A: step k at row a
    {
      Still st{};
      if (col && a >= 0 && a < src.ny) {
        collide<float, POW, LOGDA, SR>(src, a * src.nx + c, nf, ng);
        put_row(ring1, s1, t, nf, ng, st);
      }
      if (col && a + 1 >= 0 && a + 1 < src.ny && a + 1 <= y_end + 1)
        load_node<float, false>(src, c, a + 1, nf, ng);
      r1m = r10;
      r10 = r1p;
      r1p = st;
    }
    __syncthreads();
    // B: step k + 1 at row b = a - 1 (ring1 slots s1mm, s1m, s1 = rows b - 1, b, b + 1)
    const int b = a - 1;
    {
      Still st{};
      if (b >= y0 - 1 && b >= 0 && b < src.ny && col && t >= 1 && t <= TILE - 2) {
        float df[9], dg[5];
        pull_pair(src, ring1, s1mm, s1m, s1, t, c, b, r1m, r10, r1p, df, dg);
        collide<float, POW, LOGDA, SR>(src, b * src.nx + c, df, dg);
        put_row(ring2, s1m, t, df, dg, st);  // ring2 keeps row r in the slot ring1 gives row r
      }
      r2m = r20;
      r20 = r2p;
      r2p = st;
    }
    __syncthreads();
    // C: S_{k+2} at row o = a - 2 (rows o - 1, o, o + 1 = a - 3, a - 2, a - 1 in slots s1, s1mm, s1m)
    const int o = a - 2;
    if (o >= y0 && o < y_end && t >= 2 && t <= TILE - 3 && c < src.nx) {
      float df[9], dg[5];
      pull_pair(src, ring2, s1, s1mm, s1m, t, c, o, r2m, r20, r2p, df, dg);
      const int64_t off = pop_off(dst, c, o);
#pragma unroll
      for (int q = 0; q < 9; ++q) stg<float, true>(dst.f + q * dst.qs + off, df[q]);
#pragma unroll
      for (int q = 0; q < 5; ++q) stg<float, true>(dst.g + q * dst.qs + off, dg[q]);
    }
  }
}

// ---- batched parameter sweep: one launch steps every live case ----
// Workgroup b takes the (case, tile) pair of entry b of the schedule; cases
// that have met their stopping test are skipped.  A tile is tw columns by th
// rows (tw a multiple of 64, tw * th threads): thread t works on column
// t % tw, row t / tw of the tile, so every wave lies within one grid row.
// Each case runs the same per-node body as the single-case kernel, so a case
// advanced here is bitwise identical to the same case advanced alone,
// whatever the tile shape.  SR_ANY: some case rounds stochastically (FP32
// only); without it the kernel carries no stochastic-rounding branch, which
// would cost round-to-nearest sweeps registers and occupancy.
template <typename T, bool ODD, bool SR_ANY>
__global__ __launch_bounds__(TILE) void k_step_multi(const SweepCase<T>* __restrict__ cases,
                                                     const int2* __restrict__ sched,
                                                     const int* __restrict__ live, int tw, int th) {
  const int2 e = sched[blockIdx.x];  // (case, tile within the case)
  if (!live[e.x]) return;
  const SweepCase<T>& c = cases[e.x];
  const int ty = e.y / c.tiles_x;
  const int lx = (int)threadIdx.x % tw, j = ty * th + (int)threadIdx.x / tw;
  if (j >= c.p.ny) return;  // whole waves
  const int i0 = (e.y - ty * c.tiles_x) * tw;
  if constexpr (SR_ANY && std::is_same<T, float>::value) {
    if (c.p.sr) {
      if (c.pow) step_tile<T, ODD, true, false, true>(c.p, c.p, i0, j, lx);
      else step_tile<T, ODD, false, false, true>(c.p, c.p, i0, j, lx);
      return;
    }
  }
  if (c.pow) step_tile<T, ODD, true, false>(c.p, c.p, i0, j, lx);
  else step_tile<T, ODD, false, false>(c.p, c.p, i0, j, lx);
}

// Rest state: df = 0, dg_q = w_q (T_init - T_ref).  (The padding of the
// population region is cleared by the launcher.)
template <typename T, typename S>
__global__ void k_init(KParams<T, S> p, T dg_init) {
  const int64_t n = (int64_t)p.nx * p.ny;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(k / p.nx), i = (int)(k - (int64_t)j * p.nx);
    const int64_t o = pop_off(p, i, j);
#pragma unroll
    for (int q = 0; q < 9; ++q) p.f[q * p.qs + o] = S(0);
    p.g[o] = (S)(dg_init * T(2));  // w_0 = 1/3 = 2 w_1
#pragma unroll
    for (int q = 1; q < 5; ++q) p.g[q * p.qs + o] = (S)dg_init;
  }
}

// Eq. (24): one workgroup, fixed summation order (deterministic).
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_nu(KParams<T, S> p, int parity, double* out) {
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
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_resid(KParams<T, S> p, int parity, T* snap,
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

// Sweep residual: one workgroup per schedule entry (a tile of a live case,
// laid out as in k_step_multi) -> max |theta - snapshot| over the tile into
// the tile's slot of the case-major partial array, snapshot := theta.
template <typename T>
__global__ __launch_bounds__(TILE) void k_resid_multi(const SweepCase<T>* __restrict__ cases,
                                                      const int2* __restrict__ sched,
                                                      const int* __restrict__ live, int parity,
                                                      double* __restrict__ partial, int tw, int th) {
  __shared__ double red[TILE];
  const int2 e = sched[blockIdx.x];
  if (!live[e.x]) return;  // uniform over the workgroup
  const SweepCase<T>& c = cases[e.x];
  const int ty = e.y / c.tiles_x;
  const int j = ty * th + (int)threadIdx.x / tw;
  const int i = (e.y - ty * c.tiles_x) * tw + (int)threadIdx.x % tw;
  double mx = 0.0;
  if (i < c.p.nx && j < c.p.ny) {
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
  for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {  // blockDim.x = tw * th, a power of two
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

template <typename T, bool ODD, bool POW, bool LOGDA, typename O, typename S>
__global__ __launch_bounds__(TILE) void k_fields(KParams<T, S> p, O* U, O* V, O* th, O* nuo) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= p.nx) return;
  for (int j = blockIdx.y; j < p.ny; j += gridDim.y) {
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

template <typename T, bool ODD, typename O, typename S>
__global__ __launch_bounds__(TILE) void k_get_pop(KParams<T, S> p, O* f, O* g) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= p.nx) return;
  const int64_t n = (int64_t)p.nx * p.ny;
  for (int j = blockIdx.y; j < p.ny; j += gridDim.y) {
    T df[9], dg[5];
    load_node<T, ODD>(p, i, j, df, dg);
    const int64_t k = (int64_t)j * p.nx + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q * n + k] = (O)((double)df[q] + (double)w9<T>(q));
#pragma unroll
    for (int q = 0; q < 5; ++q) g[q * n + k] = (O)((double)dg[q] + (double)w5<T>(q) * (double)p.T_ref);
  }
}

template <typename T, typename I, typename S>
__global__ __launch_bounds__(TILE) void k_set_pop(KParams<T, S> p, const I* f, const I* g) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= p.nx) return;
  const int64_t n = (int64_t)p.nx * p.ny;
  for (int j = blockIdx.y; j < p.ny; j += gridDim.y) {
    const int64_t k = (int64_t)j * p.nx + i, o = pop_off(p, i, j);
#pragma unroll
    for (int q = 0; q < 9; ++q) p.f[q * p.qs + o] = (S)((double)f[q * n + k] - (double)w9<T>(q));
#pragma unroll
    for (int q = 0; q < 5; ++q)
      p.g[q * p.qs + o] = (S)((double)g[q * n + k] - (double)w5<T>(q) * (double)p.T_ref);
  }
}

template <typename T, typename I>
__global__ void k_convert(T* dst, const I* src, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = (T)src[k];
}

__global__ void k_header(int64_t* dst, int64_t steps, uint64_t tag, uint64_t phys) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = (int64_t)tag;
    dst[1] = steps;
    dst[2] = (int64_t)phys;
  }
}

// Stream function from the U field, in place: on entry psi holds U at the
// nodes, on exit psi(j) = (sum_{j' < j} U(j') + U(j) / 2) / L up each column
// (the integral of U dy from the bottom wall to the node by the midpoint
// rule), as a blocked scan with FP64 sums: (1) every thread sums one
// column over one block of R rows; (2) one thread per column turns the
// block sums into exclusive block offsets; (3) every (column, block) thread
// walks its rows from its block's offset.  A wave reads 64 adjacent columns
// of a row at a time, so every access is contiguous.
// Rows per block: 64, doubled until the block count fits a launch's y extent.
inline int psi_rows(int ny) {
  int r = 64;
  while ((ny + r - 1) / r > GRID_Y_MAX) r *= 2;
  return r;
}

template <typename O>
__global__ __launch_bounds__(256) void k_psi_blocks(const O* __restrict__ u, double* __restrict__ blk, int nx,
                                                    int ny, int R) {
  const int i = blockIdx.x * 256 + threadIdx.x, b = blockIdx.y;
  if (i >= nx) return;
  const int j1 = (int)min((int64_t)ny, (int64_t)(b + 1) * R);
  double s = 0.0;
#pragma unroll 8
  for (int j = b * R; j < j1; ++j) s += (double)u[(int64_t)j * nx + i];
  blk[(int64_t)b * nx + i] = s;
}

// Exclusive prefix over the block sums of each column, in order.  The sums
// are loaded 16 at a time before any is overwritten, so the loads of a
// group are in flight together.
__global__ __launch_bounds__(256) void k_psi_offsets(double* __restrict__ blk, int nx, int nblk) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nx) return;
  constexpr int G = 16;
  double acc = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += G) {
    double s[G];
#pragma unroll
    for (int t = 0; t < G; ++t) s[t] = b0 + t < nblk ? blk[(int64_t)(b0 + t) * nx + i] : 0.0;
#pragma unroll
    for (int t = 0; t < G; ++t) {
      if (b0 + t < nblk) blk[(int64_t)(b0 + t) * nx + i] = acc;
      acc += s[t];
    }
  }
}

template <typename O>
__global__ __launch_bounds__(256) void k_psi_apply(O* __restrict__ psi, const double* __restrict__ blk, int nx,
                                                   int ny, int R, double inv_L) {
  const int i = blockIdx.x * 256 + threadIdx.x, b = blockIdx.y;
  if (i >= nx) return;
  const int j1 = (int)min((int64_t)ny, (int64_t)(b + 1) * R);
  double acc = blk[(int64_t)b * nx + i];
#pragma unroll 8
  for (int j = b * R; j < j1; ++j) {
    const int64_t k = (int64_t)j * nx + i;
    const double u = (double)psi[k];
    psi[k] = (O)((acc + 0.5 * u) * inv_L);
    acc += u;
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

template <typename T, typename S>
hipError_t launch_step(const KParams<T, S>& p, const Launch& L, int parity, bool pow, bool logda) {
  if (!(L.step_w == 64 || L.step_w == 128 || L.step_w == 256) || L.step_w > TILE) return hipErrorInvalidValue;
  dim3 grid(L.step_ntiles), block(L.step_w);
#define PM_STEP(ODD, POW, LOG, SR) \
  hipLaunchKernelGGL((k_step<T, ODD, POW, LOG, SR, S>), grid, block, 0, L.stream, p, L.step_tiles_x, L.step_ntiles)
#define PM_STEP_ALL(SR)                                                                             \
  if (parity) {                                                                                     \
    if (pow) { if (logda) PM_STEP(true, true, true, SR); else PM_STEP(true, true, false, SR); }       \
    else { if (logda) PM_STEP(true, false, true, SR); else PM_STEP(true, false, false, SR); }        \
  } else {                                                                                          \
    if (pow) { if (logda) PM_STEP(false, true, true, SR); else PM_STEP(false, true, false, SR); }    \
    else { if (logda) PM_STEP(false, false, true, SR); else PM_STEP(false, false, false, SR); }     \
  }
  bool done = false;
  if constexpr (std::is_same<T, float>::value) {
    if (p.sr) {
      PM_STEP_ALL(true)
      done = true;
    }
  }
  if (!done) { PM_STEP_ALL(false) }
#undef PM_STEP_ALL
#undef PM_STEP
  return hipGetLastError();
}

hipError_t launch_step2(const KParams<float>& src, const KParams<float>& dst, hipStream_t s, bool pow,
                        bool logda, int rows) {
  if (rows < 1 || (src.ny + rows - 1) / rows > GRID_Y_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((src.nx + PAIR_W - 1) / PAIR_W), (unsigned)((src.ny + rows - 1) / rows));
#define PM_PAIR(POW, LOG, SR) hipLaunchKernelGGL((k_step2<POW, LOG, SR>), grid, dim3(TILE), 0, s, src, dst, rows)
  if (src.sr) {
    if (pow) { if (logda) PM_PAIR(true, true, true); else PM_PAIR(true, false, true); }
    else { if (logda) PM_PAIR(false, true, true); else PM_PAIR(false, false, true); }
  } else {
    if (pow) { if (logda) PM_PAIR(true, true, false); else PM_PAIR(true, false, false); }
    else { if (logda) PM_PAIR(false, true, false); else PM_PAIR(false, false, false); }
  }
#undef PM_PAIR
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_oop(const KParams<T>& src, const KParams<T>& dst, const Launch& L, int parity,
                           bool pow, bool logda) {
  if (!(L.step_w == 64 || L.step_w == 128 || L.step_w == 256) || L.step_w > TILE) return hipErrorInvalidValue;
  dim3 grid(L.step_ntiles), block(L.step_w);
#define PM_OOP(ODD, POW, LOG, SR) \
  hipLaunchKernelGGL((k_step_oop<T, ODD, POW, LOG, SR>), grid, block, 0, L.stream, src, dst, L.step_tiles_x)
#define PM_OOP_ALL(SR)                                                                              \
  if (parity) {                                                                                     \
    if (pow) { if (logda) PM_OOP(true, true, true, SR); else PM_OOP(true, true, false, SR); }         \
    else { if (logda) PM_OOP(true, false, true, SR); else PM_OOP(true, false, false, SR); }          \
  } else {                                                                                          \
    if (pow) { if (logda) PM_OOP(false, true, true, SR); else PM_OOP(false, true, false, SR); }      \
    else { if (logda) PM_OOP(false, false, true, SR); else PM_OOP(false, false, false, SR); }       \
  }
  bool done = false;
  if constexpr (std::is_same<T, float>::value) {
    if (src.sr) {
      PM_OOP_ALL(true)
      done = true;
    }
  }
  if (!done) { PM_OOP_ALL(false) }
#undef PM_OOP_ALL
#undef PM_OOP
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_multi(const SweepCase<T>* cases, const int2* sched, const int* live,
                             int nsched, int parity, int tw, int th, bool any_sr, hipStream_t s) {
  if (!sweep_tile_ok(tw, th)) return hipErrorInvalidValue;
  if (nsched <= 0) return hipSuccess;  // no live case scheduled
#define PM_MULTI(ODD, SR) \
  hipLaunchKernelGGL((k_step_multi<T, ODD, SR>), dim3(nsched), dim3(tw * th), 0, s, cases, sched, live, tw, th)
  bool sr = false;
  if constexpr (std::is_same<T, float>::value) {
    sr = any_sr;
    if (sr) {
      if (parity) PM_MULTI(true, true); else PM_MULTI(false, true);
    }
  }
  if (!sr) {
    if (parity) PM_MULTI(true, false); else PM_MULTI(false, false);
  }
#undef PM_MULTI
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_multi(const SweepCase<T>* cases, int ncases, const int2* sched, int* live,
                              int nsched, int parity, int tw, int th, double* partial, SweepStatus* st,
                              int64_t chunk, double tol, int64_t max_steps, hipStream_t s) {
  if (!sweep_tile_ok(tw, th)) return hipErrorInvalidValue;
  if (nsched <= 0) return hipSuccess;  // no live case scheduled
  hipLaunchKernelGGL((k_resid_multi<T>), dim3(nsched), dim3(tw * th), 0, s, cases, sched,
                     (const int*)live, parity, partial, tw, th);
  hipLaunchKernelGGL((k_retire<T>), dim3(1), dim3(64), 0, s, cases, ncases, (const double*)partial,
                     live, st, chunk, tol, max_steps);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_init(const KParams<T, S>& p, const Launch& L, T dg_init, size_t pop_bytes) {
  // whole population region first (row padding included), then the nodes
  hipError_t e = hipMemsetAsync(p.f, 0, pop_bytes, L.stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_init<T, S>), dim3(grid_for((int64_t)p.nx * p.ny)), dim3(256), 0, L.stream,
                     p, dg_init);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_nu(const KParams<T, S>& p, const Launch& L, int parity, double* out) {
  hipLaunchKernelGGL((k_nu<T, S>), dim3(1), dim3(256), 0, L.stream, p, parity, out);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_residual(const KParams<T, S>& p, const Launch& L, int parity, T* snap,
                           double* partial, double* out, int snapshot_only) {
  const int nb = grid_for((int64_t)p.nx * p.ny, 256, RED_BLOCKS);
  hipLaunchKernelGGL((k_resid<T, S>), dim3(nb), dim3(256), 0, L.stream, p, parity, snap, partial,
                     snapshot_only);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, L.stream, (const double*)partial, nb, out);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_fields(const KParams<T, S>& p, const Launch& L, int parity, bool pow, bool logda,
                         void* U, void* V, void* th, void* nu, int out_fp64) {
  dim3 grid(L.tiles_x, std::min(p.ny, GRID_Y_MAX)), block(TILE);
#define PM_F(ODD, POW, LOG, O)                                                              \
  hipLaunchKernelGGL((k_fields<T, ODD, POW, LOG, O, S>), grid, block, 0, L.stream, p, (O*)U, \
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

template <typename T, typename S>
hipError_t launch_get_pop(const KParams<T, S>& p, const Launch& L, int parity, void* f, void* g,
                          int out_fp64) {
  dim3 grid(L.tiles_x, std::min(p.ny, GRID_Y_MAX)), block(TILE);
  if (parity) {
    if (out_fp64) hipLaunchKernelGGL((k_get_pop<T, true, double, S>), grid, block, 0, L.stream, p, (double*)f, (double*)g);
    else hipLaunchKernelGGL((k_get_pop<T, true, float, S>), grid, block, 0, L.stream, p, (float*)f, (float*)g);
  } else {
    if (out_fp64) hipLaunchKernelGGL((k_get_pop<T, false, double, S>), grid, block, 0, L.stream, p, (double*)f, (double*)g);
    else hipLaunchKernelGGL((k_get_pop<T, false, float, S>), grid, block, 0, L.stream, p, (float*)f, (float*)g);
  }
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_set_pop(const KParams<T, S>& p, const Launch& L, const void* f, const void* g,
                          int in_fp64) {
  dim3 grid(L.tiles_x, std::min(p.ny, GRID_Y_MAX)), block(TILE);
  if (in_fp64)
    hipLaunchKernelGGL((k_set_pop<T, double, S>), grid, block, 0, L.stream, p, (const double*)f, (const double*)g);
  else
    hipLaunchKernelGGL((k_set_pop<T, float, S>), grid, block, 0, L.stream, p, (const float*)f, (const float*)g);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_set_logda(const KParams<T, S>& p, const Launch& L, T* dst, const void* src,
                            int in_fp64) {
  const int64_t n = (int64_t)p.nx * p.ny;
  if (in_fp64)
    hipLaunchKernelGGL((k_convert<T, double>), dim3(grid_for(n)), dim3(256), 0, L.stream, dst, (const double*)src, n);
  else
    hipLaunchKernelGGL((k_convert<T, float>), dim3(grid_for(n)), dim3(256), 0, L.stream, dst, (const float*)src, n);
  return hipGetLastError();
}

hipError_t launch_write_header(void* dst, int64_t steps, uint64_t tag, uint64_t phys, hipStream_t s) {
  hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, (int64_t*)dst, steps, tag, phys);
  return hipGetLastError();
}

size_t stream_scratch_bytes(int nx, int ny) {
  const int R = psi_rows(ny);
  return (size_t)nx * (size_t)((ny + R - 1) / R) * sizeof(double);
}

hipError_t launch_stream_y(void* psi, int nx, int ny, double inv_L, int out_fp64, double* scratch,
                           hipStream_t s) {
  const int R = psi_rows(ny), nblk = (ny + R - 1) / R;
  const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)nblk);
  if (out_fp64)
    hipLaunchKernelGGL((k_psi_blocks<double>), grid, dim3(256), 0, s, (const double*)psi, scratch, nx, ny, R);
  else
    hipLaunchKernelGGL((k_psi_blocks<float>), grid, dim3(256), 0, s, (const float*)psi, scratch, nx, ny, R);
  hipLaunchKernelGGL(k_psi_offsets, dim3(grid.x), dim3(256), 0, s, scratch, nx, nblk);
  if (out_fp64)
    hipLaunchKernelGGL((k_psi_apply<double>), grid, dim3(256), 0, s, (double*)psi, (const double*)scratch, nx,
                       ny, R, inv_L);
  else
    hipLaunchKernelGGL((k_psi_apply<float>), grid, dim3(256), 0, s, (float*)psi, (const double*)scratch, nx, ny,
                       R, inv_L);
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

#define PM_INST_S(T, S)                                                                          \
  template hipError_t launch_step<T, S>(const KParams<T, S>&, const Launch&, int, bool, bool);    \
  template hipError_t launch_init<T, S>(const KParams<T, S>&, const Launch&, T, size_t);          \
  template hipError_t launch_nu<T, S>(const KParams<T, S>&, const Launch&, int, double*);         \
  template hipError_t launch_residual<T, S>(const KParams<T, S>&, const Launch&, int, T*, double*, \
                                            double*, int);                                         \
  template hipError_t launch_fields<T, S>(const KParams<T, S>&, const Launch&, int, bool, bool,   \
                                          void*, void*, void*, void*, int);                        \
  template hipError_t launch_get_pop<T, S>(const KParams<T, S>&, const Launch&, int, void*, void*, \
                                           int);                                                   \
  template hipError_t launch_set_pop<T, S>(const KParams<T, S>&, const Launch&, const void*,      \
                                           const void*, int);                                      \
  template hipError_t launch_set_logda<T, S>(const KParams<T, S>&, const Launch&, T*, const void*, int);
#define PM_INST(T)                                                                              \
  PM_INST_S(T, T)                                                                               \
  template hipError_t launch_step_oop<T>(const KParams<T>&, const KParams<T>&, const Launch&, int, \
                                         bool, bool);                                           \
  template hipError_t launch_step_multi<T>(const SweepCase<T>*, const int2*, const int*, int, int, \
                                           int, int, bool, hipStream_t);                          \
  template hipError_t launch_resid_multi<T>(const SweepCase<T>*, int, const int2*, int*, int, int, \
                                            int, int, double*, SweepStatus*, int64_t, double,     \
                                            int64_t, hipStream_t);
PM_INST(float)
PM_INST(double)
PM_INST_S(float, _Float16)
#undef PM_INST
#undef PM_INST_S

}  // namespace pm
