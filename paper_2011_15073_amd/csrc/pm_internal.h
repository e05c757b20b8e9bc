// pm_internal.h -- device-side parameter block and kernel launchers of the
// gfx950 lattice Boltzmann library (internal; the public ABI is pmlbm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pm {

// Everything one node update needs, already converted to the compute type T;
// the populations are stored as S (T itself, or _Float16 with FP32 compute).
// Populations are stored shifted: df_q = f_q - w_q and dg_q = g_q - w_q T_ref
// (T_ref = 1/2), which keeps the storage precision on the small deviations
// from the rest state.  Population q of node (i, j) is f[q * qs + j * rs + i]
// (g likewise).  The library lays the 14 populations of a row out one after
// the other (row-interleaved: qs = padded nx, rs = 14 qs, g = f + 9 qs); the
// per-cell planes (log10 Da, the residual snapshot, both of type T) and every
// caller-facing field use the natural index k = j * nx + i.
template <typename T, typename S = T>
struct KParams {
  using compute_t = T;
  using storage_t = S;
  S* f;            // 9 populations
  S* g;            // 5 populations
  const T* logda;  // per-cell log10(Da) plane [ny][nx] or nullptr
  int64_t qs;      // population stride in elements
  int64_t rs;      // row stride in elements
  int nx, ny;
  int px, py;      // periodic axes
  // viscosity (power law, Eq. 21)
  T nu_newt;       // clamped nu0, the Newtonian value
  T nu_min, nu_max;
  T y_lo, y_hi;    // log2 of nu_min, nu_max
  T lc0;           // log2 nu0 + (n - 1) log2 gamma_scale
  T nm1, inv_n;    // n - 1, 1 / n
  T tol;           // Newton tolerance on log2(nu)
  int max_it;
  int sr;          // 1: round the population updates stochastically (FP32 or FP16 storage)
  // porous medium
  T eps, inv_eps, invK, invsK, Feps, inv_Kscale;
  // body forces: G = (gx, gy + gbeta (T - T_m))
  T gbeta, dTm;    // dTm = T_m - T_ref
  T gx, gy;
  // relaxation rates
  T s_e, s_eps, s_q, s_g, sT_e, sT_nu;
  // thermal walls in shifted form: 2 w_1 (T_wall - T_ref)
  T hotc, coldc;
  T T_ref;
  T inv_U;         // 1 / U_lb
};

// One case of a batched sweep, as the device sees it.
template <typename T>
struct SweepCase {
  KParams<T> p;
  T* snap;       // residual snapshot of theta (shifted)
  int tiles_x;   // tiles across a row of the grid: ceil(nx / tile width)
  int ntiles;    // tiles of this case: tiles_x * ceil(ny / tile height)
  int tile_base; // first slot of this case in the case-major per-tile arrays
  int pow;       // n != 1: solve the power-law viscosity
};

// Per-case progress of a sweep, kept on the device.
struct SweepStatus {
  int64_t steps;     // steps taken by this case
  double residual;   // last max |dT| over a chunk
};

// Constants of the adjoint step, in FP64 (the adjoint recomputes the
// forward node update in FP64 whatever the storage type of the state).
// Per-workgroup adjoint partials: sums of the ln nu0, n and s_g derivatives,
// then the largest |lambda| the workgroup wrote.
constexpr int ADJ_PART = 4;

struct AdjParams {
  int nx, ny, has_logda, pow;
  double eps, inv_eps, Feps, invK, invsK, inv_Kscale, gbeta, dTm, gx, gy;
  double s_e, s_eps, s_q, s_g, sT_e, sT_nu, T_ref;
  double nu0, log2nu0, y_lo, y_hi, lc0, nm1, inv_n, log2c;
  double g2_floor;  // (shear-rate floor)^2, lattice units: below it nu is held fixed
};

struct Launch {
  hipStream_t stream;
  int tiles_x;       // row tiles of TILE nodes
  int ntiles;        // tiles_x * ny
  int step_w;        // row-segment width of the step kernels' workgroups (64, 128 or 256)
  int step_tiles_x;  // ceil(nx / step_w)
  int step_ntiles;   // step_tiles_x * ny
};

#ifndef PM_TILE
#define PM_TILE 256
#endif
constexpr int TILE = PM_TILE;   // nodes per workgroup (one row segment)

// The two-step kernel: a workgroup owns PAIR_W output columns by PAIR_R
// output rows.  It pays off only with many workgroups: each marches through
// its rows with two barriers per row, and only three fit a CU (LDS), so the
// library uses it when the grid gives at least PAIR_MIN_WORKGROUPS of them
// (three full rounds of 3 workgroups on each of 256 CUs; at 4096^2 it is 20%
// faster per step than the single-step kernel, at 3072^2 and below equal or
// slower).
// PAIR_R is the nominal row count (the host tunes the actual one per grid
// between PAIR_R_MIN and PAIR_R so that the workgroups fill whole rounds).
#ifndef PM_PAIR_R
#define PM_PAIR_R 24
#endif
constexpr int PAIR_W = PM_TILE - 4;
constexpr int PAIR_R = PM_PAIR_R;
constexpr int PAIR_R_MIN = 16;
constexpr int PAIR_PER_CU = 3;  // resident workgroups per CU (LDS: 2 x 24 KB each)
constexpr int64_t PAIR_MIN_WORKGROUPS = 9 * 256;
constexpr int RED_BLOCKS = 1024; // partial-result slots of the residual
constexpr int GRID_Y_MAX = 65535; // largest gridDim.y of any launch: taller grids loop over rows

// parity 0: state in natural layout; 1: after an odd number of steps
template <typename T, typename S>
hipError_t launch_step(const KParams<T, S>& p, const Launch& L, int parity, bool pow, bool logda);
template <typename T>
hipError_t launch_step_oop(const KParams<T>& src, const KParams<T>& dst, const Launch& L, int parity,
                           bool pow, bool logda);
template <typename T, typename S>
hipError_t launch_init(const KParams<T, S>& p, const Launch& L, T dg_init, size_t pop_bytes);
template <typename T, typename S>
hipError_t launch_nu(const KParams<T, S>& p, const Launch& L, int parity, double* out);
template <typename T, typename S>
hipError_t launch_residual(const KParams<T, S>& p, const Launch& L, int parity, T* snap,
                           double* partial, double* out, int take_snapshot_only);
template <typename T, typename S>
hipError_t launch_fields(const KParams<T, S>& p, const Launch& L, int parity, bool pow, bool logda,
                         void* U, void* V, void* th, void* nu, int out_fp64);
template <typename T, typename S>
hipError_t launch_get_pop(const KParams<T, S>& p, const Launch& L, int parity, void* f, void* g,
                          int out_fp64);
template <typename T, typename S>
hipError_t launch_set_pop(const KParams<T, S>& p, const Launch& L, const void* f, const void* g,
                          int in_fp64);
template <typename T, typename S>
hipError_t launch_set_logda(const KParams<T, S>& p, const Launch& L, T* dst, const void* src,
                            int in_fp64);
// Sweep tiles are tw columns by th rows: tw in {64, 128, 256}, th in {1, 2, 4},
// tw * th <= TILE threads (a wave then lies within one grid row).  any_sr:
// some case of the sweep rounds stochastically.
inline bool sweep_tile_ok(int tw, int th) {
  return (tw == 64 || tw == 128 || tw == 256) && (th == 1 || th == 2 || th == 4) && tw * th <= TILE;
}
template <typename T>
hipError_t launch_step_multi(const SweepCase<T>* cases, const int2* sched, const int* live,
                             int nsched, int parity, int tw, int th, bool any_sr, hipStream_t s);
template <typename T>
hipError_t launch_resid_multi(const SweepCase<T>* cases, int ncases, const int2* sched, int* live,
                              int nsched, int parity, int tw, int th, double* partial, SweepStatus* st,
                              int64_t chunk, double tol, int64_t max_steps, hipStream_t s);
// L: storage type of the adjoint state (double; float for FP32 states)
template <typename S, typename L>
hipError_t launch_adjoint(const KParams<S>& st, const AdjParams& a, int parity, const L* lam_next, L* lam,
                          double* g_logda, double* partial, hipStream_t s);
template <typename L>
hipError_t launch_adjoint_seed(int nx, int ny, double seed, L* lam, hipStream_t s);
// a[0, n) := 0 (a fill kernel, so that callers may capture it in a graph)
hipError_t launch_fill_zero(double* a, int64_t n, hipStream_t s);
// the adjoint partials of nblocks workgroups reduced in workgroup order into out[ADJ_PART]
hipError_t launch_adj_reduce(const double* partial, int nblocks, double* out, hipStream_t s);
hipError_t launch_write_header(void* dst, int64_t steps, uint64_t tag, uint64_t phys, hipStream_t s);
// Two time steps of an FP32 cavity (no periodic axis) in one pass, from the
// natural-layout state in src (even step count) to dst.
hipError_t launch_step2(const KParams<float>& src, const KParams<float>& dst, hipStream_t s, bool pow,
                        bool logda, int rows);
// Stream function up each column, in place on the U field in psi; scratch:
// stream_scratch_bytes(nx, ny) bytes of device memory.
size_t stream_scratch_bytes(int nx, int ny);
hipError_t launch_stream_y(void* psi, int nx, int ny, double inv_L, int out_fp64, double* scratch,
                           hipStream_t s);
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace pm
