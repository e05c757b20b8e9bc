// pm_api.hip -- host runtime and C ABI (pmlbm.h) of the gfx950 lattice
// Boltzmann library: parameter mapping and validation, workspace carving,
// launch sequencing (with HIP-graph replay of long step runs), reductions,
// checkpoints.
#include "pmlbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include <climits>
#include <mutex>
#include <type_traits>
#include <vector>

#include "pm_internal.h"

namespace {

thread_local char g_last_err[512] = "";

void set_global_err(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_err, sizeof g_last_err, fmt, ap);
  va_end(ap);
}

constexpr size_t ALIGN = 256;
constexpr int GRAPH_PAIRS = 32;  // steps per captured graph = 2 * GRAPH_PAIRS
constexpr uint64_t STATE_TAG = 0x504d4c424d535431ull;  // "PMLBMST1"
constexpr size_t HEADER_BYTES = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t elem;       // population element size (2, 4 or 8 bytes)
  size_t pelem;      // element size of the per-cell planes (the compute type: 4 or 8 bytes)
  size_t qs, rs;     // population stride, row stride (elements), see pm::KParams
  size_t plane;      // pitch of the per-cell planes (log10 Da, snapshot), elements
  size_t pop_bytes;  // the population region (f and g, padding included)
  size_t off_f, off_g, off_logda, off_snap, off_red, off_scan, total;
  size_t off_pair;   // second population region for the two-step kernel (0: none)
};

// Populations are row-interleaved: row j holds the 9 f rows then the 5 g rows
// of that grid row, each padded to a multiple of 64 elements, so the 14
// populations a node update reads (and writes) sit within one contiguous
// 14-row block instead of 14 planes far apart.  At 4096^2 FP32 the in-place
// (even) step streams ~10% faster this way; PM_SOA_LAYOUT=1 builds the
// plane-per-population layout instead, for comparison.
#ifndef PM_SOA_LAYOUT
#define PM_SOA_LAYOUT 0
#endif

// Two time steps per pass (pm::launch_step2) for large FP32 cavities without
// a periodic axis: fewer HBM bytes per step at the price of a second
// population region.  PM_PAIR_STEP=0 builds without it, for comparison.
#ifndef PM_PAIR_STEP
#define PM_PAIR_STEP 1
#endif

// Row-segment width of the single-step kernels' workgroups (64, 128 or 256
// nodes; one lane per node either way, so the results do not depend on it).
// Measured on one MI355X (us per step, widths 256 / 128 / 64):
//   FP64 512^2 15.2 / 15.2 / 14.0, 1024^2 44.8 / 44.9 / 45.8, 4096^2 637 / 615 / 634;
//   FP32 512^2 8.3 / 8.3 / 7.5, 1024^2 21.2 / 22.1 / 23.6, 2048^2 73.0 / 76.9 / 84.1.
int step_width_for(int nx, int ny, int dtype) {
  if ((int64_t)nx * ny <= 512 * 512) return 64;
  return dtype == PM_FP64 ? 128 : 256;
}

// Rows per workgroup of the two-step kernel: the workgroups run in rounds of
// PAIR_PER_CU per CU, so a last round that is mostly empty costs nearly a
// full one; fewer rows recompute a larger share of halo rows (4 extra rows of
// step k per workgroup).  Pick the row count in [PAIR_R_MIN, PAIR_R] that
// minimises (rows + 4) / rows divided by the fraction of the last round used.
int pair_rows_for(int nx, int ny, int cus) {
  const int64_t strips = (nx + pm::PAIR_W - 1) / pm::PAIR_W, slots = (int64_t)pm::PAIR_PER_CU * cus;
  int best = pm::PAIR_R;
  double best_cost = 1e300;
  for (int r = pm::PAIR_R; r >= pm::PAIR_R_MIN; --r) {
    if ((ny + r - 1) / r > pm::GRID_Y_MAX) break;  // row groups are gridDim.y
    const int64_t wg = strips * ((ny + r - 1) / r);
    const int64_t rounds = (wg + slots - 1) / slots;
    const double fill = (double)wg / (double)(rounds * slots);
    const double cost = (double)(r + 4) / r / fill;
    if (cost < best_cost - 1e-12) {
      best_cost = cost;
      best = r;
    }
  }
  return best;
}

bool pair_capable(const pm_params& p) {
  if (!PM_PAIR_STEP || p.dtype != PM_FP32 || p.periodic_x || p.periodic_y) return false;
  if ((p.ny + pm::PAIR_R - 1) / pm::PAIR_R > pm::GRID_Y_MAX) return false;
  if (p.step_kernel == PM_STEP_PAIR) return true;
  if (p.step_kernel == PM_STEP_SINGLE) return false;
  const int64_t wg = (int64_t)((p.nx + pm::PAIR_W - 1) / pm::PAIR_W) * ((p.ny + pm::PAIR_R - 1) / pm::PAIR_R);
  return wg >= pm::PAIR_MIN_WORKGROUPS;
}

Layout layout_of(const pm_params& p, bool pair = false) {
  Layout L{};
  L.elem = p.dtype == PM_FP64 ? 8 : (p.dtype == PM_FP16 ? 2 : 4);
  L.pelem = p.dtype == PM_FP64 ? 8 : 4;
  const size_t n = (size_t)p.nx * (size_t)p.ny;
  L.plane = (n + 63) / 64 * 64;
#if PM_SOA_LAYOUT
  L.qs = L.plane;
  L.rs = (size_t)p.nx;
  L.pop_bytes = 14 * L.qs * L.elem;
#else
  L.qs = ((size_t)p.nx + 63) / 64 * 64;
  L.rs = 14 * L.qs;
  L.pop_bytes = (size_t)p.ny * L.rs * L.elem;
#endif
  size_t o = 0;
  L.off_f = o;
  L.off_g = o + 9 * L.qs * L.elem;
  o = align_up(o + L.pop_bytes);
  L.off_logda = o;
  if (p.has_logda) o = align_up(o + L.plane * L.pelem);
  L.off_snap = o;
  o = align_up(o + L.plane * L.pelem);
  L.off_red = o;
  o = align_up(o + (pm::RED_BLOCKS + 16) * sizeof(double));
  L.off_scan = o;  // block sums of the stream-function scan
  o = align_up(o + pm::stream_scratch_bytes(p.nx, p.ny));
  if (pair) {
    o = (o + (size_t(1) << 21) - 1) / (size_t(1) << 21) * (size_t(1) << 21);  // 2 MiB, like the base
    L.off_pair = o;
    o = align_up(o + L.pop_bytes);
  }
  L.total = o;
  return L;
}

// FP32 population updates are rounded stochastically (PM_ROUND_STOCHASTIC, or
// the default PM_ROUND_AUTO with FP32 storage).
bool rounds_stochastically(const pm_params& p) {
  return (p.dtype == PM_FP32 || p.dtype == PM_FP16) &&
         (p.rounding == PM_ROUND_STOCHASTIC || p.rounding == PM_ROUND_AUTO);
}

// Step 0 of the update: physical groups -> lattice values (see pmlbm.h).
int map_params(const pm_params& p, pm_lattice& L, char* msg, size_t msglen) {
  auto fail = [&](const char* m) {
    snprintf(msg, msglen, "%s", m);
    return PM_EINVAL;
  };
  if (p.nx < 2 || p.ny < 2) return fail("nx and ny must be >= 2");
  if ((double)p.nx * (double)p.ny > 2147483647.0 / 2) return fail("grid too large for 32-bit node indices");
  // the odd step's interior path addresses three rows of 14 populations with
  // 32-bit offsets: 42 padded rows must stay below 2^32 elements
  if (p.nx > 100000000) return fail("nx must be <= 1e8");
  if (p.dtype != PM_FP32 && p.dtype != PM_FP64 && p.dtype != PM_FP16)
    return fail("dtype must be PM_FP32, PM_FP64 or PM_FP16");
  if (!(p.n > 0.0 && p.n <= 4.0)) return fail("power-law index n must be in (0, 4]");
  if (!(p.Ra > 0.0) || !(p.Pr > 0.0)) return fail("Ra and Pr must be > 0");
  if (!(p.Da > 0.0)) return fail("Da must be > 0 (+inf for a clear fluid)");
  if (!(p.eps > 0.0 && p.eps <= 1.0)) return fail("eps must be in (0, 1]");
  if (!(p.mach > 0.0 && p.mach < 1.0)) return fail("mach must be in (0, 1)");
  if (!(p.nu_lo > 0.0) || !(p.nu_hi >= p.nu_lo)) return fail("need 0 < nu_lo <= nu_hi");
  if (p.clamp_mode != PM_CLAMP_NU && p.clamp_mode != PM_CLAMP_GAMMA)
    return fail("clamp_mode must be PM_CLAMP_NU or PM_CLAMP_GAMMA");
  if (p.clamp_mode == PM_CLAMP_NU && !(p.nu_lo <= 1.0 && p.nu_hi >= 1.0))
    return fail("PM_CLAMP_NU bounds must bracket 1 (nu0 itself)");
  if (!std::isfinite(p.gx) || !std::isfinite(p.gy) || !std::isfinite(p.T_init))
    return fail("gx, gy, T_init must be finite");
  if (p.step_kernel != PM_STEP_AUTO && p.step_kernel != PM_STEP_SINGLE && p.step_kernel != PM_STEP_PAIR)
    return fail("step_kernel must be PM_STEP_AUTO, PM_STEP_SINGLE or PM_STEP_PAIR");
  if (p.step_kernel == PM_STEP_PAIR && (!PM_PAIR_STEP || p.dtype != PM_FP32 || p.periodic_x || p.periodic_y))
    return fail("PM_STEP_PAIR needs FP32 and cavity walls on both axes");
  if (p.step_kernel == PM_STEP_PAIR && (p.ny + pm::PAIR_R - 1) / pm::PAIR_R > pm::GRID_Y_MAX)
    return fail("PM_STEP_PAIR: ny too large (more row groups than a launch's y dimension takes)");
  if (p.rounding != PM_ROUND_NEAREST && p.rounding != PM_ROUND_STOCHASTIC && p.rounding != PM_ROUND_AUTO)
    return fail("rounding must be PM_ROUND_AUTO, PM_ROUND_NEAREST or PM_ROUND_STOCHASTIC");
  if (p.rounding == PM_ROUND_STOCHASTIC && p.dtype == PM_FP64)
    return fail("PM_ROUND_STOCHASTIC applies to FP32 and FP16 storage only");
  const double N = (double)p.nx;
  memset(&L, 0, sizeof L);
  L.U_lb = p.mach / std::sqrt(3.0);
  L.nu0 = p.Pr / std::pow(std::sqrt(p.Ra), 2.0 - p.n) * L.U_lb * N;
  L.gamma_scale = N / L.U_lb;
  if (p.clamp_mode == PM_CLAMP_NU) {
    L.nu_min = p.nu_lo * L.nu0;
    L.nu_max = p.nu_hi * L.nu0;
  } else {
    const double a = L.nu0 * std::pow(p.nu_lo, p.n - 1.0);
    const double b = L.nu0 * std::pow(p.nu_hi, p.n - 1.0);
    L.nu_min = a < b ? a : b;
    L.nu_max = a < b ? b : a;
  }
  L.eps = p.eps;
  L.K = std::isinf(p.Da) ? INFINITY : p.Da * N * N;
  L.Feps = p.forchheimer ? 1.75 / std::sqrt(150.0 * p.eps * p.eps * p.eps) : 0.0;
  L.gbeta = p.Pr * L.U_lb * L.U_lb / N;
  L.T_m = 0.5;
  L.alpha = L.U_lb * N / std::sqrt(p.Ra);
  double nu_newt = L.nu0;
  if (nu_newt < L.nu_min) nu_newt = L.nu_min;
  if (nu_newt > L.nu_max) nu_newt = L.nu_max;
  L.tau0 = 3.0 * nu_newt + 0.5;
  L.tau_min = 3.0 * L.nu_min + 0.5;
  L.tau_max = 3.0 * L.nu_max + 0.5;
  L.tau_g = 3.0 * L.alpha + 0.5;
  L.s_e = p.s_e > 0 ? p.s_e : 1.4;
  L.s_eps = p.s_eps > 0 ? p.s_eps : 1.4;
  L.s_q = p.s_q > 0 ? p.s_q : 1.2;
  L.sT_e = p.sT_e > 0 ? p.sT_e : 1.0;
  L.sT_nu = p.sT_nu > 0 ? p.sT_nu : 1.0;
  if (!(L.nu_min > 0.0) || !std::isfinite(L.nu_max)) return fail("viscosity bounds not finite/positive");
  if (!(L.alpha > 0.0) || !std::isfinite(L.alpha)) return fail("thermal diffusivity not finite/positive");
  if (L.s_e >= 2.0 || L.s_eps >= 2.0 || L.s_q >= 2.0 || L.sT_e >= 2.0 || L.sT_nu >= 2.0)
    return fail("relaxation rates must lie in (0, 2)");
  return PM_OK;
}

template <typename T, typename S = T>
pm::KParams<T, S> kparams(const pm_params& p, const pm_lattice& L, void* ws, const Layout& lay) {
  pm::KParams<T, S> k{};
  char* base = (char*)ws;
  k.f = (S*)(base + lay.off_f);
  k.g = (S*)(base + lay.off_g);
  k.logda = p.has_logda ? (const T*)(base + lay.off_logda) : nullptr;
  k.qs = (int64_t)lay.qs;
  k.rs = (int64_t)lay.rs;
  k.nx = p.nx;
  k.ny = p.ny;
  k.px = p.periodic_x ? 1 : 0;
  k.py = p.periodic_y ? 1 : 0;
  double nu_newt = L.nu0;
  if (nu_newt < L.nu_min) nu_newt = L.nu_min;
  if (nu_newt > L.nu_max) nu_newt = L.nu_max;
  k.nu_newt = (T)nu_newt;
  k.nu_min = (T)L.nu_min;
  k.nu_max = (T)L.nu_max;
  k.y_lo = (T)std::log2(L.nu_min);
  k.y_hi = (T)std::log2(L.nu_max);
  k.lc0 = (T)(std::log2(L.nu0) + (p.n - 1.0) * std::log2(L.gamma_scale));
  k.nm1 = (T)(p.n - 1.0);
  k.inv_n = (T)(1.0 / p.n);
  k.tol = sizeof(T) == 8 ? (T)1e-13 : (T)8e-6;
  k.max_it = sizeof(T) == 8 ? 40 : 12;
  k.sr = (sizeof(T) == 4 && rounds_stochastically(p)) ? 1 : 0;
  k.eps = (T)L.eps;
  k.inv_eps = (T)(1.0 / L.eps);
  k.invK = std::isinf(L.K) ? (T)0 : (T)(1.0 / L.K);
  k.invsK = std::isinf(L.K) ? (T)0 : (T)std::sqrt(1.0 / L.K);
  k.Feps = (T)L.Feps;
  k.inv_Kscale = (T)(1.0 / ((double)p.nx * (double)p.nx));
  k.gbeta = (T)L.gbeta;
  k.T_ref = (T)0.5;
  k.dTm = (T)(L.T_m - 0.5);
  k.gx = (T)p.gx;
  k.gy = (T)p.gy;
  k.s_e = (T)L.s_e;
  k.s_eps = (T)L.s_eps;
  k.s_q = (T)L.s_q;
  k.s_g = (T)(1.0 / L.tau_g);
  k.sT_e = (T)L.sT_e;
  k.sT_nu = (T)L.sT_nu;
  k.hotc = (T)(2.0 / 6.0 * (1.0 - 0.5));
  k.coldc = (T)(2.0 / 6.0 * (0.0 - 0.5));
  k.inv_U = (T)(1.0 / L.U_lb);
  return k;
}

}  // namespace

struct pm_ctx {
  pm_params p;
  pm_lattice L;
  Layout lay;
  void* ws;
  hipStream_t stream;
  hipStream_t cap_stream;  // private stream used only for graph capture
  int device;
  int64_t steps;
  pm::KParams<float> k32;
  pm::KParams<double> k64;
  pm::KParams<float, _Float16> k16;  // FP16 storage, FP32 compute
  pm::KParams<float> k32b;  // k32 on the second population region (two-step kernel)
  bool pair;                // two-step kernel available (FP32 cavity, second region)
  int pair_rows;            // rows per workgroup of the two-step kernel
  pm::Launch launch;
  bool pow;
  hipGraphExec_t graph[2];  // chunk graphs starting at parity 0 / 1
  double* red;              // device partials + results
  char err[512];
};

namespace {

int ctx_fail(pm_ctx* c, int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(c ? c->err : g_last_err, 512, fmt, ap);
  va_end(ap);
  return code;
}

int check_hip(pm_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return PM_OK;
  return ctx_fail(c, PM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename F>
hipError_t dispatch(pm_ctx* c, F&& fn) {
  if (c->p.dtype == PM_FP64) return fn(c->k64);
  if (c->p.dtype == PM_FP16) return fn(c->k16);
  return fn(c->k32);
}

// k steps from step count start_steps.  With the two-step kernel, whole
// groups of four steps from an even step count run as two passes (region
// A -> B -> A, so the state always ends in its own region); the remaining
// steps use the single-step kernel in place.
hipError_t enqueue_steps(pm_ctx* c, hipStream_t s, int64_t k, int64_t start_steps) {
  pm::Launch L = c->launch;
  L.stream = s;
  const bool logda = c->p.has_logda != 0;
  auto single = [&](int64_t t) {
    const int parity = (int)((start_steps + t) & 1);
    return dispatch(c, [&](auto& kp) { return pm::launch_step(kp, L, parity, c->pow, logda); });
  };
  hipError_t e = hipSuccess;
  int64_t t = 0;
  if (c->pair) {
    if ((start_steps & 1) && k > 0) e = single(t++);
    for (; e == hipSuccess && k - t >= 4; t += 4) {
      e = pm::launch_step2(c->k32, c->k32b, s, c->pow, logda, c->pair_rows);
      if (e == hipSuccess) e = pm::launch_step2(c->k32b, c->k32, s, c->pow, logda, c->pair_rows);
    }
  }
  for (; e == hipSuccess && t < k; ++t) e = single(t);
  return e;
}

int build_graph(pm_ctx* c, int parity) {
  if (c->graph[parity]) return PM_OK;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return check_hip(c, e, "hipStreamBeginCapture");
  hipError_t le = enqueue_steps(c, c->cap_stream, 2 * GRAPH_PAIRS, parity);
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return check_hip(c, le, "capturing step kernels");
  }
  if (e != hipSuccess) return check_hip(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->graph[parity] = nullptr;
    return check_hip(c, e, "hipGraphInstantiate");
  }
  return PM_OK;
}

int sync_read(pm_ctx* c, double* host, const double* dev, int n) {
  hipError_t e = hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return check_hip(c, e, "reading a reduction result");
}

int dtype_ok(int d) { return d == PM_FP32 || d == PM_FP64; }  // caller-facing arrays

// Checkpoint header: [tag of grid and dtype, step count, physics hash], then
// the population region and the residual snapshot plane.
uint64_t state_tag(const pm_ctx* c) {
  return STATE_TAG ^ ((uint64_t)c->p.nx << 32) ^ (uint64_t)c->p.ny ^ ((uint64_t)c->p.dtype << 60);
}

// FNV-1a (64-bit) over the lattice values the update runs with (so that the
// same physics given with default or explicit rates hashes the same) and the
// switches that change results.  The log-Da plane's contents are not hashed.
uint64_t physics_hash(const pm_ctx* c) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto eat = [&](const void* v, size_t n) {
    const unsigned char* b = (const unsigned char*)v;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 0x100000001b3ull;
    }
  };
  const pm_lattice& L = c->L;
  const double d[] = {c->p.n, L.U_lb, L.nu0, L.nu_min, L.nu_max, L.gamma_scale, L.eps, L.K, L.Feps, L.gbeta,
                      L.alpha, L.s_e, L.s_eps, L.s_q, L.sT_e, L.sT_nu, c->p.gx, c->p.gy};
  const int32_t k[] = {c->p.has_logda, c->p.periodic_x, c->p.periodic_y, rounds_stochastically(c->p) ? 1 : 0};
  eat(d, sizeof d);
  eat(k, sizeof k);
  return h;
}

size_t snap_bytes(const pm_ctx* c) { return c->lay.plane * c->lay.pelem; }

int init_ctx(const pm_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, bool pair, pm_ctx** out);

}  // namespace

extern "C" {

int pm_params_default(pm_params* p) {
  if (!p) return PM_EINVAL;
  memset(p, 0, sizeof *p);
  p->nx = p->ny = 64;
  p->n = 1.0;
  p->Da = INFINITY;
  p->Ra = 1e3;
  p->Pr = 10.0;
  p->eps = 1.0;
  p->mach = 0.1;
  p->nu_lo = 0.1;
  p->nu_hi = 10.0;
  p->clamp_mode = PM_CLAMP_NU;
  p->dtype = PM_FP32;
  p->forchheimer = 1;
  p->T_init = 0.5;
  p->rounding = PM_ROUND_AUTO;
  return PM_OK;
}

int pm_lattice_of(const pm_params* p, pm_lattice* out) {
  if (!p || !out) {
    set_global_err("pm_lattice_of: null argument");
    return PM_EINVAL;
  }
  char msg[256];
  int rc = map_params(*p, *out, msg, sizeof msg);
  if (rc) set_global_err("%s", msg);
  return rc;
}

int pm_workspace_bytes(const pm_params* p, size_t* bytes) {
  pm_lattice L;
  int rc = pm_lattice_of(p, &L);
  if (rc) return rc;
  if (!bytes) return PM_EINVAL;
  *bytes = layout_of(*p, pair_capable(*p)).total;
  return PM_OK;
}

int pm_init(const pm_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, pm_ctx** out) {
  return p ? init_ctx(p, dev_ws, ws_bytes, hip_stream, pair_capable(*p), out) : PM_EINVAL;
}

}  // extern "C"

namespace {

// pm_init, with or without the second population region of the two-step
// kernel (contexts of a sweep go without: the sweep has its own kernels).
int init_ctx(const pm_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, bool pair, pm_ctx** out) {
  if (!out) {
    set_global_err("pm_init: null out pointer");
    return PM_EINVAL;
  }
  *out = nullptr;
  pm_lattice L;
  int rc = pm_lattice_of(p, &L);
  if (rc) return rc;
  Layout lay = layout_of(*p, pair);
  if (!dev_ws || ws_bytes < lay.total) {
    set_global_err("pm_init: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, lay.total);
    return PM_ESTATE;
  }
  if (((uintptr_t)dev_ws) % ALIGN) {
    set_global_err("pm_init: workspace must be %zu-byte aligned", ALIGN);
    return PM_EINVAL;
  }
  pm_ctx* c = new (std::nothrow) pm_ctx();
  if (!c) {
    set_global_err("pm_init: out of host memory");
    return PM_EDEVICE;
  }
  c->p = *p;
  c->L = L;
  c->lay = lay;
  c->ws = dev_ws;
  c->stream = (hipStream_t)hip_stream;
  c->steps = 0;
  c->pow = p->n != 1.0;
  (void)hipGetDevice(&c->device);
  c->k32 = kparams<float>(*p, L, dev_ws, lay);
  c->k64 = kparams<double>(*p, L, dev_ws, lay);
  c->k16 = kparams<float, _Float16>(*p, L, dev_ws, lay);
  c->pair = pair;
  if (pair) {
    c->k32b = c->k32;
    c->k32b.f = (float*)((char*)dev_ws + lay.off_pair + lay.off_f);
    c->k32b.g = (float*)((char*)dev_ws + lay.off_pair + lay.off_g);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
      cus = 256;
    c->pair_rows = pair_rows_for(p->nx, p->ny, cus);
  }
  c->launch.stream = c->stream;
  c->launch.tiles_x = (p->nx + pm::TILE - 1) / pm::TILE;
  c->launch.ntiles = c->launch.tiles_x * p->ny;
  c->launch.step_w = std::min(step_width_for(p->nx, p->ny, p->dtype), pm::TILE);
  c->launch.step_tiles_x = (p->nx + c->launch.step_w - 1) / c->launch.step_w;
  c->launch.step_ntiles = c->launch.step_tiles_x * p->ny;
  c->red = (double*)((char*)dev_ws + lay.off_red);
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    set_global_err("hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    delete c;
    return PM_EDEVICE;
  }
  const double dg_init = (1.0 / 6.0) * (p->T_init - 0.5);
  e = dispatch(c, [&](auto& kp) {
    using T = typename std::remove_reference_t<decltype(kp)>::compute_t;
    return pm::launch_init(kp, c->launch, (T)dg_init, c->lay.pop_bytes);
  });
  if (e == hipSuccess)
    e = dispatch(c, [&](auto& kp) {
      using T = typename std::remove_reference_t<decltype(kp)>::compute_t;
      T* snap = (T*)((char*)c->ws + c->lay.off_snap);
      return pm::launch_residual(kp, c->launch, 0, snap, c->red, c->red + pm::RED_BLOCKS, 1);
    });
  if (e != hipSuccess) {
    set_global_err("pm_init: %s", hipGetErrorString(e));
    (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return PM_EDEVICE;
  }
  *out = c;
  return PM_OK;
}

}  // namespace

extern "C" {

void pm_destroy(pm_ctx* c) {
  if (!c) return;
  for (auto& g : c->graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

int pm_set_logda(pm_ctx* c, const void* dev_plane, int dtype) {
  if (!c) return PM_EINVAL;
  if (!c->p.has_logda) return ctx_fail(c, PM_ESTATE, "pm_set_logda: context created with has_logda = 0");
  if (!dev_plane || !dtype_ok(dtype)) return ctx_fail(c, PM_EINVAL, "pm_set_logda: bad plane or dtype");
  hipError_t e = dispatch(c, [&](auto& kp) {
    using T = typename std::remove_reference_t<decltype(kp)>::compute_t;
    return pm::launch_set_logda(kp, c->launch, (T*)kp.logda, dev_plane, dtype == PM_FP64);
  });
  return check_hip(c, e, "pm_set_logda");
}

int pm_step(pm_ctx* c, int64_t k) {
  if (!c) return PM_EINVAL;
  if (k < 0) return ctx_fail(c, PM_EINVAL, "pm_step: k must be >= 0");
  const int64_t chunk = 2 * GRAPH_PAIRS;
  int64_t left = k;
  hipError_t e = hipSuccess;
  if (left >= 2 * chunk) {
    const int parity = (int)(c->steps & 1);
    int rc = build_graph(c, parity);
    if (rc) return rc;
    while (left >= chunk) {
      e = hipGraphLaunch(c->graph[parity], c->stream);
      if (e != hipSuccess) return check_hip(c, e, "hipGraphLaunch");
      left -= chunk;
      c->steps += chunk;  // chunk is even: parity unchanged
    }
  }
  e = enqueue_steps(c, c->stream, left, c->steps);
  if (e != hipSuccess) return check_hip(c, e, "pm_step launch");
  c->steps += left;
  return PM_OK;
}

int pm_steps_done(const pm_ctx* c, int64_t* steps) {
  if (!c || !steps) return PM_EINVAL;
  *steps = c->steps;
  return PM_OK;
}

int pm_nu(pm_ctx* c, double* nu_out) {
  if (!c || !nu_out) return PM_EINVAL;
  const int parity = (int)(c->steps & 1);
  double* dev = c->red + pm::RED_BLOCKS + 1;
  hipError_t e = dispatch(c, [&](auto& kp) { return pm::launch_nu(kp, c->launch, parity, dev); });
  if (e != hipSuccess) return check_hip(c, e, "pm_nu");
  int rc = sync_read(c, nu_out, dev, 1);
  if (rc) return rc;
  if (!std::isfinite(*nu_out)) return ctx_fail(c, PM_EDIVERGED, "pm_nu: Nusselt number is not finite");
  return PM_OK;
}

int pm_residual(pm_ctx* c, double* r_out, int64_t* at_step) {
  if (!c || !r_out) return PM_EINVAL;
  if (at_step) *at_step = c->steps;
  const int parity = (int)(c->steps & 1);
  double* dev = c->red + pm::RED_BLOCKS;
  hipError_t e = dispatch(c, [&](auto& kp) {
    using T = typename std::remove_reference_t<decltype(kp)>::compute_t;
    T* snap = (T*)((char*)c->ws + c->lay.off_snap);
    return pm::launch_residual(kp, c->launch, parity, snap, c->red, dev, 0);
  });
  if (e != hipSuccess) return check_hip(c, e, "pm_residual");
  int rc = sync_read(c, r_out, dev, 1);
  if (rc) return rc;
  if (!std::isfinite(*r_out)) return ctx_fail(c, PM_EDIVERGED, "pm_residual: NaN/Inf in the temperature field");
  return PM_OK;
}

int pm_run_to_steady(pm_ctx* c, double tol, int64_t check_every, int64_t max_steps,
                     int64_t* steps_out, double* r_out) {
  if (!c) return PM_EINVAL;
  if (check_every <= 0 || max_steps < 0) return ctx_fail(c, PM_EINVAL, "pm_run_to_steady: bad chunk or cap");
  int64_t done = 0;
  double r = INFINITY;
  int rc = PM_OK;
  while (done < max_steps) {
    int64_t k = check_every;
    if (done + k > max_steps) k = max_steps - done;
    rc = pm_step(c, k);
    if (rc) break;
    done += k;
    rc = pm_residual(c, &r, nullptr);
    if (rc) break;
    if (r < tol) break;
  }
  if (steps_out) *steps_out = done;
  if (r_out) *r_out = r;
  return rc;
}

int pm_fields(pm_ctx* c, void* U, void* V, void* theta, int dtype) {
  if (!c) return PM_EINVAL;
  if (!dtype_ok(dtype)) return ctx_fail(c, PM_EINVAL, "pm_fields: bad dtype");
  const int parity = (int)(c->steps & 1);
  hipError_t e = dispatch(c, [&](auto& kp) {
    return pm::launch_fields(kp, c->launch, parity, c->pow, c->p.has_logda != 0, U, V, theta,
                             nullptr, dtype == PM_FP64);
  });
  return check_hip(c, e, "pm_fields");
}

int pm_stream_function(pm_ctx* c, void* psi, int dtype) {
  if (!c || !psi) return PM_EINVAL;
  if (!dtype_ok(dtype)) return ctx_fail(c, PM_EINVAL, "pm_stream_function: bad dtype");
  const int parity = (int)(c->steps & 1);
  hipError_t e = dispatch(c, [&](auto& kp) {
    return pm::launch_fields(kp, c->launch, parity, c->pow, c->p.has_logda != 0, psi, nullptr,
                             nullptr, nullptr, dtype == PM_FP64);
  });
  if (e == hipSuccess)
    e = pm::launch_stream_y(psi, c->p.nx, c->p.ny, 1.0 / (double)c->p.nx, dtype == PM_FP64,
                            (double*)((char*)c->ws + c->lay.off_scan), c->stream);
  return check_hip(c, e, "pm_stream_function");
}

int pm_viscosity(pm_ctx* c, void* nu, int dtype) {
  if (!c || !nu) return PM_EINVAL;
  if (!dtype_ok(dtype)) return ctx_fail(c, PM_EINVAL, "pm_viscosity: bad dtype");
  const int parity = (int)(c->steps & 1);
  hipError_t e = dispatch(c, [&](auto& kp) {
    return pm::launch_fields(kp, c->launch, parity, c->pow, c->p.has_logda != 0, nullptr,
                             nullptr, nullptr, nu, dtype == PM_FP64);
  });
  return check_hip(c, e, "pm_viscosity");
}

int pm_get_populations(pm_ctx* c, void* f, void* g, int dtype) {
  if (!c || !f || !g) return PM_EINVAL;
  if (!dtype_ok(dtype)) return ctx_fail(c, PM_EINVAL, "pm_get_populations: bad dtype");
  const int parity = (int)(c->steps & 1);
  hipError_t e = dispatch(c, [&](auto& kp) {
    return pm::launch_get_pop(kp, c->launch, parity, f, g, dtype == PM_FP64);
  });
  return check_hip(c, e, "pm_get_populations");
}

int pm_set_populations(pm_ctx* c, const void* f, const void* g, int dtype) {
  if (!c || !f || !g) return PM_EINVAL;
  if (!dtype_ok(dtype)) return ctx_fail(c, PM_EINVAL, "pm_set_populations: bad dtype");
  hipError_t e = dispatch(c, [&](auto& kp) {
    return pm::launch_set_pop(kp, c->launch, f, g, dtype == PM_FP64);
  });
  if (e != hipSuccess) return check_hip(c, e, "pm_set_populations");
  c->steps = 0;
  return PM_OK;
}

int pm_state_bytes(const pm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return PM_EINVAL;
  *bytes = HEADER_BYTES + c->lay.pop_bytes + snap_bytes(c);
  return PM_OK;
}

int pm_save_state(pm_ctx* c, void* dst, size_t bytes) {
  if (!c || !dst) return PM_EINVAL;
  size_t need;
  pm_state_bytes(c, &need);
  if (bytes < need) return ctx_fail(c, PM_ESTATE, "pm_save_state: buffer of %zu bytes < %zu", bytes, need);
  hipError_t e = pm::launch_write_header(dst, c->steps, state_tag(c), physics_hash(c), c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)dst + HEADER_BYTES, (char*)c->ws + c->lay.off_f, c->lay.pop_bytes,
                       hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)dst + HEADER_BYTES + c->lay.pop_bytes, (char*)c->ws + c->lay.off_snap,
                       snap_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  return check_hip(c, e, "pm_save_state");
}

int pm_load_state(pm_ctx* c, const void* src, size_t bytes) {
  if (!c || !src) return PM_EINVAL;
  size_t need;
  pm_state_bytes(c, &need);
  if (bytes < need) return ctx_fail(c, PM_ESTATE, "pm_load_state: buffer of %zu bytes < %zu", bytes, need);
  int64_t hdr[3];
  hipError_t e = hipMemcpyAsync(hdr, src, sizeof hdr, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pm_load_state header");
  if ((uint64_t)hdr[0] != state_tag(c) || hdr[1] < 0)
    return ctx_fail(c, PM_ESTATE, "pm_load_state: checkpoint does not match this grid/dtype");
  if ((uint64_t)hdr[2] != physics_hash(c))
    return ctx_fail(c, PM_ESTATE,
                    "pm_load_state: checkpoint was saved with other physics (n, Da, Ra, Pr, eps, Mach, viscosity "
                    "bounds, rates, body force, log-Da plane use, periodic axes or rounding differ)");
  e = hipMemcpyAsync((char*)c->ws + c->lay.off_f, (const char*)src + HEADER_BYTES, c->lay.pop_bytes,
                     hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)c->ws + c->lay.off_snap, (const char*)src + HEADER_BYTES + c->lay.pop_bytes,
                       snap_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pm_load_state");
  c->steps = hdr[1];
  return PM_OK;
}

int pm_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst || bytes % 16) {
    set_global_err("pm_copy_probe: null buffer or size not a multiple of 16");
    return PM_EINVAL;
  }
  hipError_t e = pm::launch_copy_probe(src, dst, bytes, (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    set_global_err("pm_copy_probe: %s", hipGetErrorString(e));
    return PM_EDEVICE;
  }
  return PM_OK;
}

// ---------------------------------------------------------------------------
// Batched parameter sweep
// ---------------------------------------------------------------------------
}  // extern "C"

struct pm_sweep {
  int ncases;
  int dtype;
  int order;
  hipStream_t stream;
  hipStream_t cap_stream;
  std::vector<pm_ctx*> ctx;
  std::vector<int> ntiles, tile_base;
  int total_tiles;
  int nsched;           // schedule entries: the tiles of the cases live when it was built
  int sched_live;       // cases live when the schedule was built
  int tile_w, tile_h;   // sweep tile: tile_w columns by tile_h rows (pm_sweep_set_tile)
  bool any_sr;          // some case rounds stochastically (PM_ROUND_STOCHASTIC)
  void* d_cases;        // SweepCase<T>[ncases]
  int2* d_sched;        // schedule entries (case, tile)
  int* d_live;          // 1 while the case still runs
  pm::SweepStatus* d_st;
  double* d_partial;    // per-tile residual partials, case-major
  std::vector<unsigned char> h_cases;  // host copy of the case table (kept for the async copy)
  std::vector<int2> h_sched;
  std::vector<int> h_live;
  std::vector<pm::SweepStatus> h_st;
  int64_t gsteps;       // steps taken by the cases still live
  int64_t graph_chunk;  // steps in the captured chunk
  double graph_tol;
  int64_t graph_max;
  hipGraphExec_t graph[2];
  char err[512];
};

namespace {

constexpr size_t SWEEP_ALIGN = size_t(1) << 21;

size_t align_to(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct SweepLayout {
  std::vector<size_t> off, bytes;
  size_t off_cases, off_sched, off_live, off_st, off_partial, total;
  int total_tiles;
};

int sweep_layout(const pm_params* cases, int n, SweepLayout& L, char* msg, size_t len) {
  if (!cases || n <= 0 || n > 4096) {
    snprintf(msg, len, "sweep: need 1..4096 cases");
    return PM_EINVAL;
  }
  L.off.resize(n);
  L.bytes.resize(n);
  size_t o = 0;
  int tiles = 0;
  for (int i = 0; i < n; ++i) {
    pm_lattice lat;
    int rc = map_params(cases[i], lat, msg, len);
    if (rc) return rc;
    if (cases[i].dtype != cases[0].dtype) {
      snprintf(msg, len, "sweep: all cases must share one dtype");
      return PM_EINVAL;
    }
    if (cases[i].has_logda) {
      snprintf(msg, len, "sweep: per-cell log-Da planes are not supported in a sweep");
      return PM_EINVAL;
    }
    if (cases[i].dtype == PM_FP16) {
      snprintf(msg, len, "sweep: FP16 storage is not supported in a sweep");
      return PM_EINVAL;
    }
    L.off[i] = o;
    L.bytes[i] = layout_of(cases[i]).total;
    o = align_to(o + L.bytes[i], SWEEP_ALIGN);
    tiles += ((cases[i].nx + 63) / 64) * cases[i].ny;  // the most tiles any tile shape gives (64 x 1)
  }
  const size_t case_sz = cases[0].dtype == PM_FP64 ? sizeof(pm::SweepCase<double>) : sizeof(pm::SweepCase<float>);
  L.off_cases = o;
  o = align_up(o + n * case_sz);
  L.off_sched = o;
  o = align_up(o + (size_t)tiles * sizeof(int2));
  L.off_live = o;
  o = align_up(o + n * sizeof(int));
  L.off_st = o;
  o = align_up(o + n * sizeof(pm::SweepStatus));
  L.off_partial = o;
  o = align_up(o + (size_t)tiles * sizeof(double));
  L.total = o;
  L.total_tiles = tiles;
  return PM_OK;
}

int sweep_fail(pm_sweep* s, int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(s ? s->err : g_last_err, 512, fmt, ap);
  va_end(ap);
  return code;
}

// Only the tiles of live cases are scheduled, so cases that have stopped cost
// no workgroups (the step kernel still checks the live flag).
void build_schedule(pm_sweep* s) {
  const int n = s->ncases;
  auto live = [&](int i) { return s->h_live.empty() || s->h_live[i] != 0; };
  std::vector<int> ids;
  for (int i = 0; i < n; ++i)
    if (live(i)) ids.push_back(i);
  s->sched_live = (int)ids.size();
  if (s->order == PM_ORDER_LARGEST)
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return s->ntiles[a] > s->ntiles[b]; });
  s->h_sched.clear();
  s->h_sched.reserve(s->total_tiles);
  if (s->order == PM_ORDER_INTERLEAVE) {
    int maxt = 0;
    for (int i : ids) maxt = std::max(maxt, s->ntiles[i]);
    for (int t = 0; t < maxt; ++t)
      for (int i : ids)
        if (t < s->ntiles[i]) s->h_sched.push_back(make_int2(i, t));
  } else {
    for (int i : ids)
      for (int t = 0; t < s->ntiles[i]; ++t) s->h_sched.push_back(make_int2(i, t));
  }
  s->nsched = (int)s->h_sched.size();
}

hipError_t sweep_enqueue_chunk(pm_sweep* s, hipStream_t st, int64_t chunk, int parity0, double tol,
                               int64_t max_steps) {
  hipError_t e = hipSuccess;
  for (int64_t t = 0; t < chunk && e == hipSuccess; ++t) {
    const int par = (int)((parity0 + t) & 1);
    if (s->dtype == PM_FP64)
      e = pm::launch_step_multi<double>((const pm::SweepCase<double>*)s->d_cases, s->d_sched, s->d_live,
                                        s->nsched, par, s->tile_w, s->tile_h, s->any_sr, st);
    else
      e = pm::launch_step_multi<float>((const pm::SweepCase<float>*)s->d_cases, s->d_sched, s->d_live,
                                       s->nsched, par, s->tile_w, s->tile_h, s->any_sr, st);
  }
  if (e != hipSuccess) return e;
  const int par_end = (int)((parity0 + chunk) & 1);
  if (s->dtype == PM_FP64)
    return pm::launch_resid_multi<double>((const pm::SweepCase<double>*)s->d_cases, s->ncases, s->d_sched,
                                          s->d_live, s->nsched, par_end, s->tile_w, s->tile_h,
                                          s->d_partial, s->d_st, chunk, tol, max_steps, st);
  return pm::launch_resid_multi<float>((const pm::SweepCase<float>*)s->d_cases, s->ncases, s->d_sched,
                                       s->d_live, s->nsched, par_end, s->tile_w, s->tile_h, s->d_partial,
                                       s->d_st, chunk, tol, max_steps, st);
}

void sweep_drop_graphs(pm_sweep* s) {
  for (auto& g : s->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

int sweep_graph(pm_sweep* s, int parity, int64_t chunk, double tol, int64_t max_steps) {
  if (s->graph_chunk != chunk || s->graph_tol != tol || s->graph_max != max_steps) {
    sweep_drop_graphs(s);
    s->graph_chunk = chunk;
    s->graph_tol = tol;
    s->graph_max = max_steps;
  }
  if (s->graph[parity]) return PM_OK;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  hipError_t le = sweep_enqueue_chunk(s, s->cap_stream, chunk, parity, tol, max_steps);
  e = hipStreamEndCapture(s->cap_stream, &g);
  if (le != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return sweep_fail(s, PM_EDEVICE, "capturing the sweep chunk: %s",
                      hipGetErrorString(le != hipSuccess ? le : e));
  }
  e = hipGraphInstantiate(&s->graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    s->graph[parity] = nullptr;
    return sweep_fail(s, PM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return PM_OK;
}

template <typename T> const pm::KParams<T>& kparams_of(const pm_ctx* c);
template <> const pm::KParams<float>& kparams_of<float>(const pm_ctx* c) { return c->k32; }
template <> const pm::KParams<double>& kparams_of<double>(const pm_ctx* c) { return c->k64; }

template <typename T>
void fill_case(pm_sweep* s, int i, pm_ctx* c) {
  pm::SweepCase<T> sc{};
  sc.p = kparams_of<T>(c);
  sc.snap = (T*)((char*)c->ws + c->lay.off_snap);
  sc.tiles_x = (c->p.nx + s->tile_w - 1) / s->tile_w;
  sc.ntiles = s->ntiles[i];
  sc.tile_base = s->tile_base[i];
  sc.pow = c->pow ? 1 : 0;
  memcpy(s->h_cases.data() + i * sizeof(sc), &sc, sizeof(sc));
}

// Tile counts, the case table and the schedule for the current tile shape.
void sweep_retile(pm_sweep* s) {
  int tb = 0;
  for (int i = 0; i < s->ncases; ++i) {
    const pm_params& p = s->ctx[i]->p;
    s->ntiles[i] = ((p.nx + s->tile_w - 1) / s->tile_w) * ((p.ny + s->tile_h - 1) / s->tile_h);
    s->tile_base[i] = tb;
    tb += s->ntiles[i];
    if (s->dtype == PM_FP64) fill_case<double>(s, i, s->ctx[i]);
    else fill_case<float>(s, i, s->ctx[i]);
  }
  s->total_tiles = tb;
  build_schedule(s);
}

}  // namespace

extern "C" {

int pm_sweep_workspace_bytes(const pm_params* cases, int ncases, size_t* bytes) {
  if (!bytes) return PM_EINVAL;
  SweepLayout L;
  char msg[256];
  int rc = sweep_layout(cases, ncases, L, msg, sizeof msg);
  if (rc) {
    set_global_err("%s", msg);
    return rc;
  }
  *bytes = L.total;
  return PM_OK;
}

int pm_sweep_create(const pm_params* cases, int ncases, void* dev_ws, size_t ws_bytes, void* hip_stream,
                    pm_sweep** out) {
  if (!out) return PM_EINVAL;
  *out = nullptr;
  SweepLayout L;
  char msg[256];
  int rc = sweep_layout(cases, ncases, L, msg, sizeof msg);
  if (rc) {
    set_global_err("%s", msg);
    return rc;
  }
  if (!dev_ws || ws_bytes < L.total) {
    set_global_err("pm_sweep_create: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);
    return PM_ESTATE;
  }
  if (((uintptr_t)dev_ws) % ALIGN) {
    set_global_err("pm_sweep_create: workspace must be %zu-byte aligned", ALIGN);
    return PM_EINVAL;
  }
  pm_sweep* s = new (std::nothrow) pm_sweep();
  if (!s) return PM_EDEVICE;
  s->ncases = ncases;
  s->dtype = cases[0].dtype;
  s->order = PM_ORDER_CASE;
  s->stream = (hipStream_t)hip_stream;
  s->tile_w = pm::TILE;
  s->tile_h = 1;
  s->any_sr = false;
  for (int i = 0; i < ncases; ++i)
    if (rounds_stochastically(cases[i])) s->any_sr = true;
  char* base = (char*)dev_ws;
  s->d_cases = base + L.off_cases;
  s->d_sched = (int2*)(base + L.off_sched);
  s->d_live = (int*)(base + L.off_live);
  s->d_st = (pm::SweepStatus*)(base + L.off_st);
  s->d_partial = (double*)(base + L.off_partial);
  s->graph_chunk = -1;
  s->ctx.assign(ncases, nullptr);
  s->ntiles.resize(ncases);
  s->tile_base.resize(ncases);
  const size_t case_sz = s->dtype == PM_FP64 ? sizeof(pm::SweepCase<double>) : sizeof(pm::SweepCase<float>);
  s->h_cases.assign(ncases * case_sz, 0);
  for (int i = 0; i < ncases; ++i) {
    rc = init_ctx(&cases[i], base + L.off[i], L.bytes[i], hip_stream, false, &s->ctx[i]);
    if (rc) {
      snprintf(s->err, sizeof s->err, "case %d: %s", i, g_last_err);
      set_global_err("%s", s->err);
      pm_sweep_destroy(s);
      return rc;
    }
  }
  sweep_retile(s);
  s->h_live.assign(ncases, 1);
  s->h_st.assign(ncases, pm::SweepStatus{0, INFINITY});
  hipError_t e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_cases, s->h_cases.data(), s->h_cases.size(), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_sched, s->h_sched.data(), s->h_sched.size() * sizeof(int2), hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_live, s->h_live.data(), ncases * sizeof(int), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_st, s->h_st.data(), ncases * sizeof(pm::SweepStatus), hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    set_global_err("pm_sweep_create: %s", hipGetErrorString(e));
    pm_sweep_destroy(s);
    return PM_EDEVICE;
  }
  *out = s;
  return PM_OK;
}

int pm_sweep_set_order(pm_sweep* s, int order) {
  if (!s) return PM_EINVAL;
  if (order < PM_ORDER_CASE || order > PM_ORDER_INTERLEAVE)
    return sweep_fail(s, PM_EINVAL, "pm_sweep_set_order: unknown order %d", order);
  s->order = order;
  build_schedule(s);
  sweep_drop_graphs(s);
  hipError_t e = hipMemcpyAsync(s->d_sched, s->h_sched.data(), s->h_sched.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_set_order: %s", hipGetErrorString(e));
  return PM_OK;
}

int pm_sweep_set_tile(pm_sweep* s, int tile_w, int tile_h) {
  if (!s) return PM_EINVAL;
  if (!pm::sweep_tile_ok(tile_w, tile_h))
    return sweep_fail(s, PM_EINVAL, "pm_sweep_set_tile: %d x %d is not a supported tile (width 64, 128 or 256, "
                      "height 1, 2 or 4, at most %d threads)", tile_w, tile_h, pm::TILE);
  // the previous tile shape's launches may still read the case table
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_set_tile: %s", hipGetErrorString(e));
  s->tile_w = tile_w;
  s->tile_h = tile_h;
  sweep_retile(s);
  sweep_drop_graphs(s);
  e = hipMemcpyAsync(s->d_cases, s->h_cases.data(), s->h_cases.size(), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_sched, s->h_sched.data(), s->h_sched.size() * sizeof(int2), hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_set_tile: %s", hipGetErrorString(e));
  return PM_OK;
}

int pm_sweep_advance(pm_sweep* s, double tol, int64_t check_every, int64_t max_steps, int64_t max_chunks,
                     int* nlive) {
  if (!s) return PM_EINVAL;
  if (check_every <= 0 || max_steps < 0 || max_chunks <= 0)
    return sweep_fail(s, PM_EINVAL, "pm_sweep_advance: bad chunk, cap or chunk budget");
  hipError_t e = hipSuccess;
  int live = 0;
  for (int64_t chunk = 0;; ++chunk) {
    live = 0;
    for (int i = 0; i < s->ncases; ++i) live += s->h_live[i];
    if (!live || chunk >= max_chunks) break;
    // every live case has taken gsteps steps: stop them all at the cap, and
    // shorten the chunk that reaches it, as pm_run_to_steady shortens its last
    if (s->gsteps >= max_steps) {
      std::fill(s->h_live.begin(), s->h_live.end(), 0);
      e = hipMemcpyAsync(s->d_live, s->h_live.data(), s->ncases * sizeof(int), hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_advance: %s", hipGetErrorString(e));
      live = 0;
      break;
    }
    const int64_t k = std::min(check_every, max_steps - s->gsteps);
    const int parity = (int)(s->gsteps & 1);
    if (k == check_every) {
      int rc = sweep_graph(s, parity, check_every, tol, max_steps);
      if (rc) return rc;
      e = hipGraphLaunch(s->graph[parity], s->stream);
      if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
    } else {
      e = sweep_enqueue_chunk(s, s->stream, k, parity, tol, max_steps);
      if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_advance: %s", hipGetErrorString(e));
    }
    s->gsteps += k;
    e = hipMemcpyAsync(s->h_live.data(), s->d_live, s->ncases * sizeof(int), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_advance: %s", hipGetErrorString(e));
    // cases stopped in this chunk: schedule only the live ones from now on
    int now_live = 0;
    for (int i = 0; i < s->ncases; ++i) now_live += s->h_live[i];
    if (now_live && now_live < s->sched_live) {
      build_schedule(s);
      sweep_drop_graphs(s);
      e = hipMemcpyAsync(s->d_sched, s->h_sched.data(), s->h_sched.size() * sizeof(int2), hipMemcpyHostToDevice,
                         s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_advance: %s", hipGetErrorString(e));
    }
  }
  e = hipMemcpyAsync(s->h_st.data(), s->d_st, s->ncases * sizeof(pm::SweepStatus), hipMemcpyDeviceToHost,
                     s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_advance: %s", hipGetErrorString(e));
  for (int i = 0; i < s->ncases; ++i) s->ctx[i]->steps = s->h_st[i].steps;
  if (nlive) *nlive = live;
  return PM_OK;
}

int pm_sweep_run(pm_sweep* s, double tol, int64_t check_every, int64_t max_steps, int64_t* steps_out,
                 double* r_out) {
  int live = 1;
  while (live) {
    int rc = pm_sweep_advance(s, tol, check_every, max_steps, INT64_MAX, &live);
    if (rc) return rc;
  }
  return pm_sweep_status(s, steps_out, r_out);
}

int pm_sweep_status(const pm_sweep* s, int64_t* steps_out, double* r_out) {
  if (!s) return PM_EINVAL;
  int rc = PM_OK;
  for (int i = 0; i < s->ncases; ++i) {
    if (steps_out) steps_out[i] = s->h_st[i].steps;
    if (r_out) r_out[i] = s->h_st[i].residual;
    if (!(s->h_st[i].residual <= 1.7976931348623157e308) && !s->h_live[i] && s->h_st[i].steps > 0) rc = PM_EDIVERGED;
  }
  if (rc) sweep_fail((pm_sweep*)s, rc, "a case stopped on a NaN/Inf residual");
  return rc;
}

int pm_sweep_step(pm_sweep* s, int64_t k) {
  if (!s) return PM_EINVAL;
  if (k < 0) return sweep_fail(s, PM_EINVAL, "pm_sweep_step: k must be >= 0");
  hipError_t e = hipSuccess;
  for (int64_t t = 0; t < k && e == hipSuccess; ++t) {
    const int par = (int)((s->gsteps + t) & 1);
    if (s->dtype == PM_FP64)
      e = pm::launch_step_multi<double>((const pm::SweepCase<double>*)s->d_cases, s->d_sched, s->d_live,
                                        s->nsched, par, s->tile_w, s->tile_h, s->any_sr, s->stream);
    else
      e = pm::launch_step_multi<float>((const pm::SweepCase<float>*)s->d_cases, s->d_sched, s->d_live,
                                       s->nsched, par, s->tile_w, s->tile_h, s->any_sr, s->stream);
  }
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_step: %s", hipGetErrorString(e));
  // live cases advance together; the per-case counters follow on the device
  // only through pm_sweep_run, so keep the host copies in step here
  s->gsteps += k;
  for (int i = 0; i < s->ncases; ++i)
    if (s->h_live[i]) {
      s->ctx[i]->steps += k;
      s->h_st[i].steps += k;
    }
  e = hipMemcpyAsync(s->d_st, s->h_st.data(), s->ncases * sizeof(pm::SweepStatus), hipMemcpyHostToDevice,
                     s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return sweep_fail(s, PM_EDEVICE, "pm_sweep_step: %s", hipGetErrorString(e));
  return PM_OK;
}

int pm_sweep_case(pm_sweep* s, int i, pm_ctx** out) {
  if (!s || !out) return PM_EINVAL;
  if (i < 0 || i >= s->ncases) return sweep_fail(s, PM_EINVAL, "pm_sweep_case: index %d out of range", i);
  *out = s->ctx[i];
  return PM_OK;
}

void pm_sweep_destroy(pm_sweep* s) {
  if (!s) return;
  sweep_drop_graphs(s);
  for (pm_ctx* c : s->ctx) pm_destroy(c);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

const char* pm_sweep_last_error(const pm_sweep* s) { return s ? s->err : g_last_err; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint (gradients of the Nusselt number)
// ---------------------------------------------------------------------------
struct pm_adjoint {
  pm_ctx* ctx;
  int64_t T, C, ncp, s0;
  size_t span;          // bytes of one raw population state (the population region)
  char* cp;             // ncp checkpoints
  char* seg[2];         // C + 1 states of a replayed segment, double-buffered
  hipStream_t replay;   // segment replays run here, one segment ahead of the adjoint
  hipEvent_t ev_start, ev_rep[2], ev_used[2];
  void* lam[2];         // adjoint state, natural layout [14][ny][nx], FP64 or FP32 (lam_dtype)
  int lam_dtype;        // PM_FP64 (default) or PM_FP32
  double* partial;      // pm::ADJ_PART doubles per workgroup
  int nblocks;
  double J;
  bool have_forward;
  pm::AdjParams ap;
  char err[512];
};

namespace {

struct AdjLayout {
  size_t span, off_cp, off_seg, off_lam0, off_lam1, off_partial, total;
  int64_t ncp;
  int nblocks;
};

int adj_layout(const pm_params& p, int64_t T, int64_t C, AdjLayout& A, char* msg, size_t len) {
  pm_lattice L;
  int rc = map_params(p, L, msg, len);
  if (rc) return rc;
  if (T < 1 || C < 1 || C > T) {
    snprintf(msg, len, "adjoint: need T >= 1 and 1 <= C <= T");
    return PM_EINVAL;
  }
  if (p.periodic_x || p.periodic_y) {
    snprintf(msg, len, "adjoint: periodic axes are not supported (cavity walls only)");
    return PM_EINVAL;
  }
  if (p.clamp_mode != PM_CLAMP_NU) {
    snprintf(msg, len, "adjoint: only PM_CLAMP_NU is supported");
    return PM_EINVAL;
  }
  if (p.dtype == PM_FP16) {
    snprintf(msg, len, "adjoint: FP16 storage is not supported (FP32 or FP64 forward states)");
    return PM_EINVAL;
  }
  if (p.gx != 0.0 || p.gy != 0.0) {
    snprintf(msg, len, "adjoint: extra body forces are not supported");
    return PM_EINVAL;
  }
  const Layout lay = layout_of(p);
  const int64_t nn = (int64_t)p.nx * p.ny;
  A.span = lay.pop_bytes;
  A.ncp = (T + C - 1) / C;
  A.nblocks = ((p.nx + pm::TILE - 1) / pm::TILE) * p.ny;
  size_t o = 0;
  A.off_cp = o;
  o = align_up(o + A.ncp * align_up(A.span));
  A.off_seg = o;
  o = align_up(o + 2 * (C + 1) * align_up(A.span));
  A.off_lam0 = o;
  o = align_up(o + 14 * nn * sizeof(double));
  A.off_lam1 = o;
  o = align_up(o + 14 * nn * sizeof(double));
  A.off_partial = o;
  o = align_up(o + pm::ADJ_PART * (size_t)A.nblocks * sizeof(double));
  A.total = o;
  return PM_OK;
}

pm::AdjParams adj_params(const pm_ctx* c) {
  pm::AdjParams a{};
  const pm_params& p = c->p;
  const pm_lattice& L = c->L;
  a.nx = p.nx;
  a.ny = p.ny;
  a.has_logda = p.has_logda ? 1 : 0;
  a.pow = c->pow ? 1 : 0;
  a.eps = L.eps;
  a.inv_eps = 1.0 / L.eps;
  a.Feps = L.Feps;
  a.invK = std::isinf(L.K) ? 0.0 : 1.0 / L.K;
  a.invsK = std::sqrt(a.invK);
  a.inv_Kscale = 1.0 / ((double)p.nx * (double)p.nx);
  a.gbeta = L.gbeta;
  a.dTm = L.T_m - 0.5;
  a.gx = p.gx;
  a.gy = p.gy;
  a.s_e = L.s_e;
  a.s_eps = L.s_eps;
  a.s_q = L.s_q;
  a.s_g = 1.0 / L.tau_g;
  a.sT_e = L.sT_e;
  a.sT_nu = L.sT_nu;
  a.T_ref = 0.5;
  a.nu0 = L.nu0;
  a.log2nu0 = std::log2(L.nu0);
  a.y_lo = std::log2(L.nu_min);
  a.y_hi = std::log2(L.nu_max);
  a.nm1 = p.n - 1.0;
  a.inv_n = 1.0 / p.n;
  a.log2c = std::log2(L.gamma_scale);
  a.lc0 = a.log2nu0 + a.nm1 * a.log2c;
  a.g2_floor = 0.0;
  return a;
}

template <typename T>
pm::KParams<T> slot_params(const pm_ctx* c, const pm::KParams<T>& base, char* slot) {
  pm::KParams<T> k = base;
  k.f = (T*)slot;
  k.g = (T*)(slot + c->lay.off_g);
  return k;
}

int adj_fail(pm_adjoint* a, int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(a ? a->err : g_last_err, 512, fmt, ap);
  va_end(ap);
  return code;
}

// One adjoint step at a raw state (parity given), lam_next -> lam.
hipError_t adj_step(const pm_ctx* c, const pm::AdjParams& ap, char* state, int parity, const double* lam_next,
                    double* lam, double* g_logda, double* partial) {
  if (c->p.dtype == PM_FP64)
    return pm::launch_adjoint<double, double>(slot_params<double>(c, c->k64, state), ap, parity, lam_next, lam,
                                              g_logda, partial, c->stream);
  return pm::launch_adjoint<float, double>(slot_params<float>(c, c->k32, state), ap, parity, lam_next, lam,
                                           g_logda, partial, c->stream);
}

// The same with an FP32-stored adjoint state (FP32 forward states only).
hipError_t adj_step(const pm_ctx* c, const pm::AdjParams& ap, char* state, int parity, const float* lam_next,
                    float* lam, double* g_logda, double* partial) {
  return pm::launch_adjoint<float, float>(slot_params<float>(c, c->k32, state), ap, parity, lam_next, lam,
                                          g_logda, partial, c->stream);
}

// Chain rule from the per-node parameters (ln nu0, n at fixed nu0, s_g) to
// (n, Ra): nu0 = Pr / sqrt(Ra)^(2-n) U N, alpha = U N / sqrt(Ra),
// s_g = 1 / (3 alpha + 1/2).
// Fixed-order host sum of the per-workgroup partials; largest |lambda|.
void reduce_partials(const std::vector<double>& part, double sums[3], double& lam_max) {
  sums[0] = sums[1] = sums[2] = 0.0;
  lam_max = 0.0;
  for (size_t b = 0; b < part.size() / pm::ADJ_PART; ++b) {
    for (int q = 0; q < 3; ++q) sums[q] += part[pm::ADJ_PART * b + q];
    const double m = part[pm::ADJ_PART * b + 3];
    lam_max = (m != m) ? INFINITY : std::max(lam_max, m);
  }
}

// Bound on |lambda| relative to the seed (whose own size is 3 nx / ny): an
// adjoint state this large means the backward sweep is amplifying, not
// transporting, sensitivities.
constexpr double ADJ_LAMBDA_LIMIT = 1e12;

void chain_scalars(const pm_ctx* c, const double* sums, double* d_n, double* d_Ra) {
  const double n = c->p.n, Ra = c->p.Ra;
  const double sg = 1.0 / c->L.tau_g, alpha = c->L.alpha;
  if (d_n) *d_n = sums[1] + 0.5 * std::log(Ra) * sums[0];
  if (d_Ra) *d_Ra = -(2.0 - n) / (2.0 * Ra) * sums[0] + 1.5 * sg * sg * alpha / Ra * sums[2];
}

}  // namespace

extern "C" {

int pm_adjoint_workspace_bytes(const pm_params* p, int64_t T, int64_t C, size_t* bytes) {
  if (!p || !bytes) return PM_EINVAL;
  AdjLayout A;
  char msg[256];
  int rc = adj_layout(*p, T, C, A, msg, sizeof msg);
  if (rc) {
    set_global_err("%s", msg);
    return rc;
  }
  *bytes = A.total;
  return PM_OK;
}

int pm_adjoint_create(pm_ctx* c, int64_t T, int64_t C, void* dev_ws, size_t ws_bytes, pm_adjoint** out) {
  if (!c || !out) return PM_EINVAL;
  *out = nullptr;
  AdjLayout A;
  char msg[256];
  int rc = adj_layout(c->p, T, C, A, msg, sizeof msg);
  if (rc) {
    set_global_err("%s", msg);
    return rc;
  }
  if (!dev_ws || ws_bytes < A.total || ((uintptr_t)dev_ws) % ALIGN) {
    set_global_err("pm_adjoint_create: workspace must be %zu-byte aligned and >= %zu bytes", ALIGN, A.total);
    return PM_ESTATE;
  }
  pm_adjoint* a = new (std::nothrow) pm_adjoint();
  if (!a) return PM_EDEVICE;
  hipError_t e = hipStreamCreateWithFlags(&a->replay, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&a->ev_start, hipEventDisableTiming);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&a->ev_rep[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a->ev_used[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    set_global_err("pm_adjoint_create: %s", hipGetErrorString(e));
    pm_adjoint_destroy(a);
    return PM_EDEVICE;
  }
  a->ctx = c;
  a->T = T;
  a->C = C;
  a->ncp = A.ncp;
  a->span = A.span;
  char* b = (char*)dev_ws;
  a->cp = b + A.off_cp;
  a->seg[0] = b + A.off_seg;
  a->seg[1] = a->seg[0] + (C + 1) * align_up(A.span);
  a->lam[0] = b + A.off_lam0;
  a->lam[1] = b + A.off_lam1;
  a->lam_dtype = PM_FP64;
  a->partial = (double*)(b + A.off_partial);
  a->nblocks = A.nblocks;
  a->ap = adj_params(c);
  *out = a;
  return PM_OK;
}

int pm_adjoint_forward(pm_adjoint* a, double* J_out) {
  if (!a) return PM_EINVAL;
  pm_ctx* c = a->ctx;
  a->s0 = c->steps;
  const size_t stride = align_up(a->span);
  for (int64_t k = 0; k < a->ncp; ++k) {
    hipError_t e = hipMemcpyAsync(a->cp + k * stride, (char*)c->ws + c->lay.off_f, a->span,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return adj_fail(a, PM_EDEVICE, "checkpoint copy: %s", hipGetErrorString(e));
    const int64_t n = std::min(a->C, a->T - k * a->C);
    int rc = pm_step(c, n);
    if (rc) return adj_fail(a, rc, "forward: %s", c->err);
  }
  int rc = pm_nu(c, &a->J);
  if (rc) return adj_fail(a, rc, "forward: %s", c->err);
  a->have_forward = true;
  if (J_out) *J_out = a->J;
  return PM_OK;
}

int pm_adjoint_backward(pm_adjoint* a, double seed, void* grad_logda, double* grad_n, double* grad_Ra) {
  if (!a) return PM_EINVAL;
  if (!a->have_forward) return adj_fail(a, PM_ESTATE, "pm_adjoint_backward: run pm_adjoint_forward first");
  pm_ctx* c = a->ctx;
  if (c->p.has_logda && !grad_logda) return adj_fail(a, PM_EINVAL, "pm_adjoint_backward: grad_logda needed");
  const int64_t nn = (int64_t)c->p.nx * c->p.ny;
  hipError_t e = hipMemsetAsync(a->partial, 0, pm::ADJ_PART * (size_t)a->nblocks * sizeof(double), c->stream);
  if (e == hipSuccess && grad_logda) e = hipMemsetAsync(grad_logda, 0, nn * sizeof(double), c->stream);
  const bool lam32 = a->lam_dtype == PM_FP32;
  if (e == hipSuccess)
    e = lam32 ? pm::launch_adjoint_seed(c->p.nx, c->p.ny, seed, (float*)a->lam[0], c->stream)
              : pm::launch_adjoint_seed(c->p.nx, c->p.ny, seed, (double*)a->lam[0], c->stream);
  if (e != hipSuccess) return adj_fail(a, PM_EDEVICE, "backward setup: %s", hipGetErrorString(e));
  const size_t stride = align_up(a->span);
  const bool logda = c->p.has_logda != 0;
  // Replay of segment k: from its checkpoint, out of place, into C + 1 slots
  // (slot t holds S_{kC + t}), on the replay stream.
  pm::Launch rl = c->launch;
  rl.stream = a->replay;
  auto replay = [&](int64_t k, char* seg) -> hipError_t {
    const int64_t start = k * a->C;
    const int64_t n = std::min(a->C, a->T - start);
    hipError_t r = hipMemcpyAsync(seg, a->cp + k * stride, a->span, hipMemcpyDeviceToDevice, a->replay);
    for (int64_t t = 0; t < n && r == hipSuccess; ++t) {
      const int parity = (int)((a->s0 + start + t) & 1);
      char* src = seg + t * stride;
      char* dst = seg + (t + 1) * stride;
      if (c->p.dtype == PM_FP64)
        r = pm::launch_step_oop(slot_params<double>(c, c->k64, src), slot_params<double>(c, c->k64, dst), rl,
                                parity, c->pow, logda);
      else
        r = pm::launch_step_oop(slot_params<float>(c, c->k32, src), slot_params<float>(c, c->k32, dst), rl,
                                parity, c->pow, logda);
    }
    return r;
  };
  // The replay of segment k - 1 runs while the adjoint steps of segment k
  // run on the context's stream: buffer b holds segment k, b ^ 1 receives
  // k - 1 once segment k + 1's adjoint steps have finished reading it.
  if (e == hipSuccess) e = hipEventRecord(a->ev_start, c->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(a->replay, a->ev_start, 0);
  if (e == hipSuccess) e = replay(a->ncp - 1, a->seg[0]);
  if (e == hipSuccess) e = hipEventRecord(a->ev_rep[0], a->replay);
  int cur = 0;
  for (int64_t k = a->ncp - 1; k >= 0 && e == hipSuccess; --k) {
    const int b = (int)((a->ncp - 1 - k) & 1);
    if (k >= 1) {
      if (k + 1 <= a->ncp - 1) e = hipStreamWaitEvent(a->replay, a->ev_used[b ^ 1], 0);
      if (e == hipSuccess) e = replay(k - 1, a->seg[b ^ 1]);
      if (e == hipSuccess) e = hipEventRecord(a->ev_rep[b ^ 1], a->replay);
    }
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, a->ev_rep[b], 0);
    // adjoint steps in reverse over the segment
    const int64_t start = k * a->C;
    const int64_t n = std::min(a->C, a->T - start);
    for (int64_t t = n - 1; t >= 0 && e == hipSuccess; --t) {
      const int parity = (int)((a->s0 + start + t) & 1);
      char* st = a->seg[b] + t * stride;
      e = lam32 ? adj_step(c, a->ap, st, parity, (const float*)a->lam[cur], (float*)a->lam[cur ^ 1],
                           (double*)grad_logda, a->partial)
                : adj_step(c, a->ap, st, parity, (const double*)a->lam[cur], (double*)a->lam[cur ^ 1],
                           (double*)grad_logda, a->partial);
      cur ^= 1;
    }
    if (e == hipSuccess) e = hipEventRecord(a->ev_used[b], c->stream);
  }
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(a->replay);
    return adj_fail(a, PM_EDEVICE, "backward: %s", hipGetErrorString(e));
  }
  std::vector<double> part(pm::ADJ_PART * (size_t)a->nblocks);
  e = hipMemcpyAsync(part.data(), a->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return adj_fail(a, PM_EDEVICE, "backward: %s", hipGetErrorString(e));
  double sums[3], lam_max;
  reduce_partials(part, sums, lam_max);
  chain_scalars(c, sums, grad_n, grad_Ra);
  const double limit = ADJ_LAMBDA_LIMIT * std::fabs(seed) * std::max(1.0, (double)c->p.nx / c->p.ny);
  if (!(lam_max <= limit) || !std::isfinite(sums[0]) || !std::isfinite(sums[1]) || !std::isfinite(sums[2]))
    return adj_fail(a, PM_EDIVERGED,
                    "pm_adjoint_backward: the adjoint state grew to %.3g (limit %.3g): the linearised update "
                    "amplifies perturbations on this trajectory (for n < 1, where low shear meets the Darcy "
                    "drag); pm_adjoint_set_shear_floor gives a regularised gradient",
                    lam_max, limit);
  return PM_OK;
}

int pm_adjoint_set_shear_floor(pm_adjoint* a, double gamma_floor) {
  if (!a) return PM_EINVAL;
  if (!(gamma_floor >= 0.0) || std::isinf(gamma_floor))
    return adj_fail(a, PM_EINVAL, "pm_adjoint_set_shear_floor: need a finite gamma_floor >= 0");
  const double g = gamma_floor / a->ctx->L.gamma_scale;  // nondimensional -> lattice
  a->ap.g2_floor = g * g;
  return PM_OK;
}

int pm_adjoint_set_lambda_dtype(pm_adjoint* a, int dtype) {
  if (!a) return PM_EINVAL;
  if (dtype != PM_FP64 && dtype != PM_FP32)
    return adj_fail(a, PM_EINVAL, "pm_adjoint_set_lambda_dtype: PM_FP64 or PM_FP32");
  if (dtype == PM_FP32 && a->ctx->p.dtype != PM_FP32)
    return adj_fail(a, PM_EINVAL, "pm_adjoint_set_lambda_dtype: an FP32 adjoint state needs FP32 forward states");
  a->lam_dtype = dtype;
  return PM_OK;
}

void pm_adjoint_destroy(pm_adjoint* a) {
  if (!a) return;
  if (a->replay) {
    (void)hipStreamSynchronize(a->replay);
    (void)hipStreamDestroy(a->replay);
  }
  for (hipEvent_t ev : {a->ev_start, a->ev_rep[0], a->ev_rep[1], a->ev_used[0], a->ev_used[1]})
    if (ev) (void)hipEventDestroy(ev);
  delete a;
}

const char* pm_adjoint_last_error(const pm_adjoint* a) { return a ? a->err : g_last_err; }

size_t pm_adjoint_vjp_scratch_bytes(const pm_ctx* c) {
  if (!c) return 0;
  return pm::ADJ_PART * (size_t)c->launch.ntiles * sizeof(double);
}

int pm_adjoint_vjp(pm_ctx* c, const void* lam_next, void* lam, void* grad_logda, void* dev_scratch,
                   size_t scratch_bytes, double* grad_scalars) {
  if (!c || !lam_next || !lam || !dev_scratch) return PM_EINVAL;
  if (c->p.periodic_x || c->p.periodic_y || c->p.clamp_mode != PM_CLAMP_NU || c->p.gx != 0.0 || c->p.gy != 0.0 ||
      c->p.dtype == PM_FP16)
    return ctx_fail(c, PM_EINVAL, "pm_adjoint_vjp: cavity walls, PM_CLAMP_NU, no body force, FP32/FP64 only");
  if (c->p.has_logda && !grad_logda) return ctx_fail(c, PM_EINVAL, "pm_adjoint_vjp: grad_logda needed");
  const size_t need = pm_adjoint_vjp_scratch_bytes(c);
  if (scratch_bytes < need) return ctx_fail(c, PM_ESTATE, "pm_adjoint_vjp: scratch < %zu bytes", need);
  hipError_t e = hipMemsetAsync(dev_scratch, 0, need, c->stream);
  if (e == hipSuccess)
    e = adj_step(c, adj_params(c), (char*)c->ws + c->lay.off_f, (int)(c->steps & 1), (const double*)lam_next,
                 (double*)lam, (double*)grad_logda, (double*)dev_scratch);
  std::vector<double> part(need / sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), dev_scratch, need, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pm_adjoint_vjp");
  double sums[3], lam_max;
  reduce_partials(part, sums, lam_max);
  if (grad_scalars) chain_scalars(c, sums, &grad_scalars[0], &grad_scalars[1]);
  return PM_OK;
}

}  // extern "C"

// ---- allocation-free adjoint step ----
// The per-workgroup partials of pm_adjoint_vjp_noalloc live in this
// file-scope device array instead of caller scratch: ADJ_PART doubles for
// each of up to NOALLOC_MAX_WG workgroups, then the ADJ_PART reduced values
// (2 MiB + 32 B on each device, held until the process ends).  Host code
// never passes the array's name to a kernel: it takes the array's device
// address once per device with hipGetSymbolAddress and uses that.
namespace {

constexpr int NOALLOC_MAX_WG = 65536;
constexpr size_t NOALLOC_OUT = (size_t)pm::ADJ_PART * NOALLOC_MAX_WG;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[NOALLOC_OUT + pm::ADJ_PART];

std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES];  // device address of scratch, per device

// The address of this device's copy of scratch (looked up on the first call
// on the device, which must be current).
int noalloc_scratch(pm_ctx* c, double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(c, e, "pm_adjoint_vjp_noalloc: hipGetDevice");
  if (dev != c->device)
    return ctx_fail(c, PM_EINVAL, "pm_adjoint_vjp_noalloc: make the context's device (%d) current, not %d",
                    c->device, dev);
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return ctx_fail(c, PM_EINVAL, "pm_adjoint_vjp_noalloc: device %d beyond the %d supported", dev,
                    NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return check_hip(c, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                  "pm_adjoint_vjp_noalloc: hipGetSymbolAddress");
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return PM_OK;
}

}  // namespace

extern "C" {

int pm_adjoint_vjp_noalloc(pm_ctx* c, const void* lam_next, void* lam, void* grad_logda, double* grad_scalars) {
  if (!c || !lam_next || !lam) return PM_EINVAL;
  if (c->p.periodic_x || c->p.periodic_y || c->p.clamp_mode != PM_CLAMP_NU || c->p.gx != 0.0 || c->p.gy != 0.0 ||
      c->p.dtype == PM_FP16)
    return ctx_fail(c, PM_EINVAL,
                    "pm_adjoint_vjp_noalloc: cavity walls, PM_CLAMP_NU, no body force, FP32/FP64 only");
  if (c->p.has_logda && !grad_logda) return ctx_fail(c, PM_EINVAL, "pm_adjoint_vjp_noalloc: grad_logda needed");
  const int nblocks = c->launch.ntiles;
  if (nblocks > NOALLOC_MAX_WG)
    return ctx_fail(c, PM_EINVAL,
                    "pm_adjoint_vjp_noalloc: the grid needs %d workgroup slots, the static scratch holds %d "
                    "(ceil(nx / %d) * ny must not exceed it); use pm_adjoint_vjp with caller scratch",
                    nblocks, NOALLOC_MAX_WG, pm::TILE);
  double* ptr = nullptr;
  int rc = noalloc_scratch(c, &ptr);
  if (rc) return rc;
  hipError_t e = pm::launch_fill_zero(ptr, (int64_t)pm::ADJ_PART * nblocks, c->stream);
  if (e == hipSuccess)
    e = adj_step(c, adj_params(c), (char*)c->ws + c->lay.off_f, (int)(c->steps & 1), (const double*)lam_next,
                 (double*)lam, (double*)grad_logda, ptr);
  if (e == hipSuccess) e = pm::launch_adj_reduce(ptr, nblocks, ptr + NOALLOC_OUT, c->stream);
  double out[pm::ADJ_PART];
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, ptr + NOALLOC_OUT, sizeof out, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pm_adjoint_vjp_noalloc");
  if (grad_scalars) chain_scalars(c, out, &grad_scalars[0], &grad_scalars[1]);
  return PM_OK;
}

const char* pm_strerror(int code) {
  switch (code) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_EDEVICE: return "HIP device error";
    case PM_EDIVERGED: return "simulation diverged (NaN/Inf)";
    case PM_ESTATE: return "buffer size or state mismatch";
    default: return "unknown error";
  }
}

const char* pm_last_error(const pm_ctx* c) { return c ? c->err : g_last_err; }

}  // extern "C"
