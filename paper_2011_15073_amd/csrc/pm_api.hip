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
#include <type_traits>

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
  size_t elem, P;  // element size, plane pitch (elements)
  size_t off_f, off_g, off_logda, off_snap, off_red, total;
};

Layout layout_of(const pm_params& p) {
  Layout L{};
  L.elem = p.dtype == PM_FP64 ? 8 : 4;
  const size_t n = (size_t)p.nx * (size_t)p.ny;
  L.P = (n + 63) / 64 * 64 + PM_PITCH_SKEW;
  size_t o = 0;
  L.off_f = o;
  o = align_up(o + 9 * L.P * L.elem);
  L.off_g = o;
  o = align_up(o + 5 * L.P * L.elem);
  L.off_logda = o;
  if (p.has_logda) o = align_up(o + L.P * L.elem);
  L.off_snap = o;
  o = align_up(o + L.P * L.elem);
  L.off_red = o;
  o = align_up(o + (pm::RED_BLOCKS + 16) * sizeof(double));
  L.total = o;
  return L;
}

// Step 0 of the update: physical groups -> lattice values (see pmlbm.h).
int map_params(const pm_params& p, pm_lattice& L, char* msg, size_t msglen) {
  auto fail = [&](const char* m) {
    snprintf(msg, msglen, "%s", m);
    return PM_EINVAL;
  };
  if (p.nx < 2 || p.ny < 2) return fail("nx and ny must be >= 2");
  if ((double)p.nx * (double)p.ny > 2147483647.0 / 2) return fail("grid too large for 32-bit node indices");
  if (p.dtype != PM_FP32 && p.dtype != PM_FP64) return fail("dtype must be PM_FP32 or PM_FP64");
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

template <typename T>
pm::KParams<T> kparams(const pm_params& p, const pm_lattice& L, void* ws, const Layout& lay) {
  pm::KParams<T> k{};
  char* base = (char*)ws;
  k.f = (T*)(base + lay.off_f);
  k.g = (T*)(base + lay.off_g);
  k.logda = p.has_logda ? (const T*)(base + lay.off_logda) : nullptr;
  k.P = (int64_t)lay.P;
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
  return fn(c->k32);
}

hipError_t enqueue_steps(pm_ctx* c, hipStream_t s, int64_t k, int64_t start_steps) {
  pm::Launch L = c->launch;
  L.stream = s;
  const bool logda = c->p.has_logda != 0;
  for (int64_t t = 0; t < k; ++t) {
    const int parity = (int)((start_steps + t) & 1);
    hipError_t e = dispatch(c, [&](auto& kp) { return pm::launch_step(kp, L, parity, c->pow, logda); });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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

int dtype_ok(int d) { return d == PM_FP32 || d == PM_FP64; }

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
  *bytes = layout_of(*p).total;
  return PM_OK;
}

int pm_init(const pm_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, pm_ctx** out) {
  if (!out) {
    set_global_err("pm_init: null out pointer");
    return PM_EINVAL;
  }
  *out = nullptr;
  pm_lattice L;
  int rc = pm_lattice_of(p, &L);
  if (rc) return rc;
  Layout lay = layout_of(*p);
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
  c->launch.stream = c->stream;
  c->launch.tiles_x = (p->nx + pm::TILE - 1) / pm::TILE;
  c->launch.ntiles = c->launch.tiles_x * p->ny;
  c->red = (double*)((char*)dev_ws + lay.off_red);
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    set_global_err("hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    delete c;
    return PM_EDEVICE;
  }
  const double dg_init = (1.0 / 6.0) * (p->T_init - 0.5);
  e = dispatch(c, [&](auto& kp) {
    using T = typename std::remove_reference_t<decltype(*kp.f)>;
    return pm::launch_init(kp, c->launch, (T)dg_init);
  });
  if (e == hipSuccess)
    e = dispatch(c, [&](auto& kp) {
      using T = typename std::remove_reference_t<decltype(*kp.f)>;
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
    using T = typename std::remove_reference_t<decltype(*kp.f)>;
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

int pm_residual(pm_ctx* c, double* r_out) {
  if (!c || !r_out) return PM_EINVAL;
  const int parity = (int)(c->steps & 1);
  double* dev = c->red + pm::RED_BLOCKS;
  hipError_t e = dispatch(c, [&](auto& kp) {
    using T = typename std::remove_reference_t<decltype(*kp.f)>;
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
    rc = pm_residual(c, &r);
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
  *bytes = HEADER_BYTES + 14 * c->lay.P * c->lay.elem;
  return PM_OK;
}

int pm_save_state(pm_ctx* c, void* dst, size_t bytes) {
  if (!c || !dst) return PM_EINVAL;
  size_t need;
  pm_state_bytes(c, &need);
  if (bytes < need) return ctx_fail(c, PM_ESTATE, "pm_save_state: buffer of %zu bytes < %zu", bytes, need);
  const uint64_t tag = STATE_TAG ^ ((uint64_t)c->p.nx << 32) ^ (uint64_t)c->p.ny ^ ((uint64_t)c->p.dtype << 60);
  hipError_t e = pm::launch_write_header(dst, c->steps, tag, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)dst + HEADER_BYTES, (char*)c->ws + c->lay.off_f, 9 * c->lay.P * c->lay.elem,
                       hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)dst + HEADER_BYTES + 9 * c->lay.P * c->lay.elem, (char*)c->ws + c->lay.off_g,
                       5 * c->lay.P * c->lay.elem, hipMemcpyDeviceToDevice, c->stream);
  return check_hip(c, e, "pm_save_state");
}

int pm_load_state(pm_ctx* c, const void* src, size_t bytes) {
  if (!c || !src) return PM_EINVAL;
  size_t need;
  pm_state_bytes(c, &need);
  if (bytes < need) return ctx_fail(c, PM_ESTATE, "pm_load_state: buffer of %zu bytes < %zu", bytes, need);
  int64_t hdr[2];
  hipError_t e = hipMemcpyAsync(hdr, src, sizeof hdr, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "pm_load_state header");
  const uint64_t tag = STATE_TAG ^ ((uint64_t)c->p.nx << 32) ^ (uint64_t)c->p.ny ^ ((uint64_t)c->p.dtype << 60);
  if ((uint64_t)hdr[0] != tag || hdr[1] < 0)
    return ctx_fail(c, PM_ESTATE, "pm_load_state: checkpoint does not match this grid/dtype");
  e = hipMemcpyAsync((char*)c->ws + c->lay.off_f, (const char*)src + HEADER_BYTES, 9 * c->lay.P * c->lay.elem,
                     hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)c->ws + c->lay.off_g, (const char*)src + HEADER_BYTES + 9 * c->lay.P * c->lay.elem,
                       5 * c->lay.P * c->lay.elem, hipMemcpyDeviceToDevice, c->stream);
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
