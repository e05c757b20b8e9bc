/*
 * pmlbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for
 * natural convection of a power-law fluid in a porous square cavity
 * (Islam, Nag & Molla, ICME 2019, arXiv:2011.15073).
 *
 * Method (equation numbers count the paper's displayed equations in order):
 *   - D2Q9 MRT collision in moment space with forcing, Eq. (12), relaxation
 *     rates Eq. (13), velocities Eq. (14), nu = c_s^2 (tau - 1/2) Eq. (15),
 *     macroscopic rho and u Eqs. (16)-(17);
 *   - Boussinesq buoyancy (Eq. 9's +Pr theta) and a Brinkman-Forchheimer
 *     porous drag (Eq. 8's Darcy term -U D/Da, generalised with porosity and
 *     the Forchheimer term);
 *   - local modified power-law viscosity, Eq. (21), with the shear rate from
 *     the non-equilibrium moments, Eqs. (22)-(23);
 *   - D2Q5 MRT thermal update, Eqs. (18)-(20), hot left wall, cold right wall,
 *     adiabatic top and bottom (the text of the "Mathematical Formulations"
 *     section; Eq. (5) as printed swaps the walls);
 *   - hot-wall average Nusselt number, Eq. (24), and the steady-state
 *     residual max |T_k - T_{k-m}|.
 *
 * Lattice units: dx = dt = 1; node (i, j) at x = i + 1/2, y = j + 1/2; walls
 * halfway between nodes, so the cavity side L equals the node count N.
 * Parameter mapping (the paper gives none): U_lb = mach / sqrt(3);
 * nu0_lb = Pr / sqrt(Ra)^(2-n) * U_lb * N; alpha_lb = U_lb * N / sqrt(Ra);
 * g*beta_lb = Pr * U_lb^2 / N; K = Da * N^2; F_eps = 1.75 / sqrt(150 eps^3).
 *
 * Conventions for every call:
 *   - Return value: PM_OK (0) or a negative PM_E* code; nothing aborts or
 *     throws across the ABI.  pm_last_error(ctx) holds a message for the most
 *     recent failure on that context (pm_last_error(NULL): the most recent
 *     failure of a call that had no context yet).
 *   - Device memory is always owned by the caller: the workspace passed to
 *     pm_init, and every output buffer.  The library allocates only its host
 *     context, one private non-blocking stream on which pm_step captures its
 *     HIP graphs, and those graphs, all released by pm_destroy (a sweep or
 *     an adjoint likewise releases what it creates in its own destroy call).
 *   - A context is bound to the HIP stream given to pm_init; every call
 *     enqueues on that stream.  Calls that return host values (pm_nu,
 *     pm_residual, pm_run_to_steady) synchronise that stream.  A context is
 *     not thread-safe.
 *   - Every caller-facing array (fields, populations, log10 Da, gradients,
 *     adjoint states) is a set of planes [q][ny][nx], x fastest.  Inside the
 *     workspace the populations are row-interleaved (the 14 rows of grid row
 *     j one after the other); raw states from pm_save_state keep that
 *     internal layout.
 */
#ifndef PMLBM_H
#define PMLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM_OK 0
#define PM_EINVAL (-1)    /* invalid argument or parameters */
#define PM_EDEVICE (-2)   /* HIP runtime error (message kept) */
#define PM_EDIVERGED (-3) /* NaN/Inf met in a reduction */
#define PM_ESTATE (-4)    /* buffer size or state mismatch */

#define PM_FP32 0 /* FP32 storage and arithmetic; FP64 reductions */
#define PM_FP64 1 /* FP64 storage and arithmetic */
#define PM_FP16 2 /* FP16 population storage, FP32 arithmetic, FP64 reductions (see pm_params.dtype) */

#define PM_ROUND_NEAREST 0    /* population updates rounded to nearest */
#define PM_ROUND_STOCHASTIC 1 /* FP32/FP16 population updates rounded stochastically (see pm_params.rounding) */
#define PM_ROUND_AUTO 2       /* default: stochastic with FP32 and FP16 storage, nearest with FP64 */

#define PM_STEP_AUTO 0   /* two-step kernel where it pays off (large FP32 cavities) */
#define PM_STEP_SINGLE 1 /* always one step per pass (in place, AA pattern) */
#define PM_STEP_PAIR 2   /* two steps per pass wherever allowed (FP32, no periodic axis) */

#define PM_CLAMP_NU 0    /* nu = clamp(nu0 gamma*^(n-1), nu_lo nu0, nu_hi nu0) */
#define PM_CLAMP_GAMMA 1 /* nu = nu0 clamp(gamma*, nu_lo, nu_hi)^(n-1): the
                            thresholds gamma1, gamma2 of Eq. (21) */

typedef struct pm_ctx pm_ctx;

/* Problem parameters.  Groups of Eq. (6) plus porosity, Mach number and the
 * viscosity bounds.  Fill with pm_params_default() and override. */
typedef struct {
  int32_t nx, ny;                 /* nodes; nx = ny for the paper's cavity */
  int32_t periodic_x, periodic_y; /* 1 = periodic axis instead of walls */
  double n;        /* power-law index (> 0); 1 = Newtonian */
  double Da;       /* Darcy number K/L^2 (> 0); +inf = clear fluid */
  double Ra, Pr;   /* Rayleigh, Prandtl numbers (> 0) */
  double eps;      /* porosity in (0, 1] */
  double mach;     /* lattice Mach number (default 0.1) */
  double nu_lo, nu_hi; /* clamp bounds, see PM_CLAMP_* (default 0.1, 10) */
  int32_t clamp_mode;  /* PM_CLAMP_NU (default) or PM_CLAMP_GAMMA */
  int32_t dtype;       /* PM_FP32 (default), PM_FP64 or PM_FP16.  PM_FP16 stores the shifted
                          populations as IEEE half (56 B per node update moved instead of 112),
                          computes in FP32 and rounds every stored update stochastically (unless
                          rounding = PM_ROUND_NEAREST); the per-cell planes stay FP32.  It runs the
                          single-step kernel only, and neither sweeps nor the adjoint take it.
                          Its fields are 1e-3 to 1e-2 of the FP64 oracle's after 20 000 steps of
                          the 64^2 cavities, against about 1e-6 for FP32. */
  int32_t forchheimer; /* 1 (default): Ergun F_eps; 0: Darcy-Brinkman only */
  int32_t has_logda;   /* 1: per-cell log10(Da) plane from pm_set_logda */
  double s_e, s_eps, s_q; /* D2Q9 rates s1, s2, s4 = s6 (default 1.4, 1.4, 1.2) */
  double sT_e, sT_nu;     /* D2Q5 higher-moment rates (default 1.0, 1.0) */
  double gx, gy;          /* extra uniform body force, lattice units (default 0) */
  double T_init;          /* initial uniform theta (default 0.5) */
  int32_t step_kernel;    /* PM_STEP_AUTO (default), PM_STEP_SINGLE or PM_STEP_PAIR.  Both
                             kernels give the same populations bit for bit; the two-step
                             kernel needs a second population region in the workspace
                             (pm_workspace_bytes accounts for it).  PM_STEP_PAIR with FP64,
                             a periodic axis or ny > 24 * 65535 is PM_EINVAL (PM_STEP_AUTO
                             then takes the single-step kernel). */
  int32_t rounding;       /* PM_ROUND_AUTO (default), PM_ROUND_NEAREST or PM_ROUND_STOCHASTIC (FP32
                             and FP16 storage; PM_EINVAL with FP64).  Near a steady flow,
                             round-to-nearest FP32 storage makes the same rounding every step, and
                             the cavity's slowly decaying modes turn that fixed pattern into a bias
                             (about 5e-4 of the fields at the 256^2 power-law steady state).
                             Stochastic rounding draws one 32-bit word per node update from a hash
                             of the node and its inputs (deterministic, the same in every kernel).
                             FP32: each update is added to its stored population with a uniform
                             dither of width 2 ulp of the stored value, then rounded to nearest.
                             FP16: each update is converted by the hardware's stochastically
                             rounding FP32 -> FP16 conversion, fed the word rotated per
                             population.  Unbiased; no measurable cost per step at 4096^2. */
} pm_params;

/* Lattice values derived from pm_params (read-only description). */
typedef struct {
  double U_lb, nu0, nu_min, nu_max, gamma_scale;
  double eps, K, Feps, gbeta, T_m, alpha;
  double tau0, tau_min, tau_max, tau_g;
  double s_e, s_eps, s_q, sT_e, sT_nu;
} pm_lattice;

/* Defaults: nx = ny = 64, n = 1, Da = +inf, Ra = 1e3, Pr = 10, eps = 1,
 * mach = 0.1, nu_lo = 0.1, nu_hi = 10, PM_CLAMP_NU, PM_FP32, forchheimer = 1,
 * has_logda = 0, paper rates, no body force, T_init = 0.5, PM_STEP_AUTO,
 * PM_ROUND_AUTO. */
int pm_params_default(pm_params* p);

/* Validate p and describe the lattice it maps to.  Host only.  PM_EINVAL if
 * any tau would be <= 1/2, a bound is inverted, or a value is out of range. */
int pm_lattice_of(const pm_params* p, pm_lattice* out);

/* Device workspace size (bytes) that pm_init needs for p. */
int pm_workspace_bytes(const pm_params* p, size_t* bytes);

/* Create a context for the cavity problem of the paper's "Mathematical
 * Formulations" section: side L = nx nodes, groups n, Da, Ra, Pr of Eq. (6)
 * plus eps, mapped to lattice values as described at the top of this file.
 * Validates p, carves the caller's device workspace dev_ws (at least
 * pm_workspace_bytes, 256-byte aligned, on the current device), and enqueues
 * the rest-state initialisation (rho = 1, u = 0, theta = T_init, the
 * equilibrium populations) on hip_stream (a hipStream_t; NULL = default
 * stream).  The workspace must stay allocated until pm_destroy.  Errors:
 * PM_EINVAL for invalid parameters or a misaligned workspace, PM_ESTATE for
 * a workspace that is too small, PM_EDEVICE for a HIP failure; *out is then
 * NULL. */
int pm_init(const pm_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
            pm_ctx** out);

/* Release the host context (never frees the caller's workspace). */
void pm_destroy(pm_ctx* ctx);

/* Per-cell log10(Da) plane [ny][nx] in device memory (dtype PM_FP32 or
 * PM_FP64), copied into the workspace; K(x) = 10^logDa(x) N^2.  Requires
 * has_logda = 1.  Async. */
int pm_set_logda(pm_ctx* ctx, const void* dev_plane, int dtype);

/* Advance k >= 0 time steps.  One step is the D2Q9 MRT update of Eq. (12)
 * (collision in moment space with the relaxation rates of Eq. (13), the
 * local viscosity of Eqs. (21)-(23), buoyancy and porous drag as the forcing
 * term, then streaming with halfway bounce-back walls) and the D2Q5 MRT
 * update of Eq. (18) (hot/cold anti-bounce-back walls, adiabatic
 * bounce-back walls), for every node.  Async; PM_EINVAL for k < 0. */
int pm_step(pm_ctx* ctx, int64_t k);

/* Steps done since pm_init / the last pm_set_populations or pm_load_state. */
int pm_steps_done(const pm_ctx* ctx, int64_t* steps);

/* Hot-wall average Nusselt number of the current state, Eq. (24), summed in
 * FP64 in a fixed order.  Synchronises.  PM_EDIVERGED if not finite. */
int pm_nu(pm_ctx* ctx, double* nu_out);

/* Steady-state residual: r = max over nodes of |theta - theta_snapshot|
 * (FP64), then snapshot := theta.  The snapshot is taken at pm_init (and
 * restored by pm_load_state).  *at_step (may be NULL) = the step count at
 * which r was taken, i.e. pm_steps_done.  Synchronises.  PM_EDIVERGED (with
 * *r_out = +inf) if a NaN/Inf is met. */
int pm_residual(pm_ctx* ctx, double* r_out, int64_t* at_step);

/* Run in chunks of check_every steps, calling pm_residual after each, until
 * r < tol or max_steps steps were taken by this call.  *steps_out = steps
 * taken by this call, *r_out = last residual. */
int pm_run_to_steady(pm_ctx* ctx, double tol, int64_t check_every, int64_t max_steps,
                     int64_t* steps_out, double* r_out);

/* Nondimensional fields of Eq. (6) for the current state into caller device
 * buffers [ny][nx] of dtype PM_FP32 / PM_FP64: U = u/U_lb, V = v/U_lb (u the
 * porous velocity of the update, from rho and j of Eqs. (16)-(17)) and
 * theta = T of Eq. (20) (the walls are at theta = 1 and 0).  Any pointer may
 * be NULL.  Async.  PM_EINVAL for a bad dtype. */
int pm_fields(pm_ctx* ctx, void* U, void* V, void* theta, int dtype);

/* Stream function of the current state [ny][nx] (the streamline plots of
 * the paper's results section): psi with U = d psi / dY, V = -d psi / dX in
 * the nondimensional units of pm_fields (Y = y / L, L = nx), psi = 0 on the
 * bottom wall, integrated up each column by the midpoint rule
 * (psi_j = (sum_{j' < j} U_j' + U_j / 2) / L) with FP64 sums (a blocked
 * scan over 64-row blocks; scratch space is part of the workspace).  Closed
 * streamlines are level sets; psi on the top wall is the column's net flux
 * (0 for a steady incompressible flow).  Async. */
int pm_stream_function(pm_ctx* ctx, void* psi, int dtype);

/* Local lattice viscosity nu(x) of the current state [ny][nx].  Async. */
int pm_viscosity(pm_ctx* ctx, void* nu, int dtype);

/* Pre-collision populations of the current state, absolute values:
 * f [9][ny][nx], g [5][ny][nx] in caller device buffers of dtype.  Async. */
int pm_get_populations(pm_ctx* ctx, void* f, void* g, int dtype);

/* Replace the state by the given pre-collision populations (same layout);
 * resets the step count to 0.  Async. */
int pm_set_populations(pm_ctx* ctx, const void* f, const void* g, int dtype);

/* Raw state checkpoint: pm_state_bytes gives the size; save/load copy, between
 * the workspace and a caller device buffer, a header (grid and dtype tag, the
 * step count, a hash of the physics: the lattice values of pm_lattice, n,
 * the body force, has_logda, the periodic axes and the rounding mode), the
 * population region and the residual snapshot, so that a resumed
 * pm_run_to_steady stops where the uninterrupted run stops.  The log-Da
 * plane is not saved (set it again after loading into a new context).
 * pm_load_state checks the header synchronously: PM_ESTATE if the buffer is
 * too small, or was saved for another grid, dtype or physics (nothing is
 * loaded then).  Loading restores the step count.  The copies are async. */
int pm_state_bytes(const pm_ctx* ctx, size_t* bytes);
int pm_save_state(pm_ctx* ctx, void* dev_dst, size_t bytes);
int pm_load_state(pm_ctx* ctx, const void* dev_src, size_t bytes);

/* Read+write bandwidth probe: copies `bytes` (multiple of 16) from src to dst
 * with the library's streaming copy kernel on hip_stream.  Used to measure
 * the achievable HBM ceiling and to calibrate traffic counters.  Async. */
int pm_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream);

/* ---- Batched parameter sweep ----
 * Many independent cavities (e.g. the (n, Da, Ra) grid of the paper's
 * parametric study, Table 2, with uneven grid sides) advanced together: one
 * launch per time step covers every tile of every case still running,
 * and a chunk of check_every steps plus the per-case residual test is
 * replayed as one HIP graph.  Each case stops at the first check with
 * residual < tol (or at max_steps, or on NaN/Inf) exactly as
 * pm_run_to_steady would stop it, and is then skipped.  The per-node
 * arithmetic is the single-case kernel's, so every case ends bitwise equal to
 * the same case run alone.  All cases must share one dtype; per-cell log-Da
 * planes are not supported; every case steps one step per pass (step_kernel
 * is ignored).  FP32 cases may mix PM_ROUND_NEAREST and PM_ROUND_STOCHASTIC;
 * a sweep with no stochastic case runs a step kernel compiled without that
 * branch (fewer registers).  The workspace (caller-owned device memory,
 * 256-byte aligned) holds every case's planes plus the case table,
 * schedule, flags and partial results. */
typedef struct pm_sweep pm_sweep;

#define PM_ORDER_CASE 0       /* schedule row tiles case after case, in input order */
#define PM_ORDER_LARGEST 1    /* case after case, largest case first */
#define PM_ORDER_INTERLEAVE 2 /* round-robin over the cases, tile by tile */

/* Bytes of device workspace for these cases.  PM_EINVAL (message in
 * pm_last_error(NULL)) for ncases outside 1..4096, mixed dtypes, a case with
 * has_logda, or a case that pm_workspace_bytes rejects. */
int pm_sweep_workspace_bytes(const pm_params* cases, int ncases, size_t* bytes);
/* Validates every case, creates one context per case on its slice of the
 * workspace (rest state), uploads the case table and the schedule.
 * Synchronises the stream. */
int pm_sweep_create(const pm_params* cases, int ncases, void* dev_ws, size_t ws_bytes, void* hip_stream,
                    pm_sweep** out);
/* Choose the tile order (PM_ORDER_*); used by the autotuner. */
int pm_sweep_set_order(pm_sweep* s, int order);
/* Choose the tile shape: one workgroup of tile_w * tile_h threads per tile of
 * tile_w columns by tile_h rows of a case; tile_w in {64, 128, 256}, tile_h in
 * {1, 2, 4}, tile_w * tile_h <= 256 (default 256 x 1).  Results are bitwise
 * the same for every shape; used by the autotuner.  Synchronises the stream.
 * PM_EINVAL for any other shape. */
int pm_sweep_set_tile(pm_sweep* s, int tile_w, int tile_h);
/* Run every live case until it stops (see above).  max_steps counts every
 * step a case has taken since pm_sweep_create (all run, advance and step
 * calls together); the chunk that reaches it is shortened, as
 * pm_run_to_steady shortens its last one.  steps_out[i], r_out[i] (arrays
 * of ncases, may be NULL): steps taken and last residual of case i.
 * Returns PM_EDIVERGED if any case stopped on NaN/Inf. */
int pm_sweep_run(pm_sweep* s, double tol, int64_t check_every, int64_t max_steps, int64_t* steps_out,
                 double* r_out);
/* Same as pm_sweep_run but returns after at most max_chunks chunks;
 * *nlive = cases still running (0: done).  For progress reporting and for
 * sharing the GPU with other work between chunks. */
int pm_sweep_advance(pm_sweep* s, double tol, int64_t check_every, int64_t max_steps, int64_t max_chunks,
                     int* nlive);
/* Steps taken and last residual of every case so far (arrays of ncases, may
 * be NULL).  PM_EDIVERGED if a stopped case ended on a NaN/Inf residual. */
int pm_sweep_status(const pm_sweep* s, int64_t* steps_out, double* r_out);
/* Advance every live case by k steps with no stopping test (warm-up and
 * schedule timing).  Synchronises. */
int pm_sweep_step(pm_sweep* s, int64_t k);
/* Borrow the context of case i (fields, Nu, populations); owned by the
 * sweep, valid until pm_sweep_destroy. */
int pm_sweep_case(pm_sweep* s, int i, pm_ctx** out);
void pm_sweep_destroy(pm_sweep* s);
const char* pm_sweep_last_error(const pm_sweep* s);

/* ---- Adjoint: gradients of the Nusselt number ----
 * J = Nu_bar (Eq. 24) after T steps from the context's current state.
 * Gradients with respect to the per-cell log10(Da) field (has_logda = 1),
 * the power-law index n and the Rayleigh number Ra, by the discrete adjoint
 * of the update: transposed streaming, and the reverse-mode derivative of the
 * node update recomputed in FP64 (the viscosity of Eq. (21) differentiated
 * through its fixed-point equation, or through the active clamp).  Memory:
 * checkpoints of the state every C steps (C ~ sqrt(T)); each segment is
 * replayed out of place before its adjoint steps run in reverse, the replay
 * of the next segment overlapping the adjoint steps of the current one on a
 * second HIP stream that the adjoint creates (with five events; released by
 * pm_adjoint_destroy).  Supported: cavity walls (no periodic axes),
 * PM_CLAMP_NU, no extra body force.  The workspace (caller-owned device
 * memory, 256-byte aligned) holds the ceil(T / C) checkpoints, two buffers
 * of C + 1 replayed states, two FP64 adjoint states and per-workgroup
 * partial sums. */
typedef struct pm_adjoint pm_adjoint;

int pm_adjoint_workspace_bytes(const pm_params* p, int64_t T, int64_t C, size_t* bytes);
/* Bind an adjoint to a context (which it borrows; keep the context alive). */
int pm_adjoint_create(pm_ctx* ctx, int64_t T, int64_t C, void* dev_ws, size_t ws_bytes, pm_adjoint** out);
/* Run T steps from the context's current state, checkpointing every C
 * steps; *J_out = Nu_bar of the final state.  Synchronises. */
int pm_adjoint_forward(pm_adjoint* a, double* J_out);
/* Gradients of seed * J: grad_logda (device FP64 [ny][nx], overwritten; may
 * be NULL when has_logda = 0), *grad_n, *grad_Ra (host; may be NULL).  The
 * context's state is left at the end of the forward run.  Synchronises.
 * PM_EDIVERGED (outputs then meaningless) when the adjoint state exceeds
 * 1e12 |seed| max(1, nx / ny) or is not finite: the linearised update is
 * amplifying perturbations along this trajectory (see
 * pm_adjoint_set_shear_floor). */
int pm_adjoint_backward(pm_adjoint* a, double seed, void* grad_logda, double* grad_n, double* grad_Ra);
/* Regularised derivative (default 0: the exact discrete adjoint).  Where the
 * local nondimensional shear rate gamma* (Eq. 22 times N / U) is below
 * gamma_floor, the adjoint holds the viscosity of Eq. (21) fixed with
 * respect to the populations (its dependence on nu0 and n is kept).  For
 * n < 1 the power law's slope d nu / d gamma grows like gamma^(n-2) towards
 * zero shear, and where that meets the Darcy drag the linearised update can
 * amplify perturbations from step to step; the floor removes that channel.
 * PM_EINVAL for a negative or non-finite value. */
int pm_adjoint_set_shear_floor(pm_adjoint* a, double gamma_floor);
/* Storage of the adjoint state between steps: PM_FP64 (default) or PM_FP32,
 * for FP32 forward states only (else PM_EINVAL).  The adjoint arithmetic
 * stays FP64; with PM_FP32 each step's result is rounded to nearest FP32
 * before it is stored, which halves the adjoint state's memory traffic (the
 * adjoint step then moves 188 B per node instead of 300) at a relative cost
 * in the gradients of the order of the FP32 forward's own rounding.  The
 * workspace size does not depend on it.  Takes effect at the next
 * pm_adjoint_backward. */
int pm_adjoint_set_lambda_dtype(pm_adjoint* a, int dtype);
void pm_adjoint_destroy(pm_adjoint* a);
const char* pm_adjoint_last_error(const pm_adjoint* a);

/* One adjoint step at the context's current state S_k: given lam_next =
 * dL/dS_{k+1} (device FP64 [14][ny][nx], f planes then g planes), writes
 * lam = dL/dS_k, adds dL/dlog10(Da) of this step into grad_logda (device
 * FP64 [ny][nx]) and returns (dL/dn, dL/dRa) of this step in grad_scalars[2]
 * (host).  dev_scratch: pm_adjoint_vjp_scratch_bytes(ctx) bytes of device
 * memory.  Synchronises.  Used to check the adjoint against autograd. */
size_t pm_adjoint_vjp_scratch_bytes(const pm_ctx* ctx);
int pm_adjoint_vjp(pm_ctx* ctx, const void* lam_next, void* lam, void* grad_logda, void* dev_scratch,
                   size_t scratch_bytes, double* grad_scalars);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the adjoint
 * step of pm_adjoint_vjp, with the same arguments except the scratch buffer
 * and bit-for-bit the same results.  Its per-workgroup partial sums live in a
 * static device array of the library instead (2 MiB + 32 B on each device
 * that calls it, held until the process ends), which it clears with a kernel
 * on every call.  Limit: ceil(nx / 256) * ny <= 65536 workgroups (4096^2
 * fits); larger grids get PM_EINVAL and a message.  The context's device must
 * be current (else PM_EINVAL).  Every call on a device shares that device's
 * array, so calls that overlap on one GPU (several threads or streams) race.
 * Calls no hipMalloc, hipFree or other allocating routine.  Synchronises. */
int pm_adjoint_vjp_noalloc(pm_ctx* ctx, const void* lam_next, void* lam, void* grad_logda,
                           double* grad_scalars);

const char* pm_strerror(int code);
const char* pm_last_error(const pm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
