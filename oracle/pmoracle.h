/*
 * pmoracle.h -- FP64 CPU reference ("oracle") for the MRT lattice Boltzmann
 * model of power-law natural convection in a porous square cavity
 * (Islam, Nag & Molla, "GPU Accelerated Lattice Boltzmann Simulation of
 * Non-Newtonian Power-Law Fluid in a Porous Enclosure", ICME 2019,
 * arXiv:2011.15073).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path; it
 * is called only by the test suite, by the smoke check and by the benchmark's
 * CPU-baseline leg.  It shares no code, header, table or constant with the
 * GPU library: every constant here is written out from the paper and the
 * readings listed in the design notes.
 *
 * Lattice units throughout: dx = dt = c = 1.  Node (i, j), 0 <= i < nx,
 * 0 <= j < ny, sits at x = i + 1/2, y = j + 1/2; walls (when not periodic)
 * are halfway between nodes, at x = 0, nx and y = 0, ny, so L = N.
 * Arrays are planes [q][j][i], i fastest.
 */
#ifndef PMORACLE_H
#define PMORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Physical (nondimensional) problem parameters: Eq. (6) groups n, Ra, Pr, Da,
 * plus porosity, Mach number and the power-law clamp. */
typedef struct {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y; /* 0 = halfway walls on that axis */
  double n;          /* power-law index */
  double Da;         /* Darcy number K/L^2; +inf = clear fluid */
  double Ra, Pr;     /* Rayleigh and Prandtl numbers, Eq. (6) */
  double eps;        /* porosity (1 = clear fluid) */
  double mach;       /* lattice Mach number, U_lb = mach * c_s */
  double nu_lo, nu_hi; /* viscosity clamp as multiples of nu0 (clamp_mode 0),
                          or shear-rate thresholds gamma1, gamma2 (mode 1) */
  int32_t clamp_mode;  /* 0: clamp nu to [nu_lo, nu_hi]*nu0; 1: clamp the
                          nondimensional shear rate to [gamma1, gamma2] */
  int32_t forchheimer; /* 1: Ergun F_eps, 0: Darcy-Brinkman only */
  double s_e, s_eps, s_q; /* D2Q9 non-hydrodynamic rates (s1, s2, s4 = s6) */
  double sT_e, sT_nu;     /* D2Q5 higher-moment rates */
  double gx, gy;          /* extra uniform body force, lattice units */
  double T_init;          /* initial uniform temperature */
} orc_physics;

/* Lattice parameters: everything the update needs, in lattice units. */
typedef struct {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y;
  double nu0;          /* reference (Newtonian) lattice viscosity nu0_lb */
  double npow;         /* power-law index n */
  double nu_min, nu_max; /* absolute lattice viscosity bounds */
  double gamma_scale;  /* N / U_lb: lattice shear rate -> nondimensional */
  double eps;          /* porosity */
  double K;            /* uniform permeability (lattice units); +inf = none */
  double K_scale;      /* N^2: K = Da * K_scale for the per-cell Da plane */
  double Feps;         /* Forchheimer coefficient (0 = off) */
  double gbeta;        /* g * beta, lattice units */
  double T_m;          /* reference temperature of the buoyancy term */
  double gx, gy;       /* extra body force, lattice units */
  double alpha;        /* thermal diffusivity, lattice units */
  double s_e, s_eps, s_q; /* D2Q9 rates s1, s2, s4 = s6 */
  double sT_e, sT_nu;     /* D2Q5 rates for the two higher moments */
  double T_hot, T_cold;   /* Dirichlet wall temperatures (x = 0 and x = nx) */
  double T_init;
  double U_lb;          /* velocity scale of the nondimensional output */
} orc_lattice;

typedef struct orc_state orc_state;

/* Step 0 of the method: physical groups -> lattice parameters.  Returns 0, or
 * -1 if the parameters are invalid (message in orc_last_error()). */
int orc_map_physics(const orc_physics* phys, orc_lattice* lat);

/* Create a state at the uniform rest equilibrium (rho = 1, u = 0,
 * T = T_init).  Returns NULL on invalid input. */
orc_state* orc_new(const orc_lattice* lat);
void orc_free(orc_state* s);
const char* orc_last_error(void);

/* Per-cell log10(Da) plane [ny][nx]; K = 10^logDa * K_scale.  Pass NULL to
 * return to the uniform K. */
int orc_set_logda(orc_state* s, const double* logda);

/* Raw populations of the pre-collision state: f [9][ny][nx], g [5][ny][nx]. */
void orc_get_state(const orc_state* s, double* f, double* g);
void orc_set_state(orc_state* s, const double* f, const double* g);
int64_t orc_steps_done(const orc_state* s);

/* Advance k time steps (collide every node, then stream with the BCs). */
void orc_step(orc_state* s, int64_t k);

/* Macroscopic fields of the current pre-collision state, each [ny][nx]:
 * density, velocity (the porous velocity u of the update, lattice units),
 * temperature and the local effective lattice viscosity.  Any pointer may be
 * NULL. */
void orc_macros(const orc_state* s, double* rho, double* ux, double* uy,
                double* T, double* nu);

/* Hot-wall average Nusselt number of the current state. */
double orc_nu_bar(const orc_state* s);

/* Steady-state run: advance in chunks of `check_every` steps; after each
 * chunk r = max |T - T_prev_chunk|.  Stops at the first r < tol or when
 * max_steps is reached.  Returns the last r; *steps_out = steps done. */
double orc_run_to_steady(orc_state* s, double tol, int64_t check_every,
                         int64_t max_steps, int64_t* steps_out);

/* ---- single-node pieces, exposed for the algebraic checks ---- */

/* Collide one node: pre-collision f[9], g[5] (and local K) -> post-collision
 * fo[9], go[5]; also returns rho, ux, uy, T, nu (any may be NULL). */
void orc_collide_node(const orc_lattice* lat, double K, const double* f,
                      const double* g, double* fo, double* go, double* rho,
                      double* ux, double* uy, double* T, double* nu);

/* Equilibrium and forcing populations of the generalised (porous) model. */
void orc_feq(double eps, double rho, double ux, double uy, double* feq);
void orc_forcing(double eps, double rho, double ux, double uy, double Fx,
                 double Fy, double* Fi);
void orc_geq(double T, double ux, double uy, double* geq);

/* The transforms used by the oracle: M [9][9], its numerically computed
 * inverse, N [5][5] and its inverse (row-major). */
void orc_matrices(double* M, double* Minv, double* N, double* Ninv);

/* Squared shear-rate magnitude |gamma|^2 of one node for a given s_nu, by
 * the literal moment-space formula; f^eq taken at velocity (vx, vy). */
double orc_shear_sq(const orc_lattice* lat, const double* f, double rho,
                    double vx, double vy, double s_nu);

/* Self-consistent local viscosity of one node (the a2 solve). */
double orc_viscosity(const orc_lattice* lat, const double* f, double rho,
                     double vx, double vy);

#ifdef __cplusplus
}
#endif
#endif
