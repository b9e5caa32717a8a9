/* lam_oracle.h -- plain FP64 CPU reference ("oracle") of the hybrid lattice-Boltzmann /
 * finite-difference model of Gonnella, Lamura & Tiribocchi, "Thermal and hydrodynamic effects in
 * the ordering of lamellar fluids" (arXiv:1102.3094).
 *
 * TEST INFRASTRUCTURE.  This library exists to check the GPU implementation and to give a CPU
 * baseline; it is not part of the product path.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or constant with the GPU
 * library.
 *
 * Conventions: lattice units (dx = dt = 1, c_s^2 = 1/3, Section 2); site index
 * i = x + nx*(y + ny*z); in 2D nz = 1.  Walls, when present, are normal to the last axis (y in 2D,
 * z in 3D); the other axes are periodic.  All arrays are host FP64, owned by the caller unless
 * stated otherwise.  Functions return 0 on success and a negative code on error.
 */
#ifndef LAM_ORACLE_H
#define LAM_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim, nx, ny, nz;   /* 2 or 3; nz = 1 in 2D                                         */
  int32_t walls;             /* 1: cold flat walls on the first/last layer of the last axis  */
  int32_t hydro;             /* 1: lattice Boltzmann coupled; 0: phi and T only               */
  double tau, Gamma, b, kappa, c;
  double Tc, T0, Tw, xi;     /* xi < 0: infinitely fast quench (T = Tw everywhere at t = 0)  */
  int32_t n_phi_sub;         /* explicit Euler sub-steps of phi per LB step; 0 = automatic   */
  int32_t n_T_sub;           /* FTCS sub-steps of T per LB step; 0 = automatic               */
  int32_t force_form;        /* 0: F = -div P (pressure tensor); 1: F = -phi grad mu         */
  int32_t pad_;
  double body_force[3];      /* uniform acceleration g; the force density n*g is added       */
} orc_params;

typedef struct {
  double mass_dev;           /* sum over sites of (n - 1)                                     */
  double mom[3];             /* sum over sites of sum_q f_q e_q (bare, before the force shift) */
  double phi_sum;            /* sum over sites of phi                                          */
  double max_u;              /* max over sites of |u|, u = (sum_q f_q e_q + F/2)/n            */
  double mach;               /* max_u / c_s                                                    */
  double free_energy;        /* discrete Brazovskii free energy of phi (ideal-gas part left out) */
  int64_t step;
  int32_t nonfinite;         /* 1 if any population or phi value is NaN or infinite            */
  int32_t pad_;
} orc_obs;

typedef struct orc_sim orc_sim;

int orc_create(const orc_params* p, orc_sim** out);
void orc_destroy(orc_sim* s);
/* Number of phi and T sub-steps the simulation uses (after the automatic rule). */
int orc_substeps(const orc_sim* s, int32_t* n_phi, int32_t* n_T);
/* Lattice tables: e[Q][3], w[Q], opp[Q]; returns Q. */
int orc_lattice(int32_t dim, int32_t* e, double* w, int32_t* opp);

/* f_q = f^eq_q(n0, u0) at every site; phi = phi0.  u0 is [dim][N] (nullable: 0), n0 is [N]
 * (nullable: 1).  T starts at T0 with the wall layers at Tw (or Tw everywhere if xi < 0). */
int orc_init_fields(orc_sim* s, const double* phi0, const double* u0, const double* n0);
int orc_step(orc_sim* s, int64_t nsteps);
int orc_observables(orc_sim* s, orc_obs* out);
/* Fields at the current time.  phi [N]; u [dim][N] (force-shifted velocity); n [N]; T [N].
 * Any pointer may be NULL. */
int orc_get_fields(orc_sim* s, double* phi, double* u, double* n, double* T);
/* Populations f [Q][N] at the current time (after streaming, before collision). */
int orc_get_populations(orc_sim* s, double* f);
/* Chemical potential mu [N] and total force density F [dim][N] of the current state. */
int orc_eval_mu(orc_sim* s, double* mu);
int orc_eval_force(orc_sim* s, double* F);
/* Single-site building blocks: equilibrium f^eq_q(n, u) and forcing term F_q(u, F) [Q]. */
int orc_feq(int32_t dim, double n, const double* u, double* out);
int orc_guo(int32_t dim, double tau, const double* u, const double* F, double* out);
/* Checkpoint of the full state (f, phi, T, step). */
size_t orc_state_bytes(const orc_sim* s);
int orc_get_state(const orc_sim* s, void* buf, size_t bytes);
int orc_set_state(orc_sim* s, const void* buf, size_t bytes);
/* OpenMP threads of the loops over sites: n > 0 sets them for the calls that follow; returns the
 * number in use. */
int orc_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
