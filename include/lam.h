/* lam.h -- C-ABI of the MI355X (gfx950) library for the hybrid lattice-Boltzmann / finite-difference
 * model of lamellar fluids under cold thermal fronts (Gonnella, Lamura & Tiribocchi,
 * arXiv:1102.3094, Sections 2 and 3).
 *
 * One simulation holds populations, order parameter and temperature on a D2Q9 (2D) or D3Q19 (3D)
 * lattice in lattice units (dx = dt = 1, c_s^2 = 1/3, Section 2).  Each call of lam_step advances
 * the state by whole time steps:
 *   - reduced temperature a = (T - Tc)/Tc, eq. (aterm);
 *   - chemical potential mu = a phi + b phi^3 - kappa lap phi + c lap^2 phi, eq. (chem), with the
 *     second-order 5/7-point Laplacian and its square (13/25-point) as the biharmonic;
 *   - body force F = -div P of the pressure tensor of Section 2 without its ideal-gas term
 *     (the lattice pressure n c_s^2 stays; eq. (ff)), or F = -phi grad mu;
 *   - moments n = sum f, n u = sum f e + F/2, eq. (moment); BGK collision with the second-order
 *     equilibrium and the forcing term of eq. (latticeforceterm); streaming, with bounce-back on
 *     walls half a spacing beyond the first and last layers of the last axis;
 *   - n_phi explicit Euler sub-steps of d_t phi + div(phi u) = Gamma lap mu, eq. (massdiff),
 *     with u and a held at the step's values;
 *   - n_T forward-time centred-space sub-steps of d_t T = xi lap T with T = Tw on the wall
 *     layers (Section 2: walls at fixed temperature).
 * x (and y in 3D) are periodic; the order parameter is reflected evenly across the walls, so
 * grad phi, grad lap phi and grad lap^2 phi have zero normal component there and sum(phi) is
 * conserved exactly (Section 2).
 *
 * Memory.  Every device pointer is owned by the caller.  The library allocates no device memory:
 * the caller passes one workspace of lam_workspace_bytes() bytes to lam_create and keeps it alive
 * until lam_destroy.  The library owns only its host-side handle.  All work is queued on the
 * HIP stream given to lam_create; calls that return data to the host synchronise that stream.
 * A handle is not thread-safe; different handles on different streams are independent.
 *
 * Layouts (row-major, x fastest): scalar fields [nz][ny][nx] (nz = 1 in 2D), FP32;
 * vector fields [dim][nz][ny][nx].  Populations are stored internally as deviations f_q - w_q
 * from the rest state, in FP32 or (pop_storage = 1) FP16.
 *
 * Errors.  Every int-returning function returns 0 on success or one of the LAM_E* codes below;
 * lam_last_error gives a message (for a NULL handle: the last failure of lam_create or
 * lam_workspace_bytes on the calling thread).
 */
#ifndef LAM_H
#define LAM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAM_OK 0
#define LAM_EINVAL (-1)      /* invalid argument or parameter set                               */
#define LAM_EHIP (-2)        /* a HIP runtime call failed (message holds the HIP error string)  */
#define LAM_ESIZE (-3)       /* workspace or buffer too small                                    */
#define LAM_ENONFINITE (-4)  /* observables found a NaN or infinite value in the state          */
#define LAM_ESTATE (-5)      /* checkpoint does not match this simulation                        */
#define LAM_ECORRUPT (-6)    /* a guard band of the workspace was overwritten                     */

/* Guard bands: LAM_GUARD_BYTES of a fixed pattern before the first region of the workspace and
 * after each of its regions (populations, phi, phi scratch, u, T, reduction partials, observable
 * scratch); they are counted in lam_workspace_bytes. */
#define LAM_GUARD_BYTES 256

typedef struct lam_params {
  int32_t dim;               /* 2 (D2Q9) or 3 (D3Q19)                                              */
  int32_t nx, ny, nz;        /* lattice extents; nz = 1 in 2D; each >= 8; the site count times the
                              * population size (4 or 2 bytes) below 2^32                          */
  int32_t walls;             /* 1: cold walls on the first and last layer of the last axis        */
  int32_t hydro;             /* 1: lattice Boltzmann coupled; 0: phi and T only (Section 3 runs) */
  double tau;                /* BGK relaxation time, > 1/2; viscosity (tau - 1/2)/3 (Section 2)  */
  double Gamma;              /* mobility, eq. (massdiff), >= 0                                      */
  double b, kappa, c;        /* free-energy coefficients, eq. (fren); b > 0 and c > 0 required     */
  double Tc, T0, Tw;         /* critical, initial and wall temperatures, eq. (aterm); Tc > 0        */
  double xi;                 /* thermal conductivity; < 0 means an instantaneous quench (T = Tw)  */
  int32_t n_phi_sub;         /* Euler sub-steps of phi per step; 0 = smallest stable count        */
  int32_t n_T_sub;           /* FTCS sub-steps of T per step; 0 = ceil(xi / 0.45)                  */
  int32_t force_form;        /* 0: F = -div P; 1: F = -phi grad mu                                 */
  int32_t pop_storage;       /* 0: FP32 population deviations; 1: FP16 deviations (FP32 arithmetic,
                                round-to-nearest storage; halves the population traffic)         */
  int32_t allow_unstable;    /* 1: accept n_phi_sub / n_T_sub below the stability bound           */
  int32_t tile_hint;         /* 0: automatic; 8, 16, 32 or 64: tile height of the step kernels. The
                                per-site arithmetic is the same for every tile: bit-identical
                                fields (used to test the tiling)                                  */
  double body_force[3];      /* uniform acceleration g; the force density n g is added (tests)    */
} lam_params;

typedef struct lam_obs {
  double mass_dev;           /* sum over sites of (n - 1)                                          */
  double mom[3];             /* sum over sites of sum_q f_q e_q (before the F/2 shift)            */
  double phi_sum;            /* sum over sites of phi                                              */
  double max_u;              /* max over sites of |u|, u = (sum_q f_q e_q + F/2)/n                 */
  double mach;               /* max_u / c_s, c_s = 1/sqrt(3); Section 2 asks for Ma < 0.1          */
  double free_energy;        /* sum of a phi^2/2 + b phi^4/4 + kappa/2 |forward grad phi|^2
                                + c/2 (lap phi)^2 (eq. fren without the ideal-gas part)           */
  int64_t step;
  int32_t nonfinite;         /* 1 if a population or phi value is NaN or infinite                  */
  int32_t reserved_;
} lam_obs;

typedef struct lam_sim lam_sim;

/* Bytes of device workspace the parameter set needs (256-byte aligned start required). */
int lam_workspace_bytes(const lam_params* p, size_t* bytes);

/* Validate p and bind a simulation to the caller's workspace and HIP stream (hipStream_t passed
 * as void*, NULL = default stream).  The fields are undefined until lam_init_fields. */
int lam_create(const lam_params* p, void* d_workspace, size_t bytes, void* hip_stream,
               lam_sim** out);

/* Sub-step counts in use after the automatic rule. */
int lam_substeps(const lam_sim* s, int32_t* n_phi, int32_t* n_T);

/* Initial state: phi = d_phi0 [N]; populations at equilibrium with density d_n0 [N] (NULL: 1)
 * and velocity d_u0 [dim][N] (NULL: 0); T = T0 except T = Tw on the wall layers (everywhere if
 * xi < 0).  Device pointers; the data are copied.  Resets the step counter to 0. */
int lam_init_fields(lam_sim* s, const float* d_phi0, const float* d_u0, const float* d_n0);

/* Advance nsteps time steps; asynchronous on the simulation's stream.  On a stream of the caller
 * (not the legacy default stream), with timing off and outside a capture the caller runs on that
 * stream, pairs of steps can be replayed from a HIP graph captured on first use.  The first call
 * of at least 24 steps measures 8 directly launched steps against 4 replayed pairs (that call
 * waits for them) and keeps the faster way for the simulation's life; the fields are bit-identical
 * either way.  The roctx range "lam_step" marks every call. */
int lam_step(lam_sim* s, int64_t nsteps);

/* The launch mode lam_step settled on: *graphs = -1 (not measured yet), 0 (direct launches) or 1
 * (graph replays), and the measured microseconds per step of each (0 before the measurement). Any
 * output pointer may be NULL. */
int lam_launch_mode(const lam_sim* s, int32_t* graphs, float* direct_us, float* graph_us);

/* Conserved totals and monitors of the current state (FP64 reductions); synchronises. Returns
 * LAM_ENONFINITE (with *h_out filled) if the state holds NaN or infinite values. */
int lam_observables(lam_sim* s, lam_obs* h_out);

/* Structure factor of phi (2D only): h_S[nbins] is the mean of |DFT(phi - mean)|^2 / N over the
 * modes of each shell floor(|k| / dk), dk = 2 pi / min(nx, ny) (k = 0 left out); k_peak and
 * S_peak refine the largest shell by a parabola through it and its neighbours (shell centres at
 * (m + 1/2) dk); k_mean is the |phi_hat|^2-weighted mean |k|.  Output pointers are host memory,
 * any of the three scalars may be NULL; synchronises. */
int lam_structure_factor(lam_sim* s, double* h_S, int32_t nbins, double* k_peak, double* S_peak,
                         double* k_mean);

/* No-allocation variant of lam_structure_factor, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * structure factor, computed by the same kernels, of a caller-given FP32 field d_phi [ny][nx]
 * (device memory, row-major) on the stream hip_stream (NULL: default stream), which must belong
 * to the device current on the calling thread.  Outputs as lam_structure_factor (host memory);
 * synchronises the stream.  Its scratch (transposed spectrum and per-row shell sums, about
 * 8 nx ny + 16 nx max(nx, ny) bytes: 24 MiB at 1024^2) lives in a static device array of
 * LAM_SK_STATIC_BYTES bytes that each GPU holds from the library's first use on it until the
 * process ends; lattices needing more return LAM_ESIZE, with nothing launched.  It allocates and
 * frees nothing.  All calls on one GPU share that array: calls that overlap in time on one GPU
 * (other threads, or other streams of the same device) race and give wrong results; calls made
 * one after another are safe.  Errors are reported through lam_last_error(NULL). */
#define LAM_SK_STATIC_BYTES (32u << 20)
int lam_structure_factor_static(const float* d_phi, int32_t nx, int32_t ny, void* hip_stream,
                                double* h_S, int32_t nbins, double* k_peak, double* S_peak,
                                double* k_mean);

/* Orientation of phi gradients, the measure of lamellar order relative to the walls that the
 * paper reads off its snapshots (Section 3, Figs 1-3); 1 <= nbins <= 36.
 * 2D: h_hist[nbins] holds the fraction of sum |grad phi|^2 whose gradient angle
 * atan2(g_y, g_x) mod pi falls in each of nbins equal bins of [0, pi);
 * Q = sum(g_y^2 - g_x^2) / sum |grad phi|^2 (+1: lamellae parallel to the walls, -1
 * perpendicular); h_Qrow[ny] (nullable) is the same ratio per row.
 * 3D: the angle theta = arccos(|g_z| / |grad phi|) to the wall normal in nbins equal bins of
 * [0, pi/2]; Q = sum(g_z^2 - (g_x^2 + g_y^2)/2) / sum |grad phi|^2 (+1: parallel to the walls,
 * -1/2 perpendicular, 0 isotropic); h_Qrow[nz] per layer.
 * Central differences, even reflection at walls.  Host outputs; synchronises. */
int lam_orientation(lam_sim* s, double* h_hist, int32_t nbins, double* Q, double* h_Qrow);

/* Fields of the current state into caller device buffers (any may be NULL): phi [N],
 * u [dim][N] (force-shifted velocity of eq. moment), n [N], T [N]. Asynchronous. */
int lam_get_fields(lam_sim* s, float* d_phi, float* d_u, float* d_n, float* d_T);

/* Re-anchoring after an external update of the fields (for example the learned surrogate of
 * lam_surrogate.h): phi is replaced by d_phi [N] and the populations by the same equilibrium
 * start as lam_init_fields (density d_n, velocity d_u [dim][N]; NULL gives 1 and 0), while the
 * temperature and the step count are kept.  Asynchronous. */
int lam_set_fields(lam_sim* s, const float* d_phi, const float* d_u, const float* d_n);

/* Advance only the temperature by nsteps time steps (the FTCS sub-steps lam_step applies to T,
 * Section 2) and the step count; phi and the populations are unchanged.  Asynchronous.  At most
 * 8192 layers along the wall axis (the profile is held in LDS); LAM_EINVAL beyond. */
int lam_advance_temperature(lam_sim* s, int64_t nsteps);

/* Checkpoint: the complete state (populations, phi, T, step) in lam_state_bytes() bytes of
 * caller device memory.  lam_set_state returns LAM_ESTATE for a checkpoint of another lattice. */
int lam_state_bytes(const lam_sim* s, size_t* bytes);
int lam_get_state(lam_sim* s, void* d_buf, size_t bytes);
int lam_set_state(lam_sim* s, const void* d_buf, size_t bytes);

/* Race and bounds check.  lam_init_fields and lam_set_state fill every guard band with a fixed
 * 32-bit pattern; lam_check_guards copies the bands to the host (synchronises) and returns
 * LAM_ECORRUPT, naming the region before the first damaged band in lam_last_error and setting
 * *h_first_bad to its index (else -1; NULL allowed), if a kernel wrote past the end of a region.
 * LAM_EINVAL before the fields are initialised.  lam_guard_layout writes the byte offsets of the
 * bands within the workspace of parameter set p to h_offsets[max] and their number to *count
 * (LAM_ESIZE if max is too small; host only, no device call). */
int lam_check_guards(lam_sim* s, int32_t* h_first_bad);
int lam_guard_layout(const lam_params* p, size_t* h_offsets, int32_t max, int32_t* count);

/* Profiling aid.  With timing enabled, lam_step launches each kernel with a pair of HIP events
 * that take the kernel's own start and end timestamps (hipExtLaunchKernelGGL).  lam_kernel_times synchronises, writes the accumulated kernel time
 * in milliseconds and the launch count of each kernel class (LAM_K_LB: the fused force /
 * stream / collide kernel; LAM_K_PHI: the order-parameter kernel) into h_ms[nk] and
 * h_launches[nk] (host arrays), and resets the accumulators.  Events are created on first use
 * and released by lam_destroy. */
#define LAM_K_LB 0
#define LAM_K_PHI 1
#define LAM_NK 2
int lam_set_timing(lam_sim* s, int32_t enable);
int lam_kernel_times(lam_sim* s, double* h_ms, int64_t* h_launches, int32_t nk);

const char* lam_last_error(const lam_sim* s);
void lam_destroy(lam_sim* s);

/* Ensembles: independent 2D simulations of different sizes and parameters (for example sweeps in
 * xi and viscosity, Section 3) advanced together.  Every time step is one persistent launch of the
 * LB kernel and one of the phi kernel: a grid of a few workgroups per compute unit takes
 * (member, tile) work items from per-XCD queues until none is left (no workgroup waits for
 * another; the last one to finish resets the queues), so small lattices fill the GPU together;
 * with a non-NULL stream, pairs of steps are captured once in a HIP graph and replayed.  Each
 * member computes exactly what it computes alone (bit for bit, at the same tile height).
 * Requirements: all members 2D with the same hydro flag, pop_storage and phi sub-step count.
 * Memory: one caller workspace of lam_ensemble_workspace_bytes() bytes holds every member. */
typedef struct lam_ensemble lam_ensemble;
int lam_ensemble_workspace_bytes(const lam_params* members, int32_t count, size_t* bytes);
int lam_ensemble_create(const lam_params* members, int32_t count, void* d_workspace, size_t bytes,
                        void* hip_stream, lam_ensemble** out);
/* The member simulation i (owned by the ensemble): lam_observables, lam_get_fields,
 * lam_structure_factor, lam_orientation and checkpoints work on it; do not lam_step it alone. */
int lam_ensemble_member(lam_ensemble* e, int32_t i, lam_sim** out);
/* d_phi0: host array of count device pointers to each member's initial phi. */
int lam_ensemble_init_fields(lam_ensemble* e, const float* const* d_phi0);
int lam_ensemble_step(lam_ensemble* e, int64_t nsteps);
/* Autotuner: times `steps` steps for every tile height (8, 16, 32, 64) and grid (one workgroup
 * per tile without a queue, reported as 0 workgroups, or a persistent grid of 1, 2 or 4
 * workgroups per compute unit), keeps the fastest and returns it (either output may be NULL).
 * It must come before lam_ensemble_init_fields (LAM_EINVAL otherwise): it times a fixed state
 * (phi = 0, fluid at rest) and leaves the members uninitialised. */
int lam_ensemble_tune(lam_ensemble* e, int32_t steps, int32_t* tile_height, int32_t* workgroups);
int lam_ensemble_sites(const lam_ensemble* e, int64_t* sites);
const char* lam_ensemble_last_error(const lam_ensemble* e);
void lam_ensemble_destroy(lam_ensemble* e);

#ifdef __cplusplus
}
#endif
#endif
