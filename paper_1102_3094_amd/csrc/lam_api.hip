// lam_api.hip -- host implementation of the C-ABI in include/lam.h: parameter validation, the
// sub-step stability rule, workspace carving, launch order of one time step, observables,
// fields and checkpoints.  All device memory belongs to the caller.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/lam.h"
#include "lam_dev.hpp"

namespace lam {
enum { MODE_STEP = 0, MODE_OBS = 1, MODE_FIELDS = 2 };
// lam_2d.hip
int lb2d_blocks(const KParams& P, int ty);
hipError_t launch_lb2d(const KParams& P, int ty, int mode, const void* gin, void* gout,
                       const float* phi, const float* Trow, float* u, float* n, double* partials,
                       hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
int phi2d_max_sub();
hipError_t launch_phi2d(const KParams& P, int ty, int nsub, const float* in, float* out,
                        const float* u, const float* T, float* Tn, float* Ts, int do_T,
                        hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// lam_3d.hip
int blocks3d(const KParams& P);
int phi3d_chunk(int nx, int ny, int nz);
hipError_t launch_lb3d(const KParams& P, int mode, const void* gin, void* gout,
                       const float* phi, const float* Trow, float* u, float* n, double* partials,
                       hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_phi3d(const KParams& P, const float* in, float* out, const float* u,
                        const float* T, float* Tn, float* Ts, int do_T, hipStream_t st,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_ens_step(const EnsMember* mem, const int* tile_member, int ntiles, int ty,
                           int cur, int half, int hydro, int nphi, int grid, unsigned* q,
                           hipStream_t st);
int ens_queue_words();
// lam_util.hip
hipError_t launch_init(const KParams& P, int dim, const float* n0, const float* u0, void* g,
                       hipStream_t st);
hipError_t launch_init_T(int nrows, int walls, float T0, float Tw, int quench, float* a, float* b,
                         hipStream_t st);
hipError_t launch_finalize(const double* partials, int nblk, double* out, hipStream_t st);
hipError_t launch_temperature(int nrows, int walls, float r_T, int n_T, int64_t nsteps,
                              const float* Tin, float* Tout, hipStream_t st);
hipError_t launch_broadcast_T(const float* Trow, size_t N, size_t layer, float* out,
                              hipStream_t st);
hipError_t launch_write_header(int dim, int nx, int ny, int nz, int64_t step, int Q, int esz,
                               void* dst, hipStream_t st);
bool check_header(const void* host_copy, int dim, int nx, int ny, int nz, int Q, int esz,
                  int64_t* step);
size_t header_bytes();
// lam_spectra.hip
size_t spectra_scratch_bytes(int nx, int ny);
hipError_t structure_factor_2d(const KParams& P, const float* phi, void* scratch, int nbins,
                               double* h_S, double* h_kpeak, double* h_Speak, double* h_kmean,
                               hipStream_t st);
hipError_t orientation_2d(const KParams& P, const float* phi, void* scratch, int nbins,
                          double* h_hist, double* h_Q, double* h_Qrow, hipStream_t st);
size_t orientation3_scratch_bytes(int ny, int nz);
hipError_t orientation_3d(const KParams& P, const float* phi, void* scratch, int nbins,
                          double* h_hist, double* h_Q, double* h_Qrow, hipStream_t st);
size_t static_scratch_capacity();
hipError_t static_scratch(int device, void** out);
}  // namespace lam

using namespace lam;

static thread_local std::string g_create_error;

struct lam_sim {
  lam_params p;
  KParams k;
  int Q, nphi, nT, nrows;
  int ty_lb, ty_phi;  // tile heights of the two step kernels
  size_t N;
  hipStream_t st;
  char* ws;
  size_t ws_bytes;
  void* g[2];      // population deviations, FP32 or FP16 (pop_storage)
  size_t pop_bytes;  // bytes of one population field (Q * N * element size)
  float* phi[2];
  float* psi[2];
  float* u;
  float* T[3];
  double* partials;
  double* result;
  void* spec;
  int nblk;
  int64_t step;
  bool initialised;
  bool guards_set = false;   // the guard bands hold the pattern (set with the fields)
  size_t guard[14];          // offsets of the guard bands in the workspace
  std::string err;
  // kernel timing (profiling aid)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_cls;
  size_t ev_used = 0;
  // two time steps (even then odd) captured once and replayed by lam_step, when that measured
  // faster than direct launches (graph_mode: -1 not yet measured, 0 direct, 1 graph)
  hipGraphExec_t pair_graph = nullptr;
  int graph_mode = -1;
  float direct_us = 0.f, graph_us = 0.f;  // per step, as measured
};

namespace {

// Guard bands: LAM_GUARD_BYTES of a fixed 32-bit pattern before the first region of the workspace
// and after every region, filled when the fields are initialised or restored and compared by
// lam_check_guards.  A kernel that writes past the end of a field (a halo or tile-edge mistake)
// changes the band behind it.
constexpr int GUARD_BANDS = 14;
constexpr uint32_t GUARD_WORD = 0x7FA5C3E1u;  // a NaN with a payload no kernel writes
static_assert(sizeof(lam_sim::guard) / sizeof(size_t) == GUARD_BANDS, "one offset per band");
const char* const GUARD_AFTER[GUARD_BANDS] = {
    "the workspace start", "populations[0]", "populations[1]", "phi[0]", "phi[1]", "psi[0]",
    "psi[1]", "u", "T[0]", "T[1]", "T[2]", "partials", "result", "observable scratch"};

struct Layout {
  size_t g[2], phi[2], psi[2], u, T[3], partials, result, spec, total;
  size_t guard[GUARD_BANDS];
  int nblk;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(const lam_params& p) {
  static_assert(LAM_GUARD_BYTES % 256 == 0, "guard bands keep every region 256-byte aligned");
  Layout L{};
  const size_t N = (size_t)p.nx * p.ny * (p.dim == 3 ? p.nz : 1);
  const int Q = p.dim == 2 ? 9 : 19;
  const int nrows = p.dim == 2 ? p.ny : p.nz;
  size_t off = 0;
  int band = 0;
  auto guard = [&]() {
    L.guard[band++] = off;
    off += LAM_GUARD_BYTES;
  };
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    guard();
    return o;
  };
  guard();
  const size_t esz = p.pop_storage == 1 ? 2 : 4;
  for (int i = 0; i < 2; ++i) L.g[i] = take(esz * Q * N);
  for (int i = 0; i < 2; ++i) L.phi[i] = take(sizeof(float) * N);
  for (int i = 0; i < 2; ++i) L.psi[i] = take(sizeof(float) * N);
  L.u = take(sizeof(float) * p.dim * N);
  for (int i = 0; i < 3; ++i) L.T[i] = take(sizeof(float) * nrows);
  // one partial per workgroup of the largest grid (2D tiles 64 x 8; 3D handled by its kernels)
  L.nblk = (int)((size_t)((p.nx + 63) / 64) * ((p.ny + 7) / 8) * (p.dim == 3 ? p.nz : 1) + 1);
  L.partials = take(sizeof(double) * R_N * L.nblk);
  L.result = take(sizeof(double) * R_N);
  L.spec = take(p.dim == 2 ? spectra_scratch_bytes(p.nx, p.ny) : orientation3_scratch_bytes(p.ny, p.nz));
  L.total = off;
  return L;
}

// Smallest number of explicit Euler sub-steps that keeps the checkerboard mode of the linearised
// phi equation damped: one sub-step of length h multiplies it by
// 1 - h Gamma lambda (a_eff + kappa lambda + c lambda^2), lambda = 4 dim (largest eigenvalue of the
// lattice Laplacian); require >= -0.8.  a_eff is the largest local d mu / d phi: a itself, or
// a + 3 b A^2 in a lamellar state of single-mode amplitude A^2 = 4(-a + kappa^2/(4c))/(3b) at
// the coldest a (single-mode theory of Section 2).
int auto_nphi(const lam_params& p) {
  double a0 = (p.T0 - p.Tc) / p.Tc, aw = (p.Tw - p.Tc) / p.Tc;
  double amax = a0, amin = a0;
  if (p.xi < 0) amax = amin = aw;
  else if (p.walls) {
    amax = std::max(a0, aw);
    amin = std::min(a0, aw);
  }
  double aeff = amax;
  double A2 = 4.0 * (-amin + p.kappa * p.kappa / (4.0 * p.c)) / (3.0 * p.b);
  if (A2 > 0) aeff = std::max(aeff, amin + 3.0 * p.b * A2);
  double lam = 4.0 * p.dim;
  double x = p.Gamma * lam * (aeff + p.kappa * lam + p.c * lam * lam) / 1.8;
  int n = (int)ceil(x - 1e-12);
  return n < 1 ? 1 : n;
}

// FTCS on T, which varies only along the wall axis, is stable for xi/n_T <= 1/2; keep 0.45.
int auto_nT(const lam_params& p) {
  if (p.xi <= 0) return 1;
  int n = (int)ceil(p.xi / 0.45 - 1e-12);
  return n < 1 ? 1 : n;
}

int fail(lam_sim* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  else g_create_error = msg;
  return code;
}

int hip_fail(lam_sim* s, hipError_t e, const char* where) {
  return fail(s, LAM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(s, call)                              \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(s, e_, #call); \
  } while (0)

int validate(const lam_params* p, std::string& why) {
  if (!p) return why = "null parameters", LAM_EINVAL;
  if (p->dim != 2 && p->dim != 3) return why = "dim must be 2 or 3", LAM_EINVAL;
  if (p->nx < 8 || p->ny < 8) return why = "nx and ny must be >= 8", LAM_EINVAL;
  if (p->dim == 2 && p->nz != 1) return why = "nz must be 1 in 2D", LAM_EINVAL;
  // the step kernels address each population plane with 32-bit byte offsets
  if ((double)p->nx * p->ny * (p->dim == 3 ? p->nz : 1) * (p->pop_storage ? 2 : 4) >= 4294967296.0)
    return why = "lattice too large: a population plane must stay below 2^32 bytes", LAM_EINVAL;
  if (p->dim == 3 && p->nz < 8) return why = "nz must be >= 8 in 3D", LAM_EINVAL;
  if (!(p->tau > 0.5)) return why = "tau must exceed 1/2", LAM_EINVAL;
  if (!(p->b > 0) || !(p->c > 0)) return why = "b and c must be positive (Section 2)", LAM_EINVAL;
  if (!(p->Tc > 0)) return why = "Tc must be positive", LAM_EINVAL;
  if (!(p->Gamma >= 0)) return why = "Gamma must be non-negative", LAM_EINVAL;
  if (p->force_form != 0 && p->force_form != 1) return why = "force_form must be 0 or 1", LAM_EINVAL;
  if (p->pop_storage != 0 && p->pop_storage != 1)
    return why = "pop_storage must be 0 (FP32) or 1 (FP16)", LAM_EINVAL;
  if (p->walls != 0 && p->walls != 1) return why = "walls must be 0 or 1", LAM_EINVAL;
  if (p->hydro != 0 && p->hydro != 1) return why = "hydro must be 0 or 1", LAM_EINVAL;
  if (p->n_phi_sub < 0 || p->n_T_sub < 0) return why = "sub-step counts must be >= 0", LAM_EINVAL;
  if (p->tile_hint != 0 && p->tile_hint != 8 && p->tile_hint != 16 && p->tile_hint != 32 &&
      p->tile_hint != 64)
    return why = "tile_hint must be 0, 8, 16, 32 or 64", LAM_EINVAL;
  if (!p->allow_unstable) {
    if (p->n_phi_sub > 0 && p->n_phi_sub < auto_nphi(*p))
      return why = "n_phi_sub below the stability bound (set allow_unstable to force)", LAM_EINVAL;
    if (p->n_T_sub > 0 && p->xi > 0 && p->xi / p->n_T_sub > 0.5)
      return why = "n_T_sub gives xi/n_T > 1/2 (set allow_unstable to force)", LAM_EINVAL;
  }
  return LAM_OK;
}

int fill_guards(lam_sim* s) {
  for (int i = 0; i < GUARD_BANDS; ++i)
    HIPCHK(s, hipMemsetD32Async((hipDeviceptr_t)(s->ws + s->guard[i]), (int)GUARD_WORD,
                                LAM_GUARD_BYTES / 4, s->st));
  s->guards_set = true;
  return LAM_OK;
}

}  // namespace

extern "C" {

int lam_workspace_bytes(const lam_params* p, size_t* bytes) {
  std::string why;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  if (!bytes) return fail(nullptr, LAM_EINVAL, "null output");
  *bytes = layout(*p).total;
  return LAM_OK;
}

int lam_create(const lam_params* p, void* d_workspace, size_t bytes, void* hip_stream,
               lam_sim** out) {
  std::string why;
  if (!out) return fail(nullptr, LAM_EINVAL, "null output handle");
  *out = nullptr;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  Layout L = layout(*p);
  if (!d_workspace || bytes < L.total)
    return fail(nullptr, LAM_ESIZE, "workspace smaller than lam_workspace_bytes()");
  if (((uintptr_t)d_workspace) & 255) return fail(nullptr, LAM_EINVAL, "workspace not 256-byte aligned");
  lam_sim* s = new lam_sim();
  s->p = *p;
  s->Q = p->dim == 2 ? 9 : 19;
  s->N = (size_t)p->nx * p->ny * (p->dim == 3 ? p->nz : 1);
  s->nrows = p->dim == 2 ? p->ny : p->nz;
  s->nphi = p->n_phi_sub > 0 ? p->n_phi_sub : auto_nphi(*p);
  s->nT = p->n_T_sub > 0 ? p->n_T_sub : auto_nT(*p);
  s->st = (hipStream_t)hip_stream;
  // 2D tile height: 32 (64 x 32 tiles, measured fastest at 1024^2 and 4096^2) unless that leaves
  // fewer tiles than compute units, then 16 (512^2: lb2d 7.5 -> 6.3 us, phi2d 6.7 -> 6.5 us; the
  // halo of lower tiles costs more than the idle units they fill at 1024^2 and above)
  int ty_auto = 32;
  if (p->dim == 2 && ((p->nx + 63) / 64) * ((p->ny + 31) / 32) < 256) ty_auto = 16;
  s->ty_lb = p->tile_hint ? p->tile_hint : ty_auto;
  s->ty_phi = p->tile_hint ? p->tile_hint : ty_auto;
  s->ws = (char*)d_workspace;
  s->ws_bytes = bytes;
  for (int i = 0; i < 2; ++i) {
    s->g[i] = (void*)(s->ws + L.g[i]);
    s->phi[i] = (float*)(s->ws + L.phi[i]);
    s->psi[i] = (float*)(s->ws + L.psi[i]);
  }
  s->u = (float*)(s->ws + L.u);
  for (int i = 0; i < 3; ++i) s->T[i] = (float*)(s->ws + L.T[i]);
  s->partials = (double*)(s->ws + L.partials);
  s->result = (double*)(s->ws + L.result);
  s->spec = s->ws + L.spec;
  s->nblk = L.nblk;
  for (int i = 0; i < GUARD_BANDS; ++i) s->guard[i] = L.guard[i];
  s->pop_bytes = (p->pop_storage == 1 ? 2 : 4) * (size_t)s->Q * s->N;
  KParams& k = s->k;
  k.nx = p->nx;
  k.ny = p->ny;
  k.nz = p->dim == 3 ? p->nz : 1;
  k.walls = p->walls;
  k.hydro = p->hydro;
  k.force_form = p->force_form;
  k.omega = (float)(1.0 / p->tau);
  k.kforce = (float)(1.0 - 0.5 / p->tau);
  k.Gamma = (float)p->Gamma;
  k.b = (float)p->b;
  k.kappa = (float)p->kappa;
  k.c = (float)p->c;
  k.Tc = (float)p->Tc;
  k.h = (float)(1.0 / s->nphi);
  k.gx = (float)p->body_force[0];
  k.gy = (float)p->body_force[1];
  k.gz = (float)p->body_force[2];
  k.n_T = p->xi > 0 ? s->nT : 0;
  k.r_T = p->xi > 0 ? (float)(p->xi / s->nT) : 0.f;
  k.half_pops = p->pop_storage == 1;
  k.zch_phi = p->dim == 3 ? phi3d_chunk(p->nx, p->ny, p->nz) : 1;
  s->step = 0;
  s->initialised = false;
  *out = s;
  return LAM_OK;
}

int lam_substeps(const lam_sim* s, int32_t* n_phi, int32_t* n_T) {
  if (!s) return LAM_EINVAL;
  if (n_phi) *n_phi = s->nphi;
  if (n_T) *n_T = s->nT;
  return LAM_OK;
}

int lam_init_fields(lam_sim* s, const float* d_phi0, const float* d_u0, const float* d_n0) {
  if (!s || !d_phi0) return fail(s, LAM_EINVAL, "null simulation or phi0");
  HIPCHK(s, hipMemcpyAsync(s->phi[0], d_phi0, sizeof(float) * s->N, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(s, launch_init(s->k, s->p.dim, d_n0, d_u0, s->g[0], s->st));
  HIPCHK(s, hipMemcpyAsync(s->g[1], s->g[0], s->pop_bytes, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(s, hipMemsetAsync(s->u, 0, sizeof(float) * s->p.dim * s->N, s->st));
  HIPCHK(s, launch_init_T(s->nrows, s->p.walls, (float)s->p.T0, (float)s->p.Tw, s->p.xi < 0,
                          s->T[0], s->T[1], s->st));
  if (int rc = fill_guards(s)) return rc;
  s->step = 0;
  s->initialised = true;
  return LAM_OK;
}

}  // extern "C"
// Lattice of a simulation, for the surrogate driver in the same library (not part of the C-ABI).
namespace lam {
// True when lam_advance_temperature changes no temperature (no diffusion sub-steps).
bool sim_temperature_frozen(const lam_sim* s) { return s->k.n_T == 0; }
int sim_dims(const lam_sim* s, int* dim, int* nx, int* ny, int* walls) {
  if (!s || !s->initialised) return LAM_EINVAL;
  *dim = s->p.dim;
  *nx = s->p.nx;
  *ny = s->p.ny;
  *walls = s->p.walls;
  return LAM_OK;
}
}  // namespace lam
extern "C" {

int lam_set_fields(lam_sim* s, const float* d_phi, const float* d_u, const float* d_n) {
  if (!s || !d_phi) return fail(s, LAM_EINVAL, "null simulation or phi");
  if (!s->initialised) return fail(s, LAM_EINVAL, "fields not initialised");
  const int cur = (int)(s->step & 1);
  HIPCHK(s, hipMemcpyAsync(s->phi[cur], d_phi, sizeof(float) * s->N, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(s, launch_init(s->k, s->p.dim, d_n, d_u, s->g[cur], s->st));
  return LAM_OK;
}

int lam_advance_temperature(lam_sim* s, int64_t nsteps) {
  if (!s || nsteps < 0) return fail(s, LAM_EINVAL, "bad arguments");
  if (!s->initialised) return fail(s, LAM_EINVAL, "fields not initialised");
  if (nsteps == 0) return LAM_OK;
  if (s->nrows > 8192) return fail(s, LAM_EINVAL, "more than 8192 layers along the wall axis");
  const int cur = (int)(s->step & 1), nxt = (int)((s->step + nsteps) & 1);
  const float* src = s->T[cur];
  if (s->k.n_T > 0) {
    HIPCHK(s, launch_temperature(s->nrows, s->p.walls, s->k.r_T, s->k.n_T, nsteps, src, s->T[2], s->st));
    src = s->T[2];
  }
  if (src != s->T[nxt])
    HIPCHK(s, hipMemcpyAsync(s->T[nxt], src, sizeof(float) * s->nrows, hipMemcpyDeviceToDevice, s->st));
  // phi lives in the buffer of the current parity; move it with the step count
  if (cur != nxt)
    HIPCHK(s, hipMemcpyAsync(s->phi[nxt], s->phi[cur], sizeof(float) * s->N, hipMemcpyDeviceToDevice, s->st));
  if (cur != nxt)
    HIPCHK(s, hipMemcpyAsync(s->g[nxt], s->g[cur], s->pop_bytes, hipMemcpyDeviceToDevice, s->st));
  s->step += nsteps;
  return LAM_OK;
}

}  // extern "C"

namespace {
// Event pair of the next timed launch of class cls, or (nullptr, nullptr) when timing is off.
struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
};
EvPair timing_slot(lam_sim* s, int cls) {
  EvPair e;
  if (!s->timing) return e;
  if (s->ev_used + 2 > s->ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t h;
      if (hipEventCreate(&h) != hipSuccess) return e;
      s->ev.push_back(h);
      s->ev_cls.push_back(0);
    }
  }
  size_t slot = s->ev_used;
  s->ev_cls[slot] = cls;
  s->ev_used += 2;
  e.a = s->ev[slot];
  e.b = s->ev[slot + 1];
  return e;
}
}  // namespace

extern "C" {

int lam_set_timing(lam_sim* s, int32_t enable) {
  if (!s) return LAM_EINVAL;
  s->timing = enable != 0;
  s->ev_used = 0;
  return LAM_OK;
}

int lam_kernel_times(lam_sim* s, double* h_ms, int64_t* h_launches, int32_t nk) {
  if (!s || !h_ms || !h_launches || nk < 1) return fail(s, LAM_EINVAL, "bad arguments");
  for (int k = 0; k < nk; ++k) {
    h_ms[k] = 0.0;
    h_launches[k] = 0;
  }
  HIPCHK(s, hipStreamSynchronize(s->st));
  for (size_t i = 0; i < s->ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(s, hipEventElapsedTime(&ms, s->ev[i], s->ev[i + 1]));
    int c = s->ev_cls[i];
    if (c < nk) {
      h_ms[c] += ms;
      h_launches[c] += 1;
    }
  }
  s->ev_used = 0;
  return LAM_OK;
}

}  // extern "C"

namespace {

// The launches of one time step from parity cur (every argument depends only on the parity).
int one_step(lam_sim* s, int cur) {
  const KParams& k = s->k;
  const bool d3 = s->p.dim == 3;
  const int maxsub = d3 ? 1 : phi2d_max_sub();
  const int nxt = cur ^ 1;
  if (k.hydro) {
    EvPair ev = timing_slot(s, LAM_K_LB);
    if (d3)
      HIPCHK(s, launch_lb3d(k, MODE_STEP, s->g[cur], s->g[nxt], s->phi[cur], s->T[cur], s->u,
                            nullptr, nullptr, s->st, ev.a, ev.b));
    else
      HIPCHK(s, launch_lb2d(k, s->ty_lb, MODE_STEP, s->g[cur], s->g[nxt], s->phi[cur],
                            s->T[cur], s->u, nullptr, nullptr, s->st, ev.a, ev.b));
  }
  int remaining = s->nphi, which = 0;
  const float* src = s->phi[cur];
  while (remaining > 0) {
    int sub = std::min(remaining, maxsub);
    bool last = remaining == sub;
    float* dst = last ? s->phi[nxt] : s->psi[which];
    which ^= 1;
    EvPair ev = timing_slot(s, LAM_K_PHI);
    const int do_T = last && k.n_T > 0;
    if (d3)
      HIPCHK(s, launch_phi3d(k, src, dst, s->u, s->T[cur], s->T[nxt], s->T[2], do_T, s->st,
                             ev.a, ev.b));
    else
      HIPCHK(s, launch_phi2d(k, s->ty_phi, sub, src, dst, s->u, s->T[cur], s->T[nxt], s->T[2],
                             do_T, s->st, ev.a, ev.b));
    src = dst;
    remaining -= sub;
  }
  return LAM_OK;
}

// Captures the step pair (parity 0, then 1) on the simulation's stream into s->pair_graph.
int capture_pair(lam_sim* s) {
  hipGraph_t g = nullptr;
  hipError_t r = hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal);
  if (r != hipSuccess) return hip_fail(s, r, "hipStreamBeginCapture");
  int rc = one_step(s, 0);
  if (rc == LAM_OK) rc = one_step(s, 1);
  hipError_t r2 = hipStreamEndCapture(s->st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (r2 != hipSuccess) return hip_fail(s, r2, "hipStreamEndCapture");
  r = hipGraphInstantiate(&s->pair_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (r != hipSuccess) {
    s->pair_graph = nullptr;
    return hip_fail(s, r, "hipGraphInstantiate");
  }
  return LAM_OK;
}

}  // namespace

extern "C" {

int lam_step(lam_sim* s, int64_t nsteps) {
  if (!s || nsteps < 0) return fail(s, LAM_EINVAL, "bad arguments");
  if (!s->initialised) return fail(s, LAM_EINVAL, "fields not initialised");
  roctxRangePushA("lam_step");
  int rc = LAM_OK;
  int64_t done = 0;
  auto direct = [&](int64_t n) {
    for (int64_t i = 0; i < n && rc == LAM_OK; ++i) {
      rc = one_step(s, (int)(s->step & 1));
      if (rc == LAM_OK) {
        s->step++;
        done++;
      }
    }
  };
  auto replay = [&](int64_t pairs) {
    for (int64_t i = 0; i < pairs && rc == LAM_OK; ++i) {
      hipError_t r = hipGraphLaunch(s->pair_graph, s->st);
      if (r != hipSuccess) {
        rc = hip_fail(s, r, "hipGraphLaunch");
        break;
      }
      s->step += 2;
      done += 2;
    }
  };
  // Graph replays of step pairs are possible on a stream of the caller (not the legacy default
  // stream) with timing off, when the stream is not itself being captured by the caller (then the
  // launches go into that capture).  Whether they are faster than direct launches is measured
  // once, on the first call long enough for it: 8 direct steps against 4 replayed pairs, timed
  // with events (these are steps of the call; that call waits for them).
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool graphs = s->st != nullptr && !s->timing && s->graph_mode != 0 && nsteps >= 3 &&
                      hipStreamIsCapturing(s->st, &cs) == hipSuccess &&
                      cs == hipStreamCaptureStatusNone;
  if (graphs && (s->graph_mode == 1 || nsteps >= 24)) {
    if (s->step & 1) direct(1);  // reach an even step first
    if (rc == LAM_OK && !s->pair_graph) rc = capture_pair(s);
    if (rc == LAM_OK && s->graph_mode < 0) {
      hipEvent_t e[3] = {nullptr, nullptr, nullptr};
      hipError_t r = hipSuccess;
      for (int i = 0; i < 3 && r == hipSuccess; ++i) r = hipEventCreate(&e[i]);
      if (r == hipSuccess) r = hipEventRecord(e[0], s->st);
      if (r == hipSuccess) direct(8);
      if (r == hipSuccess && rc == LAM_OK) r = hipEventRecord(e[1], s->st);
      if (r == hipSuccess && rc == LAM_OK) replay(4);
      if (r == hipSuccess && rc == LAM_OK) r = hipEventRecord(e[2], s->st);
      float t_direct = 0.f, t_graph = 0.f;
      if (r == hipSuccess && rc == LAM_OK) r = hipEventSynchronize(e[2]);
      if (r == hipSuccess && rc == LAM_OK) r = hipEventElapsedTime(&t_direct, e[0], e[1]);
      if (r == hipSuccess && rc == LAM_OK) r = hipEventElapsedTime(&t_graph, e[1], e[2]);
      for (int i = 0; i < 3; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
      if (r != hipSuccess && rc == LAM_OK) rc = hip_fail(s, r, "graph timing");
      if (rc == LAM_OK) {
        s->direct_us = t_direct * 1e3f / 8.f;
        s->graph_us = t_graph * 1e3f / 8.f;
        s->graph_mode = t_graph < t_direct ? 1 : 0;
      }
    }
    if (rc == LAM_OK && s->graph_mode == 1) {
      roctxRangePushA("lam_step graph replays");
      replay((nsteps - done) / 2);
      roctxRangePop();
    }
  }
  direct(nsteps - done);
  roctxRangePop();
  return rc;
}

int lam_launch_mode(const lam_sim* s, int32_t* graphs, float* direct_us, float* graph_us) {
  if (!s) return fail(nullptr, LAM_EINVAL, "null simulation");
  if (graphs) *graphs = s->graph_mode;
  if (direct_us) *direct_us = s->direct_us;
  if (graph_us) *graph_us = s->graph_us;
  return LAM_OK;
}

int lam_observables(lam_sim* s, lam_obs* o) {
  if (!s || !o) return fail(s, LAM_EINVAL, "bad arguments");
  if (!s->initialised) return fail(s, LAM_EINVAL, "fields not initialised");
  const int cur = (int)(s->step & 1);
  int nblk;
  if (s->p.dim == 3) {
    nblk = blocks3d(s->k);
    HIPCHK(s, launch_lb3d(s->k, MODE_OBS, s->g[cur], nullptr, s->phi[cur], s->T[cur], nullptr,
                          nullptr, s->partials, s->st));
  } else {
    nblk = lb2d_blocks(s->k, s->ty_lb);
    HIPCHK(s, launch_lb2d(s->k, s->ty_lb, MODE_OBS, s->g[cur], nullptr, s->phi[cur], s->T[cur],
                          nullptr, nullptr, s->partials, s->st));
  }
  HIPCHK(s, launch_finalize(s->partials, nblk, s->result, s->st));
  double r[R_N];
  HIPCHK(s, hipMemcpyAsync(r, s->result, sizeof(r), hipMemcpyDeviceToHost, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  memset(o, 0, sizeof(*o));
  o->mass_dev = r[R_MASS];
  o->mom[0] = r[R_JX];
  o->mom[1] = r[R_JY];
  o->mom[2] = r[R_JZ];
  o->phi_sum = r[R_PHI];
  o->max_u = r[R_UMAX];
  o->mach = r[R_UMAX] * sqrt(3.0);
  o->free_energy = r[R_FE];
  o->step = s->step;
  o->nonfinite = r[R_BAD] != 0.0;
  if (o->nonfinite) return fail(s, LAM_ENONFINITE, "state holds NaN or infinite values");
  return LAM_OK;
}

int lam_structure_factor(lam_sim* s, double* h_S, int32_t nbins, double* k_peak, double* S_peak,
                         double* k_mean) {
  if (!s || !h_S || nbins < 3) return fail(s, LAM_EINVAL, "bad arguments (need nbins >= 3)");
  if (s->p.dim != 2) return fail(s, LAM_EINVAL, "structure factor is 2D only");
  if (nbins > std::max(s->p.nx, s->p.ny)) return fail(s, LAM_EINVAL, "nbins > max(nx, ny)");
  HIPCHK(s, structure_factor_2d(s->k, s->phi[s->step & 1], s->spec, nbins, h_S, k_peak, S_peak,
                                k_mean, s->st));
  return LAM_OK;
}

int lam_structure_factor_static(const float* d_phi, int32_t nx, int32_t ny, void* hip_stream,
                                double* h_S, int32_t nbins, double* k_peak, double* S_peak,
                                double* k_mean) {
  if (!d_phi || !h_S || nbins < 3 || nx < 1 || ny < 1)
    return fail(nullptr, LAM_EINVAL, "bad arguments (need d_phi, h_S, nbins >= 3)");
  if (nbins > std::max(nx, ny)) return fail(nullptr, LAM_EINVAL, "nbins > max(nx, ny)");
  const size_t need = spectra_scratch_bytes(nx, ny);
  if (need > static_scratch_capacity())
    return fail(nullptr, LAM_ESIZE,
                "lattice needs " + std::to_string(need) + " bytes of scratch; the static array "
                "holds " + std::to_string(static_scratch_capacity()) + " (LAM_SK_STATIC_BYTES)");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (st) {
    hipDevice_t sdev = -1;
    e = hipStreamGetDevice(st, &sdev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipStreamGetDevice");
    if (sdev != dev)
      return fail(nullptr, LAM_EINVAL, "the stream belongs to another device than the current one");
  }
  void* scr = nullptr;
  e = static_scratch(dev, &scr);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
  KParams k{};
  k.nx = nx;
  k.ny = ny;
  k.nz = 1;
  e = structure_factor_2d(k, d_phi, scr, nbins, h_S, k_peak, S_peak, k_mean, st);
  if (e != hipSuccess) return hip_fail(nullptr, e, "structure factor");
  return LAM_OK;
}

int lam_orientation(lam_sim* s, double* h_hist, int32_t nbins, double* Q, double* h_Qrow) {
  if (!s || !h_hist || nbins < 1 || nbins > 36) return fail(s, LAM_EINVAL, "bad arguments (1 <= nbins <= 36)");
  if (s->p.dim == 3)
    HIPCHK(s, orientation_3d(s->k, s->phi[s->step & 1], s->spec, nbins, h_hist, Q, h_Qrow, s->st));
  else
    HIPCHK(s, orientation_2d(s->k, s->phi[s->step & 1], s->spec, nbins, h_hist, Q, h_Qrow, s->st));
  return LAM_OK;
}

int lam_get_fields(lam_sim* s, float* d_phi, float* d_u, float* d_n, float* d_T) {
  if (!s) return fail(s, LAM_EINVAL, "null simulation");
  if (!s->initialised) return fail(s, LAM_EINVAL, "fields not initialised");
  const int cur = (int)(s->step & 1);
  if (d_phi)
    HIPCHK(s, hipMemcpyAsync(d_phi, s->phi[cur], sizeof(float) * s->N, hipMemcpyDeviceToDevice,
                             s->st));
  if ((d_u || d_n) && s->p.dim == 3)
    HIPCHK(s, launch_lb3d(s->k, MODE_FIELDS, s->g[cur], nullptr, s->phi[cur], s->T[cur],
                          d_u ? d_u : s->u, d_n, nullptr, s->st));
  else if (d_u || d_n)
    HIPCHK(s, launch_lb2d(s->k, s->ty_lb, MODE_FIELDS, s->g[cur], nullptr, s->phi[cur],
                          s->T[cur], d_u ? d_u : s->u, d_n, nullptr, s->st));
  if (d_T) {
    size_t layer = (size_t)s->p.nx * (s->p.dim == 3 ? s->p.ny : 1);
    HIPCHK(s, launch_broadcast_T(s->T[cur], s->N, layer, d_T, s->st));
  }
  return LAM_OK;
}

int lam_state_bytes(const lam_sim* s, size_t* bytes) {
  if (!s || !bytes) return LAM_EINVAL;
  *bytes = header_bytes() + s->pop_bytes + sizeof(float) * (s->N + s->nrows);
  return LAM_OK;
}

int lam_get_state(lam_sim* s, void* d_buf, size_t bytes) {
  size_t need;
  lam_state_bytes(s, &need);
  if (!s || !d_buf) return fail(s, LAM_EINVAL, "bad arguments");
  if (bytes < need) return fail(s, LAM_ESIZE, "checkpoint buffer too small");
  const int cur = (int)(s->step & 1);
  char* b = (char*)d_buf;
  HIPCHK(s, launch_write_header(s->p.dim, s->p.nx, s->p.ny, s->k.nz, s->step, s->Q,
                                (int)(s->pop_bytes / ((size_t)s->Q * s->N)), b, s->st));
  b += header_bytes();
  HIPCHK(s, hipMemcpyAsync(b, s->g[cur], s->pop_bytes, hipMemcpyDeviceToDevice, s->st));
  b += s->pop_bytes;
  HIPCHK(s, hipMemcpyAsync(b, s->phi[cur], sizeof(float) * s->N, hipMemcpyDeviceToDevice, s->st));
  b += sizeof(float) * s->N;
  HIPCHK(s, hipMemcpyAsync(b, s->T[cur], sizeof(float) * s->nrows, hipMemcpyDeviceToDevice, s->st));
  return LAM_OK;
}

int lam_set_state(lam_sim* s, const void* d_buf, size_t bytes) {
  size_t need;
  lam_state_bytes(s, &need);
  if (!s || !d_buf) return fail(s, LAM_EINVAL, "bad arguments");
  if (bytes < need) return fail(s, LAM_ESIZE, "checkpoint buffer too small");
  char hdr[256];
  HIPCHK(s, hipMemcpyAsync(hdr, d_buf, sizeof(hdr), hipMemcpyDeviceToHost, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  int64_t step;
  if (!check_header(hdr, s->p.dim, s->p.nx, s->p.ny, s->k.nz, s->Q,
                    (int)(s->pop_bytes / ((size_t)s->Q * s->N)), &step))
    return fail(s, LAM_ESTATE, "checkpoint does not match this lattice");
  const int cur = (int)(step & 1);
  const char* b = (const char*)d_buf + header_bytes();
  for (int i = 0; i < 2; ++i)
    HIPCHK(s, hipMemcpyAsync(s->g[i], b, s->pop_bytes, hipMemcpyDeviceToDevice, s->st));
  b += s->pop_bytes;
  HIPCHK(s, hipMemcpyAsync(s->phi[cur], b, sizeof(float) * s->N, hipMemcpyDeviceToDevice, s->st));
  b += sizeof(float) * s->N;
  for (int i = 0; i < 2; ++i)
    HIPCHK(s, hipMemcpyAsync(s->T[i], b, sizeof(float) * s->nrows, hipMemcpyDeviceToDevice, s->st));
  if (int rc = fill_guards(s)) return rc;
  s->step = step;
  s->initialised = true;
  return LAM_OK;
}

int lam_guard_layout(const lam_params* p, size_t* h_offsets, int32_t max, int32_t* count) {
  std::string why;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  if (!count) return fail(nullptr, LAM_EINVAL, "null count");
  *count = GUARD_BANDS;
  if (max < GUARD_BANDS || !h_offsets) return fail(nullptr, LAM_ESIZE, "offset array too small");
  const Layout L = layout(*p);
  for (int i = 0; i < GUARD_BANDS; ++i) h_offsets[i] = L.guard[i];
  return LAM_OK;
}

int lam_check_guards(lam_sim* s, int32_t* h_first_bad) {
  if (!s) return LAM_EINVAL;
  if (h_first_bad) *h_first_bad = -1;
  if (!s->guards_set) return fail(s, LAM_EINVAL, "fields not initialised (no guard bands yet)");
  std::vector<uint32_t> h((size_t)GUARD_BANDS * LAM_GUARD_BYTES / 4);
  for (int i = 0; i < GUARD_BANDS; ++i)
    HIPCHK(s, hipMemcpyAsync(h.data() + (size_t)i * LAM_GUARD_BYTES / 4, s->ws + s->guard[i],
                             LAM_GUARD_BYTES, hipMemcpyDeviceToHost, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  for (int i = 0; i < GUARD_BANDS; ++i) {
    int bad = 0;
    for (int w = 0; w < LAM_GUARD_BYTES / 4; ++w)
      bad += h[(size_t)i * LAM_GUARD_BYTES / 4 + w] != GUARD_WORD;
    if (bad) {
      if (h_first_bad) *h_first_bad = i;
      return fail(s, LAM_ECORRUPT, std::string("guard band after ") + GUARD_AFTER[i] +
                                       " overwritten (" + std::to_string(bad) + " of " +
                                       std::to_string(LAM_GUARD_BYTES / 4) + " words)");
    }
  }
  return LAM_OK;
}

const char* lam_last_error(const lam_sim* s) {
  return s ? s->err.c_str() : g_create_error.c_str();
}

void lam_destroy(lam_sim* s) {
  if (!s) return;
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  if (s->pair_graph) (void)hipGraphExecDestroy(s->pair_graph);
  delete s;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Ensembles.
struct lam_ensemble {
  std::vector<lam_sim*> sims;
  std::vector<EnsMember> host_members;
  std::vector<int> host_tiles;
  EnsMember* d_members = nullptr;
  int* d_tile_member = nullptr;
  unsigned* d_queue = nullptr;  // work-queue counters of the persistent kernels
  int ntiles = 0, ty = 32, nphi = 1, hydro = 1, half = 0;
  int cus = 256, grid = 512;  // compute units; workgroups of the persistent launches
  hipStream_t st = nullptr;
  hipGraphExec_t graph = nullptr;
  int64_t sites = 0;
  std::string err;
};

namespace {

int efail(lam_ensemble* e, int code, const std::string& msg) {
  if (e) e->err = msg;
  else g_create_error = msg;
  return code;
}

struct EnsLayout {
  std::vector<size_t> off, bytes;
  size_t members, tiles, queue, total;
};

int ens_layout(const lam_params* m, int count, EnsLayout& L, std::string& why) {
  if (!m || count < 1) return why = "need at least one member", LAM_EINVAL;
  size_t off = 0, maxtiles = 0;
  for (int i = 0; i < count; ++i) {
    int rc = validate(&m[i], why);
    if (rc) return why = "member " + std::to_string(i) + ": " + why, rc;
    if (m[i].dim != 2) return why = "ensemble members must be 2D", LAM_EINVAL;
    if (m[i].hydro != m[0].hydro || m[i].pop_storage != m[0].pop_storage)
      return why = "members differ in hydro or pop_storage", LAM_EINVAL;
    int n0 = m[0].n_phi_sub > 0 ? m[0].n_phi_sub : auto_nphi(m[0]);
    int ni = m[i].n_phi_sub > 0 ? m[i].n_phi_sub : auto_nphi(m[i]);
    if (n0 != ni) return why = "members need different phi sub-step counts", LAM_EINVAL;
    size_t b = layout(m[i]).total;
    L.off.push_back(off);
    L.bytes.push_back(b);
    off = align256(off + b);
    maxtiles += (size_t)((m[i].nx + 63) / 64) * ((m[i].ny + 7) / 8);  // smallest tile height
  }
  L.members = off;
  off = align256(off + sizeof(EnsMember) * count);
  L.tiles = off;
  off = align256(off + sizeof(int) * maxtiles);
  L.queue = off;
  off = align256(off + sizeof(unsigned) * ens_queue_words());
  L.total = off;
  return LAM_OK;
}

int ens_build_tiles(lam_ensemble* e, int ty) {
  e->host_tiles.clear();
  int t = 0;
  for (size_t i = 0; i < e->sims.size(); ++i) {
    const KParams& k = e->sims[i]->k;
    int n = ((k.nx + 63) / 64) * ((k.ny + ty - 1) / ty);
    e->host_members[i].tile0 = t;
    for (int j = 0; j < n; ++j) e->host_tiles.push_back((int)i);
    t += n;
  }
  e->ntiles = t;
  e->ty = ty;
  hipError_t r = hipMemcpy(e->d_members, e->host_members.data(),
                           sizeof(EnsMember) * e->host_members.size(), hipMemcpyHostToDevice);
  if (r == hipSuccess)
    r = hipMemcpy(e->d_tile_member, e->host_tiles.data(), sizeof(int) * e->host_tiles.size(),
                  hipMemcpyHostToDevice);
  if (r != hipSuccess) return efail(e, LAM_EHIP, std::string("tile table: ") + hipGetErrorString(r));
  if (e->graph) {
    (void)hipGraphExecDestroy(e->graph);
    e->graph = nullptr;
  }
  return LAM_OK;
}

hipError_t ens_one_step(lam_ensemble* e, int cur) {
  return launch_ens_step(e->d_members, e->d_tile_member, e->ntiles, e->ty, cur, e->half, e->hydro,
                         e->nphi, e->grid, e->d_queue, e->st);
}

}  // namespace

extern "C" {

int lam_ensemble_workspace_bytes(const lam_params* members, int32_t count, size_t* bytes) {
  EnsLayout L;
  std::string why;
  int rc = ens_layout(members, count, L, why);
  if (rc) return efail(nullptr, rc, why);
  if (!bytes) return efail(nullptr, LAM_EINVAL, "null output");
  *bytes = L.total;
  return LAM_OK;
}

int lam_ensemble_create(const lam_params* members, int32_t count, void* d_workspace, size_t bytes,
                        void* hip_stream, lam_ensemble** out) {
  if (!out) return efail(nullptr, LAM_EINVAL, "null output handle");
  *out = nullptr;
  EnsLayout L;
  std::string why;
  int rc = ens_layout(members, count, L, why);
  if (rc) return efail(nullptr, rc, why);
  if (!d_workspace || bytes < L.total)
    return efail(nullptr, LAM_ESIZE, "workspace smaller than lam_ensemble_workspace_bytes()");
  if (((uintptr_t)d_workspace) & 255) return efail(nullptr, LAM_EINVAL, "workspace not 256-byte aligned");
  lam_ensemble* e = new lam_ensemble();
  e->st = (hipStream_t)hip_stream;
  char* ws = (char*)d_workspace;
  for (int i = 0; i < count; ++i) {
    lam_sim* s = nullptr;
    rc = lam_create(&members[i], ws + L.off[i], L.bytes[i], hip_stream, &s);
    if (rc) {
      lam_ensemble_destroy(e);
      return efail(nullptr, rc, "member " + std::to_string(i) + ": " + g_create_error);
    }
    e->sims.push_back(s);
    EnsMember m{};
    m.P = s->k;
    m.g[0] = s->g[0];
    m.g[1] = s->g[1];
    m.phi[0] = s->phi[0];
    m.phi[1] = s->phi[1];
    m.psi[0] = s->psi[0];
    m.psi[1] = s->psi[1];
    m.u = s->u;
    for (int k = 0; k < 3; ++k) m.T[k] = s->T[k];
    e->host_members.push_back(m);
    e->sites += (int64_t)s->N;
  }
  e->nphi = e->sims[0]->nphi;
  e->hydro = members[0].hydro;
  e->half = members[0].pop_storage == 1;
  e->d_members = (EnsMember*)(ws + L.members);
  e->d_tile_member = (int*)(ws + L.tiles);
  e->d_queue = (unsigned*)(ws + L.queue);
  {  // the queues start at zero; afterwards every launch leaves them at zero
    int dev = 0, cus = 0;
    hipError_t r = hipGetDevice(&dev);
    if (r == hipSuccess) r = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (r == hipSuccess) r = hipMemsetAsync(e->d_queue, 0, sizeof(unsigned) * ens_queue_words(), e->st);
    if (r != hipSuccess) {
      lam_ensemble_destroy(e);
      return efail(nullptr, LAM_EHIP, std::string("ensemble queues: ") + hipGetErrorString(r));
    }
    e->cus = std::max(8, (cus + 7) / 8 * 8);
    e->grid = 2 * e->cus;  // persistent, two workgroups per compute unit, until tuned
  }
  rc = ens_build_tiles(e, 32);
  if (rc) {
    std::string msg = e->err;
    lam_ensemble_destroy(e);
    return efail(nullptr, rc, msg);
  }
  *out = e;
  return LAM_OK;
}

int lam_ensemble_member(lam_ensemble* e, int32_t i, lam_sim** out) {
  if (!e || !out || i < 0 || i >= (int)e->sims.size()) return efail(e, LAM_EINVAL, "bad member index");
  *out = e->sims[i];
  return LAM_OK;
}

int lam_ensemble_init_fields(lam_ensemble* e, const float* const* d_phi0) {
  if (!e || !d_phi0) return efail(e, LAM_EINVAL, "bad arguments");
  for (size_t i = 0; i < e->sims.size(); ++i) {
    int rc = lam_init_fields(e->sims[i], d_phi0[i], nullptr, nullptr);
    if (rc) return efail(e, rc, "member " + std::to_string(i) + ": " + e->sims[i]->err);
  }
  return LAM_OK;
}

int lam_ensemble_step(lam_ensemble* e, int64_t nsteps) {
  if (!e || nsteps < 0) return efail(e, LAM_EINVAL, "bad arguments");
  const int64_t step0 = e->sims[0]->step;
  for (lam_sim* s : e->sims) {
    if (!s->initialised) return efail(e, LAM_EINVAL, "member fields not initialised");
    if (s->step != step0) return efail(e, LAM_EINVAL, "members were stepped separately");
  }
  int64_t done = 0, step = step0;
  auto direct = [&]() -> int {
    hipError_t r = ens_one_step(e, (int)(step & 1));
    if (r != hipSuccess) return efail(e, LAM_EHIP, std::string("ensemble step: ") + hipGetErrorString(r));
    ++step;
    ++done;
    return LAM_OK;
  };
  if ((step & 1) && done < nsteps) {
    int rc = direct();
    if (rc) return rc;
  }
  if (e->st && nsteps - done >= 2) {
    if (!e->graph) {  // capture one pair of steps (parity 0 then 1) once
      hipGraph_t g;
      hipError_t r = hipStreamBeginCapture(e->st, hipStreamCaptureModeThreadLocal);
      if (r == hipSuccess) r = ens_one_step(e, 0);
      if (r == hipSuccess) r = ens_one_step(e, 1);
      hipError_t r2 = hipStreamEndCapture(e->st, &g);
      if (r == hipSuccess) r = r2;
      if (r == hipSuccess) r = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
      if (r2 == hipSuccess) (void)hipGraphDestroy(g);
      if (r != hipSuccess) return efail(e, LAM_EHIP, std::string("graph capture: ") + hipGetErrorString(r));
    }
    while (nsteps - done >= 2) {
      hipError_t r = hipGraphLaunch(e->graph, e->st);
      if (r != hipSuccess) return efail(e, LAM_EHIP, std::string("graph launch: ") + hipGetErrorString(r));
      step += 2;
      done += 2;
    }
  }
  while (done < nsteps) {
    int rc = direct();
    if (rc) return rc;
  }
  for (lam_sim* s : e->sims) s->step = step;
  return LAM_OK;
}

int lam_ensemble_tune(lam_ensemble* e, int32_t steps, int32_t* tile_height,
                      int32_t* workgroups) {
  if (!e || steps < 1) return efail(e, LAM_EINVAL, "bad arguments");
  for (lam_sim* s : e->sims)
    if (s->initialised)
      return efail(e, LAM_EINVAL, "lam_ensemble_tune must come before lam_ensemble_init_fields");
  // a fixed state to time (phi = 0, fluid at rest, T as at the start); the members are left
  // uninitialised again afterwards
  for (lam_sim* s : e->sims) {
    hipError_t r = hipMemsetAsync(s->psi[0], 0, sizeof(float) * s->N, s->st);
    if (r != hipSuccess) return efail(e, LAM_EHIP, std::string("tuning: ") + hipGetErrorString(r));
    int rc = lam_init_fields(s, s->psi[0], nullptr, nullptr);
    if (rc) return efail(e, rc, "tuning: " + s->err);
  }
  hipEvent_t a = nullptr, b = nullptr;
  int rc = LAM_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    rc = efail(e, LAM_EHIP, "event creation");
  // grids: one workgroup per tile (0), or 1, 2, 4 persistent workgroups per compute unit
  const int heights[4] = {8, 16, 32, 64}, per_cu[4] = {0, 1, 2, 4};
  int best_ty = 32, best_grid = 0;
  float best_ms = 1e30f;
  for (int hi = 0; hi < 4 && !rc; ++hi) {
    for (int gi = 0; gi < 4 && !rc; ++gi) {
      e->grid = per_cu[gi] * e->cus;
      if ((rc = ens_build_tiles(e, heights[hi])) || (rc = lam_ensemble_step(e, 2))) break;
      hipError_t h;
      if ((h = hipEventRecord(a, e->st))) {
        rc = efail(e, LAM_EHIP, std::string("tuning: ") + hipGetErrorString(h));
        break;
      }
      if ((rc = lam_ensemble_step(e, steps))) break;
      float ms = 0.f;
      if ((h = hipEventRecord(b, e->st)) || (h = hipEventSynchronize(b)) ||
          (h = hipEventElapsedTime(&ms, a, b))) {
        rc = efail(e, LAM_EHIP, std::string("tuning: ") + hipGetErrorString(h));
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best_ty = heights[hi];
        best_grid = e->grid;
      }
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  for (lam_sim* s : e->sims) {
    s->initialised = false;
    s->step = 0;
  }
  if (rc) return rc;
  e->grid = best_grid;
  rc = ens_build_tiles(e, best_ty);
  if (rc) return rc;
  if (tile_height) *tile_height = best_ty;
  if (workgroups) *workgroups = best_grid;
  return LAM_OK;
}

int lam_ensemble_sites(const lam_ensemble* e, int64_t* sites) {
  if (!e || !sites) return LAM_EINVAL;
  *sites = e->sites;
  return LAM_OK;
}

const char* lam_ensemble_last_error(const lam_ensemble* e) {
  return e ? e->err.c_str() : g_create_error.c_str();
}

void lam_ensemble_destroy(lam_ensemble* e) {
  if (!e) return;
  if (e->graph) (void)hipGraphExecDestroy(e->graph);
  for (lam_sim* s : e->sims) lam_destroy(s);
  delete e;
}

}  // extern "C"
