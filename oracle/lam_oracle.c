/* lam_oracle.c -- plain FP64 CPU reference ("oracle") of the hybrid LB/FD lamellar-fluid model of
 * Gonnella, Lamura & Tiribocchi (arXiv:1102.3094).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the product path.  It shares no code with the GPU library.
 *
 * It is written for clarity, not speed: every quantity is computed on the whole lattice in the
 * order of the method, with ghost layers filled by the boundary rule before each stencil.
 * Where the paper leaves a detail open, the reading taken is stated at the place it is used.
 *
 * One time step, state (f^n, phi^n, T^n) -> (f^{n+1}, phi^{n+1}, T^{n+1}), all right-hand sides
 * evaluated at time level n:
 *   S1  a = (T - Tc)/Tc                                   reduced temperature, eq. (aterm)
 *   S2  ghost layers: periodic along x (and y in 3D); even reflection about the wall planes,
 *       which lie half a spacing outside the first and last layer of the last axis
 *   S3  L = lap(phi), M = lap(L), mu = a phi + b phi^3 - kappa L + c M          eq. (chem)
 *   S4  F_alpha = -d_beta P_alpha,beta with the pressure tensor of Section 2 without the ideal-gas
 *       term n T (the lattice-Boltzmann pressure n c_s^2 is kept instead, eq. (ff)); or
 *       F = -phi grad mu; plus n g for an optional uniform test acceleration g
 *   S5  n = sum f, n u = sum f e + F/2                                        eq. (moment)
 *   S6  BGK collision with the second-order equilibrium and Guo forcing   eqs (evoleqn, latticeforceterm)
 *   S7  streaming; a population that would cross a wall is bounced back (halfway bounce-back)
 *   S8  n_phi explicit Euler sub-steps of  d_t phi + div(phi u) = Gamma lap mu   eq. (massdiff)
 *       with u = u^n and a = a^n held fixed and mu recomputed each sub-step
 *   S9  n_T FTCS sub-steps of d_t T = xi lap T on the non-wall layers; wall layers stay at Tw
 * Spatial operators are second-order central differences (Section 2): 5/7-point Laplacian,
 * biharmonic = Laplacian of the Laplacian (13/25 points), and first derivatives (pressure tensor,
 * force, advection) as isotropic central differences over the D2Q9/D3Q19 velocity set.  With
 * the two-point first derivative instead, the coupled update cannot run the paper's own
 * hydrodynamic workload (tau = 5, instantaneous quench, 21 000 steps at Ma < 0.1, Section 3 and
 * the Mach statement of Section 2): it diverges within a thousand steps.
 */
#include "lam_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define GH 3 /* ghost depth needed by the biharmonic stencil and by the pressure-tensor divergence */

struct orc_sim {
  orc_params p;
  int d, Q, nphi, nT, wall; /* wall: index of the wall axis, or -1 if fully periodic */
  int n[3], g[3], E[3];
  long N, NE, st[3];        /* st: strides of the ghost-extended array */
  int e[19][3];
  double w[19];
  int opp[19];
  double *f, *fs, *phi, *T, *a;
  double *X1, *X2, *X3;      /* ghost-extended scratch */
  double *L, *M, *mu, *tmp, *psi, *lapmu, *adv, *Tn;
  double *grad_phi[3], *grad_L[3], *F[3], *u[3];
  long step;
};

/* ------------------------------------------------------------------------------------------ */
/* Lattice tables.  D2Q9: |e| = 0, 1, sqrt2 with weights 4/9, 1/9, 1/36 (Section 2, after
 * eq. latticeforceterm).  D3Q19: rest 1/3, six faces 1/18, twelve edges 1/36 (the standard
 * three-dimensional counterpart; the paper's 3D runs have no hydrodynamics). */
static int lattice_tables(int dim, int e[19][3], double w[19], int opp[19]) {
  int Q = 0;
  memset(e, 0, sizeof(int) * 19 * 3);
  if (dim == 2) {
    static const int e2[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                 {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    Q = 9;
    for (int q = 0; q < 9; q++) {
      e[q][0] = e2[q][0];
      e[q][1] = e2[q][1];
      int m = abs(e2[q][0]) + abs(e2[q][1]);
      w[q] = m == 0 ? 4.0 / 9.0 : (m == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else {
    static const int e3[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                  {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    Q = 19;
    for (int q = 0; q < 19; q++) {
      int m = 0;
      for (int k = 0; k < 3; k++) {
        e[q][k] = e3[q][k];
        m += abs(e3[q][k]);
      }
      w[q] = m == 0 ? 1.0 / 3.0 : (m == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  }
  for (int q = 0; q < Q; q++)
    for (int r = 0; r < Q; r++)
      if (e[r][0] == -e[q][0] && e[r][1] == -e[q][1] && e[r][2] == -e[q][2]) opp[q] = r;
  return Q;
}

int orc_lattice(int32_t dim, int32_t* e, double* w, int32_t* opp) {
  int ee[19][3], oo[19];
  double ww[19];
  if (dim != 2 && dim != 3) return -1;
  int Q = lattice_tables(dim, ee, ww, oo);
  for (int q = 0; q < Q; q++) {
    for (int k = 0; k < 3; k++) e[3 * q + k] = ee[q][k];
    w[q] = ww[q];
    opp[q] = oo[q];
  }
  return Q;
}

/* ------------------------------------------------------------------------------------------ */
/* Index helpers and ghost filling. */
static long sidx(const orc_sim* s, int x, int y, int z) {
  return x + (long)s->n[0] * (y + (long)s->n[1] * z);
}
static long xidx(const orc_sim* s, int x, int y, int z) {
  return (x + s->g[0]) + (long)s->E[0] * ((y + s->g[1]) + (long)s->E[1] * (z + s->g[2]));
}

/* Copy an interior field into a ghost-extended array and fill the ghosts: periodic axes wrap;
 * across a wall plane the field is reflected evenly, phi(-1-m) = phi(m) (Section 2: neutral
 * wetting and zero normal derivative of lap phi and lap^2 phi at the walls, which also makes the
 * total of phi exactly conserved).  If `odd` is set the reflected value changes sign: used for
 * the wall-normal component of a vector (zero flux through the wall) and for the off-diagonal
 * pressure-tensor entries that involve the wall axis. */
static void fill_ext(const orc_sim* s, const double* in, double* ext, int odd) {
  for (int Z = -s->g[2]; Z < s->n[2] + s->g[2]; Z++)
    for (int Y = -s->g[1]; Y < s->n[1] + s->g[1]; Y++)
      for (int X = -s->g[0]; X < s->n[0] + s->g[0]; X++) {
        int c[3] = {X, Y, Z};
        double sign = 1.0;
        for (int k = 0; k < 3; k++) {
          if (c[k] >= 0 && c[k] < s->n[k]) continue;
          if (k == s->wall) {
            c[k] = c[k] < 0 ? -1 - c[k] : 2 * s->n[k] - 1 - c[k];
            if (odd) sign = -sign;
          } else {
            c[k] = ((c[k] % s->n[k]) + s->n[k]) % s->n[k];
          }
        }
        ext[xidx(s, X, Y, Z)] = sign * in[sidx(s, c[0], c[1], c[2])];
      }
}

#define FOR_SITES(s)                                 \
  for (int z = 0; z < (s)->n[2]; z++)                \
    for (int y = 0; y < (s)->n[1]; y++)              \
      for (int x = 0; x < (s)->n[0]; x++)

/* Second-order Laplacian: 5 points in 2D, 7 points in 3D. */
static void laplacian(const orc_sim* s, const double* ext, double* out) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < s->n[2]; z++)
    for (int y = 0; y < s->n[1]; y++)
      for (int x = 0; x < s->n[0]; x++) {
        long c = xidx(s, x, y, z);
        double sum = 0.0;
        for (int k = 0; k < s->d; k++) sum += ext[c + s->st[k]] + ext[c - s->st[k]];
        out[sidx(s, x, y, z)] = sum - 2.0 * s->d * ext[c];
      }
}

/* First derivative along axis k: the isotropic central difference over the lattice's own
 * velocity set, d_k phi = (1/c_s^2) sum_q w_q e_qk phi(x + e_q) with c_s^2 = 1/3.  It is second
 * order like the two-point difference (Section 2 only fixes the order), and its Fourier symbol is
 * i sin k_k (2 + cos k_j)/3 in 2D and i sin k_k (1 + cos k_j + cos k_l)/3 in 3D: equal to the
 * two-point one for modes along an axis, smaller across the diagonals, where the two-point
 * form lets the order-parameter force drive the short waves the explicit coupling cannot carry. */
static void gradient(const orc_sim* s, const double* ext, int k, double* out) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < s->n[2]; z++)
    for (int y = 0; y < s->n[1]; y++)
      for (int x = 0; x < s->n[0]; x++) {
        long c = xidx(s, x, y, z);
        double acc = 0.0;
        for (int q = 1; q < s->Q; q++) {
          if (s->e[q][k] == 0) continue;
          long o = s->e[q][0] * s->st[0] + s->e[q][1] * s->st[1] + s->e[q][2] * s->st[2];
          acc += s->w[q] * s->e[q][k] * ext[c + o];
        }
        out[sidx(s, x, y, z)] = 3.0 * acc;
      }
}

/* Chemical potential mu = a psi + b psi^3 - kappa lap psi + c lap lap psi (eq. chem), with the
 * biharmonic taken as the Laplacian of the Laplacian.  Leaves lap psi in s->L, lap^2 psi in s->M
 * and the extended psi in s->X1, extended L in s->X2. */
static void chem_pot(orc_sim* s, const double* psi, double* mu) {
  const orc_params* p = &s->p;
  fill_ext(s, psi, s->X1, 0);
  laplacian(s, s->X1, s->L);
  fill_ext(s, s->L, s->X2, 0);
  laplacian(s, s->X2, s->M);
  for (long i = 0; i < s->N; i++) {
    double v = psi[i];
    mu[i] = s->a[i] * v + p->b * v * v * v - p->kappa * s->L[i] + p->c * s->M[i];
  }
}

/* S1: reduced temperature a = (T - Tc)/Tc (eq. aterm). */
static void reduced_temperature(orc_sim* s) {
  for (long i = 0; i < s->N; i++) s->a[i] = (s->T[i] - s->p.Tc) / s->p.Tc;
}

/* S4: force density of the order parameter on the fluid, F[k] on the interior.
 * Default: F_alpha = -sum_beta d_beta P_alpha,beta (eq. ff with the n c_s^2 term cancelling the
 * lattice pressure, Section 2), where
 *   P_ab = { a/2 phi^2 + 3b/4 phi^4 - kappa [phi lap phi + |grad phi|^2 / 2]
 *            + c [phi lap^2 phi + (lap phi)^2 / 2 + grad phi . grad lap phi] } delta_ab
 *          + kappa d_a phi d_b phi - c [d_a phi d_b lap phi + d_b phi d_a lap phi]
 * is the pressure tensor of Section 2 without its ideal-gas term n T.  The gradients in P and
 * the divergence of P use the isotropic first difference, whose weights are antisymmetric, so
 * the total force telescopes to zero on a periodic lattice.
 * force_form = 1: F = -phi grad mu (same first difference). */
static void order_parameter_force(orc_sim* s) {
  const orc_params* p = &s->p;
  const int d = s->d;
  if (p->force_form == 1) {
    chem_pot(s, s->phi, s->mu);
    fill_ext(s, s->mu, s->X3, 0);
    for (int k = 0; k < d; k++) {
      gradient(s, s->X3, k, s->F[k]);
      for (long i = 0; i < s->N; i++) s->F[k][i] = -s->phi[i] * s->F[k][i];
    }
    return;
  }
  chem_pot(s, s->phi, s->mu); /* fills L, M, X1 = ext(phi), X2 = ext(L) */
  for (int k = 0; k < d; k++) {
    gradient(s, s->X1, k, s->grad_phi[k]);
    gradient(s, s->X2, k, s->grad_L[k]);
  }
  for (int k = 0; k < d; k++)
    for (long i = 0; i < s->N; i++) s->F[k][i] = 0.0;
  for (int A = 0; A < d; A++)
    for (int B = A; B < d; B++) {
      for (long i = 0; i < s->N; i++) {
        double ph = s->phi[i], L = s->L[i], M = s->M[i];
        double gg = 0.0, gL = 0.0;
        for (int k = 0; k < d; k++) {
          gg += s->grad_phi[k][i] * s->grad_phi[k][i];
          gL += s->grad_phi[k][i] * s->grad_L[k][i];
        }
        double P = p->kappa * s->grad_phi[A][i] * s->grad_phi[B][i] -
                   p->c * (s->grad_phi[A][i] * s->grad_L[B][i] + s->grad_phi[B][i] * s->grad_L[A][i]);
        if (A == B)
          P += 0.5 * s->a[i] * ph * ph + 0.75 * p->b * ph * ph * ph * ph -
               p->kappa * (ph * L + 0.5 * gg) + p->c * (ph * M + 0.5 * L * L + gL);
        s->tmp[i] = P;
      }
      /* P_AB is odd under reflection across the wall plane when exactly one of A, B is the
       * wall axis (one normal derivative in each term). */
      int odd = (A != B) && (A == s->wall || B == s->wall);
      fill_ext(s, s->tmp, s->X3, odd);
      /* F_A -= d_B P_AB and, for A != B, F_B -= d_A P_AB (the tensor is symmetric). */
      double* dP = s->lapmu; /* scratch */
      gradient(s, s->X3, B, dP);
      for (long i = 0; i < s->N; i++) s->F[A][i] -= dP[i];
      if (A != B) {
        gradient(s, s->X3, A, dP);
        for (long i = 0; i < s->N; i++) s->F[B][i] -= dP[i];
      }
    }
}

/* Density and total force density at every site: F += n g (test acceleration). */
static void density_and_force(orc_sim* s, double* nfield) {
  for (long i = 0; i < s->N; i++) {
    double n = 0.0;
    for (int q = 0; q < s->Q; q++) n += s->f[q * s->N + i];
    nfield[i] = n;
  }
  if (s->p.hydro) {
    order_parameter_force(s);
    for (int k = 0; k < s->d; k++)
      for (long i = 0; i < s->N; i++) s->F[k][i] += nfield[i] * s->p.body_force[k];
  } else {
    for (int k = 0; k < s->d; k++) memset(s->F[k], 0, sizeof(double) * s->N);
  }
}

/* S5: n u = sum_q f_q e_q + F/2 (eq. moment); u = 0 without hydrodynamics. */
static void velocity(orc_sim* s, const double* nfield) {
  for (int k = 0; k < s->d; k++)
    for (long i = 0; i < s->N; i++) {
      if (!s->p.hydro) {
        s->u[k][i] = 0.0;
        continue;
      }
      double j = 0.0;
      for (int q = 0; q < s->Q; q++) j += s->f[q * s->N + i] * s->e[q][k];
      s->u[k][i] = (j + 0.5 * s->F[k][i]) / nfield[i];
    }
}

/* Equilibrium: the second-order expansion of the Maxwell-Boltzmann distribution in u,
 * f^eq_q = w_q n [1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u.u/(2 c_s^2)], c_s^2 = 1/3 (Section 2). */
static void equilibrium(const orc_sim* s, double n, const double* u, double* out) {
  double uu = 0.0;
  for (int k = 0; k < s->d; k++) uu += u[k] * u[k];
  for (int q = 0; q < s->Q; q++) {
    double eu = 0.0;
    for (int k = 0; k < s->d; k++) eu += s->e[q][k] * u[k];
    out[q] = s->w[q] * n * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

/* Forcing term (eq. latticeforceterm):
 * F_q = (1 - 1/(2 tau)) w_q [(e_q - u)/c_s^2 + (e_q . u) e_q / c_s^4] . F. */
static void guo_term(const orc_sim* s, double tau, const double* u, const double* F, double* out) {
  for (int q = 0; q < s->Q; q++) {
    double eu = 0.0, t = 0.0;
    for (int k = 0; k < s->d; k++) eu += s->e[q][k] * u[k];
    for (int k = 0; k < s->d; k++) t += (3.0 * (s->e[q][k] - u[k]) + 9.0 * eu * s->e[q][k]) * F[k];
    out[q] = (1.0 - 0.5 / tau) * s->w[q] * t;
  }
}

/* S6 + S7: BGK collision with forcing (eq. evoleqn with dt = 1, relaxation 1/tau), then
 * streaming.  The wall sits half a spacing beyond the last fluid layer: a population whose
 * source lies beyond the wall is the opposite population of the same site after collision
 * (bounce-back; it conserves mass exactly, so no further density correction is needed). */
static void collide_and_stream(orc_sim* s, const double* nfield) {
  const int Q = s->Q;
  const long N = s->N;
  const double tau = s->p.tau;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    double u[3] = {0, 0, 0}, F[3] = {0, 0, 0}, feq[19], fq[19];
    for (int k = 0; k < s->d; k++) {
      u[k] = s->u[k][i];
      F[k] = s->F[k][i];
    }
    equilibrium(s, nfield[i], u, feq);
    guo_term(s, tau, u, F, fq);
    for (int q = 0; q < Q; q++) {
      double fi = s->f[q * N + i];
      s->fs[q * N + i] = fi - (fi - feq[q]) / tau + fq[q];
    }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < s->n[2]; z++)
    for (int y = 0; y < s->n[1]; y++)
      for (int x = 0; x < s->n[0]; x++) {
        long i = sidx(s, x, y, z);
        for (int q = 0; q < Q; q++) {
          int c[3] = {x - s->e[q][0], y - s->e[q][1], z - s->e[q][2]};
          int bounce = 0;
          for (int k = 0; k < 3; k++) {
            if (c[k] >= 0 && c[k] < s->n[k]) continue;
            if (k == s->wall) bounce = 1;
            else c[k] = ((c[k] % s->n[k]) + s->n[k]) % s->n[k];
          }
          s->f[q * N + i] = bounce ? s->fs[s->opp[q] * N + i] : s->fs[q * N + sidx(s, c[0], c[1], c[2])];
        }
      }
}

/* S8: order-parameter update, eq. (massdiff), explicit Euler with n_phi sub-steps of length
 * 1/n_phi.  Advection in conservative central form -sum_alpha d_alpha (psi u_alpha), with the
 * isotropic first derivative and the wall-normal flux odd across the wall (no flux through it);
 * diffusion Gamma lap mu(psi). */
static void order_parameter_update(orc_sim* s) {
  const double h = 1.0 / s->nphi;
  memcpy(s->psi, s->phi, sizeof(double) * s->N);
  for (int sub = 0; sub < s->nphi; sub++) {
    chem_pot(s, s->psi, s->mu);
    fill_ext(s, s->mu, s->X3, 0);
    laplacian(s, s->X3, s->lapmu);
    for (long i = 0; i < s->N; i++) s->adv[i] = 0.0;
    if (s->p.hydro) {
      for (int k = 0; k < s->d; k++) {
        for (long i = 0; i < s->N; i++) s->tmp[i] = s->psi[i] * s->u[k][i];
        fill_ext(s, s->tmp, s->X3, k == s->wall);
        gradient(s, s->X3, k, s->Tn);
        for (long i = 0; i < s->N; i++) s->adv[i] += s->Tn[i];
      }
    }
    for (long i = 0; i < s->N; i++)
      s->psi[i] = s->psi[i] + h * (-s->adv[i] + s->p.Gamma * s->lapmu[i]);
  }
  memcpy(s->phi, s->psi, sizeof(double) * s->N);
}

/* S9: temperature diffusion d_t T = xi lap T (Section 2) by forward-time centred-space sub-steps
 * of ratio xi/n_T; the wall layers keep T = Tw (Section 2: walls at fixed temperature). */
static void temperature_update(orc_sim* s) {
  if (s->p.xi <= 0.0) return;
  const double r = s->p.xi / s->nT;
  for (int sub = 0; sub < s->nT; sub++) {
    fill_ext(s, s->T, s->X3, 0);
    laplacian(s, s->X3, s->Tn);
    FOR_SITES(s) {
      long i = sidx(s, x, y, z);
      int c[3] = {x, y, z};
      if (s->wall >= 0 && (c[s->wall] == 0 || c[s->wall] == s->n[s->wall] - 1)) continue;
      s->T[i] += r * s->Tn[i];
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Sub-step counts.  Explicit Euler for phi with a unit time step is unstable for large
 * biharmonic coefficients; the largest Laplacian eigenvalue on the lattice is lambda = 4 d
 * (checkerboard), for which one Euler step of the linearised equation multiplies the mode by
 * G = 1 - h Gamma lambda (a_eff + kappa lambda + c lambda^2).  n_phi is the smallest count with
 * G >= -0.8.  a_eff is the largest local slope of mu: a itself, or a + 3 b A^2 inside a lamellar
 * state of single-mode amplitude A^2 = 4(-a + kappa^2/(4c))/(3b) (Section 2) at the coldest a.
 * FTCS for T needs xi/n_T <= 1/2 along the one direction T varies in; 0.45 leaves a margin. */
static void auto_substeps(orc_sim* s) {
  const orc_params* p = &s->p;
  if (p->n_phi_sub > 0) {
    s->nphi = p->n_phi_sub;
  } else {
    double a0 = (p->T0 - p->Tc) / p->Tc, aw = (p->Tw - p->Tc) / p->Tc;
    double amax = a0, amin = a0;
    if (p->walls || p->xi < 0) {
      if (p->xi < 0) amax = amin = aw;
      else {
        amax = fmax(a0, aw);
        amin = fmin(a0, aw);
      }
    }
    double aeff = amax;
    if (p->b > 0 && p->c > 0) {
      double A2 = 4.0 * (-amin + p->kappa * p->kappa / (4.0 * p->c)) / (3.0 * p->b);
      if (A2 > 0) aeff = fmax(aeff, amin + 3.0 * p->b * A2);
    }
    double lam = 4.0 * s->d;
    double x = p->Gamma * lam * (aeff + p->kappa * lam + p->c * lam * lam) / 1.8;
    int n = (int)ceil(x - 1e-12);
    s->nphi = n < 1 ? 1 : n;
  }
  if (p->n_T_sub > 0) s->nT = p->n_T_sub;
  else {
    int n = p->xi > 0 ? (int)ceil(p->xi / 0.45 - 1e-12) : 1;
    s->nT = n < 1 ? 1 : n;
  }
}

int orc_create(const orc_params* p, orc_sim** out) {
  if (!p || !out) return -1;
  *out = NULL;
  if (p->dim != 2 && p->dim != 3) return -1;
  if (p->nx < 4 || p->ny < 4 || (p->dim == 3 && p->nz < 4) || (p->dim == 2 && p->nz != 1)) return -1;
  if (p->tau <= 0.5 || p->b < 0 || p->c < 0 || p->Tc <= 0 || p->Gamma < 0) return -1;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  if (!s) return -2;
  s->p = *p;
  s->d = p->dim;
  s->Q = lattice_tables(p->dim, s->e, s->w, s->opp);
  s->n[0] = p->nx;
  s->n[1] = p->ny;
  s->n[2] = p->dim == 3 ? p->nz : 1;
  s->wall = p->walls ? p->dim - 1 : -1;
  for (int k = 0; k < 3; k++) {
    s->g[k] = k < s->d ? GH : 0;
    s->E[k] = s->n[k] + 2 * s->g[k];
  }
  s->st[0] = 1;
  s->st[1] = s->E[0];
  s->st[2] = (long)s->E[0] * s->E[1];
  s->N = (long)s->n[0] * s->n[1] * s->n[2];
  s->NE = (long)s->E[0] * s->E[1] * s->E[2];
  auto_substeps(s);
  long N = s->N;
  s->f = calloc((size_t)s->Q * N, sizeof(double));
  s->fs = calloc((size_t)s->Q * N, sizeof(double));
  double** fields[] = {&s->phi, &s->T, &s->a, &s->L, &s->M, &s->mu, &s->tmp, &s->psi, &s->lapmu,
                       &s->adv, &s->Tn};
  int bad = !s->f || !s->fs;
  for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); k++) {
    *fields[k] = calloc(N, sizeof(double));
    bad |= !*fields[k];
  }
  for (int k = 0; k < 3; k++) {
    s->grad_phi[k] = calloc(N, sizeof(double));
    s->grad_L[k] = calloc(N, sizeof(double));
    s->F[k] = calloc(N, sizeof(double));
    s->u[k] = calloc(N, sizeof(double));
    bad |= !s->grad_phi[k] || !s->grad_L[k] || !s->F[k] || !s->u[k];
  }
  s->X1 = calloc(s->NE, sizeof(double));
  s->X2 = calloc(s->NE, sizeof(double));
  s->X3 = calloc(s->NE, sizeof(double));
  bad |= !s->X1 || !s->X2 || !s->X3;
  if (bad) {
    orc_destroy(s);
    return -2;
  }
  *out = s;
  return 0;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  double* ptrs[] = {s->f, s->fs, s->phi, s->T, s->a, s->L, s->M, s->mu, s->tmp, s->psi, s->lapmu,
                    s->adv, s->Tn, s->X1, s->X2, s->X3};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); k++) free(ptrs[k]);
  for (int k = 0; k < 3; k++) {
    free(s->grad_phi[k]);
    free(s->grad_L[k]);
    free(s->F[k]);
    free(s->u[k]);
  }
  free(s);
}

int orc_substeps(const orc_sim* s, int32_t* n_phi, int32_t* n_T) {
  if (!s) return -1;
  if (n_phi) *n_phi = s->nphi;
  if (n_T) *n_T = s->nT;
  return 0;
}

/* Initial temperature: T0 everywhere except the wall layers, which are at Tw from t = 0
 * (Section 3: initial temperature above Tc, walls at Tw); xi < 0 means an instantaneous quench,
 * T = Tw everywhere. */
static void initial_temperature(orc_sim* s) {
  FOR_SITES(s) {
    int c[3] = {x, y, z};
    long i = sidx(s, x, y, z);
    int on_wall = s->wall >= 0 && (c[s->wall] == 0 || c[s->wall] == s->n[s->wall] - 1);
    s->T[i] = (s->p.xi < 0 || on_wall) ? s->p.Tw : s->p.T0;
  }
}

int orc_init_fields(orc_sim* s, const double* phi0, const double* u0, const double* n0) {
  if (!s || !phi0) return -1;
  memcpy(s->phi, phi0, sizeof(double) * s->N);
  for (long i = 0; i < s->N; i++) {
    double u[3] = {0, 0, 0}, feq[19];
    for (int k = 0; k < s->d; k++) u[k] = u0 ? u0[k * s->N + i] : 0.0;
    equilibrium(s, n0 ? n0[i] : 1.0, u, feq);
    for (int q = 0; q < s->Q; q++) s->f[q * s->N + i] = feq[q];
  }
  initial_temperature(s);
  s->step = 0;
  return 0;
}

int orc_step(orc_sim* s, int64_t nsteps) {
  if (!s || nsteps < 0) return -1;
  for (int64_t t = 0; t < nsteps; t++) {
    reduced_temperature(s);                 /* S1 */
    if (s->p.hydro) {
      density_and_force(s, s->adv);         /* S2-S4: F^n from phi^n */
      velocity(s, s->adv);                  /* S5 */
      collide_and_stream(s, s->adv);        /* S6, S7 */
    } else {
      for (int k = 0; k < s->d; k++) memset(s->u[k], 0, sizeof(double) * s->N);
    }
    order_parameter_update(s);              /* S8, with u^n and a^n */
    temperature_update(s);                  /* S9 */
    s->step++;
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Observables. */

/* Pairwise (cascade) summation, fixed order. */
static double pairwise(const double* v, long n) {
  if (n <= 8) {
    double t = 0.0;
    for (long i = 0; i < n; i++) t += v[i];
    return t;
  }
  long h = n / 2;
  return pairwise(v, h) + pairwise(v + h, n - h);
}

int orc_get_fields(orc_sim* s, double* phi, double* u, double* n, double* T) {
  if (!s) return -1;
  reduced_temperature(s);
  double* nfield = s->adv;
  density_and_force(s, nfield);
  velocity(s, nfield);
  if (phi) memcpy(phi, s->phi, sizeof(double) * s->N);
  if (u)
    for (int k = 0; k < s->d; k++) memcpy(u + k * s->N, s->u[k], sizeof(double) * s->N);
  if (n) memcpy(n, nfield, sizeof(double) * s->N);
  if (T) memcpy(T, s->T, sizeof(double) * s->N);
  return 0;
}

int orc_get_populations(orc_sim* s, double* f) {
  if (!s || !f) return -1;
  memcpy(f, s->f, sizeof(double) * s->Q * s->N);
  return 0;
}

int orc_eval_mu(orc_sim* s, double* mu) {
  if (!s || !mu) return -1;
  reduced_temperature(s);
  chem_pot(s, s->phi, mu);
  return 0;
}

int orc_eval_force(orc_sim* s, double* F) {
  if (!s || !F) return -1;
  reduced_temperature(s);
  int hydro = s->p.hydro;
  s->p.hydro = 1;
  density_and_force(s, s->adv);
  s->p.hydro = hydro;
  for (int k = 0; k < s->d; k++) memcpy(F + k * s->N, s->F[k], sizeof(double) * s->N);
  return 0;
}

/* Discrete free energy of eq. (fren) without the ideal-gas part:
 * sum_x [a phi^2/2 + b phi^4/4 + kappa/2 sum_alpha (phi(x+e_alpha) - phi(x))^2 + c/2 (lap phi)^2]
 * with forward differences for |grad phi|^2 (the difference across a wall vanishes under the
 * even reflection). */
static double free_energy(orc_sim* s) {
  const orc_params* p = &s->p;
  fill_ext(s, s->phi, s->X1, 0);
  laplacian(s, s->X1, s->L);
  FOR_SITES(s) {
    long i = sidx(s, x, y, z), c = xidx(s, x, y, z);
    double ph = s->phi[i], g2 = 0.0;
    for (int k = 0; k < s->d; k++) {
      double df = s->X1[c + s->st[k]] - s->X1[c];
      g2 += df * df;
    }
    s->tmp[i] = 0.5 * s->a[i] * ph * ph + 0.25 * p->b * ph * ph * ph * ph + 0.5 * p->kappa * g2 +
                0.5 * p->c * s->L[i] * s->L[i];
  }
  return pairwise(s->tmp, s->N);
}

int orc_observables(orc_sim* s, orc_obs* o) {
  if (!s || !o) return -1;
  memset(o, 0, sizeof(*o));
  reduced_temperature(s);
  double* nfield = s->adv;
  density_and_force(s, nfield);
  velocity(s, nfield);
  int nonfinite = 0;
  for (long i = 0; i < (long)s->Q * s->N; i++) nonfinite |= !isfinite(s->f[i]);
  for (long i = 0; i < s->N; i++) nonfinite |= !isfinite(s->phi[i]);
  for (long i = 0; i < s->N; i++) {
    double n = 0.0;
    for (int q = 0; q < s->Q; q++) n += s->f[q * s->N + i];
    s->tmp[i] = n - 1.0;
  }
  o->mass_dev = pairwise(s->tmp, s->N);
  for (int k = 0; k < s->d; k++) {
    for (long i = 0; i < s->N; i++) {
      double j = 0.0;
      for (int q = 0; q < s->Q; q++) j += s->f[q * s->N + i] * s->e[q][k];
      s->tmp[i] = j;
    }
    o->mom[k] = pairwise(s->tmp, s->N);
  }
  o->phi_sum = pairwise(s->phi, s->N);
  double umax = 0.0;
  for (long i = 0; i < s->N; i++) {
    double uu = 0.0;
    for (int k = 0; k < s->d; k++) uu += s->u[k][i] * s->u[k][i];
    if (sqrt(uu) > umax) umax = sqrt(uu);
  }
  o->max_u = umax;
  o->mach = umax * sqrt(3.0); /* Ma = |u|_max / c_s with c_s = 1/sqrt3 (Section 2) */
  o->free_energy = free_energy(s);
  o->step = s->step;
  o->nonfinite = nonfinite;
  return 0;
}

int orc_feq(int32_t dim, double n, const double* u, double* out) {
  orc_sim tmp;
  memset(&tmp, 0, sizeof(tmp));
  if (dim != 2 && dim != 3) return -1;
  tmp.d = dim;
  tmp.Q = lattice_tables(dim, tmp.e, tmp.w, tmp.opp);
  equilibrium(&tmp, n, u, out);
  return tmp.Q;
}

int orc_guo(int32_t dim, double tau, const double* u, const double* F, double* out) {
  orc_sim tmp;
  memset(&tmp, 0, sizeof(tmp));
  if (dim != 2 && dim != 3) return -1;
  tmp.d = dim;
  tmp.Q = lattice_tables(dim, tmp.e, tmp.w, tmp.opp);
  guo_term(&tmp, tau, u, F, out);
  return tmp.Q;
}

/* ------------------------------------------------------------------------------------------ */
/* Checkpoint: a header (magic, dims, step) then f, phi, T. */
typedef struct {
  uint64_t magic;
  int32_t dim, nx, ny, nz;
  int64_t step;
} orc_state_header;
#define ORC_MAGIC 0x4f52434c414d3031ull

size_t orc_state_bytes(const orc_sim* s) {
  return sizeof(orc_state_header) + sizeof(double) * ((size_t)s->Q * s->N + 2 * (size_t)s->N);
}

int orc_get_state(const orc_sim* s, void* buf, size_t bytes) {
  if (!s || !buf || bytes < orc_state_bytes(s)) return -3;
  orc_state_header h = {ORC_MAGIC, s->p.dim, s->p.nx, s->p.ny, s->p.nz, s->step};
  char* c = (char*)buf;
  memcpy(c, &h, sizeof(h));
  c += sizeof(h);
  memcpy(c, s->f, sizeof(double) * s->Q * s->N);
  c += sizeof(double) * s->Q * s->N;
  memcpy(c, s->phi, sizeof(double) * s->N);
  c += sizeof(double) * s->N;
  memcpy(c, s->T, sizeof(double) * s->N);
  return 0;
}

int orc_set_state(orc_sim* s, const void* buf, size_t bytes) {
  if (!s || !buf || bytes < orc_state_bytes(s)) return -3;
  orc_state_header h;
  const char* c = (const char*)buf;
  memcpy(&h, c, sizeof(h));
  if (h.magic != ORC_MAGIC || h.dim != s->p.dim || h.nx != s->p.nx || h.ny != s->p.ny ||
      h.nz != s->p.nz)
    return -5;
  c += sizeof(h);
  memcpy(s->f, c, sizeof(double) * s->Q * s->N);
  c += sizeof(double) * s->Q * s->N;
  memcpy(s->phi, c, sizeof(double) * s->N);
  c += sizeof(double) * s->N;
  memcpy(s->T, c, sizeof(double) * s->N);
  s->step = h.step;
  return 0;
}

int orc_threads(int32_t n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}
