// lam_3d.hip -- gfx950 kernels of one D3Q19 time step (arXiv:1102.3094, Section 2, with the
// standard three-dimensional velocity set; walls normal to z).
//
// Both kernels march along z over a 64 x 8 xy tile ("2.5D" blocking): LDS holds a few xy slices
// of each field in ring buffers, so the 7-point Laplacian, the 25-point biharmonic and the
// pressure-tensor divergence need halos only in x and y.  A workgroup owns a chunk of ZLB / ZPH
// slices and starts the pipeline a few slices early.
//
// lb3d: per slice, load phi (xy halo 3) -> L = lap phi (halo 2) -> pressure tensor (6 entries,
//   halo 1) -> for the output slice, -div P, pull of 19 populations (issued one iteration
//   ahead), moments, BGK + forcing collision, write 19 populations and u.
// phi3d: per slice, load psi (halo 3) and u (halo 1) -> mu with the 25-point biharmonic (halo 1)
//   -> psi' = psi + h (Gamma lap mu - div(psi u)) for the output slice.  One Euler sub-step per
//   launch; the workgroup of tile 0 of the last launch also advances the per-layer temperature.
// First derivatives (in P, its divergence and the advection) are the isotropic central
// differences over the D3Q19 set, which reach the edge neighbours in the slices z +- 1.
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include "lam_dev.hpp"

namespace lam {

constexpr int BX = 64, BY = 8, NT3 = BX * BY;
// z slices per workgroup (measured at 256^3: 16 for lb3d, whose pipeline prologue is short
// against its per-slice work, 64 for phi3d)
constexpr int ZLB = 16, ZPH = 64;
enum { MODE3_STEP = 0, MODE3_OBS = 1, MODE3_FIELDS = 2 };

// D3Q19: rest; faces +-x, +-y, +-z; edges in xy, xz, yz (opposites adjacent).
constexpr int E19[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                            {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
__host__ __device__ constexpr int opp19(int q) { return q == 0 ? 0 : (q % 2 ? q + 1 : q - 1); }
__host__ __device__ constexpr float w19(int q) {
  return q == 0 ? 1.f / 3.f : (q <= 6 ? 1.f / 18.f : 1.f / 36.f);
}

struct Tile3 {
  int x0, y0, z0, z1;
};

template <int ZCH>
__device__ __forceinline__ Tile3 tile3(const KParams& P) {
  const int nbx = (P.nx + BX - 1) / BX, nby = (P.ny + BY - 1) / BY, nbz = (P.nz + ZCH - 1) / ZCH;
  // x fastest, then y, then z: the tiles an XCD runs together are xy neighbours, so the halo
  // lines they share (x +- 1 pulls cross a cache line) are fetched from HBM once into that L2
  const int t = xcd_tile(blockIdx.x, nbx * nby * nbz);
  const int bx = t % nbx, by = (t / nbx) % nby, bz = t / (nbx * nby);
  Tile3 T;
  T.x0 = bx * BX;
  T.y0 = by * BY;
  T.z0 = bz * ZCH;
  T.z1 = min(T.z0 + ZCH, P.nz);
  return T;
}

// The pressure tensor of Section 2 without its ideal-gas term at one site (xx, yy, zz, xy, xz,
// yz into dst[k][r][c]); explicit fused multiply-adds with contraction off, as in 2D.
template <typename D>
__device__ __forceinline__ void pressure_tensor_3d(const KParams& P, float a, float ph, float L,
                                                   float M, float px, float py, float pz,
                                                   float Lx, float Ly, float Lz, D dst, int r,
                                                   int c) {
#pragma clang fp contract(off)
  const float ph2 = ph * ph;
  const float gg = fmaf(px, px, fmaf(py, py, pz * pz));
  const float gL = fmaf(px, Lx, fmaf(py, Ly, pz * Lz));
  const float tk = fmaf(ph, L, 0.5f * gg);
  const float tc = fmaf(ph, M, fmaf(0.5f * L, L, gL));
  const float bulk = ph2 * fmaf(0.75f * P.b, ph2, 0.5f * a);
  const float p0 = fmaf(P.c, tc, fmaf(-P.kappa, tk, bulk));
  const float c2 = -2.f * P.c, k = P.kappa, mc = -P.c;
  dst[0][r][c] = fmaf(k * px, px, fmaf(c2 * px, Lx, p0));
  dst[1][r][c] = fmaf(k * py, py, fmaf(c2 * py, Ly, p0));
  dst[2][r][c] = fmaf(k * pz, pz, fmaf(c2 * pz, Lz, p0));
  dst[3][r][c] = fmaf(k * px, py, mc * fmaf(px, Ly, py * Lx));
  dst[4][r][c] = fmaf(k * px, pz, mc * fmaf(px, Lz, pz * Lx));
  dst[5][r][c] = fmaf(k * py, pz, mc * fmaf(py, Lz, pz * Ly));
}

struct Lb3dSmem {
  int rowoff[BY + 6], colx[BX + 6];  // y * nx and x of the halo-3 xy tile (periodic)
  float a[ZLB + 6];                  // (T - Tc)/Tc of the chunk's slices, from slice z0 - 3
  float phi[5][BY + 6][BX + 6];
  // L and P rings of 3: a slice's slot is rewritten only after the barrier that follows the last
  // phase reading it, so three slots suffice and the workgroup fits four to a compute unit
  float L[3][BY + 4][BX + 4];
  float P[3][6][BY + 2][BX + 2];  // xx, yy, zz, xy, xz, yz (or mu in [0] for -phi grad mu)
  double red[NT3 / 64][R_N];
};

template <int MODE, typename ST>
__global__ __launch_bounds__(NT3) void lb3d_kernel(KParams P, const ST* __restrict__ gin,
                                                   ST* __restrict__ gout,
                                                   const float* __restrict__ phi,
                                                   const float* __restrict__ Trow,
                                                   float* __restrict__ uout,
                                                   float* __restrict__ nout,
                                                   double* __restrict__ partials) {
  __shared__ Lb3dSmem S;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const size_t plane = (size_t)nx * ny, N = plane * nz;
  const int tid = threadIdx.x, tx = tid % BX, ty = tid / BX;
  const Tile3 T = tile3<ZLB>(P);
  const int x = T.x0 + tx, y = T.y0 + ty;
  const bool in_xy = x < nx && y < ny;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x >= nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y >= ny - 1 ? 0 : y + 1;

  double acc[R_N];
#pragma unroll
  for (int k = 0; k < R_N; ++k) acc[k] = 0.0;
  float g2[2][19];  // populations of the output slice, pulled one iteration ahead

  static_assert(NT3 >= (BY + 6) + (BX + 6) + ZLB + 6, "one pass fills the tables");
  if (tid < BY + 6) {
    S.rowoff[tid] = wrap(T.y0 - 3 + tid, ny) * nx;
  } else if (tid < (BY + 6) + (BX + 6)) {
    S.colx[tid - (BY + 6)] = wrap(T.x0 - 3 + (tid - (BY + 6)), nx);
  } else if (tid < (BY + 6) + (BX + 6) + ZLB + 6) {
    const int i = tid - (BY + 6) - (BX + 6);
    bool f;
    S.a[i] = (Trow[wall_axis(T.z0 - 3 + i, nz, P.walls, f)] - P.Tc) / P.Tc;
  }
  __syncthreads();
  // phi slices are loaded into registers two iterations before they are stored to LDS (two
  // register buffers by iteration parity).  The memory counter drains in issue order: the pulls
  // of an iteration are issued before its phi prefetch, so the collision waits for the pulls
  // only, and the phi store of the next iteration only for the prefetch issued two iterations
  // back.  The phi loads are unconditional (clamped index) and a comes from LDS so that no
  // branch or late load forces an earlier wait.
  constexpr int CPH = (BY + 6) * (BX + 6), IPH = (CPH + NT3 - 1) / NT3;
  float pv[2][IPH];
  auto load_phi = [&](int sl, float(&pb)[IPH]) {
    bool f;
    const size_t zoff = (size_t)wall_axis(sl, nz, P.walls, f) * plane;
#pragma unroll
    for (int j = 0; j < IPH; ++j) {
      const int i = min(tid + j * NT3, CPH - 1);
      const int r = i / (BX + 6), c = i - r * (BX + 6);
      pb[j] = phi[zoff + S.rowoff[r] + S.colx[c]];
    }
  };
  const int K = T.z1 - T.z0 + 6;
  load_phi(T.z0 - 3, pv[0]);
  load_phi(T.z0 - 2, pv[1]);

  auto iteration = [&](const int k, float(&pb)[IPH], float(&g)[19], float(&gn)[19]) {
    const int s_load = T.z0 - 3 + k, s_L = s_load - 1, s_P = s_load - 2, s_out = s_load - 3;
    {  // phi slice s_load (loaded two iterations ago) into its ring slot
      float(*dst)[BX + 6] = S.phi[((s_load % 5) + 5) % 5];
#pragma unroll
      for (int j = 0; j < IPH; ++j) {
        const int i = tid + j * NT3;
        if (i < CPH) {
          const int r = i / (BX + 6), c = i - r * (BX + 6);
          dst[r][c] = pb[j];
        }
      }
    }
    const bool do_out = s_out >= T.z0 && in_xy;
    // pulls of the next iteration's output slice, issued before this iteration's phi prefetch
    // so that they have a whole iteration to arrive: f_q(x) = f*_q(x - e_q), bounce-back across
    // a wall
    if (s_out + 1 >= T.z0 && s_out + 1 < T.z1 && in_xy) {
      const int z = s_out + 1;
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        const int ex = E19[q][0], ey = E19[q][1], ez = E19[q][2];
        const int sz = z - ez;
        uint32_t idx;
        int qq = q;
        if (P.walls && (sz < 0 || sz >= nz)) {  // uniform: z is the workgroup's slice
          qq = opp19(q);
          idx = (uint32_t)((z * ny + y) * nx + x);
        } else {
          const int sx = ex == 1 ? xm : (ex == -1 ? xp : x);
          const int sy = ey == 1 ? ym : (ey == -1 ? yp : y);
          const int zz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
          idx = (uint32_t)((zz * ny + sy) * nx + sx);
        }
        gn[q] = to_f32(*plane_at(gin + (size_t)qq * N, idx));
      }
    }
    load_phi(s_load + 2, pb);
    __syncthreads();
    if (s_L >= T.z0 - 2) {  // L slice s_L with xy halo 2
      float(*pc)[BX + 6] = S.phi[((s_L % 5) + 5) % 5];
      float(*pd)[BX + 6] = S.phi[(((s_L - 1) % 5) + 5) % 5];
      float(*pu)[BX + 6] = S.phi[(((s_L + 1) % 5) + 5) % 5];
      float(*dst)[BX + 4] = S.L[((s_L % 3) + 3) % 3];
      for (int i = tid; i < (BY + 4) * (BX + 4); i += NT3) {
        int r = i / (BX + 4), c = i - r * (BX + 4);
        const int R = r + 1, C = c + 1;
        dst[r][c] = ((pc[R][C + 1] + pc[R][C - 1]) + (pc[R + 1][C] + pc[R - 1][C])) +
                    (pu[R][C] + pd[R][C]) - 6.f * pc[R][C];
      }
    }
    __syncthreads();
    if (P.hydro && s_P >= T.z0 - 1) {  // pressure tensor (or mu) of slice s_P with xy halo 1
      const float a = S.a[s_P - (T.z0 - 3)];
      float(*pc)[BX + 6] = S.phi[((s_P % 5) + 5) % 5];
      float(*pd)[BX + 6] = S.phi[(((s_P - 1) % 5) + 5) % 5];
      float(*pu)[BX + 6] = S.phi[(((s_P + 1) % 5) + 5) % 5];
      float(*lc)[BX + 4] = S.L[((s_P % 3) + 3) % 3];
      float(*ld)[BX + 4] = S.L[(((s_P - 1) % 3) + 3) % 3];
      float(*lu)[BX + 4] = S.L[(((s_P + 1) % 3) + 3) % 3];
      float(*dst)[BY + 2][BX + 2] = S.P[((s_P % 3) + 3) % 3];
      for (int i = tid; i < (BY + 2) * (BX + 2); i += NT3) {
        int r = i / (BX + 2), c = i - r * (BX + 2);
        const int R = r + 2, C = c + 2, r1 = r + 1, c1 = c + 1;
        const float ph = pc[R][C], L = lc[r1][c1];
        const float M = ((lc[r1][c1 + 1] + lc[r1][c1 - 1]) + (lc[r1 + 1][c1] + lc[r1 - 1][c1])) +
                        (lu[r1][c1] + ld[r1][c1]) - 6.f * L;
        if (P.force_form == 1) {
          dst[0][r][c] = a * ph + P.b * ph * ph * ph - P.kappa * L + P.c * M;
        } else {
          auto fp = [&](int dz, int dr, int dc) {
            return (dz == 0 ? pc : (dz > 0 ? pu : pd))[R + dr][C + dc];
          };
          auto fl = [&](int dz, int dr, int dc) {
            return (dz == 0 ? lc : (dz > 0 ? lu : ld))[r1 + dr][c1 + dc];
          };
          const float px = iso3_x(fp), py = iso3_y(fp), pz = iso3_z(fp);
          const float Lx = iso3_x(fl), Ly = iso3_y(fl), Lz = iso3_z(fl);
          pressure_tensor_3d(P, a, ph, L, M, px, py, pz, Lx, Ly, Lz, dst, r, c);
        }
      }
    }
    __syncthreads();
    if (do_out) {
      const int z = s_out, r = ty + 1, c = tx + 1;
      float(*Pc)[BY + 2][BX + 2] = S.P[((z % 3) + 3) % 3];
      float(*Pd)[BY + 2][BX + 2] = S.P[(((z - 1) % 3) + 3) % 3];
      float(*Pu)[BY + 2][BX + 2] = S.P[(((z + 1) % 3) + 3) % 3];
      float(*pc)[BX + 6] = S.phi[((z % 5) + 5) % 5];
      float Fx = 0.f, Fy = 0.f, Fz = 0.f;
      if (P.hydro) {  // isotropic first differences of P (or of mu)
        auto fP = [&](int k) {
          return [&, k](int dz, int dr, int dc) {
            return (dz == 0 ? Pc : (dz > 0 ? Pu : Pd))[k][r + dr][c + dc];
          };
        };
        if (P.force_form == 1) {
          const float ph = pc[ty + 3][tx + 3];
          Fx = -ph * iso3_x(fP(0));
          Fy = -ph * iso3_y(fP(0));
          Fz = -ph * iso3_z(fP(0));
        } else {
          Fx = -(iso3_x(fP(0)) + iso3_y(fP(3)) + iso3_z(fP(4)));
          Fy = -(iso3_x(fP(3)) + iso3_y(fP(1)) + iso3_z(fP(5)));
          Fz = -(iso3_x(fP(4)) + iso3_y(fP(5)) + iso3_z(fP(2)));
        }
      }
      float dn = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        dn += g[q];
        if (E19[q][0]) jx += E19[q][0] > 0 ? g[q] : -g[q];
        if (E19[q][1]) jy += E19[q][1] > 0 ? g[q] : -g[q];
        if (E19[q][2]) jz += E19[q][2] > 0 ? g[q] : -g[q];
      }
      const float n = 1.f + dn;
      Fx += n * P.gx;
      Fy += n * P.gy;
      Fz += n * P.gz;
      float ux = 0.f, uy = 0.f, uz = 0.f;
      if (P.hydro) {
        const float inv = 1.f / n;
        ux = (jx + 0.5f * Fx) * inv;
        uy = (jy + 0.5f * Fy) * inv;
        uz = (jz + 0.5f * Fz) * inv;
      }
      const uint32_t s = (uint32_t)((z * ny + y) * nx + x);
      if (MODE == MODE3_STEP) {
        const float usq = 1.5f * (ux * ux + uy * uy + uz * uz);
        const float uF = ux * Fx + uy * Fy + uz * Fz;
        const float om = P.omega, kf = P.kforce;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
          const float w = w19(q);
          const float eu = E19[q][0] * ux + E19[q][1] * uy + E19[q][2] * uz;
          const float eF = E19[q][0] * Fx + E19[q][1] * Fy + E19[q][2] * Fz;
          const float geq = w * (dn + n * (eu * (3.f + 4.5f * eu) - usq));
          const float frc = kf * w * (3.f * (eF - uF) + 9.f * eu * eF);
          *plane_at(gout + (size_t)q * N, s) = from_f32<ST>(g[q] + om * (geq - g[q]) + frc);
        }
        *plane_at(uout, s) = ux;
        *plane_at(uout + N, s) = uy;
        *plane_at(uout + 2 * N, s) = uz;
      } else if (MODE == MODE3_FIELDS) {
        *plane_at(uout, s) = ux;
        *plane_at(uout + N, s) = uy;
        *plane_at(uout + 2 * N, s) = uz;
        if (nout) *plane_at(nout, s) = n;
      } else {
        const float a = S.a[z - (T.z0 - 3)];
        float(*pu)[BX + 6] = S.phi[(((z + 1) % 5) + 5) % 5];
        const float ph = pc[ty + 3][tx + 3];
        const float L = S.L[((z % 3) + 3) % 3][ty + 2][tx + 2];
        const float dx = pc[ty + 3][tx + 4] - ph, dy = pc[ty + 4][tx + 3] - ph,
                    dz = pu[ty + 3][tx + 3] - ph;
        const float fe = 0.5f * a * ph * ph + 0.25f * P.b * ph * ph * ph * ph +
                         0.5f * P.kappa * (dx * dx + dy * dy + dz * dz) + 0.5f * P.c * L * L;
        acc[R_MASS] += (double)dn;
        acc[R_JX] += (double)jx;
        acc[R_JY] += (double)jy;
        acc[R_JZ] += (double)jz;
        acc[R_PHI] += (double)ph;
        acc[R_FE] += (double)fe;
        acc[R_UMAX] = fmax(acc[R_UMAX], (double)sqrtf(ux * ux + uy * uy + uz * uz));
        if (!(isfinite(dn) && isfinite(jx) && isfinite(jy) && isfinite(jz) && isfinite(ph)))
          acc[R_BAD] = 1.0;
      }
    }
  };
  for (int k = 0; k < K; k += 2) {
    iteration(k, pv[0], g2[0], g2[1]);
    if (k + 1 < K) iteration(k + 1, pv[1], g2[1], g2[0]);
  }

  if (MODE == MODE3_OBS) {
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int k = 0; k < R_N; ++k) {
      double v = (k == R_UMAX || k == R_BAD) ? wave_max(acc[k]) : wave_sum(acc[k]);
      if (lane == 0) S.red[wave][k] = v;
    }
    __syncthreads();
    if (tid < R_N) {
      double v = S.red[0][tid];
      for (int w = 1; w < NT3 / 64; ++w)
        v = (tid == R_UMAX || tid == R_BAD) ? fmax(v, S.red[w][tid]) : v + S.red[w][tid];
      partials[(size_t)blockIdx.x * R_N + tid] = v;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Two slices per iteration.  psi ring of 8: the stores of slices s + 2, s + 3 must not overwrite
// slices s - 4 .. s - 1, which slower threads may still read for the output slices of the previous
// iteration (no barrier between them).  mu and the fluxes are written after the iteration's first
// barrier and read for outputs s - 3, s - 2 (slices s - 4 .. s - 1): rings of 4.  psi is the same
// for the whole launch (one Euler sub-step), so the ring holds the fluxes psi u (formed once per
// cell when the velocity is staged) rather than u: the advection reads 30 instead of 60 values.
template <bool HYDRO>
struct Phi3dSmem {
  int rowoff[BY + 6], colx[BX + 6];
  float a[ZPH + 6];  // (T - Tc)/Tc of the chunk's slices, from slice z0 - 3
  float psi[8][BY + 6][BX + 6];
  float mu[4][BY + 2][BX + 2];
  float u[HYDRO ? 4 : 1][3][BY + 2][BX + 2];  // fluxes psi u_x, psi u_y, psi u_z
};

template <bool HYDRO>
__global__ __launch_bounds__(NT3) void phi3d_kernel(KParams P, const float* __restrict__ psi_in,
                                                    float* __restrict__ psi_out,
                                                    const float* __restrict__ u,
                                                    const float* __restrict__ Trow,
                                                    float* __restrict__ Tnext,
                                                    float* __restrict__ Tscr, int do_T) {
  __shared__ Phi3dSmem<HYDRO> S;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const size_t plane = (size_t)nx * ny, N = plane * nz;
  const int tid = threadIdx.x, tx = tid % BX, ty = tid / BX;
  const Tile3 T = tile3<ZPH>(P);
  const int x = T.x0 + tx, y = T.y0 + ty;
  const bool in_xy = x < nx && y < ny;

  static_assert(NT3 >= (BY + 6) + (BX + 6) + ZPH + 6, "one pass fills the tables");
  if (tid < BY + 6) {
    S.rowoff[tid] = wrap(T.y0 - 3 + tid, ny) * nx;
  } else if (tid < (BY + 6) + (BX + 6)) {
    S.colx[tid - (BY + 6)] = wrap(T.x0 - 3 + (tid - (BY + 6)), nx);
  } else if (tid < (BY + 6) + (BX + 6) + ZPH + 6) {
    const int i = tid - (BY + 6) - (BX + 6);
    bool f;
    S.a[i] = (Trow[wall_axis(T.z0 - 3 + i, nz, P.walls, f)] - P.Tc) / P.Tc;
  }
  __syncthreads();
  // psi slice s and u slice s - 2 are loaded into registers one iteration (two slices) before
  // their LDS store (one register buffer per slice of the pair): the memory counter of a wave
  // drains in issue order, so the store of the first slice waits only for its own loads while
  // those of the second stay in flight.  Every load is unconditional (clamped index, a u slice is
  // fetched and stored even where it goes unused, the last iteration prefetches slices it does
  // not need) so that no branch forces an early wait; the per-slice a comes from LDS for the same
  // reason.
  constexpr int CPS = (BY + 6) * (BX + 6), IPS = (CPS + NT3 - 1) / NT3;
  constexpr int CUS = (BY + 2) * (BX + 2), IUS = (CUS + NT3 - 1) / NT3;
  float pv[2][IPS], uv[2][3][IUS];
  auto load = [&](int sl, float(&pb)[IPS], float(&ub)[3][IUS]) {
    bool f;
    const size_t zoff = (size_t)wall_axis(sl, nz, P.walls, f) * plane;
#pragma unroll
    for (int j = 0; j < IPS; ++j) {
      const int i = min(tid + j * NT3, CPS - 1);
      const int r = i / (BX + 6), c = i - r * (BX + 6);
      pb[j] = psi_in[zoff + S.rowoff[r] + S.colx[c]];
    }
    if (HYDRO) {
      bool fl;
      const size_t uoff = (size_t)wall_axis(sl - 2, nz, P.walls, fl) * plane;
      const float sg = fl ? -1.f : 1.f;
#pragma unroll
      for (int j = 0; j < IUS; ++j) {
        const int i = min(tid + j * NT3, CUS - 1);
        const int r = i / (BX + 2), c = i - r * (BX + 2);
        const size_t s = uoff + S.rowoff[r + 2] + S.colx[c + 2];
        ub[0][j] = u[s];
        ub[1][j] = u[N + s];
        ub[2][j] = sg * u[2 * N + s];
      }
    }
  };
  const int K = T.z1 - T.z0 + 6;
  load(T.z0 - 3, pv[0], uv[0]);
  load(T.z0 - 2, pv[1], uv[1]);

  // Two slices per iteration (one barrier per slice): store psi slices s, s + 1 and u slices
  // s - 2, s - 1, compute mu of slices s - 2, s - 1, write the output slices s - 3, s - 2.
  auto pair = [&](const int k) {
    const int s0 = T.z0 - 3 + k;
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // psi slices s0, s0 + 1 (xy halo 3)
      float(*dst)[BX + 6] = S.psi[(((s0 + h) % 8) + 8) % 8];
#pragma unroll
      for (int j = 0; j < IPS; ++j) {
        const int i = tid + j * NT3;
        if (i < CPS) {
          const int r = i / (BX + 6), c = i - r * (BX + 6);
          dst[r][c] = pv[h][j];
        }
      }
    }
    __syncthreads();
    if (HYDRO) {  // fluxes psi u of slices s0 - 2, s0 - 1 (xy halo 1; normal component odd)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float(*jd)[BY + 2][BX + 2] = S.u[(((s0 - 2 + h) % 4) + 4) % 4];
        float(*pp)[BX + 6] = S.psi[(((s0 - 2 + h) % 8) + 8) % 8];
#pragma unroll
        for (int j = 0; j < IUS; ++j) {
          const int i = tid + j * NT3;
          if (i < CUS) {
            const int r = i / (BX + 2), c = i - r * (BX + 2);
            const float ps = pp[r + 2][c + 2];
            jd[0][r][c] = ps * uv[h][0][j];
            jd[1][r][c] = ps * uv[h][1][j];
            jd[2][r][c] = ps * uv[h][2][j];
          }
        }
      }
    }
    load(s0 + 2, pv[0], uv[0]);
    load(s0 + 3, pv[1], uv[1]);
    // mu of slices s0 - 2 and s0 - 1 with xy halo 1 (25-point biharmonic)
    for (int i = tid; i < 2 * CUS; i += NT3) {
      const int h = i >= CUS, q = i - h * CUS;
      const int s_mu = s0 - 2 + h;
      if (s_mu < T.z0 - 1 || s_mu > T.z1) continue;
      const float a = S.a[s_mu - (T.z0 - 3)];
      float(*c0)[BX + 6] = S.psi[((s_mu % 8) + 8) % 8];
      float(*m1)[BX + 6] = S.psi[(((s_mu - 1) % 8) + 8) % 8];
      float(*p1)[BX + 6] = S.psi[(((s_mu + 1) % 8) + 8) % 8];
      float(*m2)[BX + 6] = S.psi[(((s_mu - 2) % 8) + 8) % 8];
      float(*p2)[BX + 6] = S.psi[(((s_mu + 2) % 8) + 8) % 8];
      float(*dst)[BX + 2] = S.mu[((s_mu % 4) + 4) % 4];
      const int r = q / (BX + 2), cc = q - r * (BX + 2);
      const int R = r + 2, C = cc + 2;
      const float v = c0[R][C];
      const float face = ((c0[R][C + 1] + c0[R][C - 1]) + (c0[R + 1][C] + c0[R - 1][C])) +
                         (p1[R][C] + m1[R][C]);
      const float edge = ((c0[R + 1][C + 1] + c0[R + 1][C - 1]) + (c0[R - 1][C + 1] + c0[R - 1][C - 1])) +
                         ((p1[R][C + 1] + p1[R][C - 1]) + (m1[R][C + 1] + m1[R][C - 1])) +
                         ((p1[R + 1][C] + p1[R - 1][C]) + (m1[R + 1][C] + m1[R - 1][C]));
      const float far = ((c0[R][C + 2] + c0[R][C - 2]) + (c0[R + 2][C] + c0[R - 2][C])) +
                        (p2[R][C] + m2[R][C]);
      const float L = face - 6.f * v;
      const float M = 42.f * v - 12.f * face + 2.f * edge + far;
      dst[r][cc] = a * v + P.b * v * v * v - P.kappa * L + P.c * M;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int z = s0 - 3 + h;
      if (z < T.z0 || z >= T.z1 || !in_xy) continue;
      const int r = ty + 1, c = tx + 1, R = ty + 3, C = tx + 3;
      float(*mc)[BX + 2] = S.mu[((z % 4) + 4) % 4];
      float(*md)[BX + 2] = S.mu[(((z - 1) % 4) + 4) % 4];
      float(*mu_)[BX + 2] = S.mu[(((z + 1) % 4) + 4) % 4];
      float(*pc)[BX + 6] = S.psi[((z % 8) + 8) % 8];
      float(*pd)[BX + 6] = S.psi[(((z - 1) % 8) + 8) % 8];
      float(*pu)[BX + 6] = S.psi[(((z + 1) % 8) + 8) % 8];
      const float lapmu = ((mc[r][c + 1] + mc[r][c - 1]) + (mc[r + 1][c] + mc[r - 1][c])) +
                          (mu_[r][c] + md[r][c]) - 6.f * mc[r][c];
      float adv = 0.f;
      if (HYDRO) {
        float(*jc)[BY + 2][BX + 2] = S.u[((z % 4) + 4) % 4];
        float(*jd)[BY + 2][BX + 2] = S.u[(((z - 1) % 4) + 4) % 4];
        float(*ju)[BY + 2][BX + 2] = S.u[(((z + 1) % 4) + 4) % 4];
        // div(psi u), isotropic first differences of the staged fluxes
        auto flux = [&](int k) {
          return [&, k](int dz, int dr, int dc) {
            return (dz == 0 ? jc : (dz > 0 ? ju : jd))[k][r + dr][c + dc];
          };
        };
        adv = iso3_x(flux(0)) + iso3_y(flux(1)) + iso3_z(flux(2));
      }
      psi_out[((size_t)z * ny + y) * nx + x] = pc[R][C] + P.h * (-adv + P.Gamma * lapmu);
    }
  };
  for (int k = 0; k < K; k += 2) pair(k);

  // Temperature: FTCS sub-steps along z (T is uniform in x and y); wall layers held.
  if (do_T && blockIdx.x == 0 && P.n_T > 0) {
    __syncthreads();
    const float* src = Trow;
    for (int m = 0; m < P.n_T; ++m) {
      float* dst = ((P.n_T - 1 - m) % 2 == 0) ? Tnext : Tscr;
      for (int j = tid; j < nz; j += NT3) {
        float v = src[j];
        bool wall = P.walls && (j == 0 || j == nz - 1);
        if (!wall) {
          float lo = src[j == 0 ? nz - 1 : j - 1], hi = src[j == nz - 1 ? 0 : j + 1];
          v = v + P.r_T * ((lo + hi) - 2.f * v);
        }
        dst[j] = v;
      }
      __syncthreads();
      src = dst;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// workgroups of lb3d (also the count of its observable partials) and of phi3d
int blocks3d(const KParams& P) {
  return ((P.nx + BX - 1) / BX) * ((P.ny + BY - 1) / BY) * ((P.nz + ZLB - 1) / ZLB);
}
static int blocks3d_phi(const KParams& P) {
  return ((P.nx + BX - 1) / BX) * ((P.ny + BY - 1) / BY) * ((P.nz + ZPH - 1) / ZPH);
}

template <typename K, typename... A>
static void launch3(K kern, int nb, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A... args) {
  if (e0)
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(NT3), 0, st, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kern, dim3(nb), dim3(NT3), 0, st, args...);
}

template <typename ST>
static void lb3d_launch(const KParams& P, int mode, const void* gin, void* gout, const float* phi,
                        const float* Trow, float* u, float* n, double* partials, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
  const int nb = blocks3d(P);
  const ST* gi = (const ST*)gin;
  ST* go = (ST*)gout;
  if (mode == MODE3_STEP)
    launch3(lb3d_kernel<MODE3_STEP, ST>, nb, st, e0, e1, P, gi, go, phi, Trow, u, n, partials);
  else if (mode == MODE3_OBS)
    launch3(lb3d_kernel<MODE3_OBS, ST>, nb, st, e0, e1, P, gi, go, phi, Trow, u, n, partials);
  else
    launch3(lb3d_kernel<MODE3_FIELDS, ST>, nb, st, e0, e1, P, gi, go, phi, Trow, u, n, partials);
}

hipError_t launch_lb3d(const KParams& P, int mode, const void* gin, void* gout,
                       const float* phi, const float* Trow, float* u, float* n, double* partials,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (P.half_pops) lb3d_launch<__half>(P, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  else lb3d_launch<float>(P, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  return hipGetLastError();
}

hipError_t launch_phi3d(const KParams& P, const float* in, float* out, const float* u,
                        const float* T, float* Tn, float* Ts, int do_T, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
  const int nb = blocks3d_phi(P);
  if (P.hydro)
    launch3(phi3d_kernel<true>, nb, st, e0, e1, P, in, out, u, T, Tn, Ts, do_T);
  else
    launch3(phi3d_kernel<false>, nb, st, e0, e1, P, in, out, u, T, Tn, Ts, do_T);
  return hipGetLastError();
}

}  // namespace lam
