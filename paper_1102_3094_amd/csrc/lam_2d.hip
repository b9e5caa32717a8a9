// lam_2d.hip -- gfx950 kernels of one D2Q9 time step (arXiv:1102.3094, Section 2).
//
// Storage: populations as FP32 deviations g_q = f_q - w_q in SoA planes g[q][y][x]; the state
// between steps is the post-collision field of the previous step, so one kernel pulls
// (streams), takes moments, applies the force and collides.  phi[y][x] FP32; T per row.
//
// lb2d: one 64 x TY tile per workgroup of 16 TY threads (TY/4 waves; each thread owns four
//   sites of one column).  Each thread first issues the pulls of its 36 populations (halfway
//   bounce-back at walls), so that their latency overlaps the stencil work: phi is staged in LDS
//   with a halo of 3, from which the Laplacian (halo 2) and the pressure tensor (halo 1) are
//   built in LDS.  First derivatives (in P, its divergence and the phi advection) are the
//   isotropic central differences over the D2Q9 set.  Every site then takes the divergence of
//   P, its moments, collides with
//   the BGK + forcing rule and writes 9 populations and the force-shifted velocity.
// phi2d<S>: S explicit Euler sub-steps of the order-parameter equation on a tile with halo 3S,
//   all in LDS (temporal blocking), reading phi and u once and writing phi once.  The workgroup
//   of tile 0 also advances the per-row temperature.
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include "lam_dev.hpp"

namespace lam {

constexpr int TX = 64;

enum { MODE_STEP = 0, MODE_OBS = 1, MODE_FIELDS = 2 };

template <int TY>
struct Lb2dSmem {
  static constexpr int NWMAX = TY / 2;  // waves per workgroup with 2 sites per thread
  float phi[TY + 6][TX + 6];
  float L[TY + 4][TX + 4];
  float P[3][TY + 2][TX + 2];  // Pxx, Pyy, Pxy (or mu in P[0] for the -phi grad mu form)
  float a[TY + 6];
  int rowoff[TY + 6];  // y * nx of each tile row (wrapped or reflected)
  int colx[TX + 6];    // x of each tile column (wrapped)
  double red[NWMAX > 0 ? NWMAX : 1][R_N];
};

// Sites per thread of the D2Q9 step kernel (each thread owns SPT sites of one tile column): 2,
// measured 1-2 % faster than 4 at 1024^2 and 4096^2, or 4 where 2 would exceed 1024 threads.
constexpr int lb2d_spt(int ty) { return 64 * ty / 2 > 1024 ? 4 : 2; }
constexpr int lb2d_threads(int ty) { return 64 * ty / lb2d_spt(ty); }

// Pull of the 9 populations of site (x, y): f_q(x) = f*_q(x - e_q); across a wall the opposite
// population of x itself (halfway bounce-back).
template <typename ST>
__device__ __forceinline__ void pull9(const ST* __restrict__ G, size_t N, int nx, int ny,
                                      int walls, int x, int y, float g[9]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  auto ld = [&](int q, int yy, int xx) {
    return to_f32(ld_nt(plane_at(G + (size_t)q * N, (uint32_t)(yy * nx + xx))));
  };
  g[0] = ld(0, y, x);
  g[1] = ld(1, y, xm);
  g[3] = ld(3, y, xp);
  if (walls && y == 0) {
    g[2] = ld(4, y, x);
    g[5] = ld(7, y, x);
    g[6] = ld(8, y, x);
  } else {
    const int ym = y == 0 ? ny - 1 : y - 1;
    g[2] = ld(2, ym, x);
    g[5] = ld(5, ym, xm);
    g[6] = ld(6, ym, xp);
  }
  if (walls && y == ny - 1) {
    g[4] = ld(2, y, x);
    g[7] = ld(5, y, x);
    g[8] = ld(6, y, x);
  } else {
    const int yp = y == ny - 1 ? 0 : y + 1;
    g[4] = ld(4, yp, x);
    g[7] = ld(7, yp, xp);
    g[8] = ld(8, yp, xm);
  }
}

// The pressure tensor of Section 2 without its ideal-gas term, at one site, from phi, L = lap phi,
// M = lap L and the first differences of phi and L.  Written with explicit fused multiply-adds and
// contraction off, so that its rounding is fixed by this source and does not depend on how the
// compiler schedules a particular tile shape.
__device__ __forceinline__ void pressure_tensor_2d(const KParams& P, float a, float ph, float L,
                                                   float M, float px, float py, float Lx,
                                                   float Ly, float& Pxx, float& Pyy, float& Pxy) {
#pragma clang fp contract(off)
  const float ph2 = ph * ph;
  const float gg = fmaf(px, px, py * py), gL = fmaf(px, Lx, py * Ly);
  const float tk = fmaf(ph, L, 0.5f * gg);                   // phi lap phi + |grad phi|^2 / 2
  const float tc = fmaf(ph, M, fmaf(0.5f * L, L, gL));       // phi lap^2 phi + (lap phi)^2/2 + ...
  const float bulk = ph2 * fmaf(0.75f * P.b, ph2, 0.5f * a);  // a/2 phi^2 + 3b/4 phi^4
  const float p0 = fmaf(P.c, tc, fmaf(-P.kappa, tk, bulk));
  const float c2 = -2.f * P.c;
  Pxx = fmaf(P.kappa * px, px, fmaf(c2 * px, Lx, p0));
  Pyy = fmaf(P.kappa * py, py, fmaf(c2 * py, Ly, p0));
  Pxy = fmaf(P.kappa * px, py, -P.c * fmaf(px, Ly, py * Lx));
}

// One workgroup of 64*TY/SPT threads (TY/SPT waves) per 64 x TY tile; every thread owns the SPT
// sites (tx, ty + k TY/SPT), k < SPT, of one column.  ST is the storage type of the populations
// (float or __half); all arithmetic is FP32.
template <int TY, int MODE, typename ST, int SPT = lb2d_spt(TY)>
__device__ __forceinline__ void lb2d_tile(const KParams& P, const ST* __restrict__ gin,
                                          ST* __restrict__ gout, const float* __restrict__ phi,
                                          const float* __restrict__ Trow,
                                          float* __restrict__ uout, float* __restrict__ nout,
                                          double* __restrict__ partials, const int x0,
                                          const int y0, Lb2dSmem<TY>& S) {
  constexpr int NTH = 64 * TY / SPT, NW = TY / SPT;
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;

  // issue the population pulls first so that their latency overlaps the stencil phases
  float g[SPT][9];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int x = x0 + tx, y = y0 + ty + NW * j;
    if (x < nx && y < ny) pull9(gin, N, nx, ny, P.walls, x, y, g[j]);
  }

  // index tables of the halo-3 tile: periodic in x, reflected (or periodic) in y;
  // a = (T - Tc)/Tc per row
  for (int i = tid; i < (TY + 6) + (TX + 6); i += NTH) {
    if (i < TY + 6) {
      bool f;
      const int gy = wall_axis(y0 - 3 + i, ny, P.walls, f);
      S.rowoff[i] = gy * nx;
      S.a[i] = (Trow[gy] - P.Tc) / P.Tc;
    } else {
      S.colx[i - (TY + 6)] = wrap(x0 - 3 + (i - (TY + 6)), nx);
    }
  }
  __syncthreads();
  // phi tile; all loads of a thread are issued before its LDS stores, so their latencies overlap
  {
    constexpr int CNT = (TY + 6) * (TX + 6), IT = (CNT + NTH - 1) / NTH;
    float v[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int i = tid + k * NTH;
      if (i < CNT) {
        int r = i / (TX + 6), c = i - r * (TX + 6);
        v[k] = *plane_at(phi, (uint32_t)(S.rowoff[r] + S.colx[c]));
      }
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int i = tid + k * NTH;
      if (i < CNT) {
        int r = i / (TX + 6), c = i - r * (TX + 6);
        S.phi[r][c] = v[k];
      }
    }
  }
  __syncthreads();
  // L = lap phi on halo 2
  for (int i = tid; i < (TY + 4) * (TX + 4); i += NTH) {
    int r = i / (TX + 4), c = i - r * (TX + 4);
    const int R = r + 1, C = c + 1;
    S.L[r][c] = (S.phi[R][C + 1] + S.phi[R][C - 1]) + (S.phi[R + 1][C] + S.phi[R - 1][C]) -
                4.f * S.phi[R][C];
  }
  __syncthreads();
  if (P.hydro) {
    // pressure tensor (or mu) on halo 1
    for (int i = tid; i < (TY + 2) * (TX + 2); i += NTH) {
      int r = i / (TX + 2), c = i - r * (TX + 2);
      const int R = r + 2, C = c + 2;    // phi coordinates
      const int r1 = r + 1, c1 = c + 1;  // L coordinates
      float ph = S.phi[R][C], L = S.L[r1][c1];
      float M = (S.L[r1][c1 + 1] + S.L[r1][c1 - 1]) + (S.L[r1 + 1][c1] + S.L[r1 - 1][c1]) - 4.f * L;
      float a = S.a[R];
      if (P.force_form == 1) {
        S.P[0][r][c] = a * ph + P.b * ph * ph * ph - P.kappa * L + P.c * M;
      } else {
        auto fphi = [&](int dr, int dc) { return S.phi[R + dr][C + dc]; };
        auto fL = [&](int dr, int dc) { return S.L[r1 + dr][c1 + dc]; };
        const float px = iso2_x(fphi), py = iso2_y(fphi);
        const float Lx = iso2_x(fL), Ly = iso2_y(fL);
        pressure_tensor_2d(P, a, ph, L, M, px, py, Lx, Ly, S.P[0][r][c], S.P[1][r][c], S.P[2][r][c]);
      }
    }
    __syncthreads();
  }

  double acc[R_N];
#pragma unroll
  for (int k = 0; k < R_N; ++k) acc[k] = 0.0;

#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int row = ty + NW * j;
    const int x = x0 + tx, y = y0 + row;
    if (x >= nx || y >= ny) continue;
    // force density: -div P or -phi grad mu (isotropic first differences)
    float Fx = 0.f, Fy = 0.f;
    if (P.hydro) {
      const int r = row + 1, c = tx + 1;
      auto f0 = [&](int dr, int dc) { return S.P[0][r + dr][c + dc]; };
      if (P.force_form == 1) {
        float ph = S.phi[row + 3][tx + 3];
        Fx = -ph * iso2_x(f0);
        Fy = -ph * iso2_y(f0);
      } else {
        auto f1 = [&](int dr, int dc) { return S.P[1][r + dr][c + dc]; };
        auto f2 = [&](int dr, int dc) { return S.P[2][r + dr][c + dc]; };
        Fx = -(iso2_x(f0) + iso2_y(f2));
        Fy = -(iso2_x(f2) + iso2_y(f1));
      }
    }
    const float g0 = g[j][0], g1 = g[j][1], g2 = g[j][2], g3 = g[j][3], g4 = g[j][4];
    const float g5 = g[j][5], g6 = g[j][6], g7 = g[j][7], g8 = g[j][8];
    // moments n = 1 + sum g, j = sum g e; u = (j + F/2)/n
    const float dn = ((g0 + g1) + (g2 + g3)) + ((g4 + g5) + (g6 + g7)) + g8;
    const float jx = (g1 - g3) + (g5 - g6) + (g8 - g7);
    const float jy = (g2 - g4) + (g5 + g6) - (g7 + g8);
    const float n = 1.f + dn;
    Fx += n * P.gx;
    Fy += n * P.gy;
    float ux = 0.f, uy = 0.f;
    if (P.hydro) {
      const float inv = 1.f / n;
      ux = (jx + 0.5f * Fx) * inv;
      uy = (jy + 0.5f * Fy) * inv;
    }
    const uint32_t s = (uint32_t)(y * nx + x);
    if (MODE == MODE_STEP) {
      // BGK collision towards the second-order equilibrium plus the forcing term
      const float usq = 1.5f * (ux * ux + uy * uy);
      const float uF = ux * Fx + uy * Fy;
      const float om = P.omega, kf = P.kforce;
      auto coll = [&](float gq, float w, float eu, float eF) {
        float geq = w * (dn + n * (eu * (3.f + 4.5f * eu) - usq));
        float frc = kf * w * (3.f * (eF - uF) + 9.f * eu * eF);
        return gq + om * (geq - gq) + frc;
      };
      const float w0 = 4.f / 9.f, w1 = 1.f / 9.f, w2 = 1.f / 36.f;
      st_nt(plane_at(gout + 0 * N, s), from_f32<ST>(coll(g0, w0, 0.f, 0.f)));
      st_nt(plane_at(gout + 1 * N, s), from_f32<ST>(coll(g1, w1, ux, Fx)));
      st_nt(plane_at(gout + 2 * N, s), from_f32<ST>(coll(g2, w1, uy, Fy)));
      st_nt(plane_at(gout + 3 * N, s), from_f32<ST>(coll(g3, w1, -ux, -Fx)));
      st_nt(plane_at(gout + 4 * N, s), from_f32<ST>(coll(g4, w1, -uy, -Fy)));
      st_nt(plane_at(gout + 5 * N, s), from_f32<ST>(coll(g5, w2, ux + uy, Fx + Fy)));
      st_nt(plane_at(gout + 6 * N, s), from_f32<ST>(coll(g6, w2, uy - ux, Fy - Fx)));
      st_nt(plane_at(gout + 7 * N, s), from_f32<ST>(coll(g7, w2, -ux - uy, -Fx - Fy)));
      st_nt(plane_at(gout + 8 * N, s), from_f32<ST>(coll(g8, w2, ux - uy, Fx - Fy)));
      *plane_at(uout, s) = ux;
      *plane_at(uout + N, s) = uy;
    } else if (MODE == MODE_FIELDS) {
      *plane_at(uout, s) = ux;
      *plane_at(uout + N, s) = uy;
      if (nout) *plane_at(nout, s) = n;
    } else {
      const int R = row + 3, C = tx + 3;
      const float ph = S.phi[R][C], a = S.a[R], L = S.L[row + 2][tx + 2];
      const float dx = S.phi[R][C + 1] - ph, dy = S.phi[R + 1][C] - ph;
      const float fe = 0.5f * a * ph * ph + 0.25f * P.b * ph * ph * ph * ph +
                       0.5f * P.kappa * (dx * dx + dy * dy) + 0.5f * P.c * L * L;
      acc[R_MASS] += (double)dn;
      acc[R_JX] += (double)jx;
      acc[R_JY] += (double)jy;
      acc[R_PHI] += (double)ph;
      acc[R_FE] += (double)fe;
      acc[R_UMAX] = fmax(acc[R_UMAX], (double)sqrtf(ux * ux + uy * uy));
      if (!(isfinite(dn) && isfinite(jx) && isfinite(jy) && isfinite(ph))) acc[R_BAD] = 1.0;
    }
  }

  if (MODE == MODE_OBS) {
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int k = 0; k < R_N; ++k) {
      double v = (k == R_UMAX || k == R_BAD) ? wave_max(acc[k]) : wave_sum(acc[k]);
      if (lane == 0) S.red[wave][k] = v;
    }
    __syncthreads();
    if (tid < R_N) {
      double v = S.red[0][tid];
      for (int w = 1; w < NW; ++w)
        v = (tid == R_UMAX || tid == R_BAD) ? fmax(v, S.red[w][tid]) : v + S.red[w][tid];
      partials[(size_t)blockIdx.x * R_N + tid] = v;
    }
  }
}

template <int TY, int MODE, typename ST>
__global__ __launch_bounds__(lb2d_threads(TY)) void lb2d_kernel(KParams P, const ST* __restrict__ gin,
                                                       ST* __restrict__ gout,
                                                       const float* __restrict__ phi,
                                                       const float* __restrict__ Trow,
                                                       float* __restrict__ uout,
                                                       float* __restrict__ nout,
                                                       double* __restrict__ partials) {
  __shared__ Lb2dSmem<TY> S;
  const int nbx = (P.nx + TX - 1) / TX, nby = (P.ny + TY - 1) / TY;
  const int t = xcd_tile(blockIdx.x, nbx * nby);
  lb2d_tile<TY, MODE, ST>(P, gin, gout, phi, Trow, uout, nout, partials, (t % nbx) * TX,
                          (t / nbx) * TY, S);
}

// Ensembles: a persistent launch.  The grid is a few workgroups per compute unit; each takes work
// items (a member's tile) from a queue until none is left.  The items of the concatenated tile
// lists are split into eight contiguous ranges, one per XCD (workgroup b runs on XCD b mod 8), so
// that tiles sharing halo lines run under the same L2, and each range has its own counter in
// q[0..7].  A workgroup asks for its next item when it starts a tile, so the atomic's latency is
// hidden behind the tile.  No workgroup waits for another: the last one to finish (counter q[8])
// resets the counters for the next launch, so a replayed graph needs no reset node.  With q null
// the launch has one workgroup per item instead (no queue).  A tile computes the same values
// whichever workgroup takes it.
constexpr int ENS_QUEUE_WORDS = 9;

struct EnsQueue {
  unsigned* q;
  int ntiles, base, count;  // this workgroup's XCD range
  int ticket;               // thread 0: the ticket of the next item, fetched ahead

  __device__ __forceinline__ EnsQueue(unsigned* q_, int ntiles_) : q(q_), ntiles(ntiles_) {
    const int k = blockIdx.x & 7;
    const int qq = ntiles >> 3, rr = ntiles & 7;
    base = k < rr ? k * (qq + 1) : rr * (qq + 1) + (k - rr) * qq;
    count = qq + (k < rr ? 1 : 0);
    ticket = 0;
  }
  __device__ __forceinline__ void request() {
    if (q && threadIdx.x == 0) ticket = (int)atomicAdd(&q[blockIdx.x & 7], 1u);
  }
  // The item of the ticket requested last (-1: none left), broadcast to the workgroup.
  __device__ __forceinline__ int take(int* slot) {
    if (!q) return -1;
    if (threadIdx.x == 0) *slot = ticket < count ? base + ticket : -1;
    __syncthreads();
    const int t = *slot;
    __syncthreads();  // every thread has read it before thread 0 writes the next one
    return t;
  }
  __device__ __forceinline__ void finish() {
    if (q && threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(&q[8], 1u) == gridDim.x - 1) {  // every workgroup has taken its last ticket
        for (int k = 0; k < ENS_QUEUE_WORDS; ++k) atomicExch(&q[k], 0u);
        __threadfence();
      }
    }
  }
};

// Runs body(t) for every item this workgroup gets.
template <typename Body>
__device__ __forceinline__ void ens_for_each_item(unsigned* q, int ntiles, Body body) {
  __shared__ int slot;
  if (!q) {
    if ((int)blockIdx.x < ntiles) body(xcd_tile(blockIdx.x, ntiles));
    return;
  }
  EnsQueue Q(q, ntiles);
  Q.request();
  int t = Q.take(&slot);
  while (t >= 0) {
    Q.request();   // the next item, fetched while this one is computed
    body(t);
    __syncthreads();  // the next tile rewrites the LDS tables
    t = Q.take(&slot);
  }
  Q.finish();
}

template <int TY, typename ST>
__global__ __launch_bounds__(lb2d_threads(TY)) void lb2d_ens_kernel(const EnsMember* __restrict__ mem,
                                                           const int* __restrict__ tile_member,
                                                           int ntiles, int cur, unsigned* q) {
  __shared__ Lb2dSmem<TY> S;
  ens_for_each_item(q, ntiles, [&](int t) {
    const EnsMember& M = mem[tile_member[t]];
    const KParams P = M.P;
    const int lt = t - M.tile0, nbx = (P.nx + TX - 1) / TX;
    lb2d_tile<TY, MODE_STEP, ST>(P, (const ST*)M.g[cur], (ST*)M.g[cur ^ 1], M.phi[cur], M.T[cur],
                                 M.u, nullptr, nullptr, (lt % nbx) * TX, (lt / nbx) * TY, S);
  });
}

// ------------------------------------------------------------------------------------------------
// Order-parameter sub-steps.  Cell (r, c) of every LDS plane is the site (y0 - R + r, x0 - R + c);
// a plane is valid at depth d when rows d .. H-1-d and columns d .. W-1-d hold data.
template <int S_, int TY>
struct Phi2dDims {
  static constexpr int R = 3 * S_;
  static constexpr int H = TY + 2 * R;
  static constexpr int W = TX + 2 * R;
};

// Register strips of the phi sub-steps: KS cells of one column per thread, KS from 4 to PHI_KS
// per phase.
constexpr int PHI_KS = 6;

// Strip length of a phase over hh x ww cells with nth threads: the fewest cells per thread in
// sequence (rounds of strips times KS), so that a phase whose strips would need a second, mostly
// idle round takes longer strips instead (64 x 32 tiles, two sub-steps: 6, 6, 5, 4).
constexpr int phi_ks(int hh, int ww, int nth) {
  int best = 4, cost = 1 << 30;
  for (int k = 4; k <= PHI_KS; ++k) {
    const int rounds = (ww * ((hh + k - 1) / k) + nth - 1) / nth;
    if (rounds * k < cost) {
      cost = rounds * k;
      best = k;
    }
  }
  return best;
}

// Every plane has PHI_KS rows beyond its last valid row: a strip that runs past the valid rows
// reads them (unwritten values that feed only cells that are not computed), so no read is
// clamped and each strip addresses its cells from one base with constant offsets.
template <int S_, int TY, bool HYDRO>
struct Phi2dSmem {
  using D = Phi2dDims<S_, TY>;
  static constexpr int H = D::H, W = D::W, HU = H - 4, WU = W - 4;
  float A[H + PHI_KS][W];
  float B[H + PHI_KS][W];
  float Cm[HU + PHI_KS][WU];
  float Ux[HYDRO ? HU + PHI_KS : 1][HYDRO ? WU : 1];
  float Uy[HYDRO ? HU + PHI_KS : 1][HYDRO ? WU : 1];
  float sa[H];
  int rowoff[H], colx[W];
  float rowsgn[H];  // -1 on mirror-image rows (wall-normal velocity is odd)
};

// t is the tile's index within its simulation (the workgroup of tile 0 advances T).
template <int S_, int TY, bool HYDRO>
__device__ __forceinline__ void phi2d_tile(const KParams& P, const float* __restrict__ psi_in,
                                           float* __restrict__ psi_out,
                                           const float* __restrict__ u,
                                           const float* __restrict__ Trow,
                                           float* __restrict__ Tnext, float* __restrict__ Tscr,
                                           const int do_T, const int t, const int x0,
                                           const int y0, Phi2dSmem<S_, TY, HYDRO>& Sm) {
  using D = Phi2dDims<S_, TY>;
  constexpr int R = D::R, H = D::H, W = D::W;
  constexpr int NTH = 16 * TY;
  constexpr int HU = H - 4, WU = W - 4;  // planes used from depth 2 on (mu, velocity)
  auto& A = Sm.A;
  auto& B = Sm.B;
  auto& Cm = Sm.Cm;
  auto& Ux = Sm.Ux;
  auto& Uy = Sm.Uy;
  auto& sa = Sm.sa;
  auto& rowoff = Sm.rowoff;
  auto& colx = Sm.colx;
  auto& rowsgn = Sm.rowsgn;
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const int tid = threadIdx.x;
  for (int i = tid; i < H + W; i += NTH) {
    if (i < H) {
      bool f;
      const int gy = wall_axis(y0 - R + i, ny, P.walls, f);
      rowoff[i] = gy * nx;
      rowsgn[i] = f ? -1.f : 1.f;
      sa[i] = (Trow[gy] - P.Tc) / P.Tc;
    } else {
      colx[i - H] = wrap(x0 - R + (i - H), nx);
    }
  }
  __syncthreads();

  // Tile loads: psi, then the velocity, all issued before any LDS store; every load is
  // unconditional (clamped index) and its value is not touched until it is stored.  The memory
  // counter drains in issue order, so the psi stores wait for psi alone, and the velocity (which
  // the first mu phase does not need) is stored to LDS only after that phase, its loads in flight
  // meanwhile.  Rows go to waves and columns to lanes: a row is one uniform (scalar) base plus
  // the lane's column offsets (columns 0..63, then 64..W-1 on the low lanes), fixed per thread;
  // rows and columns past the tile are clamped to its last one (a duplicate load and store of
  // the same value).
  constexpr int NW = NTH / 64, JA = (H + NW - 1) / NW, JU = HYDRO ? (HU + NW - 1) / NW : 0;
  static_assert(NTH % 64 == 0 && W - 64 <= 64 && W >= 64, "whole waves; one or two columns per lane");
  const int wave = tid >> 6, lane = tid & 63;
  const uint32_t ca0 = (uint32_t)colx[lane], ca1 = (uint32_t)colx[min(64 + lane, W - 1)];
  const uint32_t cu0 = (uint32_t)colx[2 + lane], cu1 = (uint32_t)colx[2 + min(64 + lane, WU - 1)];
  float vx[JU > 0 ? JU : 1][2], vy[JU > 0 ? JU : 1][2];
  {
    float va[JA][2];
#pragma unroll
    for (int j = 0; j < JA; ++j) {
      const int r = min(wave + NW * j, H - 1);
      const float* row = psi_in + __builtin_amdgcn_readfirstlane(rowoff[r]);
      va[j][0] = *plane_at(row, ca0);
      va[j][1] = *plane_at(row, ca1);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the issue order: psi first
    // velocity at depth 2 (plane offset 2); the wall-normal component is odd across a wall (the
    // sign is applied when it is stored)
#pragma unroll
    for (int j = 0; j < JU; ++j) {
      const int r = min(wave + NW * j, HU - 1);
      const int ro = __builtin_amdgcn_readfirstlane(rowoff[r + 2]);
      const float *rx = u + ro, *ry = u + N + ro;
      vx[j][0] = *plane_at(rx, cu0);
      vx[j][1] = *plane_at(rx, cu1);
      vy[j][0] = *plane_at(ry, cu0);
      vy[j][1] = *plane_at(ry, cu1);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < JA; ++j) {
      const int r = min(wave + NW * j, H - 1);
      A[r][lane] = va[j][0];
      A[r][min(64 + lane, W - 1)] = va[j][1];
    }
  }
  __syncthreads();

  // Both phases work on vertical strips of KS cells: a thread keeps the column values its strip
  // shares in registers (with KS = 4 the 13-point biharmonic reads 7 instead of 13 LDS values per
  // cell, the update 15.5 instead of 30).  Consecutive lanes take consecutive columns.  Rows beyond a
  // plane's valid depth are clamped into the array and only feed cells that are not computed.
  // strips read psi rows up to H - dd + KS (dd >= 2) and mu / velocity rows up to
  // HU - dd + KS + 1 (dd >= 3): within the padded planes
  float(*ps)[W] = A;   // current psi
  float(*nx_)[W] = B;  // next psi
  auto sub = [&](auto sc) {
    constexpr int s = decltype(sc)::value, d = 3 * s;
    {  // mu at depth d + 2: lap^2 as the 13-point square of the 5-point Laplacian
      constexpr int dd = d + 2, hh = H - 2 * dd, ww = W - 2 * dd, KS = phi_ks(hh, ww, NTH);
      const int nst = ww * ((hh + KS - 1) / KS);
      for (int t = tid; t < nst; t += NTH) {
        const int rb = t / ww;
        const int c = dd + (t - rb * ww), r0 = dd + KS * rb;
        const int kk = min(KS, H - dd - r0);
        float cC[KS + 4], cL[KS + 2], cR[KS + 2], cLL[KS], cRR[KS];
        const float* b = &ps[r0 - 2][c - 2];  // lowest row and column the strip reads
#pragma unroll
        for (int j = 0; j < KS + 4; ++j) cC[j] = b[j * W + 2];
#pragma unroll
        for (int j = 0; j < KS + 2; ++j) {
          cL[j] = b[(j + 1) * W + 1];
          cR[j] = b[(j + 1) * W + 3];
        }
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          cLL[j] = b[(j + 2) * W];
          cRR[j] = b[(j + 2) * W + 4];
        }
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          if (i < kk) {
            const int r = r0 + i;
            const float v = cC[i + 2];
            const float e = cR[i + 1], w = cL[i + 1], n = cC[i + 3], so = cC[i + 1];
            const float L = (e + w) + (n + so) - 4.f * v;
            const float diag = (cR[i + 2] + cL[i + 2]) + (cR[i] + cL[i]);
            const float far = (cRR[i] + cLL[i]) + (cC[i + 4] + cC[i]);
            const float M = 20.f * v - 8.f * ((e + w) + (n + so)) + 2.f * diag + far;
            Cm[r - 2][c - 2] = sa[r] * v + P.b * v * v * v - P.kappa * L + P.c * M;
          }
        }
      }
    }
    if (HYDRO && s == 0) {
#pragma unroll
      for (int j = 0; j < JU; ++j) {
        const int r = min(wave + NW * j, HU - 1);
        const float sg = rowsgn[r + 2];
        Ux[r][lane] = vx[j][0];
        Ux[r][min(64 + lane, WU - 1)] = vx[j][1];
        Uy[r][lane] = sg * vy[j][0];
        Uy[r][min(64 + lane, WU - 1)] = sg * vy[j][1];
      }
    }
    __syncthreads();
    {  // psi' at depth d + 3
      constexpr int dd = d + 3, hh = H - 2 * dd, ww = W - 2 * dd, KS = phi_ks(hh, ww, NTH);
      constexpr bool last = s == S_ - 1;
      const int nst = ww * ((hh + KS - 1) / KS);
      for (int t = tid; t < nst; t += NTH) {
        const int rb = t / ww;
        const int c = dd + (t - rb * ww), r0 = dd + KS * rb;
        const int kk = min(KS, H - dd - r0);
        const int c2 = c - 2;  // column in the planes that start at depth 2 (mu, velocity)
        // mu: column c rows r0 - 1 .. r0 + KS, columns c +- 1 rows r0 .. r0 + KS - 1
        float mC[KS + 2], mL[KS], mR[KS];
        const float* bm = &Cm[r0 - 3][c2 - 1];  // lowest row and column read, per plane
#pragma unroll
        for (int j = 0; j < KS + 2; ++j) mC[j] = bm[j * WU + 1];
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          mL[j] = bm[(j + 1) * WU];
          mR[j] = bm[(j + 1) * WU + 2];
        }
        // psi in columns c - 1, c, c + 1, rows r0 - 1 .. r0 + KS, and the fluxes psi u there
        float pC[KS + 2], pL[KS + 2], pR[KS + 2];
        float jxL[KS + 2], jxR[KS + 2], jyL[KS + 2], jyC[KS + 2], jyR[KS + 2];
        const float* bp = &ps[r0 - 1][c - 1];
        const float* bx = &Ux[HYDRO ? r0 - 3 : 0][HYDRO ? c2 - 1 : 0];
        const float* by = &Uy[HYDRO ? r0 - 3 : 0][HYDRO ? c2 - 1 : 0];
#pragma unroll
        for (int j = 0; j < KS + 2; ++j) {
          pC[j] = bp[j * W + 1];
          pL[j] = bp[j * W];
          pR[j] = bp[j * W + 2];
          if (HYDRO) {
            jxL[j] = pL[j] * bx[j * WU];
            jxR[j] = pR[j] * bx[j * WU + 2];
            jyL[j] = pL[j] * by[j * WU];
            jyC[j] = pC[j] * by[j * WU + 1];
            jyR[j] = pR[j] * by[j * WU + 2];
          }
        }
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          if (i < kk) {
            const int r = r0 + i;
            const float lapmu = (mR[i] + mL[i]) + (mC[i + 2] + mC[i]) - 4.f * mC[i + 1];
            float adv = 0.f;
            if (HYDRO) {  // div(psi u), isotropic first differences
              adv = iso2_x([&](int dr, int dc) { return dc > 0 ? jxR[i + 1 + dr] : jxL[i + 1 + dr]; }) +
                    iso2_y([&](int dr, int dc) {
                      return dc == 0 ? jyC[i + 1 + dr] : (dc > 0 ? jyR[i + 1 + dr] : jyL[i + 1 + dr]);
                    });
            }
            const float v = pC[i + 1] + P.h * (-adv + P.Gamma * lapmu);
            if (last) {
              const int y = y0 - R + r, x = x0 - R + c;
              if (x < nx && y < ny) psi_out[(size_t)y * nx + x] = v;
            } else {
              nx_[r][c] = v;
            }
          }
        }
      }
    }
    __syncthreads();
    float(*tmp)[W] = ps;
    ps = nx_;
    nx_ = tmp;
  };
  sub(std::integral_constant<int, 0>{});
  if constexpr (S_ > 1) sub(std::integral_constant<int, 1>{});
  static_assert(S_ <= 2, "at most two fused sub-steps");

  // Temperature: FTCS sub-steps along the wall axis (T is uniform along x); wall layers held.
  if (do_T && t == 0 && P.n_T > 0) {
    const float* src = Trow;
    for (int m = 0; m < P.n_T; ++m) {
      float* dst = ((P.n_T - 1 - m) % 2 == 0) ? Tnext : Tscr;
      for (int j = tid; j < ny; j += NTH) {
        float v = src[j];
        bool wall = P.walls && (j == 0 || j == ny - 1);
        if (!wall) {
          float lo = src[j == 0 ? ny - 1 : j - 1], hi = src[j == ny - 1 ? 0 : j + 1];
          v = v + P.r_T * ((lo + hi) - 2.f * v);
        }
        dst[j] = v;
      }
      __syncthreads();
      src = dst;
    }
  }
}

template <int S_, int TY, bool HYDRO>
__global__ __launch_bounds__(16 * TY) void phi2d_kernel(KParams P, const float* __restrict__ psi_in,
                                                        float* __restrict__ psi_out,
                                                        const float* __restrict__ u,
                                                        const float* __restrict__ Trow,
                                                        float* __restrict__ Tnext,
                                                        float* __restrict__ Tscr, int do_T) {
  __shared__ Phi2dSmem<S_, TY, HYDRO> Sm;
  const int nbx = (P.nx + TX - 1) / TX, nby = (P.ny + TY - 1) / TY;
  const int t = xcd_tile(blockIdx.x, nbx * nby);
  phi2d_tile<S_, TY, HYDRO>(P, psi_in, psi_out, u, Trow, Tnext, Tscr, do_T, t, (t % nbx) * TX,
                            (t / nbx) * TY, Sm);
}

// Ensemble: a persistent launch over the tiles of all members (work queue as for the LB kernel);
// pass > 0 selects the member's phi scratch buffers for chained launches (more sub-steps than one
// launch fuses).
template <int S_, int TY, bool HYDRO>
__global__ __launch_bounds__(16 * TY) void phi2d_ens_kernel(const EnsMember* __restrict__ mem,
                                                            const int* __restrict__ tile_member,
                                                            int ntiles, int cur, int pass,
                                                            int last, unsigned* q) {
  __shared__ Phi2dSmem<S_, TY, HYDRO> Sm;
  ens_for_each_item(q, ntiles, [&](int t) {
    const EnsMember& M = mem[tile_member[t]];
    const KParams P = M.P;
    const int lt = t - M.tile0, nbx = (P.nx + TX - 1) / TX;
    const float* in = pass == 0 ? M.phi[cur] : M.psi[(pass - 1) & 1];
    float* out = last ? M.phi[cur ^ 1] : M.psi[pass & 1];
    phi2d_tile<S_, TY, HYDRO>(P, in, out, M.u, M.T[cur], M.T[cur ^ 1], M.T[2],
                              last && P.n_T > 0, lt, (lt % nbx) * TX, (lt / nbx) * TY, Sm);
  });
}

// ------------------------------------------------------------------------------------------------
// Host launchers.  Tile heights 8, 16, 32 and 64 are compiled; the per-site arithmetic does not
// depend on the tile, so every choice gives bit-identical fields.
static int blocks2d(const KParams& P, int ty) {
  return ((P.nx + TX - 1) / TX) * ((P.ny + ty - 1) / ty);
}

int lb2d_blocks(const KParams& P, int ty) { return blocks2d(P, ty); }

// With timing events given, the launch carries them (hipExtLaunchKernelGGL): their timestamps
// are the kernel's own start and end.
template <typename K, typename... A>
static void launch(K kern, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                   A... args) {
  if (e0)
    hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kern, grid, block, 0, st, args...);
}

template <int TY, typename ST>
static void lb2d_launch(const KParams& P, int mode, const void* gin, void* gout, const float* phi,
                        const float* Trow, float* u, float* n, double* partials, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
  dim3 grid(blocks2d(P, TY)), block(lb2d_threads(TY));
  const ST* gi = (const ST*)gin;
  ST* go = (ST*)gout;
  if (mode == MODE_STEP)
    launch(lb2d_kernel<TY, MODE_STEP, ST>, grid, block, st, e0, e1, P, gi, go, phi, Trow, u, n,
           partials);
  else if (mode == MODE_OBS)
    launch(lb2d_kernel<TY, MODE_OBS, ST>, grid, block, st, e0, e1, P, gi, go, phi, Trow, u, n,
           partials);
  else
    launch(lb2d_kernel<TY, MODE_FIELDS, ST>, grid, block, st, e0, e1, P, gi, go, phi, Trow, u, n,
           partials);
}

template <typename ST>
static hipError_t lb2d_dispatch(const KParams& P, int ty, int mode, const void* gin, void* gout,
                                const float* phi, const float* Trow, float* u, float* n,
                                double* partials, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (ty == 8) lb2d_launch<8, ST>(P, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  else if (ty == 16) lb2d_launch<16, ST>(P, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  else if (ty == 32) lb2d_launch<32, ST>(P, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  else if (ty == 64) lb2d_launch<64, ST>(P, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_lb2d(const KParams& P, int ty, int mode, const void* gin, void* gout,
                       const float* phi, const float* Trow, float* u, float* n, double* partials,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (P.half_pops)
    return lb2d_dispatch<__half>(P, ty, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
  return lb2d_dispatch<float>(P, ty, mode, gin, gout, phi, Trow, u, n, partials, st, e0, e1);
}

template <int S_, int TY>
static void phi2d_launch(const KParams& P, const float* in, float* out, const float* u,
                         const float* T, float* Tn, float* Ts, int do_T, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1) {
  dim3 grid(blocks2d(P, TY)), block(16 * TY);
  if (P.hydro)
    launch(phi2d_kernel<S_, TY, true>, grid, block, st, e0, e1, P, in, out, u, T, Tn, Ts, do_T);
  else
    launch(phi2d_kernel<S_, TY, false>, grid, block, st, e0, e1, P, in, out, u, T, Tn, Ts, do_T);
}

int phi2d_max_sub() { return 2; }

hipError_t launch_phi2d(const KParams& P, int ty, int nsub, const float* in, float* out,
                        const float* u, const float* T, float* Tn, float* Ts, int do_T,
                        hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (nsub < 1 || nsub > 2 || (ty != 8 && ty != 16 && ty != 32 && ty != 64))
    return hipErrorInvalidValue;
#define PHI_CASE(S_, TY_) phi2d_launch<S_, TY_>(P, in, out, u, T, Tn, Ts, do_T, st, e0, e1)
  if (nsub == 1) {
    if (ty == 8) PHI_CASE(1, 8);
    else if (ty == 16) PHI_CASE(1, 16);
    else if (ty == 32) PHI_CASE(1, 32);
    else PHI_CASE(1, 64);
  } else {
    if (ty == 8) PHI_CASE(2, 8);
    else if (ty == 16) PHI_CASE(2, 16);
    else if (ty == 32) PHI_CASE(2, 32);
    else PHI_CASE(2, 64);
  }
#undef PHI_CASE
  return hipGetLastError();
}

// Ensemble launchers: one LB launch and ceil(n_phi / 2) phi launches per step, all members, each a
// persistent grid of `grid` workgroups (grid 0: one workgroup per tile, no queue).  q: two queues
// of ENS_QUEUE_WORDS counters (LB, phi), zero before the first launch.
template <int TY>
static void ens_step_ty(const EnsMember* mem, const int* tile_member, int ntiles, int cur,
                        int half, int hydro, int nphi, int grid, unsigned* q, hipStream_t st) {
  if (grid == 0) q = nullptr;
  dim3 g(grid ? grid : ntiles), block(16 * TY), lb_block(lb2d_threads(TY));
  if (hydro) {
    if (half) hipLaunchKernelGGL((lb2d_ens_kernel<TY, __half>), g, lb_block, 0, st, mem, tile_member, ntiles, cur, q);
    else hipLaunchKernelGGL((lb2d_ens_kernel<TY, float>), g, lb_block, 0, st, mem, tile_member, ntiles, cur, q);
  }
  unsigned* qp = q ? q + ENS_QUEUE_WORDS : nullptr;
  int remaining = nphi, pass = 0;
  while (remaining > 0) {
    const int sub = remaining >= 2 ? 2 : 1;
    const int last = remaining == sub;
#define ENS_PHI(S_, H_)                                                                          \
  hipLaunchKernelGGL((phi2d_ens_kernel<S_, TY, H_>), g, block, 0, st, mem, tile_member, ntiles,  \
                     cur, pass, last, qp)
    if (sub == 2) {
      if (hydro) ENS_PHI(2, true);
      else ENS_PHI(2, false);
    } else {
      if (hydro) ENS_PHI(1, true);
      else ENS_PHI(1, false);
    }
#undef ENS_PHI
    remaining -= sub;
    ++pass;
  }
}

int ens_queue_words() { return 2 * ENS_QUEUE_WORDS; }

hipError_t launch_ens_step(const EnsMember* mem, const int* tile_member, int ntiles, int ty,
                           int cur, int half, int hydro, int nphi, int grid, unsigned* q,
                           hipStream_t st) {
  if (grid != 0 && (grid < 8 || (grid & 7))) return hipErrorInvalidValue;
  if (ty == 8) ens_step_ty<8>(mem, tile_member, ntiles, cur, half, hydro, nphi, grid, q, st);
  else if (ty == 16) ens_step_ty<16>(mem, tile_member, ntiles, cur, half, hydro, nphi, grid, q, st);
  else if (ty == 32) ens_step_ty<32>(mem, tile_member, ntiles, cur, half, hydro, nphi, grid, q, st);
  else if (ty == 64) ens_step_ty<64>(mem, tile_member, ntiles, cur, half, hydro, nphi, grid, q, st);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace lam
