// lam_3d.hip -- gfx950 kernels of one D3Q19 time step (arXiv:1102.3094, Section 2, with the
// standard three-dimensional velocity set; walls normal to z).
//
// Both kernels march along z over a 64 x 8 xy tile ("2.5D" blocking): LDS holds a few xy slices
// of each field in ring buffers, so the 7-point Laplacian, the 25-point biharmonic and the
// pressure-tensor divergence need halos only in x and y.  A workgroup owns a chunk of ZLB slices
// (lb3d) or of the host's chunk length (phi3d, at most ZPH) and starts the pipeline a few slices
// early.
//
// lb3d: per slice, load phi (xy halo 3) -> L = lap phi (halo 2) -> pressure tensor (6 entries,
//   halo 1) -> for the output slice, -div P, pull of 19 populations (issued one iteration
//   ahead), moments, BGK + forcing collision, write 19 populations and u.
// phi3d: per slice, load psi (halo 3) and u (halo 1) -> mu with the 25-point biharmonic (halo 1)
//   -> psi' = psi + h (Gamma lap mu - div(psi u)), each slice's mu and fluxes adding their
//   share to the outputs of the slices below, at and above it.  One Euler sub-step per launch;
//   the workgroup of tile 0 of the last launch also advances the per-layer temperature.
// First derivatives (in P, its divergence and the advection) are the isotropic central
// differences over the D3Q19 set, which reach the edge neighbours in the slices z +- 1.
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <type_traits>

#include "lam_dev.hpp"

namespace lam {

constexpr int BX = 64, BY = 8, NT3 = BX * BY;
// z slices per workgroup: 16 for lb3d (measured at 256^3; its pipeline prologue is short against
// its per-slice work); for phi3d the host picks up to ZPH (KParams::zch_phi)
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

__device__ __forceinline__ Tile3 tile3(const KParams& P, int zch) {
  const int nbx = (P.nx + BX - 1) / BX, nby = (P.ny + BY - 1) / BY, nbz = (P.nz + zch - 1) / zch;
  // x fastest, then y, then z: the tiles an XCD runs together are xy neighbours, so the halo
  // lines they share (x +- 1 pulls cross a cache line) are fetched from HBM once into that L2
  const int t = xcd_tile(blockIdx.x, nbx * nby * nbz);
  const int bx = t % nbx, by = (t / nbx) % nby, bz = t / (nbx * nby);
  Tile3 T;
  T.x0 = bx * BX;
  T.y0 = by * BY;
  T.z0 = bz * zch;
  T.z1 = min(T.z0 + zch, P.nz);
  return T;
}

// The pressure tensor of Section 2 without its ideal-gas term at one site (xx, yy, zz, xy, xz,
// yz into dst[k * stride]); explicit fused multiply-adds with contraction off, as in 2D.
__device__ __forceinline__ void pressure_tensor_3d(const KParams& P, float a, float ph, float L,
                                                   float M, float px, float py, float pz,
                                                   float Lx, float Ly, float Lz, float* dst,
                                                   int stride) {
#pragma clang fp contract(off)
  const float ph2 = ph * ph;
  const float gg = fmaf(px, px, fmaf(py, py, pz * pz));
  const float gL = fmaf(px, Lx, fmaf(py, Ly, pz * Lz));
  const float tk = fmaf(ph, L, 0.5f * gg);
  const float tc = fmaf(ph, M, fmaf(0.5f * L, L, gL));
  const float bulk = ph2 * fmaf(0.75f * P.b, ph2, 0.5f * a);
  const float p0 = fmaf(P.c, tc, fmaf(-P.kappa, tk, bulk));
  const float c2 = -2.f * P.c, k = P.kappa, mc = -P.c;
  dst[0] = fmaf(k * px, px, fmaf(c2 * px, Lx, p0));
  dst[stride] = fmaf(k * py, py, fmaf(c2 * py, Ly, p0));
  dst[2 * stride] = fmaf(k * pz, pz, fmaf(c2 * pz, Lz, p0));
  dst[3 * stride] = fmaf(k * px, py, mc * fmaf(px, Ly, py * Lx));
  dst[4 * stride] = fmaf(k * px, pz, mc * fmaf(px, Lz, pz * Lx));
  dst[5 * stride] = fmaf(k * py, pz, mc * fmaf(py, Lz, pz * Ly));
}

// LDS row lengths and cell counts of the halo-3 (phi), halo-2 (L) and halo-1 (P) xy tiles.
constexpr int W3 = BX + 6, W2 = BX + 4, W1 = BX + 2;
constexpr int C3 = (BY + 6) * W3, C2 = (BY + 4) * W2, C1 = (BY + 2) * W1;

struct Lb3dSmem {
  int rowoff[BY + 6], colx[BX + 6];  // y * nx and x of the halo-3 xy tile (periodic)
  float a[ZLB + 6];                  // (T - Tc)/Tc of the chunk's slices, from slice z0 - 3
  float phi[5][C3];
  // L and P rings of 3: a slice's slot is rewritten only after the barrier that follows the last
  // phase reading it, so three slots suffice and the workgroup fits four to a compute unit
  float L[3][C2];
  float P[3][6][C1];  // xx, yy, zz, xy, xz, yz (or mu in [0] for -phi grad mu)
  double red[NT3 / 64][R_N];
};

// e_q . (vx, vy, vz) with the zero components of e_q left out (a product with 0.f would stay).
template <int Q>
__device__ __forceinline__ float edot19(float vx, float vy, float vz) {
  float r = 0.f;
  bool any = false;
  const float v[3] = {vx, vy, vz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (E19[Q][k] == 0) continue;
    const float t = E19[Q][k] > 0 ? v[k] : -v[k];
    r = any ? r + t : t;
    any = true;
  }
  return r;
}

// The next population plane, base + stride bytes.  The empty asm makes the address opaque, so
// the compiler forms the 19 plane addresses by scalar adds where they are used instead of
// keeping them all live in (and spilling them from) scalar registers.
// The operand is a global-address-space pointer, so the accesses stay global (not flat) ones.
template <typename T>
__device__ __forceinline__ T* next_plane(T* p, size_t stride) {
  typedef __attribute__((address_space(1))) char gchar;
  gchar* r = (gchar*)((char*)p) + stride;
  asm volatile("" : "+s"(r));
  return (T*)r;
}

// Slot of the slice k - j in a ring of R slots, given m = k mod R (0 <= j < 2R).
template <int R>
__device__ __forceinline__ int ring_back(int m, int j) {
  int v = m - j;
  v += v < 0 ? R : 0;
  v += v < 0 ? R : 0;
  return v;
}

template <int MODE, typename ST>
__global__ __launch_bounds__(NT3) __attribute__((amdgpu_waves_per_eu(4, 4))) void lb3d_kernel(KParams P, const ST* __restrict__ gin,
                                                   ST* __restrict__ gout,
                                                   const float* __restrict__ phi,
                                                   const float* __restrict__ Trow,
                                                   float* __restrict__ uout,
                                                   float* __restrict__ nout,
                                                   double* __restrict__ partials) {
  __shared__ Lb3dSmem S;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const uint32_t plane = (uint32_t)nx * ny;
  const size_t N = (size_t)plane * nz;
  const int tid = threadIdx.x, tx = tid % BX, ty = tid / BX;
  const Tile3 T = tile3(P, ZLB);
  const int x = T.x0 + tx, y = T.y0 + ty;
  const bool in_xy = x < nx && y < ny;

  double acc[R_N];
#pragma unroll
  for (int k = 0; k < R_N; ++k) acc[k] = 0.0;
  float g2[2][19];  // populations of the output slice, pulled one iteration ahead

  static_assert(NT3 >= (BY + 6) + (BX + 6) + ZLB + 6, "one pass fills the tables");
  static_assert(C3 <= 2 * NT3 && C2 <= 2 * NT3 && C1 <= 2 * NT3 && C1 >= NT3 && C2 >= NT3,
                "every thread owns one or two cells of each halo tile");
  if (tid < BY + 6) {
    S.rowoff[tid] = wrap(T.y0 - 3 + tid, ny) * nx;
  } else if (tid < (BY + 6) + (BX + 6)) {
    S.colx[tid - (BY + 6)] = wrap(T.x0 - 3 + (tid - (BY + 6)), nx);
  } else if (tid < (BY + 6) + (BX + 6) + ZLB + 6) {
    const int i = tid - (BY + 6) - (BX + 6);
    bool f;
    S.a[i] = (Trow[wall_axis(T.z0 - 3 + i, nz, P.walls, f)] - P.Tc) / P.Tc;
  }
  // Per-thread offsets, the same for every slice: the in-plane source of a pull along (ex, ey)
  // ((y - ey) * nx + x - ex, periodic; xys[ey + 1][ex + 1]), the lattice cell of each of the
  // thread's halo-3 cells, and for its cells of the L and P stages the flat LDS index of the
  // centre in the halo-3 (phi) and halo-2 (L) tiles.
  uint32_t xys[3][3];
  {
    const int xc = min(x, nx - 1), yc = min(y, ny - 1);
    const int sx[3] = {xc == nx - 1 ? 0 : xc + 1, xc, xc == 0 ? nx - 1 : xc - 1};
    const int sy[3] = {yc == ny - 1 ? 0 : yc + 1, yc, yc == 0 ? ny - 1 : yc - 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) xys[a][b] = (uint32_t)(sy[a] * nx + sx[b]);
  }
  int lph[2], pph[2], pL[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i2 = min(tid + j * NT3, C2 - 1), r2 = i2 / W2;
    lph[j] = i2 + 2 * r2 + W3 + 1;  // (r + 1) * W3 + c + 1
    const int i1 = min(tid + j * NT3, C1 - 1), r1 = i1 / W1;
    pph[j] = i1 + 4 * r1 + 2 * W3 + 2;  // (r + 2) * W3 + c + 2
    pL[j] = i1 + 2 * r1 + W2 + 1;       // (r + 1) * W2 + c + 1
  }
  __syncthreads();
  constexpr int IPH = (C3 + NT3 - 1) / NT3;
  uint32_t hxy[IPH];
#pragma unroll
  for (int j = 0; j < IPH; ++j) {
    const int i = min(tid + j * NT3, C3 - 1);
    const int r = i / W3, c = i - r * W3;
    hxy[j] = (uint32_t)(S.rowoff[r] + S.colx[c]);
  }
  // phi slices are loaded into registers two iterations before they are stored to LDS (two
  // register buffers by iteration parity).  The memory counter drains in issue order: the pulls
  // of an iteration are issued before its phi prefetch, so the collision waits for the pulls
  // only, and the phi store of the next iteration only for the prefetch issued two iterations
  // back.  The phi loads are unconditional (clamped index) and a comes from LDS so that no
  // branch or late load forces an earlier wait.
  float pv[2][IPH];
  auto load_phi = [&](int sl, float(&pb)[IPH]) {
    bool f;
    const uint32_t zoff = (uint32_t)wall_axis(sl, nz, P.walls, f) * plane;
#pragma unroll
    for (int j = 0; j < IPH; ++j) pb[j] = *plane_at(phi, zoff + hxy[j]);
  };
  const int K = T.z1 - T.z0 + 6;
  load_phi(T.z0 - 3, pv[0]);
  load_phi(T.z0 - 2, pv[1]);

  // Iteration k loads slice z0 - 3 + k and works on the slices behind it: L of k - 1, P of
  // k - 2, the output slice k - 3.  A slice's ring slot is its index relative to z0 - 3 modulo
  // the ring length; m5 = k mod 5 and m3 = k mod 3 are carried by the loop.
  auto iteration = [&](const int k, const int m5, const int m3, float(&pb)[IPH], float(&g)[19],
                       float(&gn)[19]) {
    const int s_out = T.z0 - 3 + k - 3;
    {  // phi slice k (loaded two iterations ago) into its ring slot
      float* dst = S.phi[m5];
#pragma unroll
      for (int j = 0; j < IPH; ++j) {
        const int i = tid + j * NT3;
        if (i < C3) dst[i] = pb[j];
      }
    }
    const bool do_out = k >= 6 && in_xy;
    // pulls of the next iteration's output slice, issued before this iteration's phi prefetch
    // so that they have a whole iteration to arrive: f_q(x) = f*_q(x - e_q), halfway bounce-back
    // across a wall (the opposite population of the site itself)
    const int zn = s_out + 1;
    if (zn >= T.z0 && zn < T.z1 && in_xy) {
      const bool bot = P.walls && zn == 0, top = P.walls && zn == nz - 1;
      const uint32_t zc = (uint32_t)zn * plane;
      const uint32_t zlo = (uint32_t)(zn == 0 ? nz - 1 : zn - 1) * plane;  // source of ez = +1
      const uint32_t zhi = (uint32_t)(zn == nz - 1 ? 0 : zn + 1) * plane;  // source of ez = -1
      const size_t Nb = N * sizeof(ST);
      const ST* gq = gin;
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        const int ex = E19[q][0], ey = E19[q][1], ez = E19[q][2];
        const ST* src = gq;
        uint32_t idx = xys[ey + 1][ex + 1] + (ez == 0 ? zc : (ez > 0 ? zlo : zhi));
        if (ez != 0 && (ez > 0 ? bot : top)) {
          src = (q % 2) ? plane_at(gq, (uint32_t)N) : plane_at(gq, (uint32_t)0) - N;
          idx = xys[1][1] + zc;
        }
        gn[q] = to_f32(*plane_at(src, idx));
        if (q < 18) gq = next_plane(gq, Nb);
      }
    }
    load_phi(T.z0 - 3 + k + 2, pb);
    __syncthreads();
    if (k >= 2) {  // L slice k - 1 with xy halo 2
      const float* pc = S.phi[ring_back<5>(m5, 1)];
      const float* pd = S.phi[ring_back<5>(m5, 2)];
      const float* pu = S.phi[m5];
      float* dst = S.L[ring_back<3>(m3, 1)];
      // reads as a per-thread base (the lowest cell read) plus constants, which the LDS
      // instructions take as immediate offsets
      auto lap = [&](int o) {
        const float *c = pc + o - W3, *u = pu + o, *d = pd + o;
        return ((c[W3 + 1] + c[W3 - 1]) + (c[2 * W3] + c[0])) + (u[0] + d[0]) - 6.f * c[W3];
      };
      dst[tid] = lap(lph[0]);
      if (tid < C2 - NT3) dst[tid + NT3] = lap(lph[1]);
    }
    __syncthreads();
    if (P.hydro && k >= 4) {  // pressure tensor (or mu) of slice k - 2 with xy halo 1
      const float a = S.a[k - 2];
      const float* pc = S.phi[ring_back<5>(m5, 2)];
      const float* pd = S.phi[ring_back<5>(m5, 3)];
      const float* pu = S.phi[ring_back<5>(m5, 1)];
      const float* lc = S.L[ring_back<3>(m3, 2)];
      const float* ld = S.L[ring_back<3>(m3, 3)];
      const float* lu = S.L[ring_back<3>(m3, 1)];
      float* dst = &S.P[ring_back<3>(m3, 2)][0][0];
      auto item = [&](int i, int op, int ol) {
        // per-thread bases at the lowest cell read (row -1, column -1): constant offsets only
        const float *pc0 = pc + op - W3 - 1, *pu0 = pu + op - W3 - 1, *pd0 = pd + op - W3 - 1;
        const float *lc0 = lc + ol - W2 - 1, *lu0 = lu + ol - W2 - 1, *ld0 = ld + ol - W2 - 1;
        const float ph = pc0[W3 + 1], L = lc0[W2 + 1];
        const float M = ((lc0[W2 + 2] + lc0[W2]) + (lc0[2 * W2 + 1] + lc0[1])) +
                        (lu0[W2 + 1] + ld0[W2 + 1]) - 6.f * L;
        if (P.force_form == 1) {
          dst[i] = a * ph + P.b * ph * ph * ph - P.kappa * L + P.c * M;
        } else {
          auto fp = [&](int dz, int dr, int dc) {
            return (dz == 0 ? pc0 : (dz > 0 ? pu0 : pd0))[(dr + 1) * W3 + dc + 1];
          };
          auto fl = [&](int dz, int dr, int dc) {
            return (dz == 0 ? lc0 : (dz > 0 ? lu0 : ld0))[(dr + 1) * W2 + dc + 1];
          };
          const float px = iso3_x(fp), py = iso3_y(fp), pz = iso3_z(fp);
          const float Lx = iso3_x(fl), Ly = iso3_y(fl), Lz = iso3_z(fl);
          pressure_tensor_3d(P, a, ph, L, M, px, py, pz, Lx, Ly, Lz, dst + i, C1);
        }
      };
      item(tid, pph[0], pL[0]);
      if (tid < C1 - NT3) item(tid + NT3, pph[1], pL[1]);
    }
    __syncthreads();
    if (do_out) {
      const int z = s_out, o = (ty + 1) * W1 + tx + 1, oc = (ty + 3) * W3 + tx + 3;
      const float* Pc = &S.P[ring_back<3>(m3, 3)][0][0];
      const float* Pd = &S.P[ring_back<3>(m3, 4)][0][0];
      const float* Pu = &S.P[ring_back<3>(m3, 2)][0][0];
      const float* pc = S.phi[ring_back<5>(m5, 3)];
      float Fx = 0.f, Fy = 0.f, Fz = 0.f;
      if (P.hydro) {  // isotropic first differences of P (or of mu)
        // per-thread bases at the lowest cell read: constant offsets only
        const float *Pc0 = Pc + o - W1 - 1, *Pu0 = Pu + o - W1 - 1, *Pd0 = Pd + o - W1 - 1;
        auto fP = [&](int kk) {
          return [&, kk](int dz, int dr, int dc) {
            return (dz == 0 ? Pc0 : (dz > 0 ? Pu0 : Pd0))[kk * C1 + (dr + 1) * W1 + dc + 1];
          };
        };
        if (P.force_form == 1) {
          const float ph = pc[oc];
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
      const uint32_t s = (uint32_t)z * plane + (uint32_t)(y * nx + x);
      if (MODE == MODE3_STEP) {
        // BGK collision towards the second-order equilibrium plus the forcing term, per population
        // (the rounding of this form is the one the shear-wave and long-run parity tests hold to)
        const float usq = 1.5f * (ux * ux + uy * uy + uz * uz);
        const float uF = ux * Fx + uy * Fy + uz * Fz;
        const float om = P.omega, kf = P.kforce;
        const size_t Nb = N * sizeof(ST);
        ST* go = gout;
        auto coll = [&](auto qc) {
          constexpr int q = decltype(qc)::value;
          const float w = w19(q);
          const float eu = edot19<q>(ux, uy, uz), eF = edot19<q>(Fx, Fy, Fz);
          const float geq = w * (dn + n * (eu * (3.f + 4.5f * eu) - usq));
          const float frc = kf * w * (3.f * (eF - uF) + 9.f * eu * eF);
          if (q > 0) go = next_plane(go, Nb);
          *plane_at(go, s) = from_f32<ST>(g[q] + om * (geq - g[q]) + frc);
        };
        coll(std::integral_constant<int, 0>{});
        coll(std::integral_constant<int, 1>{});
        coll(std::integral_constant<int, 2>{});
        coll(std::integral_constant<int, 3>{});
        coll(std::integral_constant<int, 4>{});
        coll(std::integral_constant<int, 5>{});
        coll(std::integral_constant<int, 6>{});
        coll(std::integral_constant<int, 7>{});
        coll(std::integral_constant<int, 8>{});
        coll(std::integral_constant<int, 9>{});
        coll(std::integral_constant<int, 10>{});
        coll(std::integral_constant<int, 11>{});
        coll(std::integral_constant<int, 12>{});
        coll(std::integral_constant<int, 13>{});
        coll(std::integral_constant<int, 14>{});
        coll(std::integral_constant<int, 15>{});
        coll(std::integral_constant<int, 16>{});
        coll(std::integral_constant<int, 17>{});
        coll(std::integral_constant<int, 18>{});
        *plane_at(uout, s) = ux;
        *plane_at(uout + N, s) = uy;
        *plane_at(uout + 2 * N, s) = uz;
      } else if (MODE == MODE3_FIELDS) {
        *plane_at(uout, s) = ux;
        *plane_at(uout + N, s) = uy;
        *plane_at(uout + 2 * N, s) = uz;
        if (nout) *plane_at(nout, s) = n;
      } else {
        const float a = S.a[k - 3];
        const float* pu = S.phi[ring_back<5>(m5, 2)];
        const float ph = pc[oc];
        const float L = S.L[ring_back<3>(m3, 3)][(ty + 2) * W2 + tx + 2];
        const float dx = pc[oc + 1] - ph, dy = pc[oc + W3] - ph, dz = pu[oc] - ph;
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
  int m5 = 0, m3 = 0;
  for (int k = 0; k < K; k += 2) {
    iteration(k, m5, m3, pv[0], g2[0], g2[1]);
    m5 = m5 == 4 ? 0 : m5 + 1;
    m3 = m3 == 2 ? 0 : m3 + 1;
    if (k + 1 < K) iteration(k + 1, m5, m3, pv[1], g2[1], g2[0]);
    m5 = m5 == 4 ? 0 : m5 + 1;
    m3 = m3 == 2 ? 0 : m3 + 1;
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
// iteration (no barrier between them).  mu and the fluxes of slices s - 2, s - 1 are written after
// the iteration's first barrier and read only after its second, by the same iteration: every
// thread adds what one slice contributes to the outputs of slices s - 1, s and s + 1 into
// registers (the 7-point Laplacian and the isotropic divergence split by z offset), so their
// rings hold just the two slices of the iteration.  psi is the same for the whole launch (one
// Euler sub-step), so the ring holds the fluxes psi u (formed once per cell when the velocity is
// staged) rather than u.  Ring slots are the slice index relative to z0 - 3 masked to the ring
// length.  The rings read most per output (fluxes, mu) come first, so that their reads fit the
// 16-bit immediate offset of the LDS instructions.
template <bool HYDRO>
struct Phi3dSmem {
  float u[HYDRO ? 2 : 1][3][C1];  // fluxes psi u_x, psi u_y, psi u_z
  float mu[2][C1];
  float psi[8][C3];
  float a[ZPH + 6];  // (T - Tc)/Tc of the chunk's slices, from slice z0 - 3
  int rowoff[BY + 6], colx[BX + 6];
};

// mu = a psi + b psi^3 - kappa lap psi + c lap lap psi at the halo-3 tile cell o of slice c0, with
// slices m2, m1 below and p1, p2 above (the 25-point biharmonic is the 7-point Laplacian applied
// twice).
__device__ __forceinline__ float mu_at(const KParams& P, float a, const float* m2,
                                       const float* m1, const float* c0, const float* p1,
                                       const float* p2, int o) {
  // bases at the lowest cell read (two rows and two columns below o): constant offsets only
  const int B = 2 * W3 + 2;
  const float *c = c0 + o - B, *u = p1 + o - B, *d = m1 + o - B;
  const float v = c[B];
  const float face = ((c[B + 1] + c[B - 1]) + (c[B + W3] + c[B - W3])) + (p1[o] + m1[o]);
  const float edge = ((c[B + W3 + 1] + c[B + W3 - 1]) + (c[B - W3 + 1] + c[B - W3 - 1])) +
                     ((u[B + 1] + u[B - 1]) + (d[B + 1] + d[B - 1])) +
                     ((u[B + W3] + u[B - W3]) + (d[B + W3] + d[B - W3]));
  const float far = ((c[B + 2] + c[B - 2]) + (c[B + 2 * W3] + c[2])) + (p2[o] + m2[o]);
  const float L = face - 6.f * v;
  const float M = 42.f * v - 12.f * face + 2.f * edge + far;
  return a * v + P.b * v * v * v - P.kappa * L + P.c * M;
}

template <bool HYDRO>
__global__ __launch_bounds__(NT3) void phi3d_kernel(KParams P, const float* __restrict__ psi_in,
                                                    float* __restrict__ psi_out,
                                                    const float* __restrict__ u,
                                                    const float* __restrict__ Trow,
                                                    float* __restrict__ Tnext,
                                                    float* __restrict__ Tscr, int do_T) {
  __shared__ Phi3dSmem<HYDRO> S;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const uint32_t plane = (uint32_t)nx * ny;
  const size_t N = (size_t)plane * nz;
  const int tid = threadIdx.x, tx = tid % BX, ty = tid / BX;
  const Tile3 T = tile3(P, P.zch_phi);
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
  // Cells of the halo-1 tile (mu and the fluxes): every thread owns the interior cell above its
  // own site, threads below NH one cell of the ring around it (rows 0 and BY + 1, then columns 0
  // and BX + 1 of rows 1 .. BY).  o* index the halo-1 tile, p* the halo-3 tile.
  constexpr int NH = 2 * W1 + 2 * BY;
  static_assert(NH <= NT3 && C1 == NT3 + NH && C3 <= 2 * NT3, "cell ownership");
  const bool has_h = tid < NH;
  int hr, hc;
  if (tid < W1) {
    hr = 0;
    hc = tid;
  } else if (tid < 2 * W1) {
    hr = BY + 1;
    hc = tid - W1;
  } else {
    const int t = min(tid - 2 * W1, 2 * BY - 1);
    hr = 1 + t / 2;
    hc = (t % 2) ? BX + 1 : 0;
  }
  const int oi = (ty + 1) * W1 + tx + 1, pi = (ty + 3) * W3 + tx + 3;
  const int oh = hr * W1 + hc, ph = (hr + 2) * W3 + hc + 2;
  __syncthreads();
  // in-plane lattice offsets of the thread's halo-3 cells (psi) and of its two halo-1 cells (u)
  uint32_t gp[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = min(tid + j * NT3, C3 - 1);
    const int r = i / W3, c = i - r * W3;
    gp[j] = (uint32_t)(S.rowoff[r] + S.colx[c]);
  }
  const uint32_t gu[2] = {(uint32_t)(S.rowoff[ty + 3] + S.colx[tx + 3]),
                          (uint32_t)(S.rowoff[hr + 2] + S.colx[hc + 2])};

  // psi slice s and u slice s - 2 are loaded into registers one iteration (two slices) before
  // their LDS store (one register buffer per slice of the pair): the memory counter of a wave
  // drains in issue order, so the store of the first slice waits only for its own loads while
  // those of the second stay in flight.  Every load is unconditional (clamped cell, a u slice is
  // fetched and stored even where it goes unused, the last iteration prefetches slices it does
  // not need) so that no branch forces an early wait; the per-slice a comes from LDS for the same
  // reason.
  float pv[2][2], uv[2][2][3];
  auto load = [&](int sl, float(&pb)[2], float(&ub)[2][3]) {
    bool f;
    const uint32_t zoff = (uint32_t)wall_axis(sl, nz, P.walls, f) * plane;
    pb[0] = *plane_at(psi_in, zoff + gp[0]);
    pb[1] = *plane_at(psi_in, zoff + gp[1]);
    if (HYDRO) {
      bool fl;
      const uint32_t uoff = (uint32_t)wall_axis(sl - 2, nz, P.walls, fl) * plane;
      const float sg = fl ? -1.f : 1.f;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        ub[j][0] = *plane_at(u, uoff + gu[j]);
        ub[j][1] = *plane_at(u + N, uoff + gu[j]);
        ub[j][2] = sg * *plane_at(u + 2 * N, uoff + gu[j]);
      }
    }
  };
  const int K = T.z1 - T.z0 + 6;
  load(T.z0 - 3, pv[0], uv[0]);
  load(T.z0 - 2, pv[1], uv[1]);

  // Iteration k (even): store psi slices k, k + 1 (relative to z0 - 3) and the fluxes of slices
  // k - 2, k - 1, compute mu of slices k - 2, k - 1, write the output slices k - 3, k - 2.
  // rb, rc: partial R of slices k - 3 and k - 2 (from the slices before k - 2).
  float rb = 0.f, rc = 0.f;
  auto pair = [&](const int k) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float* dst = S.psi[(k + h) & 7];
      dst[tid] = pv[h][0];
      if (tid < C3 - NT3) dst[tid + NT3] = pv[h][1];
    }
    __syncthreads();
    if (HYDRO && k >= 4) {  // fluxes psi u of slices k - 2, k - 1 (xy halo 1; normal one odd)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float* jd = S.u[(k - 2 + h) & 1][0];
        const float* pp = S.psi[(k - 2 + h) & 7];
        const float ps = pp[pi];
        jd[oi] = ps * uv[h][0][0];
        jd[C1 + oi] = ps * uv[h][0][1];
        jd[2 * C1 + oi] = ps * uv[h][0][2];
        if (has_h) {
          const float pq = pp[ph];
          jd[oh] = pq * uv[h][1][0];
          jd[C1 + oh] = pq * uv[h][1][1];
          jd[2 * C1 + oh] = pq * uv[h][1][2];
        }
      }
    }
    load(T.z0 - 3 + k + 2, pv[0], uv[0]);
    load(T.z0 - 3 + k + 3, pv[1], uv[1]);
    if (k >= 4) {  // mu of slices k - 2 and k - 1 (from slice z0 - 1 on), sharing their reads
      const float a0 = S.a[k - 2], a1 = S.a[k - 1];
      const float* q0 = S.psi[(k - 4) & 7];
      const float* q1 = S.psi[(k - 3) & 7];
      const float* q2 = S.psi[(k - 2) & 7];
      const float* q3 = S.psi[(k - 1) & 7];
      const float* q4 = S.psi[k & 7];
      const float* q5 = S.psi[(k + 1) & 7];
      float* m0 = S.mu[(k - 2) & 1];
      float* m1 = S.mu[(k - 1) & 1];
      m0[oi] = mu_at(P, a0, q0, q1, q2, q3, q4, pi);
      m1[oi] = mu_at(P, a1, q1, q2, q3, q4, q5, pi);
      if (has_h) {
        m0[oh] = mu_at(P, a0, q0, q1, q2, q3, q4, ph);
        m1[oh] = mu_at(P, a1, q1, q2, q3, q4, q5, ph);
      }
    }
    __syncthreads();
    // Slices k - 2 + h in order: with R = Gamma lap mu - div(psi u), slice s adds `below` to
    // R(s - 1) (completing it), `cen` to R(s) and `above` to R(s + 1).  The z +- 1 terms of the
    // isotropic divergence are A +- B: A from the x and y fluxes of the xz and yz edges, B from
    // the z fluxes of the z face and the edges.
    if (k >= 4 && in_xy) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // per-thread bases at the lowest cell read (row -1, column -1): constant offsets only
        const float* m = S.mu[(k - 2 + h) & 1] + oi - W1 - 1;
        const float mc = m[W1 + 1];
        float cen = P.Gamma * (((m[W1 + 2] + m[W1]) + (m[2 * W1 + 1] + m[1])) - 6.f * mc);
        float below = P.Gamma * mc, above = below;
        if (HYDRO) {
          const float* jb = S.u[(k - 2 + h) & 1][0] + oi - W1 - 1;
          auto jx = [&](int dr, int dc) { return jb[(dr + 1) * W1 + dc + 1]; };
          auto jy = [&](int dr, int dc) { return jb[C1 + (dr + 1) * W1 + dc + 1]; };
          auto jz = [&](int dr, int dc) { return jb[2 * C1 + (dr + 1) * W1 + dc + 1]; };
          const float d0 = (jx(0, 1) - jx(0, -1)) + (jy(1, 0) - jy(-1, 0));
          const float de = ((jx(1, 1) - jx(1, -1)) + (jx(-1, 1) - jx(-1, -1))) +
                           ((jy(1, 1) - jy(-1, 1)) + (jy(1, -1) - jy(-1, -1)));
          const float A = (1.f / 12.f) * d0;
          const float B = (1.f / 6.f) * jz(0, 0) +
                          (1.f / 12.f) * ((jz(0, 1) + jz(0, -1)) + (jz(1, 0) + jz(-1, 0)));
          cen -= (1.f / 6.f) * d0 + (1.f / 12.f) * de;
          below -= A + B;
          above -= A - B;
        }
        const int j = k - 3 + h, z = T.z0 - 3 + j;  // output slice s - 1
        if (z >= T.z0 && z < T.z1) {
          const float pc = S.psi[j & 7][pi];
          *plane_at(psi_out, (uint32_t)z * plane + (uint32_t)(y * nx + x)) =
              pc + P.h * (rb + below);
        }
        rb = rc + cen;
        rc = above;
      }
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
  return ((P.nx + BX - 1) / BX) * ((P.ny + BY - 1) / BY) * ((P.nz + P.zch_phi - 1) / P.zch_phi);
}

// z slices per phi3d workgroup: enough chunks for about three workgroups per compute unit of a
// 256-unit part (the LDS allows three), each of 16 .. ZPH slices (the pipeline re-reads six
// slices per chunk).  At 256^3 this gives six chunks of 43 slices (phi3d 116 -> 107 us against
// four of 64).
int phi3d_chunk(int nx, int ny, int nz) {
  const int nxy = ((nx + BX - 1) / BX) * ((ny + BY - 1) / BY);
  const int nbz = (768 + nxy - 1) / nxy;
  return std::min(ZPH, std::max(std::min(16, nz), (nz + nbz - 1) / nbz));
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
