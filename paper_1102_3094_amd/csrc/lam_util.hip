// lam_util.hip -- initialisation, reduction finalisation and field/copy helpers (2D and 3D).
#include "lam_dev.hpp"

namespace lam {

// Velocity sets of this library (independent of any other implementation).
// D2Q9 order: rest, +x, +y, -x, -y, (+x+y), (-x+y), (-x-y), (+x-y).
__constant__ int c_e2[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                               {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
__constant__ float c_w2[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                              1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
__constant__ int c_o2[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// D3Q19 order: rest; faces +-x, +-y, +-z; edges in xy, xz, yz (opposites adjacent).
__constant__ int c_e3[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
__constant__ float c_w3[19] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                               1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                               1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};

// Equilibrium deviation g^eq_q = w_q [ (n - 1) + n (3 e.u + 4.5 (e.u)^2 - 1.5 u.u) ].
__device__ __forceinline__ float geq_dev(float w, float n, float eu, float uu) {
  return w * ((n - 1.f) + n * (eu * (3.f + 4.5f * eu) - 1.5f * uu));
}

// Post-collision field whose streaming yields f^eq(n0, u0) at every site:
// g*_q(x) = g^eq_q(x + e_q) if x + e_q is a fluid site, else g^eq_{opp q}(x).
template <int DIM, typename ST>
__global__ void init_pop_kernel(KParams P, const float* __restrict__ n0,
                                const float* __restrict__ u0, ST* __restrict__ g) {
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % P.nx), y = (int)((i / P.nx) % P.ny), z = (int)(i / ((size_t)P.nx * P.ny));
  constexpr int Q = DIM == 2 ? 9 : 19;
  auto site = [&](int xx, int yy, int zz) { return ((size_t)zz * P.ny + yy) * P.nx + xx; };
  auto eq = [&](int q, size_t s) {
    float n = n0 ? n0[s] : 1.f;
    float ux = u0 ? u0[s] : 0.f, uy = u0 ? u0[N + s] : 0.f, uz = (u0 && DIM == 3) ? u0[2 * N + s] : 0.f;
    float uu = ux * ux + uy * uy + uz * uz;
    if (DIM == 2) return geq_dev(c_w2[q], n, c_e2[q][0] * ux + c_e2[q][1] * uy, uu);
    return geq_dev(c_w3[q], n, c_e3[q][0] * ux + c_e3[q][1] * uy + c_e3[q][2] * uz, uu);
  };
  for (int q = 0; q < Q; ++q) {
    int ex = DIM == 2 ? c_e2[q][0] : c_e3[q][0];
    int ey = DIM == 2 ? c_e2[q][1] : c_e3[q][1];
    int ez = DIM == 2 ? 0 : c_e3[q][2];
    int sx = x + ex, sy = y + ey, sz = z + ez;
    int wc = DIM == 2 ? sy : sz, wn = DIM == 2 ? P.ny : P.nz;
    float v;
    if (P.walls && (wc < 0 || wc >= wn)) {
      int o = DIM == 2 ? c_o2[q] : (q == 0 ? 0 : (q % 2 ? q + 1 : q - 1));
      v = eq(o, i);
    } else {
      sx = (sx + P.nx) % P.nx;
      sy = (sy + P.ny) % P.ny;
      sz = DIM == 2 ? 0 : (sz + P.nz) % P.nz;
      v = eq(q, site(sx, sy, sz));
    }
    g[(size_t)q * N + i] = from_f32<ST>(v);
  }
}

// Initial temperature per layer of the wall axis.
__global__ void init_T_kernel(int nrows, int walls, float T0, float Tw, int quench, float* T0buf,
                              float* T1buf) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  bool wall = walls && (j == 0 || j == nrows - 1);
  float v = (quench || wall) ? Tw : T0;
  T0buf[j] = v;
  T1buf[j] = v;
}

// Temperature only: nsteps x n_T FTCS sub-steps of the per-layer profile (the same update as
// the tail of the phi kernels), wall layers held; one workgroup, profile in LDS.
__global__ __launch_bounds__(256) void temperature_kernel(int nrows, int walls, float r_T, int n_T,
                                                          int64_t nsteps, const float* __restrict__ Tin,
                                                          float* __restrict__ Tout) {
  extern __shared__ float sT[];
  float* a = sT;
  float* b = sT + nrows;
  for (int j = threadIdx.x; j < nrows; j += blockDim.x) a[j] = Tin[j];
  __syncthreads();
  for (int64_t t = 0; t < nsteps; ++t)
    for (int m = 0; m < n_T; ++m) {
      for (int j = threadIdx.x; j < nrows; j += blockDim.x) {
        float v = a[j];
        const bool wall = walls && (j == 0 || j == nrows - 1);
        if (!wall) {
          const float lo = a[j == 0 ? nrows - 1 : j - 1], hi = a[j == nrows - 1 ? 0 : j + 1];
          v = v + r_T * ((lo + hi) - 2.f * v);
        }
        b[j] = v;
      }
      __syncthreads();
      float* tmp = a;
      a = b;
      b = tmp;
    }
  for (int j = threadIdx.x; j < nrows; j += blockDim.x) Tout[j] = a[j];
}

hipError_t launch_temperature(int nrows, int walls, float r_T, int n_T, int64_t nsteps,
                              const float* Tin, float* Tout, hipStream_t st) {
  hipLaunchKernelGGL(temperature_kernel, dim3(1), dim3(256), 2 * nrows * sizeof(float), st, nrows,
                     walls, r_T, n_T, nsteps, Tin, Tout);
  return hipGetLastError();
}

// Sum block partials in a fixed order (deterministic), one workgroup of 256 threads.
__global__ void finalize_kernel(const double* __restrict__ partials, int nblk, int nslot,
                                double* __restrict__ out) {
  __shared__ double sm[256];
  for (int k = 0; k < nslot; ++k) {
    const bool mx = (k == R_UMAX || k == R_BAD);
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
      double p = partials[(size_t)b * nslot + k];
      v = mx ? fmax(v, p) : v + p;
    }
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sm[threadIdx.x] = mx ? fmax(sm[threadIdx.x], sm[threadIdx.x + o])
                                                : sm[threadIdx.x] + sm[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sm[0];
    __syncthreads();
  }
}

// T field from the per-layer profile (T is uniform across the wall-parallel axes).
__global__ void broadcast_T_kernel(const float* __restrict__ Trow, size_t N, size_t layer,
                                   float* __restrict__ out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = Trow[i / layer];
}

struct StateHeader {
  uint64_t magic;
  int32_t dim, nx, ny, nz;
  int64_t step;
  int32_t Q, pop_bytes;  // populations per site and bytes per population value
};
constexpr uint64_t STATE_MAGIC = 0x4c414d5354415431ull;

__global__ void write_header_kernel(StateHeader h, StateHeader* dst) { *dst = h; }

hipError_t launch_init(const KParams& P, int dim, const float* n0, const float* u0, void* g,
                       hipStream_t st) {
  size_t N = (size_t)P.nx * P.ny * P.nz;
  dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (P.half_pops) {
    if (dim == 2) hipLaunchKernelGGL((init_pop_kernel<2, __half>), grid, block, 0, st, P, n0, u0, (__half*)g);
    else hipLaunchKernelGGL((init_pop_kernel<3, __half>), grid, block, 0, st, P, n0, u0, (__half*)g);
  } else {
    if (dim == 2) hipLaunchKernelGGL((init_pop_kernel<2, float>), grid, block, 0, st, P, n0, u0, (float*)g);
    else hipLaunchKernelGGL((init_pop_kernel<3, float>), grid, block, 0, st, P, n0, u0, (float*)g);
  }
  return hipGetLastError();
}

hipError_t launch_init_T(int nrows, int walls, float T0, float Tw, int quench, float* a, float* b,
                         hipStream_t st) {
  hipLaunchKernelGGL(init_T_kernel, dim3((nrows + 255) / 256), dim3(256), 0, st, nrows, walls, T0,
                     Tw, quench, a, b);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblk, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, st, partials, nblk, (int)R_N, out);
  return hipGetLastError();
}

hipError_t launch_broadcast_T(const float* Trow, size_t N, size_t layer, float* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(broadcast_T_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, Trow,
                     N, layer, out);
  return hipGetLastError();
}

hipError_t launch_write_header(int dim, int nx, int ny, int nz, int64_t step, int Q, int esz,
                               void* dst, hipStream_t st) {
  StateHeader h{STATE_MAGIC, dim, nx, ny, nz, step, Q, esz};
  hipLaunchKernelGGL(write_header_kernel, dim3(1), dim3(1), 0, st, h, (StateHeader*)dst);
  return hipGetLastError();
}

bool check_header(const void* host_copy, int dim, int nx, int ny, int nz, int Q, int esz,
                  int64_t* step) {
  const StateHeader* h = (const StateHeader*)host_copy;
  if (h->magic != STATE_MAGIC || h->dim != dim || h->nx != nx || h->ny != ny || h->nz != nz ||
      h->Q != Q || h->pop_bytes != esz)
    return false;
  *step = h->step;
  return true;
}

size_t header_bytes() { return 256; }

}  // namespace lam
