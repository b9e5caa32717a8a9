// lam_spectra.hip -- observables of the 2D order parameter: structure factor S(k) and the
// orientation histogram of grad phi.  Both are reductions over the lattice computed on demand.
//
// S(k): mean of phi (FP64), then a DFT along x of every row (phi - mean) written transposed,
// then a DFT along y of every transposed row; |X|^2/N is binned into shells
// b = isqrt(floor((m_x^2 n_y^2 + m_y^2 n_x^2) / max(n_x, n_y)^2)) computed in exact integer
// arithmetic.  Powers of two use an in-place radix-2 FFT in LDS, other lengths a direct DFT; the
// twiddles are evaluated in FP64 and rounded once.  Each shell of a transposed row is summed by one thread over its own
// contiguous range of |m_y| (the shell index is monotone in |m_y|), so the sums have a fixed order;
// rows are then combined in a fixed order.
#include <mutex>

#include "../../include/lam.h"
#include "lam_dev.hpp"

namespace lam {

constexpr int SPEC_MAX = 4096;  // longest supported axis

struct SpecLayout {
  size_t mean, rowsum, buf, part, kpart, bins, total;
};

static SpecLayout spec_layout(int nx, int ny) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  SpecLayout L{};
  size_t o = 0;
  const int nb = nx > ny ? nx : ny;
  L.mean = o;  o = al(o + 8 * 4);
  L.rowsum = o; o = al(o + 8 * (size_t)(nx > ny ? nx : ny));
  L.buf = o;   o = al(o + 8 * (size_t)nx * ny);              // float2 transposed spectrum
  // per-row (sum, count) per shell; also holds the orientation row partials (ny x (36 + 2))
  const size_t part = 16 * (size_t)nx * nb, orient = 8 * (size_t)ny * 38;
  L.part = o;  o = al(o + (part > orient ? part : orient));
  L.kpart = o; o = al(o + 16 * (size_t)(nx > ny ? nx : ny)); // per-row (sum |k| P, sum P)
  L.bins = o;  o = al(o + 8 * (size_t)(nb + 8));
  L.total = o;
  return L;
}

size_t spectra_scratch_bytes(int nx, int ny) { return spec_layout(nx, ny).total; }

// ---------------------------------------------------------------------------------------------
__global__ void row_sum_kernel(const float* __restrict__ phi, int nx, double* __restrict__ rowsum) {
  __shared__ double sm[256];
  const float* r = phi + (size_t)blockIdx.x * nx;
  double v = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) v += (double)r[x];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) rowsum[blockIdx.x] = sm[0];
}

__global__ void mean_kernel(const double* __restrict__ rowsum, int nrows, double inv_n,
                            double* __restrict__ mean) {
  __shared__ double sm[256];
  double v = 0.0;
  for (int j = threadIdx.x; j < nrows; j += 256) v += rowsum[j];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[0] = sm[0] * inv_n;
}

// In-LDS transform of one row of length n.  Powers of two: the row was loaded in bit-reversed
// order into `a` and is transformed in place by radix-2 decimation-in-time butterflies (twiddles
// tw[m] = exp(-2 pi i m / n), m < n/2); other lengths: direct DFT from `a` into `b` with the full
// twiddle table (m < n).  Returns the array holding the natural-order result.
__device__ float2* lds_dft(float2* a, float2* b, const float2* tw, int n, bool pow2) {
  if (pow2) {
    for (int size = 2; size <= n; size <<= 1) {
      const int half = size >> 1, step = n / size;
      for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
        int grp = i / half, pos = i - grp * half;
        int k = grp * size + pos;
        float2 w = tw[pos * step], v = a[k + half], u = a[k];
        float2 t = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
        a[k] = make_float2(u.x + t.x, u.y + t.y);
        a[k + half] = make_float2(u.x - t.x, u.y - t.y);
      }
      __syncthreads();
    }
    return a;
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    float re = 0.f, im = 0.f;
    int idx = 0;
    for (int x = 0; x < n; ++x) {
      float2 v = a[x], w = tw[idx];
      re += v.x * w.x - v.y * w.y;
      im += v.x * w.y + v.y * w.x;
      idx += k;
      if (idx >= n) idx -= n;
    }
    b[k] = make_float2(re, im);
  }
  __syncthreads();
  return b;
}

__device__ void make_twiddles(float2* tw, int n, int count) {
  for (int m = threadIdx.x; m < count; m += blockDim.x) {
    double s, c;
    sincospi(-2.0 * m / n, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
  }
}

// position of element x in LDS before the transform
__device__ __forceinline__ int load_pos(int x, int n, bool pow2) {
  if (!pow2) return x;
  int bits = 31 - __clz(n);
  return (int)(__builtin_bitreverse32((unsigned)x) >> (32 - bits));
}

// LDS layout per workgroup: pow2 -> a[n], tw[n/2]; otherwise a[n], b[n], tw[n].
__host__ __device__ inline size_t dft_lds_bytes(int n, bool pow2) {
  return sizeof(float2) * (pow2 ? (size_t)n + n / 2 : 3 * (size_t)n);
}

// Pass 1: DFT along x of row y of (phi - mean); writes out[kx][y].
__global__ void fft_x_kernel(const float* __restrict__ phi, int nx, int ny,
                             const double* __restrict__ mean, float2* __restrict__ out, int pow2) {
  extern __shared__ float2 sh[];
  float2 *a = sh, *b = sh + nx, *tw = pow2 ? sh + nx : sh + 2 * nx;
  const int y = blockIdx.x;
  const float m = (float)mean[0];
  make_twiddles(tw, nx, pow2 ? nx / 2 : nx);
  for (int x = threadIdx.x; x < nx; x += blockDim.x)
    a[load_pos(x, nx, pow2)] = make_float2(phi[(size_t)y * nx + x] - m, 0.f);
  __syncthreads();
  float2* r = lds_dft(a, b, tw, nx, pow2);
  for (int k = threadIdx.x; k < nx; k += blockDim.x) out[(size_t)k * ny + y] = r[k];
}

__device__ __forceinline__ long long isqrt_ll(long long q) {
  long long r = (long long)sqrt((double)q);
  while (r * r > q) --r;
  while ((r + 1) * (r + 1) <= q) ++r;
  return r;
}

// Pass 2: DFT along y of transposed row kx; shell sums of |X|^2 / N for this row.
__global__ void fft_y_bin_kernel(const float2* __restrict__ buf, int nx, int ny, int nbmax,
                                 double2* __restrict__ part, double2* __restrict__ kpart,
                                 int pow2) {
  extern __shared__ float2 sh[];
  float2 *a = sh, *b = sh + ny, *tw = pow2 ? sh + ny : sh + 2 * ny;
  const int row = blockIdx.x;
  make_twiddles(tw, ny, pow2 ? ny / 2 : ny);
  for (int y = threadIdx.x; y < ny; y += blockDim.x)
    a[load_pos(y, ny, pow2)] = buf[(size_t)row * ny + y];
  __syncthreads();
  float2* X = lds_dft(a, b, tw, ny, pow2);
  const double invN = 1.0 / ((double)nx * ny);
  const long long mx = row < (nx + 1) / 2 ? row : row - nx;
  const long long Lm = nx > ny ? nx : ny;
  const long long L2 = Lm * Lm, ny2 = (long long)ny * ny, nx2 = (long long)nx * nx;
  const int half = ny / 2;  // |m_y| runs over 0 .. half
  auto power = [&](int idx) {
    float2 v = X[idx];
    return ((double)v.x * v.x + (double)v.y * v.y) * invN;
  };
  // |m_y| -> the one or two array entries holding +m_y and -m_y
  auto pair_power = [&](int my, int& cnt) {
    double p = power(my);
    cnt = 1;
    if (my != 0 && !(ny % 2 == 0 && my == half)) {
      p += power(ny - my);
      cnt = 2;
    }
    return p;
  };
  auto shell = [&](long long my) { return isqrt_ll((mx * mx * ny2 + my * my * nx2) / L2); };
  for (int bsh = threadIdx.x; bsh < nbmax; bsh += blockDim.x) {
    // first |m_y| whose shell is >= bsh: m_y^2 nx^2 >= bsh^2 L^2 - m_x^2 n_y^2
    long long need = (long long)bsh * bsh * L2 - mx * mx * ny2;
    long long lo = 0;
    if (need > 0) {
      long long q = (need + nx2 - 1) / nx2;
      lo = isqrt_ll(q);
      if (lo * lo < q) ++lo;
    }
    double s = 0.0, c = 0.0;
    for (long long my = lo; my <= half && shell(my) == bsh; ++my) {
      if (mx == 0 && my == 0) continue;
      int cnt;
      s += pair_power((int)my, cnt);
      c += cnt;
    }
    part[(size_t)row * nbmax + bsh] = make_double2(s, c);
  }
  // |k|-weighted sums over every mode of the row (k = 0 left out), fixed-order tree
  __shared__ double sk[256], sp[256];
  double ks = 0.0, ps = 0.0;
  const double kx = 6.283185307179586 * (double)mx / nx;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    int my = y < (ny + 1) / 2 ? y : y - ny;
    if (mx == 0 && my == 0) continue;
    double ky = 6.283185307179586 * (double)my / ny;
    double p = power(y);
    ks += sqrt(kx * kx + ky * ky) * p;
    ps += p;
  }
  sk[threadIdx.x] = ks;
  sp[threadIdx.x] = ps;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sk[threadIdx.x] += sk[threadIdx.x + o];
      sp[threadIdx.x] += sp[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) kpart[row] = make_double2(sk[0], sp[0]);
}

// Column sums of a row-major [nrows][ld] matrix of doubles, one workgroup per column, fixed
// order (strided per-thread sums, then a tree).
__global__ void colsum_kernel(const double* __restrict__ M, int nrows, int ld,
                              double* __restrict__ out) {
  __shared__ double sm[256];
  const int col = blockIdx.x;
  double v = 0.0;
  for (int r = threadIdx.x; r < nrows; r += 256) v += M[(size_t)r * ld + col];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = sm[0];
}

// S per shell from (sum, count) column sums; the largest shell (first one on ties), its
// parabolic refinement and <k>.  out: [0, nbins) S; nbins: k_peak; nbins+1: S_peak;
// nbins+2: k_mean.
__global__ void spec_final_kernel(const double* __restrict__ sc, const double* __restrict__ kk,
                                  int nbins, double dk, double* __restrict__ out) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int bidx = 0;
  for (int b = threadIdx.x; b < nbins; b += 256) {
    double c = sc[2 * b + 1];
    double v = c > 0 ? sc[2 * b] / c : 0.0;
    out[b] = v;
    if (v > best) {
      best = v;
      bidx = b;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      double v2 = bv[threadIdx.x + o];
      int i2 = bi[threadIdx.x + o];
      if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int m = bi[0];
    double kp = (m + 0.5) * dk, Sp = out[m];
    if (m > 0 && m < nbins - 1) {
      double den = out[m - 1] - 2.0 * out[m] + out[m + 1];
      if (den != 0.0) {
        double d = 0.5 * (out[m - 1] - out[m + 1]) / den;
        kp = (m + 0.5 + d) * dk;
        Sp = out[m] - 0.25 * (out[m - 1] - out[m + 1]) * d;
      }
    }
    out[nbins] = kp;
    out[nbins + 1] = Sp;
    out[nbins + 2] = kk[1] > 0 ? kk[0] / kk[1] : 0.0;
  }
}

hipError_t structure_factor_2d(const KParams& P, const float* phi, void* scratch, int nbins,
                               double* h_S, double* h_kpeak, double* h_Speak, double* h_kmean,
                               hipStream_t st) {
  const int nx = P.nx, ny = P.ny;
  if (nx > SPEC_MAX || ny > SPEC_MAX) return hipErrorInvalidValue;
  SpecLayout L = spec_layout(nx, ny);
  char* base = (char*)scratch;
  double* mean = (double*)(base + L.mean);
  double* rowsum = (double*)(base + L.rowsum);
  float2* buf = (float2*)(base + L.buf);
  double2* part = (double2*)(base + L.part);
  double2* kpart = (double2*)(base + L.kpart);
  double* bins = (double*)(base + L.bins);
  const int nbmax = nbins;
  hipLaunchKernelGGL(row_sum_kernel, dim3(ny), dim3(256), 0, st, phi, nx, rowsum);
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, st, rowsum, ny, 1.0 / ((double)nx * ny),
                     mean);
  int px = (nx & (nx - 1)) == 0, py = (ny & (ny - 1)) == 0;
  if (dft_lds_bytes(nx, px) > 65536 || dft_lds_bytes(ny, py) > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fft_x_kernel, dim3(ny), dim3(256), dft_lds_bytes(nx, px), st, phi, nx, ny,
                     mean, buf, px);
  hipLaunchKernelGGL(fft_y_bin_kernel, dim3(nx), dim3(256), dft_lds_bytes(ny, py), st, buf, nx, ny,
                     nbmax, part, kpart, py);
  const double dk = 6.283185307179586 / (nx < ny ? nx : ny);
  double* colsums = (double*)buf;  // the transposed spectrum is no longer needed
  hipLaunchKernelGGL(colsum_kernel, dim3(2 * nbmax), dim3(256), 0, st, (const double*)part, nx,
                     2 * nbmax, colsums);
  hipLaunchKernelGGL(colsum_kernel, dim3(2), dim3(256), 0, st, (const double*)kpart, nx, 2,
                     colsums + 2 * nbmax);
  hipLaunchKernelGGL(spec_final_kernel, dim3(1), dim3(256), 0, st, colsums, colsums + 2 * nbmax,
                     nbins, dk, bins);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double tail[3];
  e = hipMemcpyAsync(h_S, bins, sizeof(double) * nbins, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(tail, bins + nbins, sizeof(tail), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (h_kpeak) *h_kpeak = tail[0];
  if (h_Speak) *h_Speak = tail[1];
  if (h_kmean) *h_kmean = tail[2];
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------------
// Static scratch of the no-allocation structure factor (lam_structure_factor_static).  Each GPU
// the library runs on holds its own copy of this array until the process ends.  In host code
// its name is not a device address: the address comes from hipGetSymbolAddress, looked up once
// per device with that device current and kept below; only that address reaches the kernels.
// No part of it needs clearing: every value the structure-factor kernels read was written
// earlier in the same call.
static __device__ __align__(256) unsigned char scratch[LAM_SK_STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

size_t static_scratch_capacity() { return sizeof(scratch); }

hipError_t static_scratch(int device, void** out) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------------
// Orientation: one workgroup of 128 threads per row; each thread keeps its own column of the
// histogram in LDS, columns are then summed in a fixed order.
constexpr int OR_NT = 128;
constexpr int OR_MAXBINS = 36;

__global__ __launch_bounds__(OR_NT) void orient_row_kernel(const float* __restrict__ phi, int nx,
                                                           int ny, int walls, int nbins,
                                                           double* __restrict__ rowpart) {
  __shared__ double hist[OR_MAXBINS][OR_NT];
  __shared__ double sa[OR_NT], sb[OR_NT];
  const int y = blockIdx.x, t = threadIdx.x;
  for (int b = 0; b < nbins; ++b) hist[b][t] = 0.0;
  bool f;
  const int ym = wall_axis(y - 1, ny, walls, f), yp = wall_axis(y + 1, ny, walls, f);
  double sw = 0.0, sq = 0.0;
  const float binw = 3.14159265358979f / nbins;
  for (int x = t; x < nx; x += OR_NT) {
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    float gx = 0.5f * (phi[(size_t)y * nx + xp] - phi[(size_t)y * nx + xm]);
    float gy = 0.5f * (phi[(size_t)yp * nx + x] - phi[(size_t)ym * nx + x]);
    float w = gx * gx + gy * gy;
    if (w > 0.f) {
      float th = atan2f(gy, gx);
      if (th < 0.f) th += 3.14159265358979f;
      int b = (int)(th / binw);
      b = b < 0 ? 0 : (b >= nbins ? nbins - 1 : b);
      hist[b][t] += (double)w;
    }
    sw += (double)w;
    sq += (double)(gy * gy) - (double)(gx * gx);
  }
  sa[t] = sw;
  sb[t] = sq;
  __syncthreads();
  for (int o = OR_NT / 2; o > 0; o >>= 1) {
    if (t < o) {
      sa[t] += sa[t + o];
      sb[t] += sb[t + o];
      for (int b = 0; b < nbins; ++b) hist[b][t] += hist[b][t + o];
    }
    __syncthreads();
  }
  double* out = rowpart + (size_t)y * (nbins + 2);
  if (t == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
  if (t < nbins) out[2 + t] = hist[t][0];
}

// out[0] Q, out[1 .. nbins] histogram fractions, out[1+nbins ..] Q per row; tot = column sums
// of the row partials (sum |grad phi|^2, sum (g_y^2 - g_x^2), bins).
__global__ void orient_final_kernel(const double* __restrict__ rowpart,
                                    const double* __restrict__ tot, int ny, int nbins,
                                    double* __restrict__ out) {
  const int t = threadIdx.x;
  const int stride = nbins + 2;
  if (t == 0) out[0] = tot[0] > 0 ? tot[1] / tot[0] : 0.0;
  for (int b = t; b < nbins; b += blockDim.x) out[1 + b] = tot[0] > 0 ? tot[2 + b] / tot[0] : tot[2 + b];
  for (int y = t; y < ny; y += blockDim.x) {
    double w = rowpart[(size_t)y * stride], q = rowpart[(size_t)y * stride + 1];
    out[1 + nbins + y] = w > 0 ? q / w : 0.0;
  }
}

// 3D: angle of grad phi to the wall normal z, theta = arccos(|g_z| / |g|) in [0, pi/2], in nbins
// equal bins weighted by |g|^2, and the weighted second Legendre polynomial
// Q = sum(g_z^2 - (g_x^2 + g_y^2)/2) / sum |g|^2.  One workgroup per (y, z) line; the line
// partials are summed per layer and then over layers, each in a fixed order.
__global__ __launch_bounds__(OR_NT) void orient3_row_kernel(const float* __restrict__ phi, int nx,
                                                            int ny, int nz, int walls, int nbins,
                                                            double* __restrict__ rowpart) {
  __shared__ double hist[OR_MAXBINS][OR_NT];
  __shared__ double sa[OR_NT], sb[OR_NT];
  const int row = blockIdx.x, t = threadIdx.x;
  const int y = row % ny, z = row / ny;
  for (int b = 0; b < nbins; ++b) hist[b][t] = 0.0;
  bool f;
  const int zm = wall_axis(z - 1, nz, walls, f), zp = wall_axis(z + 1, nz, walls, f);
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const size_t plane = (size_t)nx * ny;
  const float* rc = phi + (size_t)z * plane + (size_t)y * nx;
  const float* ryp = phi + (size_t)z * plane + (size_t)yp * nx;
  const float* rym = phi + (size_t)z * plane + (size_t)ym * nx;
  const float* rzp = phi + (size_t)zp * plane + (size_t)y * nx;
  const float* rzm = phi + (size_t)zm * plane + (size_t)y * nx;
  double sw = 0.0, sq = 0.0;
  const float binw = 1.57079632679490f / nbins;
  for (int x = t; x < nx; x += OR_NT) {
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const float gx = 0.5f * (rc[xp] - rc[xm]);
    const float gy = 0.5f * (ryp[x] - rym[x]);
    const float gz = 0.5f * (rzp[x] - rzm[x]);
    const float w = gx * gx + gy * gy + gz * gz;
    if (w > 0.f) {
      const float th = acosf(fminf(fabsf(gz) / sqrtf(w), 1.f));
      int b = (int)(th / binw);
      b = b < 0 ? 0 : (b >= nbins ? nbins - 1 : b);
      hist[b][t] += (double)w;
    }
    sw += (double)w;
    sq += (double)(gz * gz) - 0.5 * ((double)(gx * gx) + (double)(gy * gy));
  }
  sa[t] = sw;
  sb[t] = sq;
  __syncthreads();
  for (int o = OR_NT / 2; o > 0; o >>= 1) {
    if (t < o) {
      sa[t] += sa[t + o];
      sb[t] += sb[t + o];
      for (int b = 0; b < nbins; ++b) hist[b][t] += hist[b][t + o];
    }
    __syncthreads();
  }
  double* out = rowpart + (size_t)row * (nbins + 2);
  if (t == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
  if (t < nbins) out[2 + t] = hist[t][0];
}

// Per-layer sums of the line partials: block (column, layer) sums the ny lines of its layer.
__global__ void layer_sum_kernel(const double* __restrict__ rowpart, int ny, int ld,
                                 double* __restrict__ layerpart) {
  __shared__ double sm[256];
  const int col = blockIdx.x, z = blockIdx.y;
  const double* M = rowpart + (size_t)z * ny * ld;
  double v = 0.0;
  for (int r = threadIdx.x; r < ny; r += 256) v += M[(size_t)r * ld + col];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) layerpart[(size_t)z * ld + col] = sm[0];
}

size_t orientation3_scratch_bytes(int ny, int nz) {
  const size_t ld = OR_MAXBINS + 2;
  return 8 * (ld * ((size_t)ny * nz + nz + 1) + 1 + OR_MAXBINS + nz) + 256;
}

hipError_t orientation_3d(const KParams& P, const float* phi, void* scratch, int nbins,
                          double* h_hist, double* h_Q, double* h_Qrow, hipStream_t st) {
  if (nbins > OR_MAXBINS) return hipErrorInvalidValue;
  const int ld = nbins + 2;
  double* rowpart = (double*)scratch;                      // [nz ny][nbins + 2]
  double* layerpart = rowpart + (size_t)P.ny * P.nz * ld;  // [nz][nbins + 2]
  double* tot = layerpart + (size_t)P.nz * ld;             // [nbins + 2]
  double* res = tot + ld;                                  // Q, bins, Q per layer
  hipLaunchKernelGGL(orient3_row_kernel, dim3(P.ny * P.nz), dim3(OR_NT), 0, st, phi, P.nx, P.ny,
                     P.nz, P.walls, nbins, rowpart);
  hipLaunchKernelGGL(layer_sum_kernel, dim3(ld, P.nz), dim3(256), 0, st, rowpart, P.ny, ld,
                     layerpart);
  hipLaunchKernelGGL(colsum_kernel, dim3(ld), dim3(256), 0, st, layerpart, P.nz, ld, tot);
  hipLaunchKernelGGL(orient_final_kernel, dim3(1), dim3(256), 0, st, layerpart, tot, P.nz, nbins,
                     res);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double Q;
  e = hipMemcpyAsync(&Q, res, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_hist, res + 1, sizeof(double) * nbins, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && h_Qrow)
    e = hipMemcpyAsync(h_Qrow, res + 1 + nbins, sizeof(double) * P.nz, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && h_Q) *h_Q = Q;
  return e;
}

hipError_t orientation_2d(const KParams& P, const float* phi, void* scratch, int nbins,
                          double* h_hist, double* h_Q, double* h_Qrow, hipStream_t st) {
  if (nbins > OR_MAXBINS) return hipErrorInvalidValue;
  SpecLayout L = spec_layout(P.nx, P.ny);
  double* rowpart = (double*)((char*)scratch + L.part);  // ny * (nbins + 2) doubles fit here
  double* res = (double*)((char*)scratch + L.buf);        // 1 + nbins + ny doubles fit here
  hipLaunchKernelGGL(orient_row_kernel, dim3(P.ny), dim3(OR_NT), 0, st, phi, P.nx, P.ny, P.walls,
                     nbins, rowpart);
  double* tot = res + 1 + nbins + P.ny;
  hipLaunchKernelGGL(colsum_kernel, dim3(nbins + 2), dim3(256), 0, st, rowpart, P.ny, nbins + 2,
                     tot);
  hipLaunchKernelGGL(orient_final_kernel, dim3(1), dim3(256), 0, st, rowpart, tot, P.ny, nbins,
                     res);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double Q;
  e = hipMemcpyAsync(&Q, res, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_hist, res + 1, sizeof(double) * nbins, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && h_Qrow)
    e = hipMemcpyAsync(h_Qrow, res + 1 + nbins, sizeof(double) * P.ny, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && h_Q) *h_Q = Q;
  return e;
}

}  // namespace lam
