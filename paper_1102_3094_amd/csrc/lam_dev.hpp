// lam_dev.hpp -- device-side definitions shared by the gfx950 kernels of the lamellar-fluid
// library: the kernel parameter block, index maps for periodic and wall-reflected axes, the
// XCD-aware tile order and small reduction helpers.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lam {

// Parameters as the kernels see them (FP32 arithmetic; FP64 only in reductions).
struct KParams {
  int nx, ny, nz;       // extents; nz = 1 in 2D
  int walls;            // walls normal to the last axis
  int hydro;            // lattice Boltzmann coupled
  int force_form;       // 0: -div P, 1: -phi grad mu
  float omega;          // 1/tau
  float kforce;         // 1 - 1/(2 tau), prefactor of the forcing term
  float Gamma, b, kappa, c;
  float Tc;
  float h;              // 1/n_phi, Euler sub-step length
  float gx, gy, gz;     // uniform test acceleration
  float r_T;            // xi / n_T
  int n_T;              // FTCS sub-steps (0: temperature frozen)
  int half_pops;        // populations stored as FP16 deviations
  int zch_phi;          // z slices per workgroup of the 3D phi kernel (1 .. its maximum)
};

// Storage conversions of the population deviations (FP32 or FP16 storage, FP32 arithmetic;
// FP16 rounding is to nearest even).
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__half v) { return __half2float(v); }
template <typename ST>
__device__ __forceinline__ ST from_f32(float v);
template <>
__device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ __half from_f32<__half>(float v) { return __float2half_rn(v); }

// Streaming (non-temporal) access to the population fields, which are not re-read within a step.
// Element `i` of the plane starting at `base`, addressed as base + a 32-bit byte offset (the host
// keeps every population plane below 2^32 bytes): the plane base is uniform, so the access takes
// the scalar-base form with one 32-bit vector offset instead of 64-bit vector address arithmetic.
template <typename T>
__device__ __forceinline__ T* plane_at(T* base, uint32_t i) {
  return (T*)((char*)base + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T* plane_at(const T* base, uint32_t i) {
  return (const T*)((const char*)base + i * (uint32_t)sizeof(T));
}

__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ __half ld_nt(const __half* p) {
  return __ushort_as_half(__builtin_nontemporal_load((const unsigned short*)p));
}
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(__half* p, __half v) {
  __builtin_nontemporal_store(__half_as_ushort(v), (unsigned short*)p);
}

// One member of an ensemble as the ensemble kernels see it: its parameters, its device buffers
// (populations by step parity, phi by step parity, phi scratch, u, T by parity + scratch) and the
// index of its first tile in the concatenated tile list.
struct EnsMember {
  KParams P;
  void* g[2];
  float* phi[2];
  float* psi[2];
  float* u;
  float* T[3];
  int tile0;
  int pad_;
};

// Reduction slots of the observables.
enum { R_MASS = 0, R_JX, R_JY, R_JZ, R_PHI, R_FE, R_UMAX, R_BAD, R_N };

// Periodic index for any integer.
__device__ __forceinline__ int wrap(int i, int n) {
  if (i >= 0 && i < n) return i;
  int m = i % n;
  return m < 0 ? m + n : m;
}

// Even reflection about the planes -1/2 and n - 1/2, folded with period 2n so that any integer
// maps into [0, n).  `flip` is set when the image is a mirror image (odd number of reflections).
__device__ __forceinline__ int reflect(int i, int n, bool& flip) {
  if (i >= 0 && i < n) {
    flip = false;
    return i;
  }
  int m = i % (2 * n);
  if (m < 0) m += 2 * n;
  flip = m >= n;
  return flip ? 2 * n - 1 - m : m;
}

// Index along the wall axis: reflected if walls are on, periodic otherwise.
__device__ __forceinline__ int wall_axis(int i, int n, int walls, bool& flip) {
  if (walls) return reflect(i, n, flip);
  flip = false;
  return wrap(i, n);
}

// Blocks of a 1D grid are dispatched round-robin over the 8 XCDs of an MI355X.  Give each XCD a
// contiguous range of tiles so that neighbouring tiles (which share halo reads) run under the
// same L2.  Bijective on [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int NX = 8;
  int q = nb / NX, r = nb % NX;
  int k = b % NX, j = b / NX;
  int base = k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q;
  return base + j;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// First derivatives: the isotropic central difference over the lattice's velocity set,
// d_k f(x) = 3 sum_q w_q e_qk f(x + e_q) (second order; on a mode exp(i k.x) it multiplies by
// i sin k_x (2 + cos k_y)/3 in 2D and i sin k_x (1 + cos k_y + cos k_z)/3 in 3D).  f(dr, dc) or
// f(dz, dr, dc) returns the value at the given offset (rows r = y, columns c = x).
// Contraction into fused multiply-adds is off inside these sums: otherwise a product returned by
// f (a flux psi u) is fused into the difference only where the compiler did not share it with a
// neighbouring site, which depends on the tile shape, and the results would differ in the last
// bit between tile shapes.
template <typename F>
__device__ __forceinline__ float iso2_x(F f) {
#pragma clang fp contract(off)
  return (1.f / 3.f) * (f(0, 1) - f(0, -1)) +
         (1.f / 12.f) * ((f(1, 1) - f(1, -1)) + (f(-1, 1) - f(-1, -1)));
}
template <typename F>
__device__ __forceinline__ float iso2_y(F f) {
#pragma clang fp contract(off)
  return (1.f / 3.f) * (f(1, 0) - f(-1, 0)) +
         (1.f / 12.f) * ((f(1, 1) - f(-1, 1)) + (f(1, -1) - f(-1, -1)));
}
template <typename F>
__device__ __forceinline__ float iso3_x(F f) {
#pragma clang fp contract(off)
  return (1.f / 6.f) * (f(0, 0, 1) - f(0, 0, -1)) +
         (1.f / 12.f) * (((f(0, 1, 1) - f(0, 1, -1)) + (f(0, -1, 1) - f(0, -1, -1))) +
                         ((f(1, 0, 1) - f(1, 0, -1)) + (f(-1, 0, 1) - f(-1, 0, -1))));
}
template <typename F>
__device__ __forceinline__ float iso3_y(F f) {
#pragma clang fp contract(off)
  return (1.f / 6.f) * (f(0, 1, 0) - f(0, -1, 0)) +
         (1.f / 12.f) * (((f(0, 1, 1) - f(0, -1, 1)) + (f(0, 1, -1) - f(0, -1, -1))) +
                         ((f(1, 1, 0) - f(1, -1, 0)) + (f(-1, 1, 0) - f(-1, -1, 0))));
}
template <typename F>
__device__ __forceinline__ float iso3_z(F f) {
#pragma clang fp contract(off)
  return (1.f / 6.f) * (f(1, 0, 0) - f(-1, 0, 0)) +
         (1.f / 12.f) * (((f(1, 0, 1) - f(-1, 0, 1)) + (f(1, 0, -1) - f(-1, 0, -1))) +
                         ((f(1, 1, 0) - f(-1, 1, 0)) + (f(1, -1, 0) - f(-1, -1, 0))));
}

}  // namespace lam
