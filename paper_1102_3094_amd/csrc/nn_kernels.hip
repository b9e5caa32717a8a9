// nn_kernels.hip -- gfx950 kernels of the U-Net surrogate: 3x3 convolutions (forward and input
// gradient) and their weight gradients on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16), plus
// the memory-bound pieces (input packing, pooling, upsampling, head, loss, reductions, Adam).
//
// Activations are NHWC bfloat16 (channel fastest) with a pixel stride `ld` that may exceed the
// channel count, so that a tensor can live inside a concatenation buffer.  A 3x3 layer is an
// implicit GEMM: M = pixels, N = output channels, K = 9 taps x input channels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lam_dev.hpp"
#include "nn_host.hpp"

namespace lam {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(bf16_t v) { return __uint_as_float((uint32_t)v << 16); }
// Round to nearest, ties to even (finite inputs).
__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
// Logistic function with the hardware reciprocal (one rounding more than an IEEE division,
// far below the bfloat16 rounding every activation goes through); exp overflow gives 0.
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  float s = sigm(z);
  return s * (1.f + z * (1.f - s));
}
__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

constexpr int PSTR = 40;  // LDS elements per pixel (or weight row) of a 32-channel chunk: 8 pad

// Workgroup = 4 waves; tile = (4 RW) rows x 32 columns x (32 NJ) output channels; wave w owns
// rows w RW .. w RW + RW - 1.  Per 32-channel chunk of the input: the (4 RW + 2) x 34 input
// patch and the 9 x 32 NJ x 32 weights are staged in LDS (the next chunk is loaded into
// registers while the matrix cores work on the current one).  For each column offset dx and
// 16-channel half, the wave reads RW + 2 input rows once and reuses them for the three row
// offsets dy.  The results leave through LDS (pixel-major rows) as 16-byte stores.
//
// FUSE (forward passes that keep no activations): FUSE_FIELDS builds the input from the planar
// FP32 fields (the packing of pack_input_kernel; only channels 0..15 are non-zero, so one
// 16-channel half is computed); FUSE_POOL reads a map of twice the resolution and averages 2x2
// blocks while staging (the arithmetic of pool_kernel); FUSE_HEAD applies the 1x1 head to the
// tile in LDS and writes the FP32 output instead of the activation (the arithmetic of
// head_fwd_kernel; needs all output channels in one tile).  Each gives the same bits as the
// separate kernels.
template <int MODE, int RW, int NJ, int FUSE, int WV = 4>
__global__ __launch_bounds__(64 * WV) void conv3x3_kernel(ConvArgs a) {
  // WV waves (4 or 8) per workgroup, each RW rows of 32 pixels
  constexpr int NT = 64 * WV;
  constexpr int PR = WV * RW + 2, PC = 34;
  constexpr int NPV = PR * PC * 4, NWV = 9 * 32 * NJ * 4;  // 16-byte vectors per chunk
  constexpr int LP = (NPV + NT - 1) / NT, LW = (NWV + NT - 1) / NT;
  __shared__ __align__(16) bf16_t sp[PR * PC * PSTR];
  __shared__ __align__(16) bf16_t sw[9 * 32 * NJ * PSTR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 31, kh = lane >> 5;
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int cob = L % a.nco, tile = L / a.nco;
  const int x0 = (tile % a.tiles_x) * 32, y0 = (tile / a.tiles_x) * WV * RW, co0 = cob * 32 * NJ;
  const int H = a.H, W = a.W;

  u32x4 rp[LP], rw[LW];
  // FUSE_FIELDS: one thread per patch pixel (consecutive lanes read consecutive x of each FP32
  // plane); channels 0..7 packed into one vector, channels 8..15 zero, 16..31 never read
  constexpr int NPX = PR * PC, LPX = (NPX + NT - 1) / NT;
  static_assert(LPX <= LP, "pixel registers fit the vector registers");
  auto load = [&](int c0) {
    if (FUSE == FUSE_FIELDS) {
#pragma unroll
      for (int i = 0; i < LPX; ++i) {
        const int p = tid + i * NT;
        rp[i] = u32x4{0, 0, 0, 0};
        const int pr = p / PC, col = p - pr * PC;
        const int y = y0 - 1 + pr;
        int x = x0 - 1 + col;
        x = x < 0 ? x + W : (x >= W ? x - W : x);
        if (p < NPX && y >= 0 && y < H) {
          const size_t np = (size_t)H * W, q = (size_t)y * W + x;
          float v[6];
#pragma unroll
          for (int c = 0; c < 4; ++c) v[c] = (a.fields[c * np + q] - a.pk.shift[c]) * a.pk.scale[c];
          v[4] = ((a.fields[3 * np + q] - a.pk.Tc) / a.pk.Tc - a.pk.shift[4]) * a.pk.scale[4];
          v[5] = 0.f;
          rp[i][0] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          rp[i][1] = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          rp[i][2] = (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
        }
      }
    } else {
#pragma unroll
    for (int i = 0; i < LP; ++i) {
      const int idx = tid + i * NT;
      rp[i] = u32x4{0, 0, 0, 0};
      if (idx < NPV) {
        const int pr = idx / (PC * 4), rem = idx % (PC * 4), col = rem >> 2, part = rem & 3;
        const int y = y0 - 1 + pr;
        int x = x0 - 1 + col;
        x = x < 0 ? x + W : (x >= W ? x - W : x);
        if (y >= 0 && y < H) {
          if (FUSE == FUSE_POOL) {
            float s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const size_t q = (size_t)(2 * y + (d >> 1)) * (2 * W) + 2 * x + (d & 1);
              const u32x4 v = *(const u32x4*)(a.in + q * a.in_ld + c0 + part * 8);
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                s8[2 * k] += __uint_as_float(v[k] << 16);
                s8[2 * k + 1] += __uint_as_float(v[k] & 0xFFFF0000u);
              }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
              rp[i][k] = (uint32_t)f2bf(0.25f * s8[2 * k]) | ((uint32_t)f2bf(0.25f * s8[2 * k + 1]) << 16);
          } else if (c0 < a.c_split) {
            rp[i] = *(const u32x4*)(a.in2 + ((size_t)(y >> 1) * (W >> 1) + (x >> 1)) * a.in2_ld + c0 + part * 8);
          } else {
            rp[i] = *(const u32x4*)(a.in + ((size_t)y * W + x) * a.in_ld + (c0 - a.c_split) + part * 8);
          }
        }
      }
    }
    }
#pragma unroll
    for (int i = 0; i < LW; ++i) {
      const int idx = tid + i * NT;
      if (idx < NWV) {
        const int tap = idx / (32 * NJ * 4), rem = idx % (32 * NJ * 4), co = rem >> 2, part = rem & 3;
        rw[i] = *(const u32x4*)(a.w + ((size_t)tap * a.Cout + co0 + co) * a.Cin + c0 + part * 8);
      }
    }
  };
  auto stage = [&]() {
    if (FUSE == FUSE_FIELDS) {
#pragma unroll
      for (int i = 0; i < LPX; ++i) {
        const int p = tid + i * NT;
        if (p < NPX) {
          *(u32x4*)(sp + p * PSTR) = rp[i];
          *(u32x4*)(sp + p * PSTR + 8) = u32x4{0, 0, 0, 0};
        }
      }
    } else {
#pragma unroll
    for (int i = 0; i < LP; ++i) {
      const int idx = tid + i * NT;
      if (idx < NPV) {
        const int pr = idx / (PC * 4), rem = idx % (PC * 4), col = rem >> 2, part = rem & 3;
        *(u32x4*)(sp + (pr * PC + col) * PSTR + part * 8) = rp[i];
      }
    }
    }
#pragma unroll
    for (int i = 0; i < LW; ++i) {
      const int idx = tid + i * NT;
      if (idx < NWV) {
        const int tap = idx / (32 * NJ * 4), rem = idx % (32 * NJ * 4), co = rem >> 2, part = rem & 3;
        *(u32x4*)(sw + (tap * 32 * NJ + co) * PSTR + part * 8) = rw[i];
      }
    }
  };

  f32x16 acc[RW][NJ];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[r][j][q] = 0.f;

  load(0);
  for (int c0 = 0; c0 < a.Cin; c0 += 32) {
    __syncthreads();
    stage();
    __syncthreads();
    if (c0 + 32 < a.Cin) load(c0 + 32);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
      for (int kk = 0; kk < (FUSE == FUSE_FIELDS ? 1 : 2); ++kk) {
        bf16x8 A[RW + 2];
#pragma unroll
        for (int r = 0; r < RW + 2; ++r)
          A[r] = as_bf(*(const u32x4*)(sp + ((wave * RW + r) * PC + m + dx) * PSTR + kk * 16 + kh * 8));
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int tap = dy * 3 + dx;
          bf16x8 B[NJ];
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            B[j] = as_bf(*(const u32x4*)(sw + (tap * 32 * NJ + j * 32 + m) * PSTR + kk * 16 + kh * 8));
#pragma unroll
          for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
              acc[r][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[r + dy], B[j], acc[r][j], 0, 0, 0);
        }
      }
    }
  }

  // D layout of the 32x32 MFMA: lane holds column m (output channel) and rows
  // 8 (q / 4) + 4 kh + (q % 4), q = 0..15 (pixel within the 32-column row).  Per 32-channel
  // block j (and per stored quantity: the output, then the forward pass's pre-activation) the
  // wave writes its values into LDS as [pixel][channel] and the workgroup stores 16-byte pieces.
  constexpr int TP = WV * RW * 32;  // pixels of the tile
  static_assert(TP * PSTR <= PR * PC * PSTR, "epilogue tile exceeds the patch buffer");
  bf16_t* so = sp;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int co = co0 + j * 32 + m;
    const float bco = MODE == CONV_FWD ? a.bias[co] : 0.f;
    const int passes = (MODE == CONV_FWD && a.zout) ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
      __syncthreads();
      if (FUSE == FUSE_HEAD && tid < 99) {
        // head weights into the free weight buffer: [3][32], then the 3 biases
        float* hw = (float*)sw;
        hw[tid] = a.head_w[tid];
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int pl = (wave * RW + r) * 32 + 8 * (q >> 2) + 4 * kh + (q & 3);
          const float v = acc[r][j][q];
          float o;
          if (MODE == CONV_FWD) {
            const float z = v + bco;
            o = pass == 0 ? z * sigm(z) : z;
          } else if (MODE == CONV_BWD_SILU) {
            const size_t p = (size_t)(y0 + pl / 32) * W + x0 + (pl & 31);
            o = v * dsilu(bf2f(a.zprev[p * a.Cout + co]));
          } else {
            o = v;
          }
          so[pl * PSTR + m] = f2bf(o);
        }
      }
      __syncthreads();
      if (FUSE == FUSE_HEAD) {
        // 1x1 head (3 outputs) over the Cout = 32 channels of each pixel (launched with NJ = 1
        // only; weights from LDS, read at the same address by every lane)
        const size_t np = (size_t)H * W;
        const float* hw = (const float*)sw;
        double hs0 = 0.0;
        for (int pl = tid; pl < TP; pl += NT) {
          float sacc[3];
#pragma unroll
          for (int o = 0; o < 3; ++o) sacc[o] = hw[96 + o];
#pragma unroll
          for (int k8 = 0; k8 < 4; ++k8) {
            const u32x4 v = *(const u32x4*)(so + pl * PSTR + 8 * k8);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const float x = __uint_as_float(t & 1 ? (v[t / 2] & 0xFFFF0000u) : (v[t / 2] << 16));
              const int k = 8 * k8 + t;
#pragma unroll
              for (int o = 0; o < 3; ++o) sacc[o] += hw[32 * o + k] * x;
            }
          }
          const size_t p = (size_t)(y0 + pl / 32) * W + x0 + (pl & 31);
#pragma unroll
          for (int o = 0; o < 3; ++o) a.head_out[o * np + p] = sacc[o];
          hs0 += (double)sacc[0];
        }
        if (a.head_part) {  // per-workgroup sums for the conservation shift of a surrogate step
          __shared__ double hred[WV];
          hs0 = wave_sum(hs0);
          if (lane == 0) hred[wave] = hs0;
          __syncthreads();
          if (tid == 0) {
            double s0 = 0.0;
            for (int w = 0; w < WV; ++w) s0 += hred[w];
            a.head_part[blockIdx.x] = s0;
          }
        }
        continue;
      }
      for (int t = tid; t < TP * 4; t += NT) {
        const int pl = t >> 2, part = t & 3;
        const size_t p = (size_t)(y0 + pl / 32) * W + x0 + (pl & 31);
        bf16_t* dst = pass == 0 ? a.out + p * a.out_ld : a.zout + p * a.Cout;
        *(u32x4*)(dst + co0 + j * 32 + part * 8) = *(const u32x4*)(so + pl * PSTR + part * 8);
      }
    }
  }
}

// Weight gradient of a 3x3 layer: dW[tap][co][ci] = sum_p g[p][co] X[p + off(tap)][ci], an MFMA
// GEMM with K = pixels.  Workgroup = 3 waves (wave = row offset dy); block (32 MJ output channels)
// x (32 input channels) x a range of pixel chunks (4 rows x 32 columns each).  Both operands
// need 8 consecutive pixels of one channel per lane, so each chunk is transposed into LDS
// (channel-major): g once, X three times (one copy per column offset dx, so that every MFMA
// operand read is 16-byte aligned).  Partial sums go to part[split][9][Cout][Cin] (FP32).
struct WgradArgs {
  const bf16_t* x;  // layer input (offset to its first channel), pixel stride x_ld; channels
  int x_ld;         // [0, c_split) come from x2 at half resolution (nearest upsampling)
  const bf16_t* x2;
  int x2_ld, c_split;
  const bf16_t* g;  // gradient w.r.t. the pre-activation, [pixels][Cout]
  float* part;
  int H, W, Cin, Cout;
  int nco, nci, nsplit, nchunks, cps;  // blocks, splits, chunks, chunks per split
};

constexpr int GST = 4 * 32 + 8;   // LDS stride per channel of the g chunk (elements)
constexpr int XST = 6 * 32 + 8;   // LDS stride per channel of one shifted X chunk

template <int MJ>
__global__ __launch_bounds__(192) void wgrad_kernel(WgradArgs a) {
  __shared__ __align__(16) bf16_t sg[32 * MJ * GST];
  __shared__ __align__(16) bf16_t sx[3 * 32 * XST];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;  // wave = dy index
  const int m = lane & 31, kh = lane >> 5;
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int split = L % a.nsplit, blk = L / a.nsplit;
  const int cib = blk % a.nci, cob = blk / a.nci;
  const int ci0 = cib * 32, co0 = cob * 32 * MJ;
  const int H = a.H, W = a.W, tiles_x = W / 32;

  f32x16 acc[3][MJ];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int j = 0; j < MJ; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[d][j][q] = 0.f;

  const int c_begin = split * a.cps;
  const int c_end = min(a.nchunks, c_begin + a.cps);
  for (int ch = c_begin; ch < c_end; ++ch) {
    const int x0 = (ch % tiles_x) * 32, y0 = (ch / tiles_x) * 4;
    __syncthreads();
    // g chunk: tasks (channel pair, row, group of 8 pixels) -> two 16-byte LDS rows.
    for (int t = tid; t < 16 * MJ * 4 * 4; t += 192) {
      const int cp = t % (16 * MJ), rg = t / (16 * MJ), r = rg >> 2, grp = rg & 3;
      uint32_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        v[k] = *(const uint32_t*)(a.g + ((size_t)(y0 + r) * W + x0 + grp * 8 + k) * a.Cout + co0 + 2 * cp);
      u32x4 lo, hi;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lo[k] = (v[2 * k] & 0xFFFFu) | (v[2 * k + 1] << 16);
        hi[k] = (v[2 * k] >> 16) | (v[2 * k + 1] & 0xFFFF0000u);
      }
      *(u32x4*)(sg + (2 * cp) * GST + r * 32 + grp * 8) = lo;
      *(u32x4*)(sg + (2 * cp + 1) * GST + r * 32 + grp * 8) = hi;
    }
    // X chunk, three column shifts: tasks (channel pair, dx, patch row, group).
    for (int t = tid; t < 16 * 3 * 6 * 4; t += 192) {
      const int cp = t % 16, rest = t / 16, grp = rest & 3, pr = (rest >> 2) % 6, dx = (rest >> 2) / 6;
      const int y = y0 - 1 + pr;
      uint32_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        int x = x0 + grp * 8 + k + dx - 1;
        x = x < 0 ? x + W : (x >= W ? x - W : x);
        if (y < 0 || y >= H) v[k] = 0u;
        else if (ci0 < a.c_split)
          v[k] = *(const uint32_t*)(a.x2 + ((size_t)(y >> 1) * (W >> 1) + (x >> 1)) * a.x2_ld + ci0 + 2 * cp);
        else
          v[k] = *(const uint32_t*)(a.x + ((size_t)y * W + x) * a.x_ld + (ci0 - a.c_split) + 2 * cp);
      }
      u32x4 lo, hi;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lo[k] = (v[2 * k] & 0xFFFFu) | (v[2 * k + 1] << 16);
        hi[k] = (v[2 * k] >> 16) | (v[2 * k + 1] & 0xFFFF0000u);
      }
      bf16_t* base = sx + dx * 32 * XST + pr * 32 + grp * 8;
      *(u32x4*)(base + (2 * cp) * XST) = lo;
      *(u32x4*)(base + (2 * cp + 1) * XST) = hi;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        bf16x8 A[MJ];
#pragma unroll
        for (int j = 0; j < MJ; ++j)
          A[j] = as_bf(*(const u32x4*)(sg + (j * 32 + m) * GST + r * 32 + kk * 16 + kh * 8));
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const bf16x8 B = as_bf(*(const u32x4*)(sx + dx * 32 * XST + m * XST + (r + wave) * 32 + kk * 16 + kh * 8));
#pragma unroll
          for (int j = 0; j < MJ; ++j)
            acc[dx][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[j], B, acc[dx][j], 0, 0, 0);
        }
      }
    }
  }
  // acc[dx][j] holds D[co = co0 + 32 j + row][ci = ci0 + m], row = 8 (q/4) + 4 kh + q % 4.
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) {
    const int tap = wave * 3 + dx;
#pragma unroll
    for (int j = 0; j < MJ; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int co = co0 + 32 * j + 8 * (q >> 2) + 4 * kh + (q & 3);
        a.part[(((size_t)split * 9 + tap) * a.Cout + co) * a.Cin + ci0 + m] = acc[dx][j][q];
      }
  }
}

// grad[i] += sum_s part[s][i'] in fixed order (deterministic); the partials are laid out
// [9][Cout][Cin_pad], the gradient [9][Cout][Cin_dst] (Cin_dst <= Cin_pad drops zero padding).
__global__ void reduce_splits_kernel(const float* __restrict__ part, int nsplit, int Cin_pad,
                                     int Cin_dst, size_t n_dst, float* __restrict__ grad) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_dst) return;
  const size_t src = (i / Cin_dst) * Cin_pad + i % Cin_dst;
  const size_t n_src = n_dst / Cin_dst * Cin_pad;
  float s = 0.f;
  for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * n_src + src];
  grad[i] += s;
}

// Column sums of a [npix][C] bfloat16 tensor (C <= 256, 256 % C == 0) over pixel ranges of
// `per` pixels: part[block][c] (FP64).
__global__ __launch_bounds__(256) void colsum_bf16_kernel(const bf16_t* __restrict__ g, int npix,
                                                          int C, int per, double* __restrict__ part) {
  __shared__ double sm[256];
  const int tid = threadIdx.x, c = tid % C, grp = tid / C, ngrp = 256 / C;
  const int p0 = blockIdx.x * per, p1 = min(npix, p0 + per);
  double s = 0.0;
  for (int p = p0 + grp; p < p1; p += ngrp) s += bf2f(g[(size_t)p * C + c]);
  sm[tid] = s;
  __syncthreads();
  if (grp == 0) {
    for (int k = 1; k < ngrp; ++k) s += sm[k * C + c];
    part[(size_t)blockIdx.x * C + c] = s;
  }
}

// out[i] += sum_b part[b][i] (FP64 partials into an FP32 vector), fixed order.
__global__ void reduce_blocks_f64_kernel(const double* __restrict__ part, int nblk, int n,
                                         float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + i];
  out[i] += (float)s;
}

// Input packing: fields [4][H][W] FP32 (phi, ux, uy, T) -> [H W][32] bfloat16, channels
// (f - shift) * scale, channel 4 from a = (T - Tc) / Tc, channels 5..31 zero.
__global__ void pack_input_kernel(const float* __restrict__ f, size_t npix, PackArgs pa,
                                  bf16_t* __restrict__ x) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float v[6];
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = (f[c * npix + p] - pa.shift[c]) * pa.scale[c];
  v[4] = ((f[3 * npix + p] - pa.Tc) / pa.Tc - pa.shift[4]) * pa.scale[4];
  v[5] = 0.f;
  u32x4 w0;
  w0[0] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  w0[1] = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
  w0[2] = (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
  w0[3] = 0;
  u32x4* dst = (u32x4*)(x + p * 32);
  dst[0] = w0;
  dst[1] = dst[2] = dst[3] = u32x4{0, 0, 0, 0};
}

// Gradient with respect to the planar FP32 fields from the gradient gx with respect to the packed
// input (pixel stride 32): the chain rule through the affine maps of pack_input_kernel; T enters
// channel 3 directly and channel 4 through a = (T - Tc) / Tc.
__global__ void field_grad_kernel(const bf16_t* __restrict__ gx, size_t npix, PackArgs pa,
                                  float* __restrict__ g) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const u32x4 w = *(const u32x4*)(gx + p * 32);
  float v[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[2 * k] = bf2f((bf16_t)(w[k] & 0xffffu));
    v[2 * k + 1] = bf2f((bf16_t)(w[k] >> 16));
  }
  g[p] = v[0] * pa.scale[0];
  g[npix + p] = v[1] * pa.scale[1];
  g[2 * npix + p] = v[2] * pa.scale[2];
  g[3 * npix + p] = v[3] * pa.scale[3] + v[4] * (pa.scale[4] / pa.Tc);
}

// 2x2 average pool: in [H][W] (pixel stride in_ld) -> out [H/2][W/2][C]; one thread per output
// pixel and group of 8 channels.
__global__ void pool_kernel(const bf16_t* __restrict__ in, int in_ld, int H, int W, int C,
                            bf16_t* __restrict__ out) {
  const int h = H / 2, w = W / 2, G = C / 8;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)h * w * G) return;
  const int g = (int)(i % G);
  const size_t p = i / G;
  const int y = (int)(p / w), x = (int)(p % w);
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const size_t q = (size_t)(2 * y + (d >> 1)) * W + 2 * x + (d & 1);
    const u32x4 v = *(const u32x4*)(in + q * in_ld + g * 8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s[2 * k] += __uint_as_float(v[k] << 16);
      s[2 * k + 1] += __uint_as_float(v[k] & 0xFFFF0000u);
    }
  }
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    o[k] = (uint32_t)f2bf(0.25f * s[2 * k]) | ((uint32_t)f2bf(0.25f * s[2 * k + 1]) << 16);
  *(u32x4*)(out + p * C + g * 8) = o;
}

// Nearest 2x upsampling: in [h][w][C] -> out [2h][2w] (pixel stride out_ld, channels 0..C-1).
__global__ void up_kernel(const bf16_t* __restrict__ in, int h, int w, int C,
                          bf16_t* __restrict__ out, int out_ld) {
  const int W = 2 * w, G = C / 8;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)4 * h * w * G) return;
  const int g = (int)(i % G);
  const size_t p = i / G;
  const int y = (int)(p / W), x = (int)(p % W);
  *(u32x4*)(out + p * out_ld + g * 8) = *(const u32x4*)(in + ((size_t)(y / 2) * w + x / 2) * C + g * 8);
}

// Gradient through the upsampling into a SiLU output: gz[p][c] = bf16(silu'(z[p][c]) *
// sum over the 2x2 fine pixels of gcat[.][c]) for the coarse [h][w][C] map; gcat has pixel
// stride cat_ld, the upsampled channels first.
__global__ void up_bwd_silu_kernel(const bf16_t* __restrict__ gcat, int cat_ld, int h, int w, int C,
                                   const bf16_t* __restrict__ z, bf16_t* __restrict__ gz) {
  const int W = 2 * w, G = C / 8;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)h * w * G) return;
  const int g = (int)(i % G);
  const size_t p = i / G;
  const int y = (int)(p / w), x = (int)(p % w);
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const size_t q = (size_t)(2 * y + (d >> 1)) * W + 2 * x + (d & 1);
    const u32x4 v = *(const u32x4*)(gcat + q * cat_ld + g * 8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s[2 * k] += __uint_as_float(v[k] << 16);
      s[2 * k + 1] += __uint_as_float(v[k] & 0xFFFF0000u);
    }
  }
  const u32x4 zv = *(const u32x4*)(z + p * C + g * 8);
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float z0 = __uint_as_float(zv[k] << 16), z1 = __uint_as_float(zv[k] & 0xFFFF0000u);
    o[k] = (uint32_t)f2bf(s[2 * k] * dsilu(z0)) | ((uint32_t)f2bf(s[2 * k + 1] * dsilu(z1)) << 16);
  }
  *(u32x4*)(gz + p * C + g * 8) = o;
}

// Gradient into an encoder output that feeds both the skip connection and the pool:
// gz[p][c] = bf16(silu'(z[p][c]) (gskip[p][c] + gpool[p/2][c] / 4)) on the fine [H][W][C] map;
// gskip has pixel stride skip_ld.
__global__ void pool_bwd_silu_kernel(const bf16_t* __restrict__ gskip, int skip_ld,
                                     const bf16_t* __restrict__ gpool, int H, int W, int C,
                                     const bf16_t* __restrict__ z, bf16_t* __restrict__ gz) {
  const int G = C / 8;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)H * W * G) return;
  const int g = (int)(i % G);
  const size_t p = i / G;
  const int y = (int)(p / W), x = (int)(p % W);
  const u32x4 a = *(const u32x4*)(gskip + p * skip_ld + g * 8);
  const u32x4 b = *(const u32x4*)(gpool + ((size_t)(y / 2) * (W / 2) + x / 2) * C + g * 8);
  const u32x4 zv = *(const u32x4*)(z + p * C + g * 8);
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float v0 = __uint_as_float(a[k] << 16) + 0.25f * __uint_as_float(b[k] << 16);
    float v1 = __uint_as_float(a[k] & 0xFFFF0000u) + 0.25f * __uint_as_float(b[k] & 0xFFFF0000u);
    v0 *= dsilu(__uint_as_float(zv[k] << 16));
    v1 *= dsilu(__uint_as_float(zv[k] & 0xFFFF0000u));
    o[k] = (uint32_t)f2bf(v0) | ((uint32_t)f2bf(v1) << 16);
  }
  *(u32x4*)(gz + p * C + g * 8) = o;
}

// Head: out[c][p] = b[c] + sum_k Wh[c][k] d[p][k] for c < nout (<= 4), FP32 planar output, C = d's
// channels (<= 64).
__global__ void head_fwd_kernel(const bf16_t* __restrict__ d, int C, int nout, size_t npix,
                                const float* __restrict__ Wh, float* __restrict__ out) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float sacc[4];
#pragma unroll
  for (int o = 0; o < 4; ++o) sacc[o] = o < nout ? Wh[nout * C + o] : 0.f;
  for (int k = 0; k < C; k += 8) {
    const u32x4 v = *(const u32x4*)(d + p * C + k);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float x = __uint_as_float(t & 1 ? (v[t / 2] & 0xFFFF0000u) : (v[t / 2] << 16));
#pragma unroll
      for (int o = 0; o < 4; ++o)
        if (o < nout) sacc[o] += Wh[o * C + k + t] * x;
    }
  }
#pragma unroll
  for (int o = 0; o < 4; ++o)
    if (o < nout) out[o * npix + p] = sacc[o];
}

// Loss gradient: gout[c][p] = 2 (out - t) / (nout npix); per-block FP64 partial of sum (out - t)^2.
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* __restrict__ out,
                                                        const float* __restrict__ t,
                                                        const float* __restrict__ extra, int nout,
                                                        size_t npix, float* __restrict__ gout,
                                                        double* __restrict__ part) {
  __shared__ double sm[4];
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (p < npix) {
    const float inv = 2.f / ((float)nout * (float)npix);
    for (int c = 0; c < nout; ++c) {
      const float d = out[c * npix + p] - t[c * npix + p];
      s += (double)d * d;
      gout[c * npix + p] = extra ? inv * d + extra[c * npix + p] : inv * d;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

// Head weight gradient partials over pixel ranges: part[b][c C + k] = sum_p gout[c][p] d[p][k],
// part[b][nout C + c] = sum_p gout[c][p], c < nout (<= 4).  Thread = (k, pixel group); C <= 64.
__global__ __launch_bounds__(256) void head_wgrad_kernel(const bf16_t* __restrict__ d, int C,
                                                         int nout, size_t npix, int per,
                                                         const float* __restrict__ gout,
                                                         double* __restrict__ part) {
  __shared__ double sm[256][4];
  const int tid = threadIdx.x, k = tid % C, grp = tid / C, ngrp = 256 / C;
  const size_t p0 = (size_t)blockIdx.x * per, p1 = min(npix, p0 + per);
  double sacc[4] = {0, 0, 0, 0}, bacc[4] = {0, 0, 0, 0};
  for (size_t p = p0 + grp; p < p1; p += ngrp) {
    const float x = bf2f(d[p * C + k]);
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if (o < nout) {
        const float g = gout[o * npix + p];
        sacc[o] += (double)g * x;
        if (k == 0) bacc[o] += g;
      }
    }
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) sm[tid][o] = sacc[o];
  __syncthreads();
  double* ob = part + (size_t)blockIdx.x * (nout * C + nout);
  if (grp == 0) {
    for (int q = 1; q < ngrp; ++q)
#pragma unroll
      for (int o = 0; o < 4; ++o) sacc[o] += sm[q * C + k][o];
    for (int o = 0; o < nout; ++o) ob[o * C + k] = sacc[o];
  }
  __syncthreads();
  if (k == 0)
#pragma unroll
    for (int o = 0; o < 4; ++o) sm[grp][o] = bacc[o];
  __syncthreads();
  if (tid == 0)
    for (int o = 0; o < nout; ++o) {
      double c = 0;
      for (int q = 0; q < ngrp; ++q) c += sm[q][o];
      ob[nout * C + o] = c;
    }
}

// Gradient into the last decoder output: gz[p][k] = bf16(silu'(z[p][k]) sum_c gout[c][p] Wh[c][k]).
__global__ void head_dgrad_kernel(const float* __restrict__ gout, size_t npix, int C, int nout,
                                  const float* __restrict__ Wh, const bf16_t* __restrict__ z,
                                  bf16_t* __restrict__ gz) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix * C) return;
  const size_t p = i / C;
  const int k = (int)(i % C);
  float g = gout[p] * Wh[k];
  for (int o = 1; o < nout; ++o) g += gout[o * npix + p] * Wh[o * C + k];
  gz[i] = f2bf(g * dsilu(bf2f(z[i])));
}

// bfloat16 copies of one 3x3 layer's FP32 weights W[9][Cout][Cin]: wf[9][Cout][Cin_pad] (zero
// beyond Cin) for the forward pass and, if wd is given, wd[8 - tap][ci][co] (ci < Cin_pad, zero
// beyond Cin) for the input gradient (the same kernel run backwards: taps mirrored, channel roles
// swapped).
__global__ void refresh_weights_kernel(const float* __restrict__ W, int Cout, int Cin, int Cin_pad,
                                       bf16_t* __restrict__ wf, bf16_t* __restrict__ wd) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)9 * Cout * Cin_pad) return;
  const int ci = (int)(i % Cin_pad);
  const size_t r = i / Cin_pad;
  const int co = (int)(r % Cout), tap = (int)(r / Cout);
  const size_t id = ((size_t)(8 - tap) * Cin_pad + ci) * Cout + co;
  if (ci >= Cin) {
    wf[i] = 0;
    if (wd) wd[id] = 0;
    return;
  }
  const bf16_t v = f2bf(W[((size_t)tap * Cout + co) * Cin + ci]);
  wf[i] = v;
  if (wd) wd[id] = v;
}

// Adam (Kingma & Ba, 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// theta -= lr (m / c1) / (sqrt(v / c2) + eps), g = grad * gscale; c1, c2 the bias corrections.
__global__ void adam_kernel(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ grad, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2, float gscale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i] * gscale;
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Training target: t[c][p] = (later - earlier) / out_scale[c] for the output channels phi, u_x,
// u_y (the first three field planes).
__global__ void make_target_kernel(const float* __restrict__ e, const float* __restrict__ l,
                                   size_t npix, float s0, float s1, float s2,
                                   float* __restrict__ t) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * npix) return;
  const int c = (int)(i / npix);
  const float s = c == 0 ? s0 : (c == 1 ? s1 : s2);
  t[i] = (l[i] - e[i]) / s;
}

// Per-block FP64 sums of one FP32 plane (an increment in units of its output scale).
__global__ __launch_bounds__(256) void sum_f32_kernel(const float* __restrict__ x, size_t n,
                                                      double* __restrict__ part) {
  __shared__ double sm[4];
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  double s = i < n ? (double)x[i] : 0.0;
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

// Mean of the per-block sums (phi increment or clamp excess): fixed-order tree
// over the blocks (one workgroup), written to part[nblk].
__global__ __launch_bounds__(256) void mean_kernel(double* __restrict__ part, int nblk, size_t npix) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[b];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[nblk] = sm[0] / (double)npix;
}

// One surrogate step applied in place: f[c] += out[c] s_c for phi, u_x, u_y, with phi shifted by
// the mean of its increment so that its sum is unchanged.
__global__ void apply_kernel(float* __restrict__ f, const float* __restrict__ out, size_t npix,
                             float s0, float s1, float s2, const double* __restrict__ mean_phi) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const float mu = (float)*mean_phi;
  f[p] += (out[p] - mu) * s0;
  f[npix + p] += out[npix + p] * s1;
  f[2 * npix + p] += out[2 * npix + p] * s2;
}

// Order-parameter limiter of a rollout.  absmax: per-block max |phi| into part, then the block
// maxima into part[nblk] (one workgroup, fixed order).
__global__ __launch_bounds__(256) void absmax_f32_kernel(const float* __restrict__ x, size_t n,
                                                         double* __restrict__ part) {
  __shared__ double sm[4];
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  double m = i < n ? fabs((double)x[i]) : 0.0;
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}
__global__ __launch_bounds__(256) void max_final_kernel(double* __restrict__ part, int nblk,
                                                        double* __restrict__ out) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) m = fmax(m, part[b]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}
// phi <- clamp(phi, -b, b) with b = factor * (*bound); per-block FP64 sums of the removed excess.
__global__ __launch_bounds__(256) void clamp_excess_kernel(float* __restrict__ phi, size_t n,
                                                           const double* __restrict__ bound,
                                                           float factor, double* __restrict__ part) {
  __shared__ double sm[4];
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const float b = factor * (float)*bound, v = phi[i];
    const float c = fminf(fmaxf(v, -b), b);
    phi[i] = c;
    e = (double)v - (double)c;
  }
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}
// phi += mean excess (part[nblk]): the clamped field keeps its sum.
__global__ void add_mean_kernel(float* __restrict__ phi, size_t n, const double* __restrict__ mean) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) phi[i] += (float)*mean;
}

// ------------------------------------------------------------------------------------------
// Launchers

static unsigned nblocks(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Tile shapes: rows per wave RW in {1, 2, 4} (the tile has 4 RW rows, which must divide H) and
// NJ in {1, 2} blocks of 32 output channels (NJ = 2 needs Cout % 64 == 0).
int conv_shapes(int H, int Cout, int* codes, int max_codes) {
  int n = 0;
  for (int rw : {1, 2, 4})
    for (int nj : {1, 2})
      if (H % (4 * rw) == 0 && Cout % (32 * nj) == 0 && n < max_codes) codes[n++] = 10 * rw + nj;
  for (int rw : {1, 2})  // eight waves per workgroup: twice the rows per staged weight tile
    for (int nj : {1, 2})
      if (H % (8 * rw) == 0 && Cout % (32 * nj) == 0 && n < max_codes) codes[n++] = 100 + 10 * rw + nj;
  return n;
}

// Default pick: the largest register tile (RW 2, NJ 2) unless the grid would leave compute
// units idle, then smaller tiles.
int conv_default_shape(int H, int W, int Cout) {
  const int tx = W / 32;
  int nj = Cout % 64 == 0 ? 2 : 1;
  int rw = H % 8 == 0 ? 2 : 1;
  auto blocks = [&]() { return (long)tx * (H / (4 * rw)) * (Cout / (32 * nj)); };
  if (blocks() < 512 && rw == 2) rw = 1;
  if (blocks() < 256 && nj == 2) nj = 1;
  return 10 * rw + nj;
}

template <int MODE, int RW, int NJ, int FUSE, int WV = 4>
static void conv_launch(ConvArgs a, hipStream_t st) {
  a.tiles_x = a.W / 32;
  a.nco = a.Cout / (32 * NJ);
  const unsigned grid = (unsigned)((a.W / 32) * (a.H / (WV * RW)) * a.nco);
  hipLaunchKernelGGL((conv3x3_kernel<MODE, RW, NJ, FUSE, WV>), grid, 64 * WV, 0, st, a);
}

template <int MODE, int FUSE>
static hipError_t conv_shape_dispatch(const ConvArgs& a, int code, hipStream_t st) {
  switch (code) {
    case 11: conv_launch<MODE, 1, 1, FUSE>(a, st); break;
    case 12: conv_launch<MODE, 1, 2, FUSE>(a, st); break;
    case 21: conv_launch<MODE, 2, 1, FUSE>(a, st); break;
    case 22: conv_launch<MODE, 2, 2, FUSE>(a, st); break;
    case 41: conv_launch<MODE, 4, 1, FUSE>(a, st); break;
    case 42: conv_launch<MODE, 4, 2, FUSE>(a, st); break;
    case 111: conv_launch<MODE, 1, 1, FUSE, 8>(a, st); break;
    case 112: conv_launch<MODE, 1, 2, FUSE, 8>(a, st); break;
    case 121: conv_launch<MODE, 2, 1, FUSE, 8>(a, st); break;
    case 122: conv_launch<MODE, 2, 2, FUSE, 8>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
static hipError_t conv_mode(const ConvArgs& a, hipStream_t st) {
  int code = a.shape ? a.shape : conv_default_shape(a.H, a.W, a.Cout);
  if (a.fuse == FUSE_HEAD) code = ((code % 100) / 10) * 10 + 1;  // 4 waves, 32 channels per tile
  const int wv = code >= 100 ? 8 : 4, rw = (code % 100) / 10, nj = code % 10;
  if (a.H % (wv * rw) || a.Cout % (32 * nj) || a.W % 32 || a.Cin % 32 || a.c_split % 32)
    return hipErrorInvalidValue;
  if (MODE != CONV_FWD && a.fuse != FUSE_NONE) return hipErrorInvalidValue;
  if ((a.fuse == FUSE_FIELDS && a.Cin != 32) || (a.fuse == FUSE_HEAD && a.Cout != 32) ||
      (a.fuse != FUSE_NONE && a.c_split))
    return hipErrorInvalidValue;
  switch (a.fuse) {
    case FUSE_NONE: return conv_shape_dispatch<MODE, FUSE_NONE>(a, code, st);
    case FUSE_FIELDS: return conv_shape_dispatch<MODE, FUSE_FIELDS>(a, code, st);
    case FUSE_POOL: return conv_shape_dispatch<MODE, FUSE_POOL>(a, code, st);
    case FUSE_HEAD: return conv_shape_dispatch<MODE, FUSE_HEAD>(a, code, st);
    default: return hipErrorInvalidValue;
  }
}

int conv_blocks(const ConvArgs& a) {
  int code = a.shape ? a.shape : conv_default_shape(a.H, a.W, a.Cout);
  if (a.fuse == FUSE_HEAD) code = ((code % 100) / 10) * 10 + 1;
  const int wv = code >= 100 ? 8 : 4, rw = (code % 100) / 10, nj = code % 10;
  return (a.W / 32) * (a.H / (wv * rw)) * (a.Cout / (32 * nj));
}

hipError_t launch_conv(int mode, const ConvArgs& a, hipStream_t st) {
  if (mode == CONV_FWD) return conv_mode<CONV_FWD>(a, st);
  if (a.fuse != FUSE_NONE) return hipErrorInvalidValue;
  if (mode == CONV_BWD_SILU) return conv_shape_dispatch<CONV_BWD_SILU, FUSE_NONE>(
      a, a.shape ? a.shape : conv_default_shape(a.H, a.W, a.Cout), st);
  return conv_shape_dispatch<CONV_BWD_PLAIN, FUSE_NONE>(
      a, a.shape ? a.shape : conv_default_shape(a.H, a.W, a.Cout), st);
}

// Splits of the weight-gradient GEMM: about 1024 workgroups, partials within `max_floats`.
void wgrad_shape(int H, int W, int Cin, int Cout, size_t max_floats, int* nsplit, int* cps) {
  const int mj = Cout % 64 == 0 ? 2 : 1;
  const int blocks = (Cout / (32 * mj)) * (Cin / 32);
  const int nchunks = (H / 4) * (W / 32);
  int ns = (1024 + blocks - 1) / blocks;
  const size_t per = (size_t)9 * Cout * Cin;
  ns = (int)std::min<size_t>((size_t)ns, std::max<size_t>(1, max_floats / per));
  ns = std::max(1, std::min(ns, nchunks));
  *cps = (nchunks + ns - 1) / ns;
  *nsplit = (nchunks + *cps - 1) / *cps;
}

hipError_t launch_wgrad(const bf16_t* x, int x_ld, const bf16_t* x2, int x2_ld, int c_split,
                        const bf16_t* g, int H, int W, int Cin, int Cout, int Cin_dst, float* part,
                        size_t max_floats, float* grad_w, hipStream_t st) {
  WgradArgs a;
  a.x = x;
  a.x_ld = x_ld;
  a.x2 = x2;
  a.x2_ld = x2_ld;
  a.c_split = c_split;
  a.g = g;
  a.part = part;
  a.H = H;
  a.W = W;
  a.Cin = Cin;
  a.Cout = Cout;
  const int mj = Cout % 64 == 0 ? 2 : 1;
  a.nco = Cout / (32 * mj);
  a.nci = Cin / 32;
  a.nchunks = (H / 4) * (W / 32);
  wgrad_shape(H, W, Cin, Cout, max_floats, &a.nsplit, &a.cps);
  const unsigned grid = (unsigned)(a.nco * a.nci * a.nsplit);
  if (mj == 2) hipLaunchKernelGGL((wgrad_kernel<2>), grid, 192, 0, st, a);
  else hipLaunchKernelGGL((wgrad_kernel<1>), grid, 192, 0, st, a);
  const size_t n = (size_t)9 * Cout * Cin_dst;
  hipLaunchKernelGGL(reduce_splits_kernel, nblocks(n, 256), 256, 0, st, part, a.nsplit, Cin, Cin_dst,
                     n, grad_w);
  return hipGetLastError();
}

// Bias gradient: grad_b[c] += sum_p g[p][c]; `part` holds at least nblk * C doubles.
int bias_blocks(size_t npix) { return (int)std::min<size_t>(512, (npix + 255) / 256); }
hipError_t launch_bias_grad(const bf16_t* g, size_t npix, int C, double* part, float* grad_b,
                            hipStream_t st) {
  const int nb = bias_blocks(npix);
  const int per = (int)((npix + nb - 1) / nb);
  hipLaunchKernelGGL(colsum_bf16_kernel, nb, 256, 0, st, g, (int)npix, C, per, part);
  hipLaunchKernelGGL(reduce_blocks_f64_kernel, nblocks(C, 256), 256, 0, st, part, nb, C, grad_b);
  return hipGetLastError();
}

hipError_t launch_pack(const float* f, size_t npix, const PackArgs& pa, bf16_t* x, hipStream_t st) {
  hipLaunchKernelGGL(pack_input_kernel, nblocks(npix, 256), 256, 0, st, f, npix, pa, x);
  return hipGetLastError();
}
hipError_t launch_pool(const bf16_t* in, int in_ld, int H, int W, int C, bf16_t* out, hipStream_t st) {
  hipLaunchKernelGGL(pool_kernel, nblocks((size_t)H / 2 * (W / 2) * (C / 8), 256), 256, 0, st, in,
                     in_ld, H, W, C, out);
  return hipGetLastError();
}
hipError_t launch_up(const bf16_t* in, int h, int w, int C, bf16_t* out, int out_ld, hipStream_t st) {
  hipLaunchKernelGGL(up_kernel, nblocks((size_t)4 * h * w * (C / 8), 256), 256, 0, st, in, h, w, C,
                     out, out_ld);
  return hipGetLastError();
}
hipError_t launch_up_bwd_silu(const bf16_t* gcat, int cat_ld, int h, int w, int C, const bf16_t* z,
                              bf16_t* gz, hipStream_t st) {
  hipLaunchKernelGGL(up_bwd_silu_kernel, nblocks((size_t)h * w * (C / 8), 256), 256, 0, st, gcat,
                     cat_ld, h, w, C, z, gz);
  return hipGetLastError();
}
hipError_t launch_pool_bwd_silu(const bf16_t* gskip, int skip_ld, const bf16_t* gpool, int H, int W,
                                int C, const bf16_t* z, bf16_t* gz, hipStream_t st) {
  hipLaunchKernelGGL(pool_bwd_silu_kernel, nblocks((size_t)H * W * (C / 8), 256), 256, 0, st, gskip,
                     skip_ld, gpool, H, W, C, z, gz);
  return hipGetLastError();
}
hipError_t launch_head_fwd(const bf16_t* d, int C, int nout, size_t npix, const float* Wh,
                           float* out, hipStream_t st) {
  hipLaunchKernelGGL(head_fwd_kernel, nblocks(npix, 256), 256, 0, st, d, C, nout, npix, Wh, out);
  return hipGetLastError();
}
int loss_blocks(size_t npix) { return (int)((npix + 255) / 256); }
hipError_t launch_loss_grad(const float* out, const float* t, const float* extra, int nout,
                            size_t npix, float* gout, double* part, hipStream_t st) {
  hipLaunchKernelGGL(loss_grad_kernel, loss_blocks(npix), 256, 0, st, out, t, extra, nout, npix,
                     gout, part);
  return hipGetLastError();
}
hipError_t launch_field_grad(const bf16_t* gx, size_t npix, const PackArgs& pa, float* g,
                             hipStream_t st) {
  hipLaunchKernelGGL(field_grad_kernel, nblocks(npix, 256), 256, 0, st, gx, npix, pa, g);
  return hipGetLastError();
}
hipError_t launch_head_bwd(const bf16_t* d, int C, int nout, size_t npix, const float* gout,
                           const float* Wh, const bf16_t* z, bf16_t* gz, double* part,
                           float* grad_head, hipStream_t st) {
  const int nb = bias_blocks(npix);
  const int per = (int)((npix + nb - 1) / nb);
  const int n = nout * C + nout;
  hipLaunchKernelGGL(head_wgrad_kernel, nb, 256, 0, st, d, C, nout, npix, per, gout, part);
  hipLaunchKernelGGL(reduce_blocks_f64_kernel, nblocks(n, 256), 256, 0, st, part, nb, n, grad_head);
  hipLaunchKernelGGL(head_dgrad_kernel, nblocks(npix * C, 256), 256, 0, st, gout, npix, C, nout, Wh,
                     z, gz);
  return hipGetLastError();
}
hipError_t launch_refresh(const float* W, int Cout, int Cin, int Cin_pad, bf16_t* wf, bf16_t* wd,
                          hipStream_t st) {
  hipLaunchKernelGGL(refresh_weights_kernel, nblocks((size_t)9 * Cout * Cin_pad, 256), 256, 0, st, W,
                     Cout, Cin, Cin_pad, wf, wd);
  return hipGetLastError();
}
hipError_t launch_adam(float* th, float* m, float* v, const float* g, size_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, float gscale, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, nblocks(n, 256), 256, 0, st, th, m, v, g, n, lr, b1, b2, eps, c1,
                     c2, gscale);
  return hipGetLastError();
}
hipError_t launch_make_target(const float* e, const float* l, size_t npix, const float* s,
                              float* t, hipStream_t st) {
  hipLaunchKernelGGL(make_target_kernel, nblocks(3 * npix, 256), 256, 0, st, e, l, npix, s[0], s[1],
                     s[2], t);
  return hipGetLastError();
}
hipError_t launch_apply(float* f, const float* out, size_t npix, const float* s, double* part,
                        int parts, hipStream_t st) {
  const int nb = (int)((npix + 255) / 256);
  const int np = parts > 0 ? parts : nb;  // partial sums of the phi increment
  if (parts <= 0) hipLaunchKernelGGL(sum_f32_kernel, nb, 256, 0, st, out, npix, part);
  hipLaunchKernelGGL(mean_kernel, 1, 256, 0, st, part, np, npix);
  hipLaunchKernelGGL(apply_kernel, nb, 256, 0, st, f, out, npix, s[0], s[1], s[2],
                     (const double*)(part + np));
  return hipGetLastError();
}

hipError_t launch_absmax(const float* x, size_t n, double* part, double* out, hipStream_t st) {
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(absmax_f32_kernel, nb, 256, 0, st, x, n, part);
  hipLaunchKernelGGL(max_final_kernel, 1, 256, 0, st, part, nb, out);
  return hipGetLastError();
}
hipError_t launch_clamp_conserve(float* phi, size_t n, const double* bound, float factor,
                                 double* part, hipStream_t st) {
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(clamp_excess_kernel, nb, 256, 0, st, phi, n, bound, factor, part);
  hipLaunchKernelGGL(mean_kernel, 1, 256, 0, st, part, nb, n);
  hipLaunchKernelGGL(add_mean_kernel, nb, 256, 0, st, phi, n, (const double*)(part + nb));
  return hipGetLastError();
}

}  // namespace nn
}  // namespace lam
