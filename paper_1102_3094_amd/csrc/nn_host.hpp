// nn_host.hpp -- argument blocks and launchers of the U-Net surrogate kernels (nn_kernels.hip),
// shared with the host implementation of the surrogate's C-ABI (nn_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lam {
namespace nn {

typedef uint16_t bf16_t;  // bfloat16 bit pattern

enum { CONV_FWD = 0, CONV_BWD_SILU = 1, CONV_BWD_PLAIN = 2 };
// Forward-pass fusions (see conv3x3_kernel): none, input packed from the planar fields, input
// pooled 2x2 from a map of twice the resolution, 1x1 head applied to the output.
enum { FUSE_NONE = 0, FUSE_FIELDS = 1, FUSE_POOL = 2, FUSE_HEAD = 3 };

struct PackArgs {
  float shift[5], scale[5];
  float Tc;
};

struct ConvArgs {
  const bf16_t* in;     // input (offset to its first channel), pixel stride in_ld
  int in_ld;
  const bf16_t* in2;    // optional second input at half resolution, nearest-upsampled: it
  int in2_ld;           // supplies input channels [0, c_split), `in` the channels from c_split
  int c_split;
  const bf16_t* w;      // [9][Cout][Cin]
  const float* bias;    // CONV_FWD: [Cout]
  bf16_t* out;          // output (offset to its first channel), pixel stride out_ld
  int out_ld;
  bf16_t* zout;         // CONV_FWD, optional: pre-activation [pixels][Cout]
  const bf16_t* zprev;  // CONV_BWD_SILU: pre-activation [pixels][Cout]; the result is multiplied by silu'
  int H, W, Cin, Cout;
  int shape;            // tile shape 10 RW + NJ (rows per wave, 32-channel output blocks), + 100:
                        // eight waves; 0: default
  int fuse;             // FUSE_*; forward passes only
  const float* fields;  // FUSE_FIELDS: planar FP32 [4][H][W] and its normalisation
  PackArgs pk;
  const float* head_w;  // FUSE_HEAD: head weights [3][32] then biases [3]; output [3][H][W]
  float* head_out;
  double* head_part;    // FUSE_HEAD, optional: per-workgroup FP64 sums of output 0 at [block]
                        // (the conservation shift of a step)
  int tiles_x, nco;     // set by the launcher
};

// Tile shapes a 3x3 layer of these sizes can use (codes 10 RW + NJ, + 100 for eight waves), and
// the default pick.
int conv_shapes(int H, int Cout, int* codes, int max_codes);
int conv_default_shape(int H, int W, int Cout);

hipError_t launch_conv(int mode, const ConvArgs& a, hipStream_t st);
void wgrad_shape(int H, int W, int Cin, int Cout, size_t max_floats, int* nsplit, int* cps);
hipError_t launch_wgrad(const bf16_t* x, int x_ld, const bf16_t* x2, int x2_ld, int c_split,
                        const bf16_t* g, int H, int W, int Cin, int Cout, int Cin_dst, float* part,
                        size_t max_floats, float* grad_w, hipStream_t st);
int bias_blocks(size_t npix);
hipError_t launch_bias_grad(const bf16_t* g, size_t npix, int C, double* part, float* grad_b,
                            hipStream_t st);
hipError_t launch_pack(const float* f, size_t npix, const PackArgs& pa, bf16_t* x, hipStream_t st);
hipError_t launch_pool(const bf16_t* in, int in_ld, int H, int W, int C, bf16_t* out, hipStream_t st);
hipError_t launch_up(const bf16_t* in, int h, int w, int C, bf16_t* out, int out_ld, hipStream_t st);
hipError_t launch_up_bwd_silu(const bf16_t* gcat, int cat_ld, int h, int w, int C, const bf16_t* z,
                              bf16_t* gz, hipStream_t st);
hipError_t launch_pool_bwd_silu(const bf16_t* gskip, int skip_ld, const bf16_t* gpool, int H, int W,
                                int C, const bf16_t* z, bf16_t* gz, hipStream_t st);
hipError_t launch_head_fwd(const bf16_t* d, int C, int nout, size_t npix, const float* Wh, float* out,
                           hipStream_t st);
int loss_blocks(size_t npix);
// gout = d loss / d out (+ extra, nullable: a gradient of later uses of the output)
hipError_t launch_loss_grad(const float* out, const float* t, const float* extra, int nout,
                            size_t npix, float* gout, double* part, hipStream_t st);
// Gradient with respect to the planar fields [4][npix] from that of the packed input.
hipError_t launch_field_grad(const bf16_t* gx, size_t npix, const PackArgs& pa, float* g,
                             hipStream_t st);
hipError_t launch_head_bwd(const bf16_t* d, int C, int nout, size_t npix, const float* gout,
                           const float* Wh, const bf16_t* z, bf16_t* gz, double* part,
                           float* grad_head, hipStream_t st);
hipError_t launch_refresh(const float* W, int Cout, int Cin, int Cin_pad, bf16_t* wf, bf16_t* wd,
                          hipStream_t st);
hipError_t launch_adam(float* th, float* m, float* v, const float* g, size_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, float gscale, hipStream_t st);
hipError_t launch_make_target(const float* e, const float* l, size_t npix, const float* s,
                              float* t, hipStream_t st);
// Rollout limiter: *out = max |x| (part: ceil(n / 256) doubles); phi clamped to +-factor * *bound
// with the removed excess spread evenly so that sum phi is unchanged (part: ceil(n/256) + 1).
hipError_t launch_absmax(const float* x, size_t n, double* part, double* out, hipStream_t st);
hipError_t launch_clamp_conserve(float* phi, size_t n, const double* bound, float factor,
                                 double* part, hipStream_t st);
// part: at least max(parts, ceil(npix / 256)) + 1 doubles.  parts > 0: the per-block sums of the
// phi increment are already in part (written by the fused head of the forward pass).
hipError_t launch_apply(float* f, const float* out, size_t npix, const float* s,
                        double* part, int parts, hipStream_t st);
// Workgroups of a forward convolution launch (the grid launch_conv uses for these arguments).
int conv_blocks(const ConvArgs& a);

}  // namespace nn
}  // namespace lam
