/* lam_surrogate.h -- C-ABI of the learned surrogate of the lamellar-fluid update (gfx950).
 *
 * A U-Net maps the fields (phi, u_x, u_y, T, a = (T - Tc)/Tc) of a 2D lattice with walls normal
 * to y to the increments of (phi, u_x, u_y) over a fixed number of lattice steps.  The paper has
 * no network: this is an accelerator around its method (Section 2 defines the fields, Section 3
 * the geometry: periodic in x, walls at y = 0 and y = H - 1).  The plain solver (lam.h) stays the
 * reference that re-anchors the state and judges the error.
 *
 * Network: L levels of widths base * 2^l; each encoder level has two 3x3 convolutions with SiLU,
 * levels are joined by 2x2 average pooling; each decoder level upsamples 2x (nearest), prepends
 * the upsampled channels to the encoder output of the level and applies two 3x3 convolutions
 * with SiLU; a 1x1 head gives 3 outputs.  Convolutions are cross-correlations, periodic in x,
 * zero-padded across the walls.  Weights and activations are stored in bfloat16, sums are FP32
 * on the matrix cores; master weights, gradients and Adam moments are FP32.
 *
 * Parameter vector (FP32, lsn_param_count entries): for each 3x3 layer in the order e1a, e1, e2a,
 * e2, ..., eLa, eL, d(L-1)a, d(L-1), ..., d1a, d1 the weights [9][C_out][C_in] (tap = 3 (dy+1) +
 * (dx+1)) then the biases [C_out]; then the head weights [NOUT][base] and biases [NOUT].  C_in of
 * e1a is 5; C_in of d(l)a is width(l+1) + width(l).
 *
 * Fields are planar FP32 in device memory: [4][H][W] = phi, u_x, u_y, T (x fastest), the layout
 * lam_get_fields writes.  Network inputs are (field - shift) * scale per channel: phi, u_x, u_y,
 * T and a (from T); outputs are normalised increments of phi, u_x, u_y: field += out * out_scale.
 * NF = 4 field planes, NOUT = 3 outputs.
 *
 * Ownership: the caller owns every device buffer (one workspace of lsn_workspace_bytes); the
 * library allocates no device memory.  All work is queued on the caller's HIP stream; functions
 * that return host values synchronise it.  Calls on one network are not thread-safe.
 * Errors: return codes as lam.h (LAM_EINVAL bad sizes or arguments, LAM_EHIP a HIP error,
 * LAM_ESIZE workspace too small, LAM_ENONFINITE non-finite loss); lsn_last_error gives text. */
#ifndef LAM_SURROGATE_H
#define LAM_SURROGATE_H
#include <stddef.h>
#include <stdint.h>

#include "lam.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsn_net lsn_net;

typedef struct {
  int32_t height, width;  /* lattice; height % (4 * 2^(levels-1)) == 0, width % (32 * 2^(levels-1)) == 0 */
  int32_t levels;         /* 1 .. 5 */
  int32_t base_width;     /* channels of level 1: 32 or 64 */
  int32_t training;       /* 1: keep activations, gradients and Adam moments */
  float Tc;               /* critical temperature, for a = (T - Tc)/Tc */
  float in_shift[5], in_scale[5];  /* input normalisation of phi, u_x, u_y, T, a */
  float out_scale[3];              /* increments of phi, u_x, u_y per unit output */
} lsn_config;

int lsn_param_count(const lsn_config* cfg, int64_t* count);
int lsn_workspace_bytes(const lsn_config* cfg, size_t* bytes);
int lsn_create(const lsn_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
               lsn_net** out);

/* Parameters in and out (FP32 device vectors of lsn_param_count entries).  Setting them resets
 * the Adam moments and step count. */
int lsn_set_params(lsn_net* net, const float* d_params);
int lsn_get_params(lsn_net* net, float* d_params);

/* Network output for the fields d_fields [NF][H][W]: d_out [NOUT][H][W] FP32 (normalised
 * increments). */
int lsn_forward(lsn_net* net, const float* d_fields, float* d_out);

/* One surrogate step in place on d_fields [NF][H][W]: phi, u_x, u_y += out * out_scale,
 * then phi is shifted by a constant so that its sum over the lattice is unchanged
 * (the exact conservation of sum phi, eq. massdiff, and of the mass).  T is left alone. */
int lsn_advance(lsn_net* net, float* d_fields);

/* Training target from two snapshots [NF][H][W] taken the surrogate's step count apart:
 * d_target [NOUT][H][W] = (later - earlier) / out_scale for phi, u_x, u_y. */
int lsn_make_target(lsn_net* net, const float* d_earlier, const float* d_later, float* d_target);

/* Loss and gradient (training networks only): loss = mean over the NOUT H W outputs of
 * (out - target)^2; its gradient with respect to the parameters is ADDED to the gradient buffer
 * (cleared by lsn_zero_grad, read by lsn_get_grads).  h_loss (nullable) receives the loss and
 * the call synchronises; LAM_ENONFINITE if it is not finite. */
int lsn_zero_grad(lsn_net* net);
int lsn_loss_backward(lsn_net* net, const float* d_fields, const float* d_target, double* h_loss);
/* The same, chained with later uses of the output (training through several surrogate steps):
 * d_out_grad (nullable, FP32 [NOUT][H][W], read only) is added to the loss gradient with respect
 * to the output before back-propagation, and d_field_grad (nullable, FP32 [NF][H][W], written,
 * must not alias an input) receives the gradient with respect to d_fields: of phi, u_x, u_y (and
 * n) through their input channels, of T through both T and a = (T - Tc) / Tc.  It is computed from
 * the bfloat16 gradient of the packed input (relative precision 2^-8).  LAM_EINVAL on a null
 * network, fields or target, an inference network or an aliased d_field_grad. */
int lsn_loss_backward_ex(lsn_net* net, const float* d_fields, const float* d_target,
                         const float* d_out_grad, float* d_field_grad, double* h_loss);
int lsn_get_grads(lsn_net* net, float* d_grads);

/* One Adam step (Kingma & Ba, 2015, with bias correction) on the accumulated gradient scaled by
 * grad_scale (for example 1/batch), then the bfloat16 weight copies are refreshed. */
int lsn_adam(lsn_net* net, float lr, float beta1, float beta2, float eps, float grad_scale);

/* Surrogate-accelerated run of the solver s (2D, walls normal to y, the network's lattice),
 * `cycles` times: read phi, u, T of s into d_fields [NF][H][W] (caller scratch), apply
 * `calls` surrogate steps (lsn_advance), each standing for `steps_per_call` lattice steps during
 * which T advances exactly (lam_advance_temperature), then re-anchor s on the result
 * (lam_set_fields: populations restarted from the equilibrium at n = 1 and the predicted u) and run
 * `anchor_steps` plain steps (lam_step).  The simulated time advances by
 * cycles * (calls * steps_per_call + anchor_steps) steps.  Asynchronous on the network's stream,
 * which must be the stream of s.
 *
 * Order-parameter limiter (on unless lsn_set_limiter turns it off): before each re-anchoring, phi
 * is clamped to +-factor * M, M = max |phi| of s when the call starts, and the clamped-off excess
 * is spread evenly over the lattice so that sum phi is unchanged.  Without it the surrogate's phi
 * drifts past the bulk values of the free energy (eq. free) and the coupled solver can blow up
 * after a re-anchoring. */
int lsn_rollout(lsn_net* net, lam_sim* s, float* d_fields, int32_t cycles, int32_t calls,
                int32_t steps_per_call, int32_t anchor_steps);

/* Limiter factor of lsn_rollout (default 1.05); factor <= 0 turns the limiter off; LAM_EINVAL for
 * a non-finite factor. */
int lsn_set_limiter(lsn_net* net, float factor);

/* Tile-shape autotuner: coordinate descent over the 3x3 layers from the default shapes (at most
 * three sweeps, until one changes nothing): each layer tries every tile shape its sizes allow
 * (and, for the first layer of a coarser level of an inference network, its 2x2 pool fused into
 * the staging or run as a kernel of its own), timed in place inside whole forward passes on
 * d_fields (its own kernels, best of `reps` passes), and keeps the fastest.  The shapes change
 * the speed only: every output is summed in the same order.  Synchronises.  lsn_get_shapes
 * writes the shape codes (10 x rows per wave + 32-channel output blocks, + 100 for workgroups of
 * eight waves instead of four) of the 3x3 layers in parameter order into codes[count].
 * lsn_set_shapes sets them (count = the number of 3x3 layers, 4 levels - 2; code 0 = the layer's
 * default), for example to reuse an earlier tuning; LAM_EINVAL, and no change, if a code is not
 * one the layer's sizes allow. */
int lsn_tune(lsn_net* net, const float* d_fields, int32_t reps);
int lsn_get_shapes(const lsn_net* net, int32_t* codes, int32_t count);
int lsn_set_shapes(lsn_net* net, const int32_t* codes, int32_t count);

/* Kernel timing: with timing enabled, the next forward's kernels are bracketed by HIP events
 * and lsn_forward_time returns its duration in ms (synchronises). */
int lsn_set_timing(lsn_net* net, int32_t enable);
int lsn_forward_time(lsn_net* net, float* ms);

const char* lsn_last_error(const lsn_net* net);
void lsn_destroy(lsn_net* net);

#ifdef __cplusplus
}
#endif
#endif
