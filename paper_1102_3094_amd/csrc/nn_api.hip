// nn_api.hip -- host implementation of include/lam_surrogate.h: configuration checks, workspace
// carving, the launch sequences of the U-Net forward pass, its backward pass and the Adam step.
// All device memory belongs to the caller.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/lam.h"
#include "../../include/lam_surrogate.h"
#include "lam_dev.hpp"
#include "nn_host.hpp"

namespace lam {
int sim_dims(const lam_sim* s, int* dim, int* nx, int* ny, int* walls);
bool sim_temperature_frozen(const lam_sim* s);
}

using namespace lam::nn;

namespace {
constexpr int MAXL = 5;
constexpr int IN_PAD = 32;                    // packed input channels (5 or 6 used)
constexpr size_t WGRAD_MAX_FLOATS = 16u << 20;  // weight-gradient partials: 64 MB

struct Layer {
  int cin, cout, cin_pad;
  size_t w_off, b_off;  // offsets in the parameter vector
  bf16_t* wf;           // [9][cout][cin_pad]
  bf16_t* wd;           // [9][cin_pad][cout], taps mirrored (training: input gradient)
  int shape;            // tile shape of the forward convolution (0: default)
  bool pool_apart;      // first layer of a coarser level: 2x2 pool as its own kernel instead of
                        // fused into the staging (inference; chosen by the tuner, same bits)
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace pieces in carve order; `base` null only sizes them.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t o = off;
    off = align256(off + count * sizeof(T));
    return base ? (T*)(base + o) : nullptr;
  }
};
}  // namespace

static thread_local std::string g_nn_error;

struct lsn_net {
  lsn_config c;
  int L, H, W, wid[MAXL];
  int nf, nout;    // field planes (4) and output channels (3)
  size_t P[MAXL];  // pixels per level
  hipStream_t st;
  size_t nparam, head_off;
  std::vector<Layer> layers;
  float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  bf16_t* x0 = nullptr;
  bf16_t *ta[MAXL] = {}, *za[MAXL] = {}, *ze[MAXL] = {}, *enc_out[MAXL] = {}, *pool[MAXL] = {};
  int enc_ld[MAXL] = {};
  bf16_t *da[MAXL] = {}, *dd[MAXL] = {}, *zda[MAXL] = {}, *zdd[MAXL] = {};
  bf16_t *gA = nullptr, *gB = nullptr, *gcat[MAXL] = {}, *gp[MAXL] = {};
  float *out = nullptr, *gout = nullptr, *part = nullptr;
  double* dpart = nullptr;
  int head_parts = 0;     // per-workgroup sums left in dpart by the last fused forward pass
  double* lim = nullptr;  // rollout limiter: [0] max |phi| at the start of the call
  float lim_factor = 1.05f;
  int64_t adam_t = 0;
  const float* fields = nullptr;  // fields of the forward pass in flight (fused input packing)
  // HIP graph of one surrogate step (forward + apply) on a given fields buffer
  hipGraphExec_t step_graph = nullptr;
  const float* step_graph_fields = nullptr;
  uint64_t shapes_version = 0, step_graph_version = 0;
  bool timing = false, timed = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // tuner: events around the work of one layer (its pool kernel included) inside a full pass
  int time_layer = -1;
  hipEvent_t tl0 = nullptr, tl1 = nullptr;
  std::string err;
};

namespace {

int fail(lsn_net* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  else g_nn_error = msg;
  return code;
}
int hip_fail(lsn_net* n, hipError_t e, const char* what) {
  return fail(n, LAM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_config(const lsn_config* c) {
  if (!c) return fail(nullptr, LAM_EINVAL, "null config");
  if (c->levels < 1 || c->levels > MAXL) return fail(nullptr, LAM_EINVAL, "levels must be 1..5");
  if (c->base_width != 32 && c->base_width != 64)
    return fail(nullptr, LAM_EINVAL, "base_width must be 32 or 64");
  const int s = 1 << (c->levels - 1);
  if (c->height <= 0 || c->width <= 0 || c->height % (4 * s) || c->width % (32 * s))
    return fail(nullptr, LAM_EINVAL,
                "height must be a multiple of 4 * 2^(levels-1) and width of 32 * 2^(levels-1)");
  if (!(c->Tc != 0.f) || !isfinite(c->Tc)) return fail(nullptr, LAM_EINVAL, "Tc must be finite and non-zero");
  for (int i = 0; i < 5; ++i)
    if (!isfinite(c->in_shift[i]) || !isfinite(c->in_scale[i]))
      return fail(nullptr, LAM_EINVAL, "input normalisation must be finite");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(c->out_scale[i]) || c->out_scale[i] == 0.f)
      return fail(nullptr, LAM_EINVAL, "out_scale must be finite and non-zero");
  return LAM_OK;
}

// Layer table in parameter order (see the header) and the parameter count.
void build_layers(const lsn_config& c, std::vector<Layer>& ly, size_t* nparam, size_t* head_off) {
  const int L = c.levels;
  int w[MAXL];
  for (int l = 0; l < L; ++l) w[l] = c.base_width << l;
  ly.clear();
  auto add = [&](int cin, int cout, int cin_pad) { ly.push_back(Layer{cin, cout, cin_pad, 0, 0, nullptr, nullptr, 0, false}); };
  for (int l = 0; l < L; ++l) {
    if (l == 0) add(5, w[0], IN_PAD);
    else add(w[l - 1], w[l], w[l - 1]);
    add(w[l], w[l], w[l]);
  }
  for (int l = L - 2; l >= 0; --l) {
    add(w[l + 1] + w[l], w[l], w[l + 1] + w[l]);
    add(w[l], w[l], w[l]);
  }
  size_t o = 0;
  for (auto& q : ly) {
    q.w_off = o;
    o += (size_t)9 * q.cout * q.cin;
    q.b_off = o;
    o += q.cout;
  }
  *head_off = o;
  *nparam = o + 3 * (size_t)w[0] + 3;
}

int enc_a(int l) { return 2 * l; }
int enc_b(int l) { return 2 * l + 1; }
int dec_a(int L, int l) { return 2 * L + 2 * (L - 2 - l); }
int dec_b(int L, int l) { return 2 * L + 2 * (L - 2 - l) + 1; }

// Carve (or size) the workspace.
size_t carve(lsn_net* n, char* base) {
  Carver cv{base};
  const lsn_config& c = n->c;
  const bool tr = c.training != 0;
  const int L = n->L;
  n->master = cv.take<float>(n->nparam);
  if (tr) {
    n->grad = cv.take<float>(n->nparam);
    n->m = cv.take<float>(n->nparam);
    n->v = cv.take<float>(n->nparam);
  }
  for (size_t i = 0; i < n->layers.size(); ++i) {
    Layer& q = n->layers[i];
    q.wf = cv.take<bf16_t>((size_t)9 * q.cout * q.cin_pad);
    q.wd = tr ? cv.take<bf16_t>((size_t)9 * q.cout * q.cin_pad) : nullptr;
  }
  n->x0 = cv.take<bf16_t>(n->P[0] * IN_PAD);
  for (int l = 0; l < L; ++l) {
    const size_t P = n->P[l];
    const int w = n->wid[l];
    n->ta[l] = cv.take<bf16_t>(P * w);
    if (tr) {
      n->za[l] = cv.take<bf16_t>(P * w);
      n->ze[l] = cv.take<bf16_t>(P * w);
    }
    n->enc_out[l] = cv.take<bf16_t>(P * w);
    n->enc_ld[l] = w;
    if (l < L - 1) {
      const int cld = n->wid[l + 1] + w;
      n->pool[l] = cv.take<bf16_t>(n->P[l + 1] * w);
      n->da[l] = cv.take<bf16_t>(P * w);
      n->dd[l] = cv.take<bf16_t>(P * w);
      if (tr) {
        n->zda[l] = cv.take<bf16_t>(P * w);
        n->zdd[l] = cv.take<bf16_t>(P * w);
        n->gcat[l] = cv.take<bf16_t>(P * cld);
        n->gp[l] = cv.take<bf16_t>(n->P[l + 1] * w);
      }
    }
  }
  n->out = cv.take<float>(n->nout * n->P[0]);
  // FP64 partials: the loss, then (from loss_blocks + 1 on) per-block partials of the bias and
  // head gradients; and, never in flight with those, the two conservation shifts of a step:
  // 2 (blocks + 1) with up to npix / 128 blocks (the fused head's workgroups).
  size_t nd = 2 * (n->P[0] / 128 + 1);
  if (tr) {
    n->gA = cv.take<bf16_t>(n->P[0] * n->wid[0]);
    n->gB = cv.take<bf16_t>(n->P[0] * n->wid[0]);
    n->gout = cv.take<float>(n->nout * n->P[0]);
    size_t need = 0;
    // weight-gradient partials: the largest split buffer over the layers
    for (int i = 0; i < (int)n->layers.size(); ++i) {
      const Layer& q = n->layers[i];
      int lev = 0;
      for (int l = 0; l < L; ++l)
        if (i == enc_a(l) || i == enc_b(l) || (l < L - 1 && (i == dec_a(L, l) || i == dec_b(L, l)))) lev = l;
      int ns, cps;
      wgrad_shape(n->H >> lev, n->W >> lev, q.cin_pad, q.cout, WGRAD_MAX_FLOATS, &ns, &cps);
      need = std::max(need, (size_t)ns * 9 * q.cout * q.cin_pad);
    }
    n->part = cv.take<float>(need);
    nd += (size_t)bias_blocks(n->P[0]) * std::max(n->nout * n->wid[0] + n->nout, 256);
  }
  n->dpart = cv.take<double>(nd);
  n->lim = cv.take<double>(4);
  return cv.off;
}

int level_of(const lsn_net* n, int i) {
  for (int l = 0; l < n->L; ++l)
    if (i == enc_a(l) || i == enc_b(l) || (l < n->L - 1 && (i == dec_a(n->L, l) || i == dec_b(n->L, l))))
      return l;
  return 0;
}

ConvArgs conv_args(const lsn_net* n, int lev, const bf16_t* in, int in_ld, int Cin, const bf16_t* w,
                   int Cout) {
  ConvArgs a{};
  a.in = in;
  a.in_ld = in_ld;
  a.w = w;
  a.H = n->H >> lev;
  a.W = n->W >> lev;
  a.Cin = Cin;
  a.Cout = Cout;
  return a;
}

// Buffers of forward layer i: input (and, for a decoder layer, the coarse map it upsamples),
// output and pre-activation store.
struct LayerIO {
  const bf16_t *in, *in2;
  int in_ld, in2_ld, c_split;
  bf16_t *out, *z;
  int out_ld;
};

LayerIO layer_io(const lsn_net* n, int i, bool keep) {
  const int L = n->L;
  LayerIO io{};
  for (int l = 0; l < L; ++l) {
    if (i == enc_a(l)) {
      io.in = l == 0 ? n->x0 : n->pool[l - 1];
      io.in_ld = l == 0 ? IN_PAD : n->wid[l - 1];
      io.out = n->ta[l];
      io.z = keep ? n->za[l] : nullptr;
    } else if (i == enc_b(l)) {
      io.in = n->ta[l];
      io.in_ld = n->wid[l];
      io.out = n->enc_out[l];
      io.z = keep ? n->ze[l] : nullptr;
    } else if (l < L - 1 && i == dec_a(L, l)) {
      io.in = n->enc_out[l];
      io.in_ld = n->wid[l];
      io.in2 = l == L - 2 ? n->enc_out[L - 1] : n->dd[l + 1];
      io.in2_ld = n->wid[l + 1];
      io.c_split = n->wid[l + 1];
      io.out = n->da[l];
      io.z = keep ? n->zda[l] : nullptr;
    } else if (l < L - 1 && i == dec_b(L, l)) {
      io.in = n->da[l];
      io.in_ld = n->wid[l];
      io.out = n->dd[l];
      io.z = keep ? n->zdd[l] : nullptr;
    } else {
      continue;
    }
    io.out_ld = n->wid[l];
  }
  return io;
}

PackArgs pack_args(const lsn_net* n) {
  PackArgs pa;
  for (int i = 0; i < 5; ++i) {
    pa.shift[i] = n->c.in_shift[i];
    pa.scale[i] = n->c.in_scale[i];
  }
  pa.Tc = n->c.Tc;
  return pa;
}

int top_layer(const lsn_net* n) { return n->L > 1 ? dec_b(n->L, 0) : enc_b(0); }

// Without kept activations the forward pass fuses the input packing into e1a, each 2x2 pool into
// the next level's first convolution and (32-channel networks) the head into the last layer.
bool fuses_head(const lsn_net* n, bool keep) { return !keep && n->wid[0] == 32; }

// Forward pass of layer i (3x3, SiLU), with its tile shape `shape` (0: the layer's own).
hipError_t fwd_layer(lsn_net* n, int i, bool keep, int shape = 0) {
  const Layer& q = n->layers[i];
  const LayerIO io = layer_io(n, i, keep);
  ConvArgs a = conv_args(n, level_of(n, i), io.in, io.in_ld, q.cin_pad, q.wf, q.cout);
  a.in2 = io.in2;
  a.in2_ld = io.in2_ld;
  a.c_split = io.c_split;
  a.bias = n->master + q.b_off;
  a.out = io.out;
  a.out_ld = io.out_ld;
  a.zout = io.z;
  a.shape = shape ? shape : q.shape;
  a.fuse = FUSE_NONE;
  if (!keep) {
    for (int l = 0; l < n->L; ++l)
      if (i == enc_a(l)) {
        if (l == 0) {
          a.fuse = FUSE_FIELDS;
          a.fields = n->fields;
          a.pk = pack_args(n);
        } else if (!q.pool_apart) {
          a.fuse = FUSE_POOL;
          a.in = n->enc_out[l - 1];  // the pool is applied while staging
          a.in_ld = n->wid[l - 1];
        }
      }
    if (i == top_layer(n) && fuses_head(n, keep)) {
      a.fuse = FUSE_HEAD;
      a.head_w = n->master + n->head_off;
      a.head_out = n->out;
      a.head_part = n->dpart;
      n->head_parts = conv_blocks(a);
    }
  }
  return launch_conv(CONV_FWD, a, n->st);
}

hipError_t forward(lsn_net* n, const float* fields, bool keep) {
  hipError_t e;
  const int L = n->L;
  n->fields = fields;
  n->head_parts = 0;
  if (keep && (e = launch_pack(fields, n->P[0], pack_args(n), n->x0, n->st))) return e;
  // layer i, preceded by the 2x2 pool of its input when that runs as a kernel of its own
  auto layer = [&](int i, int pool_level) -> hipError_t {
    hipError_t r;
    if (i == n->time_layer && (r = hipEventRecord(n->tl0, n->st))) return r;
    if (pool_level >= 0 && (keep || n->layers[i].pool_apart) &&
        (r = launch_pool(n->enc_out[pool_level], n->wid[pool_level], n->H >> pool_level,
                         n->W >> pool_level, n->wid[pool_level], n->pool[pool_level], n->st)))
      return r;
    if ((r = fwd_layer(n, i, keep))) return r;
    if (i == n->time_layer && (r = hipEventRecord(n->tl1, n->st))) return r;
    return hipSuccess;
  };
  for (int l = 0; l < L; ++l)
    if ((e = layer(enc_a(l), l - 1)) || (e = layer(enc_b(l), -1))) return e;
  for (int l = L - 2; l >= 0; --l)
    if ((e = layer(dec_a(L, l), -1)) || (e = layer(dec_b(L, l), -1))) return e;
  if (fuses_head(n, keep)) return hipSuccess;
  const bf16_t* top = L > 1 ? n->dd[0] : n->enc_out[0];
  return launch_head_fwd(top, n->wid[0], n->nout, n->P[0], n->master + n->head_off, n->out, n->st);
}

// Backward of layer i given gz = gradient w.r.t. its pre-activation: weight and bias gradients,
// then (if gin) the gradient w.r.t. its input, multiplied by silu'(zin) when zin is given.
hipError_t bwd_layer(lsn_net* n, int i, const bf16_t* gz, bf16_t* gin, int gin_ld, const bf16_t* zin) {
  hipError_t e;
  const Layer& q = n->layers[i];
  const int lev = level_of(n, i);
  const int H = n->H >> lev, W = n->W >> lev;
  const LayerIO io = layer_io(n, i, true);
  if ((e = launch_wgrad(io.in, io.in_ld, io.in2, io.in2_ld, io.c_split, gz, H, W, q.cin_pad, q.cout,
                        q.cin, n->part, WGRAD_MAX_FLOATS, n->grad + q.w_off, n->st)))
    return e;
  if ((e = launch_bias_grad(gz, n->P[lev], q.cout, n->dpart + loss_blocks(n->P[0]) + 1,
                            n->grad + q.b_off, n->st)))
    return e;
  if (!gin) return hipSuccess;
  ConvArgs a = conv_args(n, lev, gz, q.cout, q.cout, q.wd, q.cin_pad);
  a.out = gin;
  a.out_ld = gin_ld;
  a.zprev = zin;
  return launch_conv(zin ? CONV_BWD_SILU : CONV_BWD_PLAIN, a, n->st);
}

// Back-propagation of the loss (plus `extra`, nullable: a gradient with respect to the output
// from its later uses) after a forward pass that kept its activations; with field_grad the
// gradient with respect to the input fields as well.
hipError_t backward(lsn_net* n, const float* target, const float* extra, float* field_grad) {
  hipError_t e;
  const int L = n->L;
  const size_t P0 = n->P[0];
  if ((e = launch_loss_grad(n->out, target, extra, n->nout, P0, n->gout, n->dpart, n->st))) return e;
  const bf16_t* top = L > 1 ? n->dd[0] : n->enc_out[0];
  const bf16_t* ztop = L > 1 ? n->zdd[0] : n->ze[0];
  // the loss partials stay in dpart[0 .. loss_blocks): head partials go after them
  double* hpart = n->dpart + loss_blocks(P0) + 1;
  if ((e = launch_head_bwd(top, n->wid[0], n->nout, P0, n->gout, n->master + n->head_off, ztop, n->gA, hpart,
                           n->grad + n->head_off, n->st)))
    return e;
  // gA: gradient w.r.t. the pre-activation of the top layer.
  for (int l = 0; l < L - 1; ++l) {
    const int w = n->wid[l];
    const int cld = n->wid[l + 1] + w;
    if ((e = bwd_layer(n, dec_b(L, l), n->gA, n->gB, w, n->zda[l]))) return e;
    if ((e = bwd_layer(n, dec_a(L, l), n->gB, n->gcat[l], cld, nullptr))) return e;
    const bf16_t* zc = l + 1 < L - 1 ? n->zdd[l + 1] : n->ze[L - 1];
    if ((e = launch_up_bwd_silu(n->gcat[l], cld, n->H >> (l + 1), n->W >> (l + 1), n->wid[l + 1], zc,
                                n->gA, n->st)))
      return e;
  }
  for (int l = L - 1; l >= 0; --l) {
    const int w = n->wid[l];
    if (l < L - 1 &&
        (e = launch_pool_bwd_silu(n->gcat[l] + n->wid[l + 1], n->wid[l + 1] + w, n->gp[l], n->H >> l,
                                  n->W >> l, w, n->ze[l], n->gA, n->st)))
      return e;
    if ((e = bwd_layer(n, enc_b(l), n->gA, n->gB, w, n->za[l]))) return e;
    // level 0: gA (consumed by the layer above) takes the gradient of the packed input
    bf16_t* gin = l > 0 ? n->gp[l - 1] : field_grad ? n->gA : nullptr;
    if ((e = bwd_layer(n, enc_a(l), n->gB, gin, l > 0 ? n->wid[l - 1] : IN_PAD, nullptr))) return e;
  }
  if (field_grad && (e = launch_field_grad(n->gA, P0, pack_args(n), field_grad, n->st))) return e;
  return hipGetLastError();
}

hipError_t refresh(lsn_net* n) {
  hipError_t e;
  for (auto& q : n->layers)
    if ((e = launch_refresh(n->master + q.w_off, q.cout, q.cin, q.cin_pad, q.wf, q.wd, n->st))) return e;
  return hipSuccess;
}

}  // namespace

extern "C" {

int lsn_param_count(const lsn_config* cfg, int64_t* count) {
  int r = check_config(cfg);
  if (r) return r;
  if (!count) return fail(nullptr, LAM_EINVAL, "null output");
  std::vector<Layer> ly;
  size_t np, ho;
  build_layers(*cfg, ly, &np, &ho);
  *count = (int64_t)np;
  return LAM_OK;
}

static void init_dims(lsn_net* n, const lsn_config* cfg) {
  n->c = *cfg;
  n->L = cfg->levels;
  n->H = cfg->height;
  n->W = cfg->width;
  n->nf = 4;
  n->nout = 3;
  for (int l = 0; l < n->L; ++l) {
    n->wid[l] = cfg->base_width << l;
    n->P[l] = (size_t)(n->H >> l) * (n->W >> l);
  }
  build_layers(*cfg, n->layers, &n->nparam, &n->head_off);
}

int lsn_workspace_bytes(const lsn_config* cfg, size_t* bytes) {
  int r = check_config(cfg);
  if (r) return r;
  if (!bytes) return fail(nullptr, LAM_EINVAL, "null output");
  lsn_net n;
  init_dims(&n, cfg);
  *bytes = carve(&n, nullptr);
  return LAM_OK;
}

int lsn_create(const lsn_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
               lsn_net** out) {
  int r = check_config(cfg);
  if (r) return r;
  if (!out) return fail(nullptr, LAM_EINVAL, "null output");
  if (((uintptr_t)d_workspace) & 255) return fail(nullptr, LAM_EINVAL, "workspace not 256-byte aligned");
  lsn_net* n = new lsn_net();
  init_dims(n, cfg);
  const size_t need = carve(n, nullptr);
  if (!d_workspace || bytes < need) {
    delete n;
    return fail(nullptr, LAM_ESIZE, "workspace too small");
  }
  carve(n, (char*)d_workspace);
  n->st = (hipStream_t)hip_stream;
  hipError_t e;
  if ((e = hipMemsetAsync(d_workspace, 0, need, n->st))) {
    delete n;
    return fail(nullptr, LAM_EHIP, std::string("clear: ") + hipGetErrorString(e));
  }
  *out = n;
  return LAM_OK;
}

int lsn_set_params(lsn_net* n, const float* d_params) {
  if (!n || !d_params) return fail(n, LAM_EINVAL, "null argument");
  hipError_t e;
  if ((e = hipMemcpyAsync(n->master, d_params, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->st)))
    return hip_fail(n, e, "set params");
  if (n->c.training) {
    if ((e = hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->st)) ||
        (e = hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->st)))
      return hip_fail(n, e, "reset moments");
    n->adam_t = 0;
  }
  if ((e = refresh(n))) return hip_fail(n, e, "weights");
  return LAM_OK;
}

int lsn_get_params(lsn_net* n, float* d_params) {
  if (!n || !d_params) return fail(n, LAM_EINVAL, "null argument");
  hipError_t e = hipMemcpyAsync(d_params, n->master, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->st);
  return e ? hip_fail(n, e, "get params") : LAM_OK;
}

int lsn_forward(lsn_net* n, const float* d_fields, float* d_out) {
  if (!n || !d_fields || !d_out) return fail(n, LAM_EINVAL, "null argument");
  hipError_t e;
  if (n->timing && (e = hipEventRecord(n->ev0, n->st))) return hip_fail(n, e, "event");
  if ((e = forward(n, d_fields, n->c.training != 0))) return hip_fail(n, e, "forward");
  if (n->timing) {
    if ((e = hipEventRecord(n->ev1, n->st))) return hip_fail(n, e, "event");
    n->timed = true;
  }
  if (d_out != n->out &&
      (e = hipMemcpyAsync(d_out, n->out, n->nout * n->P[0] * sizeof(float), hipMemcpyDeviceToDevice,
                          n->st)))
    return hip_fail(n, e, "output");
  return LAM_OK;
}

int lsn_advance(lsn_net* n, float* d_fields) {
  if (!n || !d_fields) return fail(n, LAM_EINVAL, "null argument");
  hipError_t e;
  if (n->timing && (e = hipEventRecord(n->ev0, n->st))) return hip_fail(n, e, "event");
  if ((e = forward(n, d_fields, n->c.training != 0))) return hip_fail(n, e, "forward");
  if ((e = launch_apply(d_fields, n->out, n->P[0], n->c.out_scale, n->dpart, n->head_parts, n->st)))
    return hip_fail(n, e, "apply");
  if (n->timing) {
    if ((e = hipEventRecord(n->ev1, n->st))) return hip_fail(n, e, "event");
    n->timed = true;
  }
  return LAM_OK;
}

int lsn_make_target(lsn_net* n, const float* d_earlier, const float* d_later, float* d_target) {
  if (!n || !d_earlier || !d_later || !d_target) return fail(n, LAM_EINVAL, "null argument");
  hipError_t e = launch_make_target(d_earlier, d_later, n->P[0], n->c.out_scale, d_target,
                                    n->st);
  return e ? hip_fail(n, e, "target") : LAM_OK;
}

int lsn_zero_grad(lsn_net* n) {
  if (!n) return fail(n, LAM_EINVAL, "null argument");
  if (!n->c.training) return fail(n, LAM_EINVAL, "not a training network");
  hipError_t e = hipMemsetAsync(n->grad, 0, n->nparam * sizeof(float), n->st);
  return e ? hip_fail(n, e, "zero grad") : LAM_OK;
}

int lsn_loss_backward(lsn_net* n, const float* d_fields, const float* d_target, double* h_loss) {
  return lsn_loss_backward_ex(n, d_fields, d_target, nullptr, nullptr, h_loss);
}

int lsn_loss_backward_ex(lsn_net* n, const float* d_fields, const float* d_target,
                         const float* d_out_grad, float* d_field_grad, double* h_loss) {
  if (!n || !d_fields || !d_target) return fail(n, LAM_EINVAL, "null argument");
  if (!n->c.training) return fail(n, LAM_EINVAL, "not a training network");
  if (d_field_grad && (d_field_grad == d_fields || d_field_grad == d_target || d_field_grad == d_out_grad))
    return fail(n, LAM_EINVAL, "d_field_grad must not alias an input");
  hipError_t e;
  if ((e = forward(n, d_fields, true))) return hip_fail(n, e, "forward");
  if ((e = backward(n, d_target, d_out_grad, d_field_grad))) return hip_fail(n, e, "backward");
  if (h_loss) {
    const int nb = loss_blocks(n->P[0]);
    std::vector<double> part(nb);
    if ((e = hipMemcpyAsync(part.data(), n->dpart, nb * sizeof(double), hipMemcpyDeviceToHost, n->st)) ||
        (e = hipStreamSynchronize(n->st)))
      return hip_fail(n, e, "loss");
    double s = 0.0;
    for (double p : part) s += p;
    *h_loss = s / ((double)n->nout * (double)n->P[0]);
    if (!isfinite(*h_loss)) return fail(n, LAM_ENONFINITE, "loss is not finite");
  }
  return LAM_OK;
}

int lsn_get_grads(lsn_net* n, float* d_grads) {
  if (!n || !d_grads) return fail(n, LAM_EINVAL, "null argument");
  if (!n->c.training) return fail(n, LAM_EINVAL, "not a training network");
  hipError_t e = hipMemcpyAsync(d_grads, n->grad, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->st);
  return e ? hip_fail(n, e, "get grads") : LAM_OK;
}

int lsn_adam(lsn_net* n, float lr, float beta1, float beta2, float eps, float grad_scale) {
  if (!n) return fail(n, LAM_EINVAL, "null argument");
  if (!n->c.training) return fail(n, LAM_EINVAL, "not a training network");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(n, LAM_EINVAL, "bad Adam hyper-parameters");
  n->adam_t += 1;
  const float c1 = (float)(1.0 - pow((double)beta1, (double)n->adam_t));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)n->adam_t));
  hipError_t e;
  if ((e = launch_adam(n->master, n->m, n->v, n->grad, n->nparam, lr, beta1, beta2, eps, c1, c2,
                       grad_scale, n->st)))
    return hip_fail(n, e, "adam");
  if ((e = refresh(n))) return hip_fail(n, e, "weights");
  return LAM_OK;
}

namespace {
// One surrogate step on d_fields, replayed from a HIP graph when the stream can be captured (the
// graph is rebuilt when the buffer or the tile shapes change); otherwise launched directly.  Both
// run the same kernels on the same data.
int advance_step(lsn_net* n, float* d_fields) {
  if (!n->timing && !n->c.training) {
    if (n->step_graph && (n->step_graph_fields != d_fields || n->step_graph_version != n->shapes_version)) {
      (void)hipGraphExecDestroy(n->step_graph);
      n->step_graph = nullptr;
    }
    if (!n->step_graph) {
      hipGraph_t g;
      hipError_t r = hipStreamBeginCapture(n->st, hipStreamCaptureModeThreadLocal);
      if (r == hipSuccess) {
        hipError_t r1 = forward(n, d_fields, false);
        if (r1 == hipSuccess) r1 = launch_apply(d_fields, n->out, n->P[0], n->c.out_scale, n->dpart, n->head_parts, n->st);
        hipError_t r2 = hipStreamEndCapture(n->st, &g);
        if (r1 == hipSuccess && r2 == hipSuccess) {
          hipGraphExec_t ex;
          if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
            n->step_graph = ex;
            n->step_graph_fields = d_fields;
            n->step_graph_version = n->shapes_version;
          }
        }
        if (r2 == hipSuccess) (void)hipGraphDestroy(g);
        if (r1 != hipSuccess) return hip_fail(n, r1, "capture");
      }
      (void)hipGetLastError();  // a stream that cannot be captured leaves the direct path
    }
    if (n->step_graph) {
      hipError_t e = hipGraphLaunch(n->step_graph, n->st);
      return e ? hip_fail(n, e, "graph launch") : LAM_OK;
    }
  }
  return lsn_advance(n, d_fields);
}
}  // namespace

int lsn_rollout(lsn_net* n, lam_sim* s, float* d_fields, int32_t cycles, int32_t calls,
                int32_t steps_per_call, int32_t anchor_steps) {
  if (!n || !s || !d_fields) return fail(n, LAM_EINVAL, "null argument");
  if (cycles < 0 || calls < 0 || steps_per_call < 1 || anchor_steps < 0)
    return fail(n, LAM_EINVAL, "bad rollout counts");
  int dim, nx, ny, walls;
  if (lam::sim_dims(s, &dim, &nx, &ny, &walls) != LAM_OK || dim != 2 || nx != n->W || ny != n->H)
    return fail(n, LAM_EINVAL, "the simulation is not an initialised 2D run on the network's lattice");
  const size_t N = n->P[0];
  const bool frozen = lam::sim_temperature_frozen(s);
  const bool limit = n->lim_factor > 0.f;
  int r;
  hipError_t e;
  for (int c = 0; c < cycles; ++c) {
    if ((r = lam_get_fields(s, d_fields, d_fields + N, nullptr, d_fields + 3 * N)))
      return fail(n, r, std::string("solver: ") + lam_last_error(s));
    if (c == 0 && limit && (e = launch_absmax(d_fields, N, n->dpart, n->lim, n->st)))
      return hip_fail(n, e, "limiter");
    for (int k = 0; k < calls; ++k) {
      if ((r = advance_step(n, d_fields))) return r;
      if ((r = lam_advance_temperature(s, steps_per_call)))
        return fail(n, r, std::string("solver: ") + lam_last_error(s));
      if (!frozen && (r = lam_get_fields(s, nullptr, nullptr, nullptr, d_fields + 3 * N)))
        return fail(n, r, std::string("solver: ") + lam_last_error(s));
    }
    if (limit && (e = launch_clamp_conserve(d_fields, N, n->lim, n->lim_factor, n->dpart, n->st)))
      return hip_fail(n, e, "limiter");
    if ((r = lam_set_fields(s, d_fields, d_fields + N, nullptr)) || (r = lam_step(s, anchor_steps)))
      return fail(n, r, std::string("solver: ") + lam_last_error(s));
  }
  return LAM_OK;
}

int lsn_set_limiter(lsn_net* n, float factor) {
  if (!n) return fail(n, LAM_EINVAL, "null argument");
  if (!isfinite(factor)) return fail(n, LAM_EINVAL, "limiter factor must be finite");
  n->lim_factor = factor > 0.f ? factor : 0.f;
  return LAM_OK;
}

int lsn_tune(lsn_net* n, const float* d_fields, int32_t reps) {
  if (!n || !d_fields || reps < 1) return fail(n, LAM_EINVAL, "bad arguments");
  hipError_t e;
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a))) return hip_fail(n, e, "events");
  if ((e = hipEventCreate(&b))) {
    (void)hipEventDestroy(a);
    return hip_fail(n, e, "events");
  }
  int rc = LAM_OK;
  const bool keep = n->c.training != 0;
  // time of layer i's work inside a whole forward pass (best of reps after one warm-up): the
  // layer runs on the input the layer before has just written, as in a real pass
  n->tl0 = a;
  n->tl1 = b;
  auto layer_ms = [&](int i, float* out) -> int {
    float t = 1e30f;
    n->time_layer = i;
    for (int r = 0; r <= reps; ++r) {
      float ms = 0.f;
      if ((e = forward(n, d_fields, keep)) || (e = hipEventSynchronize(b)) ||
          (e = hipEventElapsedTime(&ms, a, b))) {
        n->time_layer = -1;
        return hip_fail(n, e, "tuning");
      }
      if (r) t = std::min(t, ms);
    }
    n->time_layer = -1;
    *out = t;
    return LAM_OK;
  };
  // coordinate descent from the default shapes (pools fused), until a sweep changes nothing (at
  // most three); the first layer of each coarser level also tries its pool as a kernel apart
  for (auto& q : n->layers) {
    q.shape = 0;
    q.pool_apart = false;
  }
  for (int sweep = 0; rc == LAM_OK && sweep < 3; ++sweep) {
    bool changed = false;
    for (int i = 0; rc == LAM_OK && i < (int)n->layers.size(); ++i) {
      const int lev = level_of(n, i);
      int codes[16];
      const int nc = conv_shapes(n->H >> lev, n->layers[i].cout, codes, 16);
      const int before = n->layers[i].shape;
      const bool before_apart = n->layers[i].pool_apart;
      bool pooled = false;
      for (int l = 1; l < n->L; ++l) pooled |= i == enc_a(l);
      float best = 1e30f;
      int pick = 0;
      bool pick_apart = false;
      for (int apart = 0; rc == LAM_OK && apart <= (pooled && !keep ? 1 : 0); ++apart)
        for (int k = 0; rc == LAM_OK && k < nc; ++k) {
          n->layers[i].shape = codes[k];
          n->layers[i].pool_apart = apart != 0;
          float t;
          if ((rc = layer_ms(i, &t)) != LAM_OK) break;
          if (t < best) {
            best = t;
            pick = codes[k];
            pick_apart = apart != 0;
          }
        }
      n->layers[i].shape = pick;
      n->layers[i].pool_apart = pick_apart;
      changed |= pick != before || pick_apart != before_apart;
    }
    if (!changed) break;
  }
  n->shapes_version++;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

int lsn_get_shapes(const lsn_net* n, int32_t* codes, int32_t count) {
  if (!n || !codes || count < (int)n->layers.size()) return LAM_EINVAL;
  for (size_t i = 0; i < n->layers.size(); ++i)
    codes[i] = n->layers[i].shape ? n->layers[i].shape
                                   : conv_default_shape(n->H >> level_of(n, (int)i), n->W >> level_of(n, (int)i),
                                                        n->layers[i].cout);
  return LAM_OK;
}

int lsn_set_shapes(lsn_net* n, const int32_t* codes, int32_t count) {
  if (!n || !codes) return fail(n, LAM_EINVAL, "null argument");
  if (count != (int32_t)n->layers.size()) return fail(n, LAM_EINVAL, "one code per 3x3 layer");
  for (size_t i = 0; i < n->layers.size(); ++i) {
    if (codes[i] == 0) continue;
    const int lev = level_of(n, (int)i);
    int cand[16];
    const int nc = conv_shapes(n->H >> lev, n->layers[i].cout, cand, 16);
    bool ok = false;
    for (int k = 0; k < nc; ++k) ok |= cand[k] == codes[i];
    if (!ok) return fail(n, LAM_EINVAL, "tile shape " + std::to_string(codes[i]) + " not available for layer " +
                                            std::to_string(i));
  }
  for (size_t i = 0; i < n->layers.size(); ++i) n->layers[i].shape = codes[i];
  n->shapes_version++;
  return LAM_OK;
}

int lsn_set_timing(lsn_net* n, int32_t enable) {
  if (!n) return fail(n, LAM_EINVAL, "null argument");
  hipError_t e;
  if (enable && !n->ev0) {
    if ((e = hipEventCreate(&n->ev0)) || (e = hipEventCreate(&n->ev1))) return hip_fail(n, e, "events");
  }
  n->timing = enable != 0;
  n->timed = false;
  return LAM_OK;
}

int lsn_forward_time(lsn_net* n, float* ms) {
  if (!n || !ms) return fail(n, LAM_EINVAL, "null argument");
  if (!n->timed) return fail(n, LAM_EINVAL, "no timed forward pass");
  hipError_t e;
  if ((e = hipEventSynchronize(n->ev1)) || (e = hipEventElapsedTime(ms, n->ev0, n->ev1)))
    return hip_fail(n, e, "timing");
  return LAM_OK;
}

const char* lsn_last_error(const lsn_net* n) { return n ? n->err.c_str() : g_nn_error.c_str(); }

void lsn_destroy(lsn_net* n) {
  if (!n) return;
  if (n->step_graph) (void)hipGraphExecDestroy(n->step_graph);
  if (n->ev0) (void)hipEventDestroy(n->ev0);
  if (n->ev1) (void)hipEventDestroy(n->ev1);
  delete n;
}

}  // extern "C"
