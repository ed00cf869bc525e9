// sur_capi.cpp -- C ABI of the warm-start network (include/lem_surrogate.h):
// argument checks, workspace carving and the order of the kernel launches of
// the forward pass, the backward pass and the Adam step.  All arithmetic runs
// in the kernels of sur_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "../../include/lem_surrogate.h"
#include "sur_internal.h"

namespace {

constexpr int kChannels[4] = {32, 64, 128, 256};
constexpr int kNumConv = 14;
constexpr int64_t kPartCap = int64_t(64) << 20;  // floats of split partials
constexpr int kBiasBlocks = 1024;   // pixel ranges of the bias gradient's partials
constexpr int kLossBlocks = 1024;
constexpr int kHeadBlocks = 2048;

struct Layer {
  int cin, cout;
  int64_t off;  // weights at off, bias at off + cout * 9 * cin
};

struct Table {
  Layer conv[kNumConv];
  int64_t head_off;
  int64_t total;
  Table() {
    int i = 0;
    auto add = [&](int cin, int cout) { conv[i].cin = cin; conv[i].cout = cout; ++i; };
    add(sur::kInChannels, kChannels[0]);
    add(kChannels[0], kChannels[0]);
    for (int l = 1; l < 4; ++l) {
      add(kChannels[l - 1], kChannels[l]);
      add(kChannels[l], kChannels[l]);
    }
    for (int l = 2; l >= 0; --l) {
      add(kChannels[l + 1] + kChannels[l], kChannels[l]);
      add(kChannels[l], kChannels[l]);
    }
    int64_t off = 0;
    for (int k = 0; k < kNumConv; ++k) {
      conv[k].off = off;
      off += (int64_t)conv[k].cout * 9 * conv[k].cin + conv[k].cout;
    }
    head_off = off;
    total = off + sur::kHeadChannels + 1;
  }
};

const Table& table() {
  static const Table t;
  return t;
}

// Layer indices.
constexpr int kEncA[4] = {0, 2, 4, 6}, kEncB[4] = {1, 3, 5, 7};
constexpr int kDecA[3] = {12, 10, 8}, kDecB[3] = {13, 11, 9};  // by level 0, 1, 2

}  // namespace

struct lem_sur_ctx {
  int B, H, W;
  hipStream_t s;
  std::string err;
  int64_t np;
  int64_t adam_t;
  bool wd_fresh;  // transposed weights match the current parameters
  float *p, *m, *v, *g;
  uint16_t *pb, *wd;
  uint16_t* x0;
  uint16_t *a_enc[4], *e[4], *pool[3], *a_dec[3], *d[3];
  float *y, *dy;
  float *gw[2], *gcat[3];  // gradients of level outputs (ping-pong), skip parts
  uint16_t *dz, *dz2;  // output gradients in bfloat16 (two layers of a block)
  float* part;
  // Split sums queued during a backward pass; their partials occupy
  // part[0, part_used).
  sur::ReduceJob jobs[sur::kMaxReduceJobs];
  int njobs;
  int64_t part_used;
  double* lpart;
  double* loss;
};

namespace {

int64_t px(const lem_sur_ctx* c, int level) {
  return (int64_t)c->B * (c->H >> level) * (c->W >> level);
}

// Carves the workspace; with base == nullptr only measures it.
size_t carve(lem_sur_ctx* c, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* r = base ? base + off : nullptr;
    off += bytes;
    return r;
  };
  const Table& t = table();
  const int64_t np = t.total;
  c->np = np;
  c->p = (float*)take(4 * np);
  c->m = (float*)take(4 * np);
  c->v = (float*)take(4 * np);
  c->g = (float*)take(4 * np);
  c->pb = (uint16_t*)take(2 * np);
  c->wd = (uint16_t*)take(2 * np);
  const int64_t P0 = px(c, 0);
  c->x0 = (uint16_t*)take(2 * P0 * sur::kInChannels);
  for (int l = 0; l < 4; ++l) {
    c->a_enc[l] = (uint16_t*)take(2 * px(c, l) * kChannels[l]);
    c->e[l] = (uint16_t*)take(2 * px(c, l) * kChannels[l]);
  }
  for (int l = 0; l < 3; ++l) {
    c->pool[l] = (uint16_t*)take(2 * px(c, l + 1) * kChannels[l]);
    c->a_dec[l] = (uint16_t*)take(2 * px(c, l) * kChannels[l]);
    c->d[l] = (uint16_t*)take(2 * px(c, l) * kChannels[l]);
    c->gcat[l] = (float*)take(4 * px(c, l) * kChannels[l]);  // skip part of the gradient
  }
  c->y = (float*)take(4 * P0);
  c->dy = (float*)take(4 * P0);
  for (int k = 0; k < 2; ++k) c->gw[k] = (float*)take(4 * P0 * kChannels[0]);
  c->dz = (uint16_t*)take(2 * P0 * kChannels[0]);
  c->dz2 = (uint16_t*)take(2 * P0 * kChannels[0]);
  c->part = (float*)take(4 * kPartCap);
  c->lpart = (double*)take(8 * kLossBlocks);
  c->loss = (double*)take(8);
  return off + 256;
}

bool valid_shape(int32_t B, int32_t H, int32_t W) {
  return B >= 1 && H >= 8 && W >= 8 && H % 8 == 0 && W % 8 == 0 &&
         (int64_t)B * H * W <= (int64_t(1) << 27);
}

lem_status fail(lem_sur_ctx* c, lem_status st, const std::string& m) {
  if (c) c->err = m;
  return st;
}

#define SUR_CHECK(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) return fail(c, LEM_E_HIP, std::string(#call) + ": " +  \
                                             hipGetErrorString(e_));             \
  } while (0)

// Sums the queued split partials into their outputs; the partial buffer is
// then free again.
lem_status flush_reduce(lem_sur_ctx* c) {
  if (c->njobs) SUR_CHECK(sur::launch_reduce_batch(c->jobs, c->njobs, c->s));
  c->njobs = 0;
  c->part_used = 0;
  return LEM_OK;
}

// Reserves room for `splits` partials of n values (and their group sums) and
// queues their sum into out; *part receives the partials' address.  Queued
// sums run in stream order before the space is reused.
lem_status queue_reduce(lem_sur_ctx* c, int splits, int64_t n, float* out, float** part) {
  lem_status st;
  const int64_t groups = sur::reduce_scratch_groups(splits);
  const int64_t need = ((n * (splits + groups)) + 63) & ~int64_t(63);
  if (need > kPartCap) return fail(c, LEM_E_SIZE, "split partials exceed the partial buffer");
  if (c->njobs == sur::kMaxReduceJobs || c->part_used + need > kPartCap)
    if ((st = flush_reduce(c)) != LEM_OK) return st;
  float* p = c->part + c->part_used;
  c->jobs[c->njobs++] = sur::ReduceJob{p, groups ? p + (int64_t)splits * n : nullptr, out, n, splits};
  c->part_used += need;
  *part = p;
  return LEM_OK;
}

// x may be the concatenation [upsampled xu (cu channels), x] (xu null: x alone).
lem_status conv(lem_sur_ctx* c, int B, int level, const uint16_t* x, int cin, const uint16_t* w,
                const float* bias, int cout, bool relu, uint16_t* outb, float* outf,
                const uint16_t* xu = nullptr, int cu = 0, float* outu = nullptr,
                int cu_out = 0) {
  sur::ConvArgs a{};
  a.x = x;
  a.xu = xu;
  a.Cu = cu;
  a.outu = outu;
  a.Cu_out = cu_out;
  a.w = w;
  a.bias = bias;
  a.outb = outb;
  a.outf = outf;
  a.B = B;
  a.H = c->H >> level;
  a.W = c->W >> level;
  a.Cin = cin;
  a.Cout = cout;
  a.relu = relu ? 1 : 0;
  a.out_f32 = outf ? 1 : 0;
  SUR_CHECK(sur::launch_conv(a, c->s));
  return LEM_OK;
}

lem_status conv_layer(lem_sur_ctx* c, int B, int level, int li, const uint16_t* x, uint16_t* out,
                      const uint16_t* xu = nullptr, int cu = 0) {
  const Layer& L = table().conv[li];
  return conv(c, B, level, x, L.cin, c->pb + L.off,
              c->p + L.off + (int64_t)L.cout * 9 * L.cin, L.cout, true, out, nullptr, xu, cu);
}

// The lower-resolution input of decoder level l: the encoder's bottom output
// for l = 2, else the decoder output of level l + 1.
const uint16_t* decoder_low(const lem_sur_ctx* c, int l) { return l == 2 ? c->e[3] : c->d[l + 1]; }

lem_status forward(lem_sur_ctx* c, int B, const double* K, const double* U, const double* h0) {
  lem_status st;
  const int64_t P0 = (int64_t)B * c->H * c->W;
  SUR_CHECK(sur::launch_features(K, U, h0, c->x0, P0, c->s));
  const uint16_t* x = c->x0;
  for (int l = 0; l < 4; ++l) {
    if ((st = conv_layer(c, B, l, kEncA[l], x, c->a_enc[l])) != LEM_OK) return st;
    if ((st = conv_layer(c, B, l, kEncB[l], c->a_enc[l], c->e[l])) != LEM_OK) return st;
    if (l < 3) {
      SUR_CHECK(sur::launch_pool(c->e[l], c->pool[l], B, c->H >> (l + 1), c->W >> (l + 1),
                                 kChannels[l], c->s));
      x = c->pool[l];
    }
  }
  // Decoder: the first convolution of level l reads the concatenation
  // [upsampled lower level, skip] straight from the two maps.
  for (int l = 2; l >= 0; --l) {
    if ((st = conv_layer(c, B, l, kDecA[l], c->e[l], c->a_dec[l], decoder_low(c, l),
                         kChannels[l + 1])) != LEM_OK)
      return st;
    if ((st = conv_layer(c, B, l, kDecB[l], c->a_dec[l], c->d[l])) != LEM_OK) return st;
  }
  const int64_t ho = table().head_off;
  SUR_CHECK(sur::launch_head(c->d[0], c->pb + ho, c->p + ho + sur::kHeadChannels, c->y, P0, c->s));
  return LEM_OK;
}

// Weight gradient of layer li into c->g (split partials, then their sum).
lem_status wgrad(lem_sur_ctx* c, int B, int level, int li, const uint16_t* x, const uint16_t* dz,
                 const uint16_t* xu = nullptr, int cu = 0) {
  const Layer& L = table().conv[li];
  const int H = c->H >> level, W = c->W >> level;
  const int64_t n = (int64_t)L.cout * 9 * L.cin;
  const int per = sur::wgrad_blocks_per_split(L.cin, L.cout);
  const int patches = sur::wgrad_patches(B, H, W);
  // One round of resident workgroups: a second, partly filled round would
  // cost as long as the first.
  int splits = std::max(1, sur::wgrad_resident(L.cout) / per);
  splits = std::min(splits, patches);
  // Partials and their group sums must fit the partial buffer.
  while (splits > 1 &&
         n * (splits + sur::reduce_scratch_groups(splits)) > kPartCap)
    --splits;
  float* part;
  lem_status st;
  if ((st = queue_reduce(c, splits, n, c->g + L.off, &part)) != LEM_OK) return st;
  sur::WgradArgs a{};
  a.x = x;
  a.xu = xu;
  a.Cu = cu;
  a.dz = dz;
  a.part = part;
  a.B = B;
  a.H = H;
  a.W = W;
  a.Cin = L.cin;
  a.Cout = L.cout;
  a.splits = splits;
  SUR_CHECK(sur::launch_wgrad(a, c->s));
  return LEM_OK;
}

// ReLU backward of layer li's output y (level `level`) given its gradient g
// (plus 0.25 g2 spread over 2x2 blocks when g2 is set): dz (bfloat16) for the
// weight and input gradients, and the bias gradient into c->g.
lem_status relu_bias_bwd(lem_sur_ctx* c, int level, int li, const float* g, const uint16_t* y,
                         int64_t P, const float* g2 = nullptr) {
  const Layer& L = table().conv[li];
  float* part;
  lem_status st;
  if ((st = queue_reduce(c, kBiasBlocks, L.cout, c->g + L.off + (int64_t)L.cout * 9 * L.cin,
                         &part)) != LEM_OK)
    return st;
  SUR_CHECK(sur::launch_relu_bwd_bias(g, g2, c->H >> level, c->W >> level, y, c->dz, P, L.cout,
                                      part, kBiasBlocks, c->s));
  return LEM_OK;
}

// Input gradient of layer lb (from c->dz) fused with the ReLU backward of
// layer la, whose stored output is a: c->dz2 = bf16 of the gradient where a
// is positive, and la's bias gradient from the convolution's per-workgroup
// sums.
lem_status dgrad_relu_bwd(lem_sur_ctx* c, int B, int level, int lb, int la, const uint16_t* a) {
  const Layer& Lb = table().conv[lb];
  const Layer& La = table().conv[la];
  sur::ConvArgs g{};
  g.x = c->dz;
  g.w = c->wd + Lb.off;
  g.outb = c->dz2;
  g.mask_y = a;
  g.B = B;
  g.H = c->H >> level;
  g.W = c->W >> level;
  g.Cin = Lb.cout;
  g.Cout = Lb.cin;
  const int groups = sur::conv_groups(g);
  lem_status st;
  if ((st = queue_reduce(c, groups, La.cout, c->g + La.off + (int64_t)La.cout * 9 * La.cin,
                         &g.bias_part)) != LEM_OK)
    return st;
  SUR_CHECK(sur::launch_conv(g, c->s));
  return LEM_OK;
}

// Backward through conv(lb)(relu(conv(la)(x))) + ReLU given the gradient ge of
// its output e (plus 0.25 ge2 over 2x2 blocks when ge2, half resolution, is
// set); gx (float32, cin(la) channels) may be null.  x may be the
// concatenation [upsampled xu (cu channels), x]; then, with gxu set, the
// gradient of its upsampled part goes to gxu (the lower level's map: sums of
// 2x2 blocks) instead of gx.
lem_status block_bwd(lem_sur_ctx* c, int B, int level, const uint16_t* x, const uint16_t* a,
                     const uint16_t* e, const float* ge, int la, int lb, float* gx,
                     const uint16_t* xu = nullptr, int cu = 0, float* gxu = nullptr,
                     const float* ge2 = nullptr) {
  lem_status st;
  const Layer& A = table().conv[la];
  const int64_t P = (int64_t)B * (c->H >> level) * (c->W >> level);
  if ((st = relu_bias_bwd(c, level, lb, ge, e, P, ge2)) != LEM_OK) return st;
  if ((st = wgrad(c, B, level, lb, a, c->dz)) != LEM_OK) return st;
  if ((st = dgrad_relu_bwd(c, B, level, lb, la, a)) != LEM_OK) return st;
  if ((st = wgrad(c, B, level, la, x, c->dz2, xu, cu)) != LEM_OK) return st;
  if (gx && (st = conv(c, B, level, c->dz2, A.cout, c->wd + A.off, nullptr, A.cin, false, nullptr,
                       gx, nullptr, 0, gxu, gxu ? cu : 0)) != LEM_OK)
    return st;
  return LEM_OK;
}

lem_status backward(lem_sur_ctx* c, int B, const double* U, const double* target) {
  lem_status st;
  const Table& t = table();
  if (!c->wd_fresh) {
    // Every layer but the first (whose input gradient is never needed).
    sur::DgradLayers L{};
    for (int k = 1; k < kNumConv; ++k) {
      const int m = L.nlayers++;
      L.off[m] = t.conv[k].off;
      L.cin[m] = t.conv[k].cin;
      L.cout[m] = t.conv[k].cout;
      L.first[m + 1] = L.first[m] + (int64_t)t.conv[k].cout * 9 * t.conv[k].cin;
    }
    SUR_CHECK(sur::launch_dgrad_weights(c->pb, c->wd, L, c->s));
    c->wd_fresh = true;
  }
  const int64_t P0 = (int64_t)B * c->H * c->W;
  const double n = (double)B * (c->H - 2) * (c->W - 2);
  SUR_CHECK(sur::launch_loss(c->y, target, U, B, c->H, c->W, c->dy, c->lpart, kLossBlocks, c->s));
  SUR_CHECK(sur::launch_reduce_f64(c->lpart, kLossBlocks, 1.0 / n, c->loss, c->s));
  // Every split sum of the pass is queued and run at its end (or earlier when
  // the partial buffer fills); nothing reads c->g before.
  c->njobs = 0;
  c->part_used = 0;
  float* hpart;
  if ((st = queue_reduce(c, kHeadBlocks, sur::kHeadChannels + 1, c->g + t.head_off, &hpart)) !=
      LEM_OK)
    return st;
  SUR_CHECK(sur::launch_head_bwd(c->dy, c->d[0], c->pb + t.head_off, c->gw[0], hpart,
                                 kHeadBlocks, P0, c->s));
  // Decoder, level 0 up to 2: the concatenation's skip part lands in gcat[l];
  // its upsampled part becomes the gradient of the level below's output.
  float* g = c->gw[0];
  for (int l = 0; l < 3; ++l) {
    // The upsampled part's gradient goes straight to the lower level as 2x2
    // block sums; gcat[l] keeps the skip part.
    float* glow = (g == c->gw[0]) ? c->gw[1] : c->gw[0];
    if ((st = block_bwd(c, B, l, c->e[l], c->a_dec[l], c->d[l], g, kDecA[l], kDecB[l],
                        c->gcat[l], decoder_low(c, l), kChannels[l + 1], glow)) != LEM_OK)
      return st;
    g = glow;
  }
  // Encoder, level 3 down to 0: an encoder output's gradient is its skip
  // part plus the pooled path's (a quarter of the level above's input
  // gradient on each pixel of its 2x2 block), added in the ReLU backward.
  const float* g2 = nullptr;
  for (int l = 3; l >= 0; --l) {
    const float* busy = g2 ? g2 : g;
    float* gx = (l > 0) ? ((busy == c->gw[0]) ? c->gw[1] : c->gw[0]) : nullptr;
    const uint16_t* x = (l > 0) ? c->pool[l - 1] : c->x0;
    if ((st = block_bwd(c, B, l, x, c->a_enc[l], c->e[l], g, kEncA[l], kEncB[l], gx, nullptr, 0,
                        nullptr, g2)) != LEM_OK)
      return st;
    if (l > 0) {
      g = c->gcat[l - 1];
      g2 = gx;
    }
  }
  return flush_reduce(c);
}

lem_status check_call(lem_sur_ctx* c, int32_t batch, const void* K, const void* U,
                      const void* h0) {
  if (!c) return LEM_E_ARG;
  if (batch < 1 || batch > c->B) return fail(c, LEM_E_ARG, "batch must be in [1, context batch]");
  if (!K || !U || !h0) return fail(c, LEM_E_ARG, "K, U and h0 must not be NULL");
  return LEM_OK;
}

lem_status read_loss(lem_sur_ctx* c, double* h_loss) {
  if (!h_loss) return LEM_OK;
  SUR_CHECK(hipMemcpyAsync(h_loss, c->loss, sizeof(double), hipMemcpyDeviceToHost, c->s));
  SUR_CHECK(hipStreamSynchronize(c->s));
  return LEM_OK;
}

}  // namespace

extern "C" {

int64_t lem_sur_param_count(void) { return table().total; }

lem_status lem_sur_layer(int32_t i, int32_t* cin, int32_t* cout, int64_t* offset) {
  if (!cin || !cout || !offset || i < 0 || i > kNumConv) return LEM_E_ARG;
  const Table& t = table();
  if (i == kNumConv) {
    *cin = sur::kHeadChannels;
    *cout = 1;
    *offset = t.head_off;
  } else {
    *cin = t.conv[i].cin;
    *cout = t.conv[i].cout;
    *offset = t.conv[i].off;
  }
  return LEM_OK;
}

size_t lem_sur_workspace_bytes(int32_t batch, int32_t ny, int32_t nx) {
  if (!valid_shape(batch, ny, nx)) return 0;
  lem_sur_ctx c{};
  c.B = batch;
  c.H = ny;
  c.W = nx;
  return carve(&c, nullptr);
}

lem_status lem_sur_create(int32_t batch, int32_t ny, int32_t nx, void* d_ws, size_t bytes,
                          void* hip_stream, lem_sur_ctx** out) {
  if (!out) return LEM_E_ARG;
  *out = nullptr;
  if (!valid_shape(batch, ny, nx)) return LEM_E_SIZE;
  if (!d_ws || ((uintptr_t)d_ws & 255u) != 0) return LEM_E_WORKSPACE;
  if (bytes < lem_sur_workspace_bytes(batch, ny, nx)) return LEM_E_WORKSPACE;
  lem_sur_ctx* c = new (std::nothrow) lem_sur_ctx();
  if (!c) return LEM_E_ARG;
  c->B = batch;
  c->H = ny;
  c->W = nx;
  c->s = (hipStream_t)hip_stream;
  carve(c, (char*)d_ws);
  c->adam_t = 0;
  c->wd_fresh = false;
  hipError_t e = hipMemsetAsync(c->p, 0, 4 * c->np, c->s);
  if (e == hipSuccess) e = hipMemsetAsync(c->pb, 0, 2 * c->np, c->s);
  if (e != hipSuccess) {
    delete c;
    return LEM_E_HIP;
  }
  *out = c;
  return LEM_OK;
}

lem_status lem_sur_set_params(lem_sur_ctx* c, const float* d_params) {
  if (!c || !d_params) return LEM_E_ARG;
  SUR_CHECK(hipMemcpyAsync(c->p, d_params, 4 * c->np, hipMemcpyDeviceToDevice, c->s));
  SUR_CHECK(hipMemsetAsync(c->m, 0, 4 * c->np, c->s));
  SUR_CHECK(hipMemsetAsync(c->v, 0, 4 * c->np, c->s));
  SUR_CHECK(sur::launch_to_bf16(c->p, c->pb, c->np, c->s));
  c->adam_t = 0;
  c->wd_fresh = false;
  return LEM_OK;
}

lem_status lem_sur_get_params(lem_sur_ctx* c, float* d_params) {
  if (!c || !d_params) return LEM_E_ARG;
  SUR_CHECK(hipMemcpyAsync(d_params, c->p, 4 * c->np, hipMemcpyDeviceToDevice, c->s));
  return LEM_OK;
}

lem_status lem_sur_predict(lem_sur_ctx* c, int32_t batch, const double* d_K, const double* d_U,
                           const double* d_h0, double* d_h, float* d_y) {
  lem_status st = check_call(c, batch, d_K, d_U, d_h0);
  if (st != LEM_OK) return st;
  if ((st = forward(c, batch, d_K, d_U, d_h0)) != LEM_OK) return st;
  if (d_h) SUR_CHECK(sur::launch_heights(c->y, d_U, d_h, batch, c->H, c->W, c->s));
  if (d_y)
    SUR_CHECK(hipMemcpyAsync(d_y, c->y, 4 * (size_t)batch * c->H * c->W, hipMemcpyDeviceToDevice,
                             c->s));
  return LEM_OK;
}

lem_status lem_sur_loss_grad(lem_sur_ctx* c, int32_t batch, const double* d_K,
                             const double* d_U, const double* d_h0, const double* d_target,
                             float* d_grad, double* h_loss) {
  lem_status st = check_call(c, batch, d_K, d_U, d_h0);
  if (st != LEM_OK) return st;
  if (!d_target) return fail(c, LEM_E_ARG, "target must not be NULL");
  if ((st = forward(c, batch, d_K, d_U, d_h0)) != LEM_OK) return st;
  if ((st = backward(c, batch, d_U, d_target)) != LEM_OK) return st;
  if (d_grad) SUR_CHECK(hipMemcpyAsync(d_grad, c->g, 4 * c->np, hipMemcpyDeviceToDevice, c->s));
  return read_loss(c, h_loss);
}

lem_status lem_sur_train_step(lem_sur_ctx* c, int32_t batch, const double* d_K,
                              const double* d_U, const double* d_h0, const double* d_target,
                              float lr, double* h_loss) {
  lem_status st = check_call(c, batch, d_K, d_U, d_h0);
  if (st != LEM_OK) return st;
  if (!d_target) return fail(c, LEM_E_ARG, "target must not be NULL");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(c, LEM_E_ARG, "lr must be finite and > 0");
  if ((st = forward(c, batch, d_K, d_U, d_h0)) != LEM_OK) return st;
  if ((st = backward(c, batch, d_U, d_target)) != LEM_OK) return st;
  c->adam_t += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)c->adam_t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)c->adam_t));
  SUR_CHECK(sur::launch_adam(c->p, c->g, c->m, c->v, c->pb, c->np, lr, c1, c2, c->s));
  c->wd_fresh = false;
  return read_loss(c, h_loss);
}

lem_status lem_sur_activation(lem_sur_ctx* c, int32_t index, int32_t batch, uint16_t* d_dst,
                              int32_t* channels, int32_t* height, int32_t* width) {
  if (!c) return LEM_E_ARG;
  if (batch < 1 || batch > c->B) return fail(c, LEM_E_ARG, "batch must be in [1, context batch]");
  const uint16_t* src = nullptr;
  int ch = 0, level = 0;
  if (index == 0) {
    src = c->x0;
    ch = sur::kInChannels;
  } else if (index >= 1 && index <= 8) {
    level = (index - 1) / 2;
    src = (index % 2) ? c->a_enc[level] : c->e[level];
    ch = kChannels[level];
  } else if (index >= 9 && index <= 11) {
    const int l = index - 9;
    src = c->pool[l];
    level = l + 1;
    ch = kChannels[l];
  } else if (index >= 12 && index <= 20) {
    level = 2 - (index - 12) / 3;
    const int k = (index - 12) % 3;
    src = k == 0 ? nullptr : (k == 1 ? c->a_dec[level] : c->d[level]);
    ch = k == 0 ? kChannels[level + 1] + kChannels[level] : kChannels[level];
  } else {
    return fail(c, LEM_E_ARG, "unknown activation index");
  }
  const int h = c->H >> level, w = c->W >> level;
  if (channels) *channels = ch;
  if (height) *height = h;
  if (width) *width = w;
  if (d_dst && src) {
    SUR_CHECK(hipMemcpyAsync(d_dst, src, 2 * (size_t)batch * h * w * ch, hipMemcpyDeviceToDevice,
                             c->s));
  } else if (d_dst) {
    // The decoder's concatenated input is never stored: it is assembled here
    // from the two maps its convolution reads.
    SUR_CHECK(sur::launch_upcat(decoder_low(c, level), c->e[level], d_dst, batch, h, w,
                                kChannels[level + 1], kChannels[level], c->s));
  }
  return LEM_OK;
}

lem_status lem_sur_sync(lem_sur_ctx* c) {
  if (!c) return LEM_E_ARG;
  SUR_CHECK(hipStreamSynchronize(c->s));
  SUR_CHECK(hipGetLastError());
  return LEM_OK;
}

lem_status lem_sur_destroy(lem_sur_ctx* c) {
  if (!c) return LEM_OK;
  (void)hipStreamSynchronize(c->s);
  delete c;
  return LEM_OK;
}

const char* lem_sur_last_error(const lem_sur_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
