// sur_internal.h -- launch interface of the warm-start network kernels
// (sur_kernels.hip), used by the C ABI in sur_capi.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sur {

// Reference scales of the features and of the output (heights in metres).
constexpr double kKRef = 1e-5;
constexpr double kURef = 1e-3;
constexpr double kHRef = 100.0;
constexpr double kLnKSigma = 0.5;
constexpr int kInChannels = 32;   // three features, zero-padded
constexpr int kHeadChannels = 32;

// 3x3 convolution (zero padding 1) as an implicit GEMM on MFMA:
// out[p, co] = bias[co] + sum_{tap, ci} x[p + tap offset, ci] * w[co, tap, ci],
// optionally followed by ReLU.  x is bfloat16 NHWC with Cin channels
// (a multiple of 32), w bfloat16 [Cout][9][Cin], out bfloat16 or float32
// NHWC with Cout channels (a multiple of 32).  With xu set, the input is the
// concatenation [nearest 2x upsample of xu (H/2 x W/2, Cu channels), x (Cin -
// Cu channels)], read from the two maps directly (Cu a multiple of 32).
struct ConvArgs {
  const uint16_t* x;
  const uint16_t* xu;  // may be null (then Cu = 0)
  int Cu;
  const uint16_t* w;
  const float* bias;   // may be null
  uint16_t* outb;      // bfloat16 output (out_f32 == 0)
  float* outf;         // float32 output (out_f32 == 1)
  // With outu set (float32 output, no bias or ReLU): output channels below
  // Cu_out are not written; outu (H/2 x W/2, Cu_out channels) gets the sums
  // of their 2x2 pixel blocks instead, and outf holds channels Cu_out..Cout-1
  // (Cout - Cu_out per pixel).
  float* outu;
  int Cu_out;
  // With mask_y set (bfloat16 output, no bias or ReLU): the ReLU backward of
  // the layer whose stored output mask_y (NHWC, Cout channels) is: outb gets
  // bf16(r) where mask_y > 0, else 0, and bias_part[g][co] (conv_groups(a) x
  // Cout floats) the per-workgroup sums of those masked values (float32).
  const uint16_t* mask_y;
  float* bias_part;
  int B, H, W, Cin, Cout;
  int relu, out_f32;
};

// Weight gradient partials: part[s][co][tap][ci] = sum over the pixels of
// split s of dz[p, co] * x[p + tap offset, ci].
struct WgradArgs {
  const uint16_t* x;   // bfloat16 NHWC, Cin channels (Cin - Cu with xu set)
  const uint16_t* xu;  // may be null; else channels [0, Cu) upsampled from it, as in ConvArgs
  int Cu;
  const uint16_t* dz;  // bfloat16 NHWC, Cout channels
  float* part;
  int B, H, W, Cin, Cout, splits;
};

hipError_t launch_conv(const ConvArgs& a, hipStream_t s);
int conv_groups(const ConvArgs& a);  // tile groups of launch_conv's persistent grid
hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s);
int wgrad_blocks_per_split(int Cin, int Cout);
int wgrad_resident(int Cout);  // workgroups the weight-gradient kernel keeps resident
int wgrad_patches(int B, int H, int W);

// Split partials are summed in groups of kReduceGroup consecutive splits,
// then over the groups (in order both times); a job with more than
// kReduceGroup splits needs reduce_scratch_groups(splits) * n floats of group
// sums (tmp).
constexpr int kReduceGroup = 32;
int reduce_scratch_groups(int splits);

// One split sum: out[i] = sum of part[s * n + i] over s < splits (tmp: its
// group sums, or null if splits <= kReduceGroup).
struct ReduceJob {
  const float* part;
  float* tmp;
  float* out;
  int64_t n;
  int splits;
};
constexpr int kMaxReduceJobs = 32;
// Runs up to kMaxReduceJobs independent split sums in two launches.
hipError_t launch_reduce_batch(const ReduceJob* jobs, int njobs, hipStream_t s);
hipError_t launch_to_bf16(const float* p, uint16_t* pb, int64_t n, hipStream_t s);
// Layers whose flipped, channel-transposed weights launch_dgrad_weights
// builds: weights of layer k at off[k] (cin[k] x 9 x cout[k] values); first
// holds the running element counts (first[0] = 0).
constexpr int kMaxDgradLayers = 16;
struct DgradLayers {
  int64_t off[kMaxDgradLayers];
  int64_t first[kMaxDgradLayers + 1];
  int cin[kMaxDgradLayers], cout[kMaxDgradLayers];
  int nlayers;
};
hipError_t launch_dgrad_weights(const uint16_t* w, uint16_t* wd, const DgradLayers& L,
                                hipStream_t s);
hipError_t launch_features(const double* K, const double* U, const double* h0, uint16_t* x0,
                           int64_t P, hipStream_t s);
hipError_t launch_pool(const uint16_t* x, uint16_t* out, int B, int Ho, int Wo, int C,
                       hipStream_t s);
hipError_t launch_upcat(const uint16_t* low, const uint16_t* skip, uint16_t* out, int B, int H,
                        int W, int Cu, int Cs, hipStream_t s);
hipError_t launch_relu_bwd_bias(const float* g, const float* g2, int H, int W, const uint16_t* y,
                                uint16_t* dz, int64_t P, int C, float* part, int nblk,
                                hipStream_t s);
hipError_t launch_head(const uint16_t* d0, const uint16_t* wb, const float* bias, float* y,
                       int64_t P, hipStream_t s);
hipError_t launch_loss(const float* y, const double* target, const double* U, int B, int H,
                       int W, float* dy, double* part, int nblk, hipStream_t s);
hipError_t launch_reduce_f64(const double* part, int n, double scale, double* out,
                             hipStream_t s);
hipError_t launch_head_bwd(const float* dy, const uint16_t* d0, const uint16_t* wb, float* g,
                           float* part, int nblk, int64_t P, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int64_t n,
                       float lr, float c1, float c2, hipStream_t s);
hipError_t launch_heights(const float* y, const double* U, double* h, int B, int H, int W,
                          hipStream_t s);

}  // namespace sur
