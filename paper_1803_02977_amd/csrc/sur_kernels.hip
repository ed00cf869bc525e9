// sur_kernels.hip -- kernels of the warm-start network (lem_surrogate.h) for
// gfx950.  Convolutions are implicit GEMMs on the bfloat16 matrix cores
// (v_mfma_f32_16x16x32_bf16: 16x16 tiles, K = 32, float32 accumulation);
// everything else is elementwise or a reduction over pixels with a fixed
// summation order, so results do not depend on the schedule.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sur_internal.h"

namespace sur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FP64 -> bfloat16 with one rounding: keep 8 significant bits, ties to even.
__device__ __forceinline__ uint16_t d2bf(double v) {
  int e;
  const double m = frexp(v, &e);
  return f2bf((float)ldexp(rint(m * 256.0) / 256.0, e));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Channels c..c+7 of pixel (b, y, x) of a convolution input that may be the
// concatenation [nearest 2x upsample of xu (Cu channels), x (Cin - Cu
// channels)] (Cu = 0: all of x).
__device__ __forceinline__ const uint16_t* conv_input(const uint16_t* x, const uint16_t* xu,
                                                      int Cu, int Cin, int H, int W, int b,
                                                      int y, int xx, int c) {
  if (c < Cu)
    return xu + (((int64_t)b * (H >> 1) + (y >> 1)) * (W >> 1) + (xx >> 1)) * Cu + c;
  return x + (((int64_t)b * H + y) * W + xx) * (Cin - Cu) + (c - Cu);
}

// ---------------------------------------------------------------------------
// 3x3 convolution.  A workgroup (4 waves) computes 16x16-pixel tiles for
// COB output channels.  Per chunk of 32 input channels it stages the tile's
// 18x18 input halo and the COB x 9 x 32 weights in LDS; for each of the nine
// taps every wave multiplies weights (A: 16 output channels x 32 input
// channels) by shifted input pixels (B: 32 input channels x 16 pixels of one
// tile row).  A wave owns two 16-channel output blocks and NR tile rows (NR =
// 8 for COB = 64, 4 for COB = 32) and takes the taps by column shift kx: the
// three row-shift weights of one kx stay in registers while the halo rows
// stream past, each loaded once and used for every (row, ky) pair it
// serves.  The accumulator of a tile holds 4 consecutive output channels of
// one pixel per lane, stored as one 8-byte (bfloat16) or 16-byte (float32)
// write.
//
// The grid is persistent: workgroup (g, cob) of G x (Cout / COB) takes output
// channel block cob and tiles g, g + G, ...; its steps are (tile, input
// chunk) pairs, and each step's global loads are issued into registers
// before the previous step's MFMAs, so memory latency hides behind them.
// With a single input chunk (ONE) the weights are staged once.
constexpr int kT = 16;
constexpr int kHalo = kT + 2;
constexpr int kKC = 32;
constexpr int kXP = 40;   // LDS pitch of one pixel's 32 channels (bank spread)
constexpr int kWP = 40;   // LDS pitch of one (output channel, tap) row

template <int COB, bool ONE>
__global__ __launch_bounds__(256, 2) void k_conv3x3(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[kHalo * kHalo * kXP];
  __shared__ __attribute__((aligned(16))) uint16_t ws[COB * 9 * kWP];
  __shared__ float red[4][COB];    // per-wave channel sums (ReLU-backward mode)
  constexpr int MB = COB / 16;     // 16-channel output blocks of the workgroup
  constexpr int MBW = 2;           // of them per wave
  constexpr int NR = MB * kT / (4 * MBW);  // tile rows per wave
  constexpr int XN = kHalo * kHalo * 4, WN = COB * 9 * 4;  // 16-byte items
  constexpr int XI = (XN + 255) / 256, WI = (WN + 255) / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_x = (a.W + kT - 1) / kT, tiles_y = (a.H + kT - 1) / kT;
  const int ntiles = a.B * tiles_x * tiles_y;
  const int nco = a.Cout / COB;
  const int cob = blockIdx.x % nco, g = blockIdx.x / nco, G = gridDim.x / nco;
  const int co0 = cob * COB;
  const int nchunk = ONE ? 1 : a.Cin / kKC;
  const int nsteps = (g < ntiles ? (ntiles - g + G - 1) / G : 0) * nchunk;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  const int cb0 = (wave % (MB / MBW)) * MBW, row0 = (wave / (MB / MBW)) * NR;

  f32x4 acc[MBW][NR];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[MBW][4];  // ReLU-backward mode: this lane's sums of its masked outputs
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) bsum[i][j] = 0.f;

  uint4 xr[XI], wr[ONE ? 1 : WI];
  auto load_w = [&](int ci0, int j) {
    const int i = tid + j * 256;
    const int row = i >> 2, part = i & 3;  // row = co * 9 + tap
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i < WN)
      v = *reinterpret_cast<const uint4*>(a.w + ((int64_t)co0 * 9 + row) * a.Cin + ci0 + part * 8);
    return v;
  };
  auto load = [&](int k) {
    int t = g + (k / nchunk) * G;
    const int ci0 = (k % nchunk) * kKC;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y, b = t / tiles_y;
    const int y0 = ty * kT, x0 = tx * kT;
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      const int i = tid + j * 256;
      const int pix = i >> 2, part = i & 3;
      const int gy = y0 + pix / kHalo - 1, gx = x0 + pix % kHalo - 1;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (i < XN && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
        v = *reinterpret_cast<const uint4*>(
            conv_input(a.x, a.xu, a.Cu, a.Cin, a.H, a.W, b, gy, gx, ci0 + part * 8));
      xr[j] = v;
    }
    if (!ONE) {
#pragma unroll
      for (int j = 0; j < WI; ++j) wr[j] = load_w(ci0, j);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      const int i = tid + j * 256;
      if (i < XN) *reinterpret_cast<uint4*>(xs + (i >> 2) * kXP + (i & 3) * 8) = xr[j];
    }
    if (!ONE) {
#pragma unroll
      for (int j = 0; j < WI; ++j) {
        const int i = tid + j * 256;
        if (i < WN) *reinterpret_cast<uint4*>(ws + (i >> 2) * kWP + (i & 3) * 8) = wr[j];
      }
    }
  };

  if (ONE) {
#pragma unroll
    for (int j = 0; j < WI; ++j) {
      const int i = tid + j * 256;
      const uint4 v = load_w(0, j);
      if (i < WN) *reinterpret_cast<uint4*>(ws + (i >> 2) * kWP + (i & 3) * 8) = v;
    }
  }
  if (nsteps > 0) load(0);
  for (int k = 0; k < nsteps; ++k) {
    __syncthreads();
    store();
    __syncthreads();
    if (k + 1 < nsteps) load(k + 1);
#pragma unroll 1
    for (int kx = 0; kx < 3; ++kx) {
      bf16x8 av[3][MBW];
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb)
          av[ky][mb] = *reinterpret_cast<const bf16x8*>(
              ws + (((cb0 + mb) * 16 + lr) * 9 + ky * 3 + kx) * kWP + lk);
      // Halo row row0 + r serves output row nb = r - ky of tap (ky, kx).
#pragma unroll
      for (int r = 0; r < NR + 2; ++r) {
        const bf16x8 bv =
            *reinterpret_cast<const bf16x8*>(xs + ((row0 + r) * kHalo + lr + kx) * kXP + lk);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          const int nb = r - ky;
          if (nb < 0 || nb >= NR) continue;
#pragma unroll
          for (int mb = 0; mb < MBW; ++mb) acc[mb][nb] = mfma(av[ky][mb], bv, acc[mb][nb]);
        }
      }
    }
    if (k % nchunk != nchunk - 1) continue;

    int t = g + (k / nchunk) * G;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y, b = t / tiles_y;
    if (a.outu && co0 < a.Cu_out) {
      // Output channels below Cu_out: only their 2x2 block sums are stored,
      // at half resolution.  Rows nb, nb + 1 of a block are this lane's
      // accumulators, columns lr, lr ^ 1 neighbouring lanes; the sum is
      // ((top left + top right) + bottom left) + bottom right.
#pragma unroll
      for (int nb = 0; nb < NR; nb += 2) {
        const int py = ty * kT + row0 + nb, px = tx * kT + lr;
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
          const f32x4 top = acc[mb][nb], bot = acc[mb][nb + 1];
          acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
          acc[mb][nb + 1] = f32x4{0.f, 0.f, 0.f, 0.f};
          float o[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float tr = __shfl_xor(top[j], 1, 64), br = __shfl_xor(bot[j], 1, 64);
            o[j] = ((top[j] + tr) + bot[j]) + br;
          }
          if ((lr & 1) || py >= a.H || px >= a.W) continue;
          const int co = co0 + (cb0 + mb) * 16 + (lane >> 4) * 4;
          const int64_t q = ((int64_t)b * (a.H >> 1) + (py >> 1)) * (a.W >> 1) + (px >> 1);
          *reinterpret_cast<float4*>(a.outu + q * a.Cu_out + co) = make_float4(o[0], o[1], o[2], o[3]);
        }
      }
      continue;
    }
#pragma unroll
    for (int nb = 0; nb < NR; ++nb) {
      const int py = ty * kT + row0 + nb, px = tx * kT + lr;
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) {
        const f32x4 r = acc[mb][nb];
        acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (py >= a.H || px >= a.W) continue;
        const int64_t p = ((int64_t)b * a.H + py) * a.W + px;
        const int co = co0 + (cb0 + mb) * 16 + (lane >> 4) * 4;
        if (a.mask_y) {
          // ReLU backward of the layer whose stored output is mask_y: keep
          // the gradient where that output is positive, store it in
          // bfloat16, and sum it per channel for the bias gradient.
          const uint2 yv = *reinterpret_cast<const uint2*>(a.mask_y + p * a.Cout + co);
          float m[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t yw = (j < 2) ? yv.x : yv.y;
            m[j] = bf2f((uint16_t)(yw >> (16 * (j & 1)))) > 0.f ? r[j] : 0.f;
            bsum[mb][j] += m[j];
          }
          uint2 pk;
          pk.x = (uint32_t)f2bf(m[0]) | ((uint32_t)f2bf(m[1]) << 16);
          pk.y = (uint32_t)f2bf(m[2]) | ((uint32_t)f2bf(m[3]) << 16);
          *reinterpret_cast<uint2*>(a.outb + p * a.Cout + co) = pk;
          continue;
        }
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          v[j] = r[j] + (a.bias ? a.bias[co + j] : 0.f);
          if (a.relu) v[j] = fmaxf(v[j], 0.f);
        }
        if (a.out_f32) {
          // Channels below Cu_out (block sums, if any) are not part of outf.
          *reinterpret_cast<float4*>(a.outf + p * (a.Cout - a.Cu_out) + (co - a.Cu_out)) =
              make_float4(v[0], v[1], v[2], v[3]);
        } else {
          uint2 pk;
          pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          *reinterpret_cast<uint2*>(a.outb + p * a.Cout + co) = pk;
        }
      }
    }
  }

  if (a.mask_y) {
    // Channel sums: over the 16 lanes of a channel group (a fixed xor tree),
    // then over the waves holding the same channels, in wave order.
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v = bsum[mb][j];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        if (lr == 0) red[wave][(cb0 + mb) * 16 + (lane >> 4) * 4 + j] = v;
      }
    __syncthreads();
    if (tid < COB) {
      const int blk = tid / 16;
      float t = 0.f;
      for (int w = 0; w < 4; ++w)
        if ((w % (MB / MBW)) * MBW <= blk && blk < (w % (MB / MBW)) * MBW + MBW) t += red[w][tid];
      a.bias_part[(int64_t)g * a.Cout + co0 + tid] = t;
    }
  }
}

// Workgroups of 256 threads of kernel fn that the device keeps resident at
// once (computed on first use; *cache holds it).
template <typename F>
int resident_groups(F fn, int* cache) {
  if (*cache == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess ||
        cus < 1 || per < 1)
      return 256;
    *cache = cus * per;
  }
  return *cache;
}

// Tile groups G of a persistent launch (grid G x Cout / COB).
template <int COB, bool ONE>
int conv_groups_cob(const ConvArgs& a) {
  const int tiles = a.B * ((a.H + kT - 1) / kT) * ((a.W + kT - 1) / kT);
  const int nco = a.Cout / COB;
  static int resident = 0;
  return std::max(1, std::min(tiles, resident_groups(k_conv3x3<COB, ONE>, &resident) / nco));
}

template <int COB, bool ONE>
hipError_t launch_conv_cob(const ConvArgs& a, hipStream_t s) {
  const int G = conv_groups_cob<COB, ONE>(a);
  hipLaunchKernelGGL((k_conv3x3<COB, ONE>), dim3(G * (a.Cout / COB)), dim3(256), 0, s, a);
  return hipGetLastError();
}

int conv_groups(const ConvArgs& a) {
  if (a.Cout % 64 == 0)
    return a.Cin == kKC ? conv_groups_cob<64, true>(a) : conv_groups_cob<64, false>(a);
  return a.Cin == kKC ? conv_groups_cob<32, true>(a) : conv_groups_cob<32, false>(a);
}

// A concatenated input needs whole 32-channel chunks from each part and an
// even-sized map.
static bool valid_split(const uint16_t* xu, int Cu, int Cin, int H, int W) {
  if (!xu) return Cu == 0;
  return Cu > 0 && Cu < Cin && Cu % 32 == 0 && H % 2 == 0 && W % 2 == 0;
}

hipError_t launch_conv(const ConvArgs& a, hipStream_t s) {
  if (a.Cin % 32 != 0 || a.Cout % 32 != 0 || a.B < 1 || a.H < 1 || a.W < 1 ||
      !valid_split(a.xu, a.Cu, a.Cin, a.H, a.W))
    return hipErrorInvalidValue;
  // Block sums: float32 output without bias or ReLU, whole channel blocks,
  // an even-sized map.
  const int cob = a.Cout % 64 == 0 ? 64 : 32;
  if (a.outu && (!a.out_f32 || a.bias || a.relu || a.Cu_out <= 0 || a.Cu_out > a.Cout ||
                 a.Cu_out % cob != 0 || a.H % 2 != 0 || a.W % 2 != 0))
    return hipErrorInvalidValue;
  // ReLU-backward mode: bfloat16 output, no bias, ReLU or block sums.
  if (a.mask_y && (a.out_f32 || !a.outb || a.bias || a.relu || a.outu || !a.bias_part))
    return hipErrorInvalidValue;
  if (a.Cout % 64 == 0)
    return a.Cin == kKC ? launch_conv_cob<64, true>(a, s) : launch_conv_cob<64, false>(a, s);
  return a.Cin == kKC ? launch_conv_cob<32, true>(a, s) : launch_conv_cob<32, false>(a, s);
}

// ---------------------------------------------------------------------------
// Weight gradient of a 3x3 convolution:
// dW[co, tap, ci] = sum_p dz[p, co] * x[p + tap offset, ci], a GEMM with
// M = output channels, N = input channels and K = pixels for each tap.  A
// workgroup owns (COB output channels, 32 input channels, split s), computes
// all nine taps, and loops over the 16x16-pixel patches s, s + splits, ....
// Per patch it stages, channel-major (pixels contiguous), the patch's dz and
// the 18x18 input halo around it; the halo rows are 16-byte aligned, so the
// three column shifts of one tap row come from one aligned 16-byte read of
// the row and one 4-byte read of its tail (columns 8-9 or 16-17, also stored
// apart; shifts by one pixel via alignbit).  The next patch's global loads
// are issued before the current patch's MFMAs.  Results go to per-split
// partials, summed later in split order.
constexpr int kPP = 264;  // LDS pitch of one output channel's 256 patch pixels

// Position of patch pixel px in the LDS row of output channel ch: the
// 32-pixel groups are permuted by channel, so that the 64 lanes of one
// transposing 8-byte write (8-channel parts of 8 quads) hit each bank at most
// twice, the minimum for 512 bytes; an aligned 8-pixel block stays aligned.
__device__ __forceinline__ int dz_pos(int ch, int px) { return px ^ (32 * ((ch >> 4) & 3)); }
constexpr int kHR = 24;   // LDS pitch of one 18-pixel halo row (16-byte aligned)
constexpr int kHP = 456;  // LDS pitch of one input channel's 18 halo rows
constexpr int kHaloPairs = kHalo * kHalo / 2 * 4;  // (pixel pair, 8-channel part) items
// Tails of the halo rows (columns 8-9 and 16-17, read for the one-pixel
// shifts), also kept apart: 2 per row, pitch kTP per channel, so that the 64
// lanes' 4-byte reads of one row fall on 64 different banks.
constexpr int kTP = 36;

int wgrad_blocks_per_split(int Cin, int Cout) {
  const int cob = (Cout % 64 == 0) ? 64 : 32;
  return (Cout / cob) * (Cin / 32);
}

int wgrad_patches(int B, int H, int W) {
  return B * ((H + kT - 1) / kT) * ((W + kT - 1) / kT);
}

__device__ __forceinline__ uint32_t lo_pair(uint32_t a, uint32_t b) {
  return (a & 0xFFFFu) | (b << 16);
}
__device__ __forceinline__ uint32_t hi_pair(uint32_t a, uint32_t b) {
  return (a >> 16) | (b & 0xFFFF0000u);
}
__device__ __forceinline__ uint32_t word(const uint4& v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

template <int COB>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t dzt[COB * kPP];
  __shared__ __attribute__((aligned(16))) uint16_t xt[32 * kHP];
  __shared__ uint32_t xtail[32 * kTP];
  constexpr int NCB = COB == 64 ? 2 : 1;    // 16-channel input blocks per wave
  constexpr int PARTS = COB / 8;            // 8-channel parts of one dz pixel
  constexpr int DZ_ITEMS = 64 * PARTS / 256;  // (4-pixel quad, part) items per thread
  constexpr int X_ITEMS = (kHaloPairs + 255) / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, grp = lane >> 4;
  int bid = blockIdx.x;
  const int s = bid % a.splits;
  bid /= a.splits;
  const int ncit = a.Cin / 32;
  const int cit = bid % ncit;
  const int cot = bid / ncit;
  const int ci0 = cit * 32, co0 = cot * COB;
  const int tiles_x = (a.W + kT - 1) / kT, tiles_y = (a.H + kT - 1) / kT;
  const int npatch = a.B * tiles_x * tiles_y;
  const int mb = COB == 64 ? wave : (wave >> 1);
  const int cb0 = COB == 64 ? 0 : (wave & 1);

  f32x4 acc[9][NCB];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < NCB; ++i) acc[t][i] = f32x4{0.f, 0.f, 0.f, 0.f};

  uint4 dzr[DZ_ITEMS][4], xr[X_ITEMS][2];
  auto load = [&](int pt) {
    const int tx = pt % tiles_x, ty = (pt / tiles_x) % tiles_y, b = pt / (tiles_x * tiles_y);
    const int y0 = ty * kT, x0 = tx * kT;
#pragma unroll
    for (int k = 0; k < DZ_ITEMS; ++k) {
      const int i = tid + k * 256;
      const int quad = i / PARTS, part = i % PARTS;
      const int gy = y0 + quad / 4, gx = x0 + (quad % 4) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy < a.H && gx + j < a.W)
          v = *reinterpret_cast<const uint4*>(
              a.dz + (((int64_t)b * a.H + gy) * a.W + gx + j) * a.Cout + co0 + part * 8);
        dzr[k][j] = v;
      }
    }
#pragma unroll
    for (int k = 0; k < X_ITEMS; ++k) {
      const int i = tid + k * 256;
      const int pair = i >> 2, part = i & 3;
      const int gy = y0 + pair / (kHalo / 2) - 1, gx = x0 + (pair % (kHalo / 2)) * 2 - 1;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (i < kHaloPairs && gy >= 0 && gy < a.H && gx + j >= 0 && gx + j < a.W)
          v = *reinterpret_cast<const uint4*>(
              conv_input(a.x, a.xu, a.Cu, a.Cin, a.H, a.W, b, gy, gx + j, ci0 + part * 8));
        xr[k][j] = v;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < DZ_ITEMS; ++k) {
      const int i = tid + k * 256;
      const int quad = i / PARTS, part = i % PARTS;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int w = c >> 1;
        uint2 pk;
        if (c & 1) {
          pk.x = hi_pair(word(dzr[k][0], w), word(dzr[k][1], w));
          pk.y = hi_pair(word(dzr[k][2], w), word(dzr[k][3], w));
        } else {
          pk.x = lo_pair(word(dzr[k][0], w), word(dzr[k][1], w));
          pk.y = lo_pair(word(dzr[k][2], w), word(dzr[k][3], w));
        }
        *reinterpret_cast<uint2*>(dzt + (part * 8 + c) * kPP + dz_pos(part * 8 + c, quad * 4)) =
            pk;
      }
    }
#pragma unroll
    for (int k = 0; k < X_ITEMS; ++k) {
      const int i = tid + k * 256;
      if (i >= kHaloPairs) continue;
      const int pair = i >> 2, part = i & 3;
      const int hy = pair / (kHalo / 2), hx = (pair % (kHalo / 2)) * 2;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int w = c >> 1;
        const uint32_t v = (c & 1) ? hi_pair(word(xr[k][0], w), word(xr[k][1], w))
                                   : lo_pair(word(xr[k][0], w), word(xr[k][1], w));
        *reinterpret_cast<uint32_t*>(xt + (part * 8 + c) * kHP + hy * kHR + hx) = v;
        if (hx == 8 || hx == 16) xtail[(part * 8 + c) * kTP + hy * 2 + (hx >> 4)] = v;
      }
    }
  };

  if (s < npatch) load(s);
  for (int pt = s; pt < npatch; pt += a.splits) {
    __syncthreads();
    store();
    __syncthreads();
    if (pt + a.splits < npatch) load(pt + a.splits);
    // Halo row 2 ks + grp / 2 + 2 (tap row ky = 2 of K step ks) is row ky = 0
    // of step ks + 1: it is carried in registers instead of read again.
    uint4 cv[NCB];
    uint32_t ce[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int ci = (cb0 + cb) * 16 + lr;
      cv[cb] = *reinterpret_cast<const uint4*>(xt + ci * kHP + (grp >> 1) * kHR + (grp & 1) * 8);
      ce[cb] = xtail[ci * kTP + (grp >> 1) * 2 + (grp & 1)];
    }
#pragma unroll 1
    for (int ks = 0; ks < 8; ++ks) {
      // K step ks: patch pixels 32 ks .. 32 ks + 31; lane group grp holds
      // pixels 32 ks + 8 grp .. + 7 = row 2 ks + grp / 2, columns 8 (grp % 2) ...
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(
          dzt + (mb * 16 + lr) * kPP + dz_pos(mb * 16 + lr, ks * 32 + grp * 8));
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int ci = (cb0 + cb) * 16 + lr;
        const uint16_t* col = xt + ci * kHP + (2 * ks + (grp >> 1)) * kHR + (grp & 1) * 8;
        const uint32_t* tail = xtail + ci * kTP + (2 * ks + (grp >> 1)) * 2 + (grp & 1);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          uint4 v;
          uint32_t e;
          if (ky == 0) {
            v = cv[cb];
            e = ce[cb];
          } else {
            v = *reinterpret_cast<const uint4*>(col + ky * kHR);
            e = tail[ky * 2];
          }
          if (ky == 2) {
            cv[cb] = v;
            ce[cb] = e;
          }
          const uint4 v1 = make_uint4(__builtin_amdgcn_alignbit(v.y, v.x, 16),
                                      __builtin_amdgcn_alignbit(v.z, v.y, 16),
                                      __builtin_amdgcn_alignbit(v.w, v.z, 16),
                                      __builtin_amdgcn_alignbit(e, v.w, 16));
          const uint4 v2 = make_uint4(v.y, v.z, v.w, e);
          acc[ky * 3 + 0][cb] = mfma(av, __builtin_bit_cast(bf16x8, v), acc[ky * 3 + 0][cb]);
          acc[ky * 3 + 1][cb] = mfma(av, __builtin_bit_cast(bf16x8, v1), acc[ky * 3 + 1][cb]);
          acc[ky * 3 + 2][cb] = mfma(av, __builtin_bit_cast(bf16x8, v2), acc[ky * 3 + 2][cb]);
        }
      }
    }
  }

#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int ci = ci0 + (cb0 + cb) * 16 + lr;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = co0 + mb * 16 + grp * 4 + j;
        a.part[(((int64_t)s * a.Cout + co) * 9 + t) * a.Cin + ci] = acc[t][cb][j];
      }
    }
}

int wgrad_resident(int Cout) {
  static int r64 = 0, r32 = 0;
  return (Cout % 64 == 0) ? resident_groups(k_wgrad<64>, &r64) : resident_groups(k_wgrad<32>, &r32);
}

hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s) {
  if (a.Cin % 32 != 0 || a.Cout % 32 != 0 || a.splits < 1 ||
      !valid_split(a.xu, a.Cu, a.Cin, a.H, a.W))
    return hipErrorInvalidValue;
  const int blocks = wgrad_blocks_per_split(a.Cin, a.Cout) * a.splits;
  if (a.Cout % 64 == 0)
    hipLaunchKernelGGL(k_wgrad<64>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_wgrad<32>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions and elementwise kernels.

__device__ __forceinline__ int reduce_scratch_groups_dev(int splits) {
  return splits <= kReduceGroup ? 0 : (splits + kReduceGroup - 1) / kReduceGroup;
}

int reduce_scratch_groups(int splits) {
  return splits <= kReduceGroup ? 0 : (splits + kReduceGroup - 1) / kReduceGroup;
}

// Up to kMaxReduceJobs split sums, out[i] = sum of part[s * n + i] over the
// splits, in one launch per stage; one thread per (value, group).  Stage 1:
// jobs of at most kReduceGroup splits are summed whole, in split order, into
// out; the others in groups of kReduceGroup consecutive splits, each in split
// order, into tmp.  Stage 2 adds a job's group sums in group order into out.
// first[j] is the first block of job j (first[njobs] = all blocks).
struct ReduceBatchArgs {
  ReduceJob job[kMaxReduceJobs];
  int first[kMaxReduceJobs + 1];
  int njobs, stage;
};

__global__ void k_reduce_batch(ReduceBatchArgs a) {
  int j = 0;
  while (j + 1 < a.njobs && (int)blockIdx.x >= a.first[j + 1]) ++j;
  const ReduceJob& J = a.job[j];
  const int local = (int)blockIdx.x - a.first[j];
  const int chunks = (int)((J.n + 255) / 256);
  const int G = reduce_scratch_groups_dev(J.splits);
  if (a.stage == 1) {
    const int g = local / chunks;
    const int64_t i = (int64_t)(local % chunks) * 256 + threadIdx.x;
    if (i >= J.n) return;
    const int s0 = G ? g * kReduceGroup : 0, s1 = G ? min(J.splits, s0 + kReduceGroup) : J.splits;
    float acc = 0.f;
#pragma unroll 8
    for (int s = s0; s < s1; ++s) acc += J.part[(int64_t)s * J.n + i];
    if (G) J.tmp[(int64_t)g * J.n + i] = acc;
    else J.out[i] = acc;
  } else {
    const int64_t i = (int64_t)local * 256 + threadIdx.x;
    if (i >= J.n) return;
    float acc = 0.f;
    for (int g = 0; g < G; ++g) acc += J.tmp[(int64_t)g * J.n + i];
    J.out[i] = acc;
  }
}

hipError_t launch_reduce_batch(const ReduceJob* jobs, int njobs, hipStream_t s) {
  if (njobs < 0 || njobs > kMaxReduceJobs) return hipErrorInvalidValue;
  for (int stage = 1; stage <= 2; ++stage) {
    ReduceBatchArgs a{};
    a.stage = stage;
    int64_t blocks = 0;
    for (int k = 0; k < njobs; ++k) {
      const ReduceJob& J = jobs[k];
      if (J.splits < 1 || J.n < 1 || !J.part || !J.out) return hipErrorInvalidValue;
      const int G = reduce_scratch_groups(J.splits);
      if (G && !J.tmp) return hipErrorInvalidValue;
      if (stage == 2 && G == 0) continue;
      const int64_t chunks = (J.n + 255) / 256;
      a.job[a.njobs] = J;
      a.first[a.njobs] = (int)blocks;
      ++a.njobs;
      blocks += (stage == 1 && G) ? chunks * G : chunks;
    }
    if (a.njobs == 0) continue;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    a.first[a.njobs] = (int)blocks;
    hipLaunchKernelGGL(k_reduce_batch, dim3((unsigned)blocks), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_to_bf16(const float* p, uint16_t* pb, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    pb[i] = f2bf(p[i]);
}

hipError_t launch_to_bf16(const float* p, uint16_t* pb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(2048), dim3(256), 0, s, p, pb, n);
  return hipGetLastError();
}

// wd[ci][t][co] = w[co][8 - t][ci] for every listed layer (its weights at
// off[k] in both arrays): the input gradient of a 3x3 convolution is the
// convolution of the output gradient with the spatially flipped,
// channel-transposed kernel.  One launch covers all layers; element i of the
// concatenated layers belongs to layer k when first[k] <= i < first[k + 1].
__global__ void k_dgrad_weights(const uint16_t* w, uint16_t* wd, DgradLayers L) {
  const int64_t n = L.first[L.nlayers];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int k = 0;
    while (k + 1 < L.nlayers && i >= L.first[k + 1]) ++k;
    const int64_t j = i - L.first[k];
    const int Cin = L.cin[k], Cout = L.cout[k];
    const int co = (int)(j % Cout);
    const int t = (int)((j / Cout) % 9);
    const int ci = (int)(j / ((int64_t)Cout * 9));
    wd[L.off[k] + j] = w[L.off[k] + ((int64_t)co * 9 + (8 - t)) * Cin + ci];
  }
}

hipError_t launch_dgrad_weights(const uint16_t* w, uint16_t* wd, const DgradLayers& L,
                                hipStream_t s) {
  if (L.nlayers < 1 || L.nlayers > kMaxDgradLayers) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dgrad_weights, dim3(1024), dim3(256), 0, s, w, wd, L);
  return hipGetLastError();
}

// Input features: (ln K - ln K_ref)/sigma, U/U_ref, h0, then zeros.
__global__ void k_features(const double* K, const double* U, const double* h0, uint16_t* x0,
                           int64_t P) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double f0 = (log(K[p]) - log(kKRef)) / kLnKSigma;
  const double f1 = U[p] / kURef;
  const double f2 = h0[p];
  uint4* dst = reinterpret_cast<uint4*>(x0 + p * kInChannels);
  dst[0] = make_uint4((uint32_t)d2bf(f0) | ((uint32_t)d2bf(f1) << 16), (uint32_t)d2bf(f2), 0u, 0u);
  dst[1] = make_uint4(0u, 0u, 0u, 0u);
  dst[2] = make_uint4(0u, 0u, 0u, 0u);
  dst[3] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_features(const double* K, const double* U, const double* h0, uint16_t* x0,
                           int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, K, U, h0,
                     x0, P);
  return hipGetLastError();
}

// Channel groups per pixel must be a power of two (the channel counts of the
// network are); lg is its log2, so a flat index splits by shifts.
static bool pow2_groups(int C, int per, int* lg) {
  if (C < per || C % per != 0) return false;
  const int g = C / per;
  if (g & (g - 1)) return false;
  int l = 0;
  while ((1 << l) < g) ++l;
  *lg = l;
  return true;
}

// 2x2 average pool of bfloat16 maps (C channels; Ho x Wo output), 8 channels
// (16 bytes) per thread and iteration.
__global__ void k_pool(const uint16_t* x, uint16_t* out, int B, int Ho, int Wo, int C, int lg) {
  const int64_t n = ((int64_t)B * Ho * Wo) << lg;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i & ((1 << lg) - 1)) * 8;
    const int q = (int)(i >> lg);
    const int xo = q % Wo, yo = (q / Wo) % Ho, b = q / (Wo * Ho);
    const int W = 2 * Wo;
    const int64_t r0 = ((int64_t)b * 2 * Ho + 2 * yo) * W + 2 * xo, r1 = r0 + W;
    const uint4 v00 = *reinterpret_cast<const uint4*>(x + r0 * C + c);
    const uint4 v01 = *reinterpret_cast<const uint4*>(x + (r0 + 1) * C + c);
    const uint4 v10 = *reinterpret_cast<const uint4*>(x + r1 * C + c);
    const uint4 v11 = *reinterpret_cast<const uint4*>(x + (r1 + 1) * C + c);
    uint32_t o[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t a0 = word(v00, w), a1 = word(v01, w), a2 = word(v10, w), a3 = word(v11, w);
      uint32_t r = 0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int sh = 16 * h;
        const float t = ((bf2f((uint16_t)(a0 >> sh)) + bf2f((uint16_t)(a1 >> sh))) +
                         bf2f((uint16_t)(a2 >> sh))) +
                        bf2f((uint16_t)(a3 >> sh));
        r |= (uint32_t)f2bf(t * 0.25f) << sh;
      }
      o[w] = r;
    }
    *reinterpret_cast<uint4*>(out + (int64_t)q * C + c) = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

hipError_t launch_pool(const uint16_t* x, uint16_t* out, int B, int Ho, int Wo, int C,
                       hipStream_t s) {
  int lg;
  if (!pow2_groups(C, 8, &lg)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pool, dim3(2048), dim3(256), 0, s, x, out, B, Ho, Wo, C, lg);
  return hipGetLastError();
}

// out = [nearest 2x upsample of low (Cu channels), skip (Cs channels)],
// moved in 8-channel (16-byte) pieces.
__global__ void k_upcat(const uint16_t* low, const uint16_t* skip, uint16_t* out, int B, int H,
                        int W, int Cu, int Cs) {
  const int C = Cu + Cs, pieces = C / 8;
  const int64_t n = (int64_t)B * H * W * pieces;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % pieces) * 8;
    const int64_t p = i / pieces;
    uint4 v;
    if (c < Cu) {
      const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((int64_t)W * H));
      const int64_t q = ((int64_t)b * (H / 2) + y / 2) * (W / 2) + x / 2;
      v = *reinterpret_cast<const uint4*>(low + q * Cu + c);
    } else {
      v = *reinterpret_cast<const uint4*>(skip + p * Cs + (c - Cu));
    }
    *reinterpret_cast<uint4*>(out + p * C + c) = v;
  }
}

hipError_t launch_upcat(const uint16_t* low, const uint16_t* skip, uint16_t* out, int B, int H,
                        int W, int Cu, int Cs, hipStream_t s) {
  hipLaunchKernelGGL(k_upcat, dim3(2048), dim3(256), 0, s, low, skip, out, B, H, W, Cu, Cs);
  return hipGetLastError();
}

// ReLU backward with the bias gradient's partial sums: v = g where the
// stored output y > 0, else 0; dz = bf16(v); part[blk][c] = sum of v[p, c]
// over pixels p of block blk's range [blk P / nblk, (blk + 1) P / nblk).
// With g2 set, the gradient is g + 0.25 g2 at the pixel's 2x2 block (g2 is
// H/2 x W/2, C channels: the pooled path's gradient spread over the block).
// A thread handles 4 consecutive channels of one pixel (C / 4 threads per
// pixel, 1024 / C pixels per pass, each thread summing its pixels in order);
// the per-thread sums are then added in LDS in pixel order.
__global__ __launch_bounds__(256) void k_relu_bwd_bias(const float* g, const float* g2, int H,
                                                       int W, const uint16_t* y, uint16_t* dz,
                                                       int64_t P, int C, float* part, int nblk) {
  __shared__ float4 red[256];
  const int Q = C / 4, R = 256 / Q;
  const int r = threadIdx.x / Q, q = threadIdx.x % Q;
  const int64_t p0 = P * blockIdx.x / nblk, p1 = P * (blockIdx.x + 1) / nblk;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t p = p0 + r; p < p1; p += R) {
    const int64_t e = p * C + q * 4;
    float4 gv = *reinterpret_cast<const float4*>(g + e);
    if (g2) {
      const int pp = (int)p;
      const int xx = pp % W, yy = (pp / W) % H, bb = pp / (W * H);
      const int64_t qq = ((int64_t)bb * (H / 2) + yy / 2) * (W / 2) + xx / 2;
      const float4 u = *reinterpret_cast<const float4*>(g2 + qq * C + q * 4);
      gv = make_float4(gv.x + 0.25f * u.x, gv.y + 0.25f * u.y, gv.z + 0.25f * u.z,
                       gv.w + 0.25f * u.w);
    }
    const uint2 yv = *reinterpret_cast<const uint2*>(y + e);
    const float v0 = bf2f((uint16_t)(yv.x & 0xFFFFu)) > 0.f ? gv.x : 0.f;
    const float v1 = bf2f((uint16_t)(yv.x >> 16)) > 0.f ? gv.y : 0.f;
    const float v2 = bf2f((uint16_t)(yv.y & 0xFFFFu)) > 0.f ? gv.z : 0.f;
    const float v3 = bf2f((uint16_t)(yv.y >> 16)) > 0.f ? gv.w : 0.f;
    acc.x += v0;
    acc.y += v1;
    acc.z += v2;
    acc.w += v3;
    uint2 pk;
    pk.x = (uint32_t)f2bf(v0) | ((uint32_t)f2bf(v1) << 16);
    pk.y = (uint32_t)f2bf(v2) | ((uint32_t)f2bf(v3) << 16);
    *reinterpret_cast<uint2*>(dz + e) = pk;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < Q) {
    float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = 0; k < R; ++k) {
      const float4 u = red[k * Q + q];
      t.x += u.x;
      t.y += u.y;
      t.z += u.z;
      t.w += u.w;
    }
    *reinterpret_cast<float4*>(part + (int64_t)blockIdx.x * C + q * 4) = t;
  }
}

hipError_t launch_relu_bwd_bias(const float* g, const float* g2, int H, int W, const uint16_t* y,
                                uint16_t* dz, int64_t P, int C, float* part, int nblk,
                                hipStream_t s) {
  if (C < 4 || C > 1024 || 1024 % C != 0 || nblk < 1 || P < 1) return hipErrorInvalidValue;
  if (g2 && (H < 2 || W < 2 || H % 2 != 0 || W % 2 != 0 || P % ((int64_t)H * W) != 0 ||
             P > INT32_MAX))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_relu_bwd_bias, dim3(nblk), dim3(256), 0, s, g, g2, H, W, y, dz, P, C, part,
                     nblk);
  return hipGetLastError();
}

// Head: y[p] = (sum_c w[c] d0[p, c]) + bias.
__global__ void k_head(const uint16_t* d0, const uint16_t* wb, const float* bias, float* y,
                       int64_t P) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < kHeadChannels; ++c) acc += bf2f(wb[c]) * bf2f(d0[p * kHeadChannels + c]);
  y[p] = acc + bias[0];
}

hipError_t launch_head(const uint16_t* d0, const uint16_t* wb, const float* bias, float* y,
                       int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_head, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, d0, wb, bias, y,
                     P);
  return hipGetLastError();
}

// Loss: over interior cells, diff = y - h/((U/U_ref) H_ref); dy = 2 diff / N
// and per-block partial sums of diff^2 (FP64).
__global__ __launch_bounds__(256) void k_loss(const float* y, const double* target,
                                              const double* U, int B, int H, int W, float* dy,
                                              double* part) {
  __shared__ double red[256];
  const int64_t P = (int64_t)B * H * W;
  const double n = (double)B * (H - 2) * (W - 2);
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(p % W), yy = (int)((p / W) % H);
    double diff = 0.0;
    if (x > 0 && x < W - 1 && yy > 0 && yy < H - 1)
      diff = (double)y[p] - target[p] / ((U[p] / kURef) * kHRef);
    dy[p] = (float)(2.0 * diff / n);
    acc += diff * diff;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

hipError_t launch_loss(const float* y, const double* target, const double* U, int B, int H,
                       int W, float* dy, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(256), 0, s, y, target, U, B, H, W, dy, part);
  return hipGetLastError();
}

// out = scale * (sum of part[0..n)): thread t sums part[t], part[t + 256], ...
// in order, then the 256 sums are added pairwise in a fixed tree.
__global__ __launch_bounds__(256) void k_reduce_f64(const double* part, int n, double scale,
                                                    double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

hipError_t launch_reduce_f64(const double* part, int n, double scale, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, s, part, n, scale, out);
  return hipGetLastError();
}

// Head backward: g[p, c] = dy[p] w[c]; per-block partials of
// dw[c] = sum_p dy[p] d0[p, c] (part[blk][c]) and db = sum_p dy[p] (part[blk][32]).
__global__ __launch_bounds__(256) void k_head_bwd(const float* dy, const uint16_t* d0,
                                                  const uint16_t* wb, float* g, float* part,
                                                  int nblk, int64_t P) {
  __shared__ float red[8][kHeadChannels + 1];
  const int c = threadIdx.x & 31, r = threadIdx.x >> 5;
  const int64_t p0 = P * blockIdx.x / nblk, p1 = P * (blockIdx.x + 1) / nblk;
  const float w = bf2f(wb[c]);
  float acc = 0.f, accb = 0.f;
  for (int64_t p = p0 + r; p < p1; p += 8) {
    const float d = dy[p];
    g[p * kHeadChannels + c] = d * w;
    acc += d * bf2f(d0[p * kHeadChannels + c]);
    if (c == 0) accb += d;
  }
  red[r][c] = acc;
  if (c == 0) red[r][kHeadChannels] = accb;
  __syncthreads();
  if (threadIdx.x <= kHeadChannels) {
    float s = 0.f;
    for (int k = 0; k < 8; ++k) s += red[k][threadIdx.x];
    part[(int64_t)blockIdx.x * (kHeadChannels + 1) + threadIdx.x] = s;
  }
}

hipError_t launch_head_bwd(const float* dy, const uint16_t* d0, const uint16_t* wb, float* g,
                           float* part, int nblk, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3(nblk), dim3(256), 0, s, dy, d0, wb, g, part, nblk, P);
  return hipGetLastError();
}

// Adam with bias correction (c1 = 1 - beta1^t, c2 = 1 - beta2^t); refreshes
// the bfloat16 copy of each parameter.
__global__ void k_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int64_t n,
                       float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
  }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int64_t n,
                       float lr, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(2048), dim3(256), 0, s, p, g, m, v, pb, n, lr, c1, c2);
  return hipGetLastError();
}

// Predicted heights: y (U/U_ref) H_ref inside the grid, 0 on its perimeter.
__global__ void k_heights(const float* y, const double* U, double* h, int B, int H, int W) {
  const int64_t P = (int64_t)B * H * W;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int x = (int)(p % W), yy = (int)((p / W) % H);
  h[p] = (x > 0 && x < W - 1 && yy > 0 && yy < H - 1) ? (double)y[p] * ((U[p] / kURef) * kHRef)
                                                       : 0.0;
}

hipError_t launch_heights(const float* y, const double* U, double* h, int B, int H, int W,
                          hipStream_t s) {
  const int64_t P = (int64_t)B * H * W;
  hipLaunchKernelGGL(k_heights, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, y, U, h, B, H,
                     W);
  return hipGetLastError();
}

}  // namespace sur
