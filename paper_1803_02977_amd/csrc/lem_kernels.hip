// lem_kernels.hip -- gfx950 kernels of the landscape-evolution hot path.
//
// One time step (Barnes, arXiv:1803.02977, Steps 2 to 7) is two launches:
//
//  k_receivers + k_donors   dense row-major sweeps over the grid:
//      Step 2 / Algorithm 1: receiver code per cell (strict ">" over the
//      slopes (h_c - h_n)/dist in neighbour order, first maximum wins);
//      Step 3 / Algorithm 2: donor bit mask per cell, over every cell.
//
//  k_order_accum_erode      one cooperative (persistent) kernel whose level
//      loops run on the device with grid-wide barriers between levels:
//      Step 4 / Algorithm 3: breadth-first levels.  Level 0 is every cell
//        without a receiver; level l+1 is the donors of level l.  Each chunk
//        of a level is expanded with a workgroup prefix scan and reserves its
//        output range with one atomic add, so the queue is written with no
//        per-cell atomics.  Alongside the queue it records, per position,
//        the receiver's position, the first donor's position, the donor mask
//        and the receiver code, so that the later phases read the tree in
//        queue order instead of gathering it from the grid.
//      Step 5 / Algorithm 4 (Equation "flow_acc"): upstream cell counts,
//        levels deepest first; each position pulls its donors' counts, which
//        sit contiguously in the next level.
//      Step 6 / Algorithm 5 and Step 7 / Algorithm 6: uplift and the
//        implicit n = 1 update h <- (h0 + F*h_rec)/(1 + F), levels from the
//        roots outward; the receiver's new height is read from the
//        queue-order copy written by the previous level.
//
// Arithmetic that decides results is written operation by operation in the
// same order as the problem's definition and compiled without FP contraction
// (-ffp-contract=off), so receivers, levels and counts are exact and heights
// round the same way on every run.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "lem_internal.h"

namespace cg = cooperative_groups;

namespace lem {

namespace {

__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive prefix sum of v over the workgroup; *total receives the sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const int s = wsum[k];
    off += (k < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__device__ __forceinline__ int64_t neighbour_offset(int k, int nx) {
  // (dy,dx) in code order: (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1)
  const int dy = (k < 3) ? -1 : (k < 5 ? 0 : 1);
  const int dx = (k == 0 || k == 3 || k == 5) ? -1 : ((k == 1 || k == 6) ? 0 : 1);
  return (int64_t)dy * nx + dx;
}

// A^m: sqrt for m = 0.5 and A itself for m = 1 (both exact), pow otherwise.
__device__ __forceinline__ double area_power(double area, const StepArgs& a) {
  return a.use_sqrt ? sqrt(area) : (a.m == 1.0 ? area : pow(area, a.m));
}

__device__ __forceinline__ double code_distance(int k, double dx, double dy, double ddiag) {
  return (k == 1 || k == 6) ? dy : ((k == 3 || k == 4) ? dx : ddiag);
}

// ---------------------------------------------------------------------------
// Step 2 / Algorithm 1: receivers.
__global__ __launch_bounds__(256) void k_receivers(StepArgs a) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx;
  const int64_t c = (int64_t)y * nx + x;
  uint8_t code;
  if (y == 0 || x == 0 || y == a.ny - 1 || x == nx - 1) {
    code = kBase;
  } else {
    const double* h = a.h;
    const double hc = h[c];
    const double dxv = a.dx, dyv = a.dy, dd = a.ddiag;
    const double s0 = (hc - h[c - nx - 1]) / dd;
    const double s1 = (hc - h[c - nx]) / dyv;
    const double s2 = (hc - h[c - nx + 1]) / dd;
    const double s3 = (hc - h[c - 1]) / dxv;
    const double s4 = (hc - h[c + 1]) / dxv;
    const double s5 = (hc - h[c + nx - 1]) / dd;
    const double s6 = (hc - h[c + nx]) / dyv;
    const double s7 = (hc - h[c + nx + 1]) / dd;
    double smax = 0.0;
    code = kSink;
    if (s0 > smax) { smax = s0; code = 0; }
    if (s1 > smax) { smax = s1; code = 1; }
    if (s2 > smax) { smax = s2; code = 2; }
    if (s3 > smax) { smax = s3; code = 3; }
    if (s4 > smax) { smax = s4; code = 4; }
    if (s5 > smax) { smax = s5; code = 5; }
    if (s6 > smax) { smax = s6; code = 6; }
    if (s7 > smax) { smax = s7; code = 7; }
  }
  a.w.rcode[c] = code;
}

// Fixed routing (test hook): copy caller codes, checking that each stays in
// the grid and that perimeter cells have none.  Bad codes raise LEM_E_ARG on
// the device and are treated as "no receiver".
__global__ __launch_bounds__(256) void k_fixed_routing(StepArgs a, const uint8_t* user) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int64_t c = (int64_t)y * a.nx + x;
  const uint8_t u = user[c];
  const bool perim = (y == 0 || x == 0 || y == a.ny - 1 || x == a.nx - 1);
  uint8_t code;
  if (perim) {
    code = kBase;
    if (u != 8) atomicMax(&a.w.ctrl->status, 1);
  } else if (u <= 7) {
    code = u;
  } else {
    code = kSink;
    if (u != 8) atomicMax(&a.w.ctrl->status, 1);
  }
  a.w.rcode[c] = code;
}

// Step 3 / Algorithm 2 over every cell: bit k of the mask is set when the
// neighbour at offset k has this cell as its receiver (code 7-k).
__global__ __launch_bounds__(256) void k_donors(StepArgs a) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    a.w.lcnt[0] = 0;
    a.w.lcnt[1] = 0;
  }
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx;
  const int64_t c = (int64_t)y * nx + x;
  const uint8_t* r = a.w.rcode;
  const bool up = y > 0, dn = y < a.ny - 1, lf = x > 0, rt = x < nx - 1;
  uint32_t m = 0;
  if (up && lf && r[c - nx - 1] == 7) m |= 1u << 0;
  if (up && r[c - nx] == 6) m |= 1u << 1;
  if (up && rt && r[c - nx + 1] == 5) m |= 1u << 2;
  if (lf && r[c - 1] == 4) m |= 1u << 3;
  if (rt && r[c + 1] == 3) m |= 1u << 4;
  if (dn && lf && r[c + nx - 1] == 2) m |= 1u << 5;
  if (dn && r[c + nx] == 1) m |= 1u << 6;
  if (dn && rt && r[c + nx + 1] == 0) m |= 1u << 7;
  a.w.dmask[c] = (uint8_t)m;
}

__device__ __forceinline__ int32_t load_acquire(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Steps 4 to 7 in one cooperative launch.
__global__ __launch_bounds__(kBlock) void k_order_accum_erode(StepArgs a) {
  cg::grid_group grid = cg::this_grid();
  __shared__ int wsum[kBlock / 64];
  __shared__ int s_base;
  const Work w = a.w;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int nx = a.nx;
  const bool lead = (blockIdx.x == 0 && tid == 0);
  uint64_t t0 = 0, t1 = 0, t2 = 0;
  if (lead && a.timers) t0 = wall_clock64();

  // Level 0: every cell without a receiver, compacted chunk by chunk.
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < n;
       base += (int64_t)gridDim.x * kChunk) {
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t c = base + (int64_t)j * kBlock + tid;
      if (c < n && w.rcode[c] >= kSink) bits |= 1u << j;
    }
    int tot;
    const int pre = block_exclusive_scan(__popc(bits), wsum, &tot);
    if (tid == 0) s_base = tot ? atomicAdd(&w.lcnt[0], tot) : 0;
    __syncthreads();
    int pos = s_base + pre;
    while (bits) {
      const int j = __ffs(bits) - 1;
      bits &= bits - 1;
      const int64_t c = base + (int64_t)j * kBlock + tid;
      w.q[pos] = (int32_t)c;
      w.par[pos] = -1;
      w.kq[pos] = w.rcode[c];
      ++pos;
    }
  }
  grid.sync();

  // Breadth-first expansion, one level per grid-wide barrier.  The number of
  // cells appended to level L+1 accumulates in lcnt[L+1]; the workgroup 0
  // lead clears lcnt[L+2] while level L runs, so nobody else touches it.
  int32_t lo = 0;
  int32_t hi = load_acquire(&w.lcnt[0]);
  int32_t L = 0;
  if (lead) w.lev[0] = 0;
  while (true) {
    if (lead) {
      w.lev[L + 1] = hi;
      w.lcnt[L + 2] = 0;
    }
    for (int64_t base = lo + (int64_t)blockIdx.x * kChunk; base < hi;
         base += (int64_t)gridDim.x * kChunk) {
      int32_t cs[kItems];
      uint32_t ms[kItems];
      int cntv = 0;
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + (int64_t)j * kBlock + tid;
        cs[j] = 0;
        ms[j] = 0;
        if (i < hi) {
          cs[j] = w.q[i];
          ms[j] = w.dmask[cs[j]];
          cntv += __popc(ms[j]);
        }
      }
      int tot;
      const int pre = block_exclusive_scan(cntv, wsum, &tot);
      if (tid == 0) s_base = tot ? atomicAdd(&w.lcnt[L + 1], tot) : 0;
      __syncthreads();
      int32_t pos = hi + s_base + pre;
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + (int64_t)j * kBlock + tid;
        if (i < hi) {
          uint32_t m = ms[j];
          w.mq[i] = (uint8_t)m;
          w.fc[i] = pos;
          while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1;
            w.q[pos] = (int32_t)(cs[j] + neighbour_offset(b, nx));
            w.par[pos] = (int32_t)i;
            w.kq[pos] = (uint8_t)(7 - b);
            ++pos;
          }
        }
      }
    }
    grid.sync();
    const int32_t added = load_acquire(&w.lcnt[L + 1]);
    if (added == 0) break;
    lo = hi;
    hi += added;
    ++L;
  }
  const int32_t nlevels = L + 1;
  const int32_t total = hi;
  if (lead && a.timers) t1 = wall_clock64();

  // Step 5: counts, deepest level first (levels >= 1).
  for (int32_t l = nlevels - 1; l >= 1; --l) {
    const int32_t a0 = w.lev[l], a1 = w.lev[l + 1];
    for (int64_t i = a0 + (int64_t)blockIdx.x * kBlock + tid; i < a1;
         i += (int64_t)gridDim.x * kBlock) {
      const uint32_t m = w.mq[i];
      uint32_t s = 1u;
      if (m) {
        const int32_t f = w.fc[i];
        const int k = __popc(m);
        for (int j = 0; j < k; ++j) s += w.cnt[f + j];
      }
      w.cnt[i] = s;
    }
    grid.sync();
  }
  if (lead && a.timers) t2 = wall_clock64();

  // Level 0: counts of the roots, and uplift of the interior roots (Step 6).
  {
    const int32_t a1 = w.lev[1];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < a1;
         i += (int64_t)gridDim.x * kBlock) {
      const uint32_t m = w.mq[i];
      uint32_t s = 1u;
      if (m) {
        const int32_t f = w.fc[i];
        const int k = __popc(m);
        for (int j = 0; j < k; ++j) s += w.cnt[f + j];
      }
      w.cnt[i] = s;
      const int32_t c = w.q[i];
      double hv = a.h[c];
      if (w.kq[i] == kSink) {
        hv = hv + (a.Uf ? a.Uf[c] * a.dt : a.udt);
        a.h[c] = hv;
      }
      w.hq[i] = hv;
    }
  }

  // Steps 6 and 7 for levels >= 1: uplift, then the implicit update against
  // the receiver's new height (from the previous level).
  for (int32_t l = 1; l < nlevels; ++l) {
    grid.sync();
    const int32_t a0 = w.lev[l], a1 = w.lev[l + 1];
    for (int64_t i = a0 + (int64_t)blockIdx.x * kBlock + tid; i < a1;
         i += (int64_t)gridDim.x * kBlock) {
      const int32_t c = w.q[i];
      const int32_t p = w.par[i];
      const double hr = w.hq[p];
      const double d = code_distance(w.kq[i], a.dx, a.dy, a.ddiag);
      const double area = (double)w.cnt[i] * a.dxdy;
      const double am = area_power(area, a);
      const double kc = a.Kf ? a.Kf[c] : a.K;
      const double f = ((kc * a.dt) * am) / d;
      const double h0 = a.h[c] + (a.Uf ? a.Uf[c] * a.dt : a.udt);
      const double hn = (h0 + f * hr) / (1.0 + f);
      w.hq[i] = hn;
      a.h[c] = hn;
    }
  }

  if (lead) {
    Ctrl* ct = w.ctrl;
    ct->nlevels = nlevels;
    ct->total = total;
    if (nlevels > ct->max_nlevels) ct->max_nlevels = nlevels;
    if (a.step < kHistCap) w.hist[a.step] = nlevels;
    ct->steps = a.step + 1;
    if (total != n) atomicMax(&ct->status, 5);
    if (a.timers) {
      const uint64_t t3 = wall_clock64();
      ct->ticks[1] += t1 - t0;
      ct->ticks[2] += t2 - t1;
      ct->ticks[3] += t3 - t2;
    }
  }
}

__global__ void k_begin_run(Ctrl* ct) {
  ct->max_nlevels = 0;
  ct->steps = 0;
  for (int k = 0; k < 4; ++k) ct->ticks[k] = 0;
}

// Routing export: receiver index, level and upstream count per cell.
__global__ __launch_bounds__(256) void k_export(StepArgs a, int32_t* rec, int32_t* depth,
                                                uint32_t* count) {
  const Work w = a.w;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t nlev = w.ctrl->nlevels;
  const int32_t total = w.ctrl->total;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    if (rec) {
      const uint8_t k = w.rcode[i];
      rec[i] = (k >= kSink) ? (int32_t)i : (int32_t)(i + neighbour_offset(k, a.nx));
    }
    if (i < total && (depth || count)) {
      int32_t lo = 0, hi = nlev;  // largest l with lev[l] <= i
      while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (w.lev[mid] <= i) lo = mid; else hi = mid;
      }
      const int32_t c = w.q[i];
      if (depth) depth[c] = lo;
      if (count) count[c] = w.cnt[i];
    }
  }
}

__global__ __launch_bounds__(256) void k_validate(const double* x, int64_t n, int32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    bad |= !isfinite(x[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

dim3 grid2d(const StepArgs& a) {
  return dim3((unsigned)((a.nx + 63) / 64), (unsigned)((a.ny + 3) / 4));
}

}  // namespace

static int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

size_t workspace_bytes(int64_t n) {
  int64_t b = 0;
  b += align256(n);                       // rcode
  b += align256(n);                       // dmask
  b += align256(4 * n);                   // q
  b += align256(4 * n);                   // par
  b += align256(4 * n);                   // fc
  b += align256(n);                       // mq
  b += align256(n);                       // kq
  b += align256(4 * n);                   // cnt
  b += align256(8 * n);                   // hq
  b += align256(4 * (n + 2));             // lcnt
  b += align256(4 * (n + 2));             // lev
  b += align256(4 * kHistCap);            // hist
  b += align256(sizeof(Ctrl));            // ctrl
  b += align256(4 * kScratchInts);        // scratch
  return (size_t)b;
}

void carve(void* base, int64_t n, Work* w) {
  char* p = (char*)base;
  auto take = [&](int64_t bytes) { char* r = p; p += align256(bytes); return (void*)r; };
  w->rcode = (uint8_t*)take(n);
  w->dmask = (uint8_t*)take(n);
  w->q = (int32_t*)take(4 * n);
  w->par = (int32_t*)take(4 * n);
  w->fc = (int32_t*)take(4 * n);
  w->mq = (uint8_t*)take(n);
  w->kq = (uint8_t*)take(n);
  w->cnt = (uint32_t*)take(4 * n);
  w->hq = (double*)take(8 * n);
  w->lcnt = (int32_t*)take(4 * (n + 2));
  w->lev = (int32_t*)take(4 * (n + 2));
  w->hist = (int32_t*)take(4 * kHistCap);
  w->ctrl = (Ctrl*)take(sizeof(Ctrl));
  w->scratch = (int32_t*)take(4 * kScratchInts);
}

hipError_t launch_route(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_receivers, grid2d(a), dim3(64, 4), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_donors, grid2d(a), dim3(64, 4), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fixed_routing(const StepArgs& a, const uint8_t* user, hipStream_t s) {
  hipLaunchKernelGGL(k_fixed_routing, grid2d(a), dim3(64, 4), 0, s, a, user);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_donors, grid2d(a), dim3(64, 4), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_order_accum_erode(const StepArgs& a, int grid, hipStream_t s) {
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_order_accum_erode, dim3(grid), dim3(kBlock),
                                    args, 0, s);
}

hipError_t launch_begin_run(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_begin_run, dim3(1), dim3(1), 0, s, a.w.ctrl);
  return hipGetLastError();
}

hipError_t launch_export(const StepArgs& a, int32_t* rec, int32_t* depth, uint32_t* count,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_export, dim3(2048), dim3(256), 0, s, a, rec, depth, count);
  return hipGetLastError();
}

hipError_t launch_validate(const double* x, int64_t n, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(2048), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

hipError_t order_kernel_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                      (const void*)k_order_accum_erode,
                                                      kBlock, 0);
}

}  // namespace lem
