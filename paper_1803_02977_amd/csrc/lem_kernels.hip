// lem_kernels.hip -- gfx950 kernels of the landscape-evolution hot path.
//
// One time step (Barnes, arXiv:1803.02977, Steps 2 to 7) is three launches.
//
//  k_tile_step   one workgroup of 512 threads per 64x64 tile.  The tile's heights and a
//      2-cell halo are staged in LDS once; each thread owns a vertical strip
//      of 8 cells of one column.  In LDS the workgroup computes Step 2 /
//      Algorithm 1 (receivers) for the tile and its 1-cell ring, Step 3 /
//      Algorithm 2 (donor masks) for the tile, and, by walks down the
//      receivers, each cell's tile-local root, its depth below that root and
//      the number of cells upstream of it.  A tree whose root has no
//      receiver and which has no donor outside the tile is a whole tree of
//      the method: its depths are its levels (Step 4 / Algorithm 3) and its
//      counts its drainage areas (Step 5 / Algorithm 4), so the workgroup
//      finishes it -- uplift and the implicit n = 1 update level by level
//      from the root (Steps 6-7 / Algorithms 5-6) -- and writes the new
//      heights.  Every other tree ("crossing": it leaves or enters the tile)
//      is handed on: its root is queued.  Heights are read from one buffer
//      and written to the other, so halo reads never see a neighbouring
//      tile's new values.
//
//  k_chunk_trees   persistent workgroups of 256 threads take chunks of
//      queued crossing roots from a work counter and carry out Steps 4-7 for
//      their whole trees in LDS, with workgroup barriers only.  A chunk whose
//      trees outgrow the stage's capacity (cells or levels) is staged for
//      the level pass below.
//
//  k_global_levels   (one grid) a cooperative kernel of at most kGlobalMaxWGs
//      workgroups of 1024 threads for the trees the chunk stage handed on,
//      with device-side level loops: breadth-first expansion (a workgroup
//      prefix scan per chunk and one atomic add per chunk to reserve its
//      output), counts in reverse level order (each queue position pulls its
//      donors' counts, which sit contiguously in the next level), then uplift
//      and erosion from the roots outward.  Large levels are shared by all
//      workgroups and end in a grid-wide barrier; runs of small levels are
//      done by one workgroup with workgroup barriers only.  It returns at
//      once when nothing was handed on.
//  k_grid_levels   (batches) the same level pass with one workgroup per grid.
//
// The results of the method do not depend on the order cells are processed
// in (receivers, levels and counts are exact; each height depends only on
// its own inputs and its receiver's new height), so resolving a tree inside
// its tile gives the same bits as resolving it in the global queue.
//
// Arithmetic that decides results is written operation by operation in the
// order of the problem's definition and compiled without FP contraction
// (-ffp-contract=off).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "lem_internal.h"

namespace cg = cooperative_groups;

namespace lem {

namespace {

constexpr uint32_t kSpinLimit = 1u << 26;  // about 2 s of polling

// Row and column offsets of neighbour k, as 2-bit fields (offset + 1) packed
// in one word so that a run-time k costs a shift and a mask, not branches:
// dy + 1 = 0 0 0 1 1 2 2 2 and dx + 1 = 0 1 2 0 2 0 1 2 for k = 0..7.
__device__ __forceinline__ int code_dy(int k) { return (int)((0xA940u >> (2 * k)) & 3u) - 1; }
__device__ __forceinline__ int code_dx(int k) { return (int)((0x9224u >> (2 * k)) & 3u) - 1; }
// Distance class of a receiver code: 0 vertical (dy), 1 horizontal (dx), 2 diagonal.
__device__ __forceinline__ int code_class(int k) {
  return (int)((0x8962u >> (2 * k)) & 3u);  // 2 0 2 1 1 2 0 2 for k = 0..7
}

__device__ __forceinline__ int64_t neighbour_offset(int k, int nx) {
  return (int64_t)code_dy(k) * nx + code_dx(k);
}

// A^m: sqrt for m = 0.5 and A itself for m = 1 (both exact), pow otherwise.
__device__ __forceinline__ double area_power(double area, int use_sqrt, double m) {
  return use_sqrt ? sqrt(area) : (m == 1.0 ? area : pow(area, m));
}
__device__ __noinline__ double area_power_call(double area, int use_sqrt, double m) {
  return area_power(area, use_sqrt, m);
}

// Step 2 / Algorithm 1 by the definition: eight quotients (h_c - h_k)/dist
// in neighbour order, strict ">" against a running maximum starting at 0.
// hk are the neighbours' heights in neighbour order k = 0..7.
__device__ __noinline__ uint8_t receiver_code_by_definition(double hc, double h0, double h1,
                                                            double h2, double h3, double h4,
                                                            double h5, double h6, double h7,
                                                            double dx, double dy, double dd) {
  const double s0 = (hc - h0) / dd;
  const double s1 = (hc - h1) / dy;
  const double s2 = (hc - h2) / dd;
  const double s3 = (hc - h3) / dx;
  const double s4 = (hc - h4) / dx;
  const double s5 = (hc - h5) / dd;
  const double s6 = (hc - h6) / dy;
  const double s7 = (hc - h7) / dd;
  double smax = 0.0;
  uint8_t code = kSink;
  if (s0 > smax) { smax = s0; code = 0; }
  if (s1 > smax) { smax = s1; code = 1; }
  if (s2 > smax) { smax = s2; code = 2; }
  if (s3 > smax) { smax = s3; code = 3; }
  if (s4 > smax) { smax = s4; code = 4; }
  if (s5 > smax) { smax = s5; code = 5; }
  if (s6 > smax) { smax = s6; code = 6; }
  if (s7 > smax) { smax = s7; code = 7; }
  return code;
}

// Reciprocals of the three neighbour distances (fl(1/d)).
struct RecvConst {
  double dx, dy, dd;
  double inv_dx, inv_dy, inv_dd;
};

// The same result as the definition, usually without any division.  The
// definition picks the first neighbour whose rounded quotient
// s_k = fl(a_k / d_k) (a_k = fl(h_c - h_k)) equals the largest one, S, when
// S > 0.  Neighbours fall in distance classes with one divisor each (with
// dx == dy the four orthogonal neighbours form one class), and rounding is
// monotone, so a class's largest quotient belongs to its largest numerator.
//  - Classes are ranked by m_c * fl(1/d_c), which is within 3 units in the
//    last place of fl(m_c / d_c); if the best class leads every other by a
//    relative 2^-48, its rounded quotient is strictly the largest.
//  - Inside the winning class the first neighbour holding the class maximum
//    wins, unless another member is within a relative 2^-49 of it (its
//    rounded quotient could then equal S).
//  - All numerators <= 0 means no receiver.
// Anything else (near-ties across classes, near-ties inside the class, or
// quotients outside [2^-1000, 2^1000]) is decided by the definition itself.
template <bool kSquare>
__device__ __forceinline__ uint8_t receiver_code(double hc, double h0, double h1, double h2,
                                                 double h3, double h4, double h5, double h6,
                                                 double h7, const RecvConst& rk) {
  const double a0 = hc - h0, a1 = hc - h1, a2 = hc - h2, a3 = hc - h3, a4 = hc - h4;
  const double a5 = hc - h5, a6 = hc - h6, a7 = hc - h7;
  constexpr double kNear = 1.0 - 0x1p-49;
  constexpr double kMargin = 1.0 - 0x1p-48;
  const double md = fmax(fmax(a0, a2), fmax(a5, a7));
  const double qd = md * rk.inv_dd;
  double m, q, q2, q3;
  uint32_t eq, near;
  if (kSquare) {
    const double mo = fmax(fmax(a1, a3), fmax(a4, a6));
    if (!(mo > 0.0) && !(md > 0.0)) return kSink;
    const double qo = mo * rk.inv_dx;
    const bool orth = qo > qd || md != md;
    m = orth ? mo : md;
    q = orth ? qo : qd;
    q2 = orth ? qd : qo;
    q3 = -1.0;
    const double b0 = orth ? a1 : a0, b1 = orth ? a3 : a2, b2 = orth ? a4 : a5, b3 = orth ? a6 : a7;
    const uint32_t k0 = orth ? 1 : 0, k1 = orth ? 3 : 2, k2 = orth ? 4 : 5, k3 = orth ? 6 : 7;
    eq = ((b0 == m) << k0) | ((b1 == m) << k1) | ((b2 == m) << k2) | ((b3 == m) << k3);
    near = ((b0 != m && b0 > m * kNear) << k0) | ((b1 != m && b1 > m * kNear) << k1) |
           ((b2 != m && b2 > m * kNear) << k2) | ((b3 != m && b3 > m * kNear) << k3);
  } else {
    const double mv = fmax(a1, a6), mh = fmax(a3, a4);
    if (!(mv > 0.0) && !(mh > 0.0) && !(md > 0.0)) return kSink;
    const double qv = mv * rk.inv_dy, qh = mh * rk.inv_dx;
    // Rank the classes (NaN classes never win).
    int win = 2;
    q = qd;
    if (qv > q || q != q) { win = 0; q = qv; }
    if (qh > q || q != q) { win = 1; q = qh; }
    q2 = win == 0 ? qh : qv;
    q3 = win == 2 ? qh : qd;
    m = win == 0 ? mv : (win == 1 ? mh : md);
    const double b0 = win == 0 ? a1 : (win == 1 ? a3 : a0);
    const double b1 = win == 0 ? a6 : (win == 1 ? a4 : a2);
    const uint32_t k0 = win == 0 ? 1 : (win == 1 ? 3 : 0);
    const uint32_t k1 = win == 0 ? 6 : (win == 1 ? 4 : 2);
    eq = ((b0 == m) << k0) | ((b1 == m) << k1);
    near = ((b0 != m && b0 > m * kNear) << k0) | ((b1 != m && b1 > m * kNear) << k1);
    if (win == 2) {
      eq |= ((a5 == m) << 5) | ((a7 == m) << 7);
      near |= ((a5 != m && a5 > m * kNear) << 5) | ((a7 != m && a7 > m * kNear) << 7);
    }
  }
  const bool fast = q >= 0x1p-1000 && q <= 0x1p1000 && !(q2 >= q * kMargin) &&
                    !(q3 >= q * kMargin) && near == 0u;
  if (fast) return (uint8_t)(__ffs(eq) - 1);
  return receiver_code_by_definition(hc, h0, h1, h2, h3, h4, h5, h6, h7, rk.dx, rk.dy, rk.dd);
}

// Receiver code of the cell at index ci of a row-major array of heights with
// row stride W (every neighbour present).
template <bool kSquare>
__device__ __forceinline__ uint8_t receiver_code_at(const double* h, int ci, int W,
                                                    const RecvConst& rk) {
  return receiver_code<kSquare>(h[ci], h[ci - W - 1], h[ci - W], h[ci - W + 1], h[ci - 1],
                                h[ci + 1], h[ci + W - 1], h[ci + W], h[ci + W + 1], rk);
}

// F = K*dt*A^m/d and 1 + F for a cell of grid gi (descriptor G) with
// `count` upstream cells that drains along code k (A = count*dx*dy).
// Scalar K and small counts read the grid's tables, built at the start of
// the run from the same expressions.
__device__ __forceinline__ void erosion_factor(const StepArgs& a, const GridDev& G, int gi,
                                               uint32_t count, int k, int64_t c, double* f,
                                               double* g) {
  const int cls = code_class(k);
  if (!a.Kf && count < (uint32_t)kAmTab) {
    *f = a.w.ftab[(gi * 3 + cls) * kAmTab + count];
    *g = a.w.gtab[(gi * 3 + cls) * kAmTab + count];
    return;
  }
  // A select, not an index: a runtime index into a local copy of the
  // descriptor would move that copy to scratch memory.
  const double d = cls == 0 ? G.dn[0] : (cls == 1 ? G.dn[1] : G.dn[2]);
  const double am = count < (uint32_t)kAmTab
                        ? a.w.amtab[gi * kAmTab + count]
                        : area_power_call((double)count * G.dxdy, G.use_sqrt, G.m);
  const double kc = a.Kf ? a.Kf[c] : G.K;
  *f = ((kc * G.dt) * am) / d;
  *g = 1.0 + *f;
}

// Step 7 for one cell: the implicit update of h0 (uplift included) towards
// its already updated receiver height hr.  For n = 1 the Newton iteration of
// Algorithm 6 started at h0 reaches (h0 + F*hr)/(1 + F) in one step, so that
// closed form is used; otherwise the loop runs until two iterates differ by
// at most eps or the iteration limit is reached.  The residual
// h - h0 + F*(h - hr)^n has one root in (hr, h0] when h0 > hr; an iterate
// that does not lie above the receiver (n < 1 can overshoot) is replaced by
// the midpoint between the receiver and the previous iterate.  A cell not
// above its receiver keeps h0.
__device__ __noinline__ double newton_height(double h0, double hr, double f, double nexp,
                                             double eps, int max_iter) {
  double hnew = h0, delta = 2.0 * eps;
  if (!(h0 - hr > 0.0)) return h0;
  for (int it = 0; fabs(delta) > eps && it < max_iter; ++it) {
    const double gap = hnew - hr;
    double next = hnew - (hnew - h0 + f * pow(gap, nexp)) / (1.0 + f * nexp * pow(gap, nexp - 1.0));
    if (!(next - hr > 0.0)) next = 0.5 * (hnew + hr);
    delta = next - hnew;
    hnew = next;
  }
  return hnew;
}

__device__ __forceinline__ double eroded_height(const GridDev& G, double h0, double hr, double f,
                                                double g) {
  return G.newton ? newton_height(h0, hr, f, G.nexp, G.eps, G.max_newton) : (h0 + f * hr) / g;
}

// Steady-state projection of one cell (an accelerator of runs to steady
// state, not part of a time step of the method): the height at which the
// implicit update leaves the cell unchanged given its receiver's new height
// hr, F (h - hr)^n = udt (udt = U*dt of the cell): hr + udt/F for n = 1,
// hr + (udt/F)^(1/n) otherwise.  F = 0 keeps the uplifted height h0.
__device__ __forceinline__ double steady_height(const GridDev& G, double h0, double hr, double f,
                                                double udt) {
  if (!(f > 0.0)) return h0;
  return G.newton ? hr + pow(udt / f, 1.0 / G.nexp) : hr + udt / f;
}

// Step 7, or the projection, for one cell.
__device__ __forceinline__ double new_height(const GridDev& G, bool project, double h0, double hr,
                                             double f, double g, double udt) {
  return project ? steady_height(G, h0, hr, f, udt) : eroded_height(G, h0, hr, f, g);
}

// Step 7 for one cell of grid gi in full generality (per-cell K, counts past
// the tables, n != 1): erosion_factor and eroded_height in one out-of-line
// call, for kernels whose common case reads F from a table in LDS.
__device__ __noinline__ double eroded_height_general(const GridDev* grids, int gi,
                                                     const double* Kf, const double* amtab,
                                                     uint32_t count, int k, int64_t c, double h0,
                                                     double hr, int project, double udt) {
  const GridDev& G = grids[gi];
  const int cls = code_class(k);
  const double d = cls == 0 ? G.dn[0] : (cls == 1 ? G.dn[1] : G.dn[2]);
  const double am = count < (uint32_t)kAmTab ? amtab[gi * kAmTab + count]
                                             : area_power((double)count * G.dxdy, G.use_sqrt, G.m);
  const double kc = Kf ? Kf[c] : G.K;
  const double f = ((kc * G.dt) * am) / d;
  const double g = 1.0 + f;
  return new_height(G, project != 0, h0, hr, f, g, udt);
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP: shifts by 1,
// 2, 4 and 8 inside each row of 16 lanes (lanes shifted in from outside the
// row add 0), then the last lane of row 0 (of rows 0-1) is added to rows 1
// and 3 (to rows 2 and 3).  Every lane of the wave must be active.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Maximum over the lanes 0..l of the wave (unsigned), the same pattern.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return v;
}

// Exclusive prefix sum of v over a workgroup of NT threads; *total gets the sum.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const int s = wsum[k];
    off += (k < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__device__ __forceinline__ uint64_t wave_inclusive_scan64(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Output positions in item order for 4W items per thread (W <= 4), item j
// of thread t being queue position base + j * NT + t.  v[g] packs the counts of
// items 4g..4g+3 (each at most 8) in 16-bit fields; pre[g] receives, field by
// field, the exclusive prefix over the threads and tot[g] the workgroup
// totals (at most 8 * NT < 2^16, so fields never carry).  Item j of thread t
// then starts at sum_{j' < j} total_{j'} + prefix_j(t).  wsum64 holds
// 4 * NT / 64 + 4 words.
__device__ __forceinline__ int item_field(uint64_t x, int i) {
  return (int)((x >> (16 * i)) & 0xFFFFu);
}

// Donor counts of four items from their masks packed in one word (8 bits
// each), as block_scan_items wants them (16 bits each).
__device__ __forceinline__ uint64_t counts_of_masks(uint32_t mk) {
  uint64_t v = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) v |= (uint64_t)__popc((mk >> (8 * i)) & 0xFFu) << (16 * i);
  return v;
}

template <int NT, int W>
__device__ __forceinline__ void block_scan_items(const uint64_t* v, uint64_t* wsum64,
                                                 uint64_t* pre, uint64_t* tot) {
  static_assert(8 * NT < 65536, "16-bit fields");
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < W; ++g) {
    pre[g] = wave_inclusive_scan64(v[g]);
    if (lane == 63) wsum64[g * NW + w] = pre[g];
  }
  __syncthreads();
  if (w == 0) {  // one wave turns the wave totals into offsets and the workgroup totals
#pragma unroll 1
    for (int g = 0; g < W; ++g) {
      const uint64_t x = lane < NW ? wsum64[g * NW + lane] : 0;
      const uint64_t y = wave_inclusive_scan64(x);
      if (lane < NW) wsum64[g * NW + lane] = y - x;
      if (lane == NW - 1) wsum64[4 * NW + g] = y;
    }
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < W; ++g) {
    pre[g] += wsum64[g * NW + w] - v[g];
    tot[g] = wsum64[4 * NW + g];
  }
  __syncthreads();
}

template <int W>
__device__ __forceinline__ int items_total(const uint64_t* tot) {
  int s = 0;
#pragma unroll
  for (int g = 0; g < W; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) s += item_field(tot[g], i);
  return s;
}

__device__ __forceinline__ int32_t load_acquire(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous run of tiles so that tiles sharing halo rows share an L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int xcd = b & 7, k = b >> 3;
  int start = 0;
  for (int j = 0; j < xcd; ++j) start += (ntiles - j + 7) >> 3;
  return start + k;
}

// ---------------------------------------------------------------------------
// Tile pass.  Every per-cell LDS array uses the row stride of the staged
// region (the tile plus a 2-cell halo), so one index serves them all.  Each
// thread owns a vertical strip of kStrip cells of one column: the wave's 64
// lanes are the tile's 64 columns, so LDS rows are read without conflicts
// and the receivers of a strip reuse a sliding 3x3 window of registers.
constexpr int kSW = kTW + 4;
constexpr int kSH = kTH + 4;
constexpr int kSN = kSW * kSH;
constexpr int kStrip = kTH / (kTileThreads / kTW);
constexpr int kRing = 2 * (kTW + 2) + 2 * kTH;  // cells of the ring around the tile
constexpr uint32_t kRingFlag = 0x10;            // rc bit: the cell lies on the ring
static_assert(kTileThreads % kTW == 0 && kTH % (kTileThreads / kTW) == 0, "strip layout");
static_assert(kStrip == 8, "codes packed 4 bits a cell in one word, levels 8 bits in two");
static_assert(kRing <= kTileThreads, "one ring cell per thread");
static_assert(kSN % 4 == 0, "byte arrays cleared as words");
static_assert(kSN <= 0x2000, "level-list entries: 13-bit LDS index and 3-bit code");

// Offset of neighbour k in the tile pass's LDS layout: eight signed bytes in
// one word, so a run-time k costs a shift and a sign extension.
constexpr uint64_t lds_off_table() {
  uint64_t t = 0;
  for (int k = 0; k < 8; ++k) {
    const int dy = (int)((0xA940u >> (2 * k)) & 3u) - 1, dx = (int)((0x9224u >> (2 * k)) & 3u) - 1;
    t |= (uint64_t)(uint8_t)(int8_t)(dy * kSW + dx) << (8 * k);
  }
  return t;
}
static_assert(kSW + 1 <= 127, "neighbour offsets fit a signed byte");
__device__ __forceinline__ int lds_off(int k) {
  return (int)(int8_t)(uint8_t)(lds_off_table() >> (8 * k));
}

// Codes of the kStrip cells of a strip whose first cell has LDS index li0,
// from the staged heights (a sliding window of three rows of three), stored
// in rc and returned 4 bits a cell.  Cells outside the grid get kNone and
// perimeter cells kBase; `inner` says neither occurs.
template <bool kSquare>
__device__ __forceinline__ uint32_t strip_codes(const double* hs, uint8_t* rc, int li0,
                                                const RecvConst& rk, bool inner, int gy0, int gx,
                                                int ny, int nx) {
  double l0 = hs[li0 - kSW - 1], c0 = hs[li0 - kSW], r0 = hs[li0 - kSW + 1];
  double l1 = hs[li0 - 1], c1 = hs[li0], r1 = hs[li0 + 1];
  uint32_t codes = 0;
#pragma unroll 2
  for (int t = 0; t < kStrip; ++t) {
    const int li = li0 + t * kSW;
    const double l2 = hs[li + kSW - 1], c2 = hs[li + kSW], r2 = hs[li + kSW + 1];
    uint32_t code;
    const int gy = gy0 + t;
    if (!inner && (gy >= ny || gx >= nx))
      code = kNone;
    else if (!inner && (gy == 0 || gx == 0 || gy == ny - 1 || gx == nx - 1))
      code = kBase;
    else
      code = receiver_code<kSquare>(c1, l0, c0, r0, l1, r1, l2, c2, r2, rk);
    codes |= code << (4 * t);
    rc[li] = (uint8_t)code;
    l0 = l1; c0 = c1; r0 = r1;
    l1 = l2; c1 = c2; r1 = r2;
  }
  return codes;
}

// Geometry of tile b of the launch (tiles are visited in XCD-contiguous order).
struct TileGeo {
  int gi, y0, x0;
  bool inner;    // tile, ring and 2-cell halo inside the grid
  bool paired;   // inner, and every staged row starts 16-byte aligned
};

__device__ __forceinline__ TileGeo tile_geo(const StepArgs& a, int b) {
  TileGeo t;
  const int k = xcd_tile(b, a.ntiles);
  // Uniform over the workgroup: scalar registers, so the descriptor and
  // everything derived from it stay scalar.
  const int tile = __builtin_amdgcn_readfirstlane(a.w.tiles[k]);
  t.gi = __builtin_amdgcn_readfirstlane(a.w.tgrid[k]);
  const GridDev& G = a.grids[t.gi];
  const int lt = tile - G.tile_base;
  t.y0 = (lt / G.tiles_x) * kTH;
  t.x0 = (lt % G.tiles_x) * kTW;
  t.inner = t.y0 >= 2 && t.x0 >= 2 && t.y0 + kTH + 2 <= G.ny && t.x0 + kTW + 2 <= G.nx;
  t.paired = t.inner && (G.nx & 1) == 0 && ((G.offset + t.x0) & 1) == 0;
  return t;
}

// Staged heights of a paired tile as pairs of doubles, loaded by one thread.
constexpr int kPairs = kSW / 2;
constexpr int kPairTotal = kSH * kPairs;
constexpr int kPairLoads = (kPairTotal + kTileThreads - 1) / kTileThreads;

__device__ __forceinline__ void load_pairs(const double* hin, int nx, int y0, int x0, int tid,
                                           double2* v) {
#pragma unroll
  for (int j = 0; j < kPairLoads; ++j) {
    // Threads past the region reload its last pair (never stored), so that
    // every element is written and the array stays in registers.
    const int p = min(tid + j * kTileThreads, kPairTotal - 1);
    const int r = p / kPairs, cp = p - r * kPairs;
    v[j] = *(const double2*)(hin + (int64_t)(y0 - 2 + r) * nx + (x0 - 2) + 2 * cp);
  }
}

__device__ __forceinline__ void store_pairs(double* hs, int tid, const double2* v) {
#pragma unroll
  for (int j = 0; j < kPairLoads; ++j) {
    const int p = tid + j * kTileThreads;
    if (p < kPairTotal) {
      const int r = p / kPairs, cp = p - r * kPairs;
      *(double2*)(hs + r * kSW + 2 * cp) = v[j];
    }
  }
}

// One round of up to NS walks in lockstep (slot t active when bit t of act
// is set).  A walk's state is one word: its cell's LDS index (bits 0-15),
// that cell's code (16-19) and its steps so far (24-31).  A round moves each
// active walk to its cell's receiver and adds one to that receiver's count;
// a walk ends at a cell without a receiver, when the receiver is on the ring
// (bit t of exitm: it leaves the tile), or at kLocalDepthCap steps (then the
// whole tile goes to the crossing-tree passes: *all = 1).
constexpr int kLockRounds = 2;       // rounds in place before the survivors are gathered
constexpr uint32_t kWalkExit = 1u << 20;  // gathered state: the walk left the tile
template <int NS>
__device__ __forceinline__ void walk_round(uint32_t (&wk)[NS], uint32_t& act, uint32_t& exitm,
                                           const uint8_t* rc, uint32_t* clw, int* all) {
  uint32_t cu[NS];
  int un[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int v = (int)(wk[t] & 0xFFFFu);
    // A finished walk re-reads its own cell (in bounds, result unused).
    un[t] = ((act >> t) & 1u) ? v + lds_off((int)((wk[t] >> 16) & 15u)) : v;
    cu[t] = rc[un[t]];
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    if (!((act >> t) & 1u)) continue;
    const int u = un[t];
    if (cu[t] & kRingFlag) {
      exitm |= 1u << t;
      act &= ~(1u << t);
      continue;
    }
    atomicAdd(&clw[u >> 1], 1u << ((u & 1) * 16));
    const uint32_t d = (wk[t] >> 24) + 1u;
    wk[t] = (uint32_t)u | (cu[t] << 16) | (d << 24);
    if (cu[t] >= kSink) {
      act &= ~(1u << t);
    } else if (d >= (uint32_t)kLocalDepthCap) {
      *all = 1;
      act &= ~(1u << t);
    }
  }
}

__global__ __launch_bounds__(kTileThreads, 4) void k_tile_step(StepArgs a) {
  __shared__ __align__(16) double hs[kSN];  // heights, tile + 2-cell halo; new heights
  __shared__ uint32_t clw[kSN / 2];         // upstream counts, two 16-bit halves a word
  __shared__ uint32_t rc32[kSN / 4];        // receiver codes, tile and ring (ring: | kRingFlag)
  __shared__ __align__(8) uint32_t xr32[kSN / 4];  // per local root: its tree crosses the tile edge
  __shared__ double ftl[3 * kAmTab];        // F for small counts (scalar K), per distance class
  __shared__ __align__(4) uint16_t wlist[kTH * kTW];  // per wave: its cells of one level
  __shared__ int wsum[kTileThreads / 64];
  __shared__ int s_all, s_clean, s_cmax, s_base;
  uint8_t* rc = (uint8_t*)rc32;
  uint8_t* xr = (uint8_t*)xr32;

  const int tid = threadIdx.x, tx = tid % kTW, ty = tid / kTW, lane = tid & 63;
  const Work& w = a.w;
  const int sy0 = kStrip * ty;                // first strip row within the tile
  const int li0 = (sy0 + 2) * kSW + tx + 2;   // LDS index of the strip's first cell
  uint16_t* wl = wlist + (tid / 64) * (64 * kStrip);
  const bool clock = a.tile_clocks && tid == 0;  // per-phase device clock (LEM_F_TILE_CLOCKS)
  static_assert(3 * kAmTab <= 2 * kTileThreads, "at most two table entries per thread");
  const bool has_ft0 = tid < 3 * kAmTab, has_ft1 = tid + kTileThreads < 3 * kAmTab;
  {
    const TileGeo tg = tile_geo(a, blockIdx.x);
    const int gi = tg.gi, y0 = tg.y0, x0 = tg.x0;
    const bool inner = tg.inner;
    const GridDev& G = a.grids[gi];  // read through the scalar cache, not copied
    const int ny = G.ny, nx = G.nx;
    const int64_t off = G.offset;
    uint64_t tk[kTilePhases + 1];
    if (clock) tk[0] = wall_clock64();

    if (tid == 0) {
      s_all = 0;
      s_clean = 0;
      s_cmax = 0;
    }
    for (int i = tid; i < kSN / 2; i += kTileThreads) clw[i] = 0x00010001u;  // counts start at 1
    for (int i = tid; i < kSN / 4; i += kTileThreads) xr32[i] = 0u;
    // The grid's F table goes to LDS; its loads are issued first and stored
    // after the staging stores.
    const bool new_table = !a.Kf;
    double ft0 = 0.0, ft1 = 0.0;
    if (new_table) {
      if (has_ft0) ft0 = w.ftab[gi * 3 * kAmTab + tid];
      if (has_ft1) ft1 = w.ftab[gi * 3 * kAmTab + tid + kTileThreads];
    }

    // Heights of the tile and a 2-cell halo (positions outside the grid hold
    // 0 and are never used).  All loads are issued before the LDS stores.
    const double* hin = a.h_in + off;
    if (tg.paired) {
      double2 pr[kPairLoads];
      load_pairs(hin, nx, y0, x0, tid, pr);
      store_pairs(hs, tid, pr);
    } else {
      // Two rounds of loads then stores (one round's values in registers).
      constexpr int kN = (kSN + kTileThreads - 1) / kTileThreads, kHalf = (kN + 1) / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double v[kHalf];
#pragma unroll
        for (int j = 0; j < kHalf; ++j) {
          const int i = tid + (h * kHalf + j) * kTileThreads;
          const int r = i / kSW, cl = i - r * kSW;
          const int gy = y0 - 2 + r, gxh = x0 - 2 + cl;
          const bool in = i < kSN && gy >= 0 && gy < ny && gxh >= 0 && gxh < nx;
          v[j] = in ? hin[(int64_t)gy * nx + gxh] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kHalf; ++j) {
          const int i = tid + (h * kHalf + j) * kTileThreads;
          if (i < kSN) hs[i] = v[j];
        }
      }
    }
    if (new_table) {
      if (has_ft0) ftl[tid] = ft0;
      if (has_ft1) ftl[tid + kTileThreads] = ft1;
    }
    __syncthreads();
    if (clock) tk[1] = wall_clock64();

    // Step 2 / Algorithm 1: receiver codes of the thread's strip, then one
    // cell of the ring per thread.
    RecvConst rk;
    rk.dx = G.dx;
    rk.dy = G.dy;
    rk.dd = G.ddiag;
    rk.inv_dx = G.inv_dx;
    rk.inv_dy = G.inv_dy;
    rk.inv_dd = G.inv_dd;
    const bool square = G.square != 0;
    const int gx = x0 + tx;
    uint32_t codes = 0;
    if (a.fixed) {
#pragma unroll
      for (int t = 0; t < kStrip; ++t) {
        const int gy = y0 + sy0 + t;
        const uint32_t code = (gy < ny && gx < nx) ? w.rcode[off + (int64_t)gy * nx + gx] : kNone;
        codes |= code << (4 * t);
        rc[li0 + t * kSW] = (uint8_t)code;
      }
    } else if (square) {
      codes = strip_codes<true>(hs, rc, li0, rk, inner, y0 + sy0, gx, ny, nx);
    } else {
      codes = strip_codes<false>(hs, rc, li0, rk, inner, y0 + sy0, gx, ny, nx);
    }
    if (tid < kRing) {
      int ly, lx;  // ring cell within the tile's frame: rows -1 and kTH, columns -1 and kTW
      if (tid < kTW + 2) {
        ly = -1;
        lx = tid - 1;
      } else if (tid < 2 * (kTW + 2)) {
        ly = kTH;
        lx = tid - (kTW + 2) - 1;
      } else if (tid < 2 * (kTW + 2) + kTH) {
        ly = tid - 2 * (kTW + 2);
        lx = -1;
      } else {
        ly = tid - 2 * (kTW + 2) - kTH;
        lx = kTW;
      }
      const int li = (ly + 2) * kSW + lx + 2;
      const int gy = y0 + ly, gxr = x0 + lx;
      uint32_t code;
      if (gy < 0 || gy >= ny || gxr < 0 || gxr >= nx)
        code = kNone;
      else if (a.fixed)
        code = w.rcode[off + (int64_t)gy * nx + gxr];
      else if (gy == 0 || gxr == 0 || gy == ny - 1 || gxr == nx - 1)
        code = kBase;
      else if (square)
        code = receiver_code_at<true>(hs, li, kSW, rk);
      else
        code = receiver_code_at<false>(hs, li, kSW, rk);
      rc[li] = (uint8_t)(code | kRingFlag);
    }
    __syncthreads();
    if (clock) tk[2] = wall_clock64();

    // Step 3 / Algorithm 2: donor masks of the strip (neighbour k drains
    // here when its code is 7 - k), from a sliding window of the codes.
    uint64_t dms = 0;
    {
      uint32_t l0 = rc[li0 - kSW - 1] & 15u, c0 = rc[li0 - kSW] & 15u,
               r0 = rc[li0 - kSW + 1] & 15u;
      uint32_t l1 = rc[li0 - 1] & 15u, r1 = rc[li0 + 1] & 15u;
#pragma unroll
      for (int t = 0; t < kStrip; ++t) {
        const int li = li0 + t * kSW;
        const uint32_t l2 = rc[li + kSW - 1] & 15u, c2 = rc[li + kSW] & 15u,
                       r2 = rc[li + kSW + 1] & 15u;
        const uint32_t m = (uint32_t)(l0 == 7u) | ((uint32_t)(c0 == 6u) << 1) |
                           ((uint32_t)(r0 == 5u) << 2) | ((uint32_t)(l1 == 4u) << 3) |
                           ((uint32_t)(r1 == 3u) << 4) | ((uint32_t)(l2 == 2u) << 5) |
                           ((uint32_t)(c2 == 1u) << 6) | ((uint32_t)(r2 == 0u) << 7);
        dms |= (uint64_t)m << (8 * t);
        l0 = l1; c0 = (codes >> (4 * t)) & 15u; r0 = r1;
        l1 = l2; r1 = r2;
      }
    }

    // Steps 4-5 inside the tile: each cell walks down its receivers to its
    // tile-local root -- a cell without a receiver, or one whose receiver is
    // outside the tile -- adding one to the count of every cell it passes (a
    // cell's count = the cells upstream of it, itself included) and counting
    // its steps (its level in the local tree).  A tree crosses the tile edge
    // if its local root drains out of the tile or one of its border cells
    // has a donor outside; such trees are marked at their local root.  A
    // walk longer than kLocalDepthCap (a receiver cycle under fixed routing,
    // or a very deep tree) sends the whole tile to the crossing-tree passes.
    // The thread's eight walks advance one step per round, so their LDS
    // reads are in flight together.  A walk's state is one word: its cell
    // (bits 0-15), that cell's code (16-19) and its steps so far (24-31).
    uint32_t wk[kStrip];
    uint32_t act = 0, exitm = 0;
#pragma unroll
    for (int t = 0; t < kStrip; ++t) {
      const uint32_t cv = (codes >> (4 * t)) & 15u;
      wk[t] = (uint32_t)(li0 + t * kSW) | (cv << 16);
      act |= (uint32_t)(cv < kSink) << t;
    }
    // Tile-local trees are shallow: after the first rounds only a few walks
    // of the wave's 512 are still going (about 44 on a noise raster), and
    // the eight slots of a lane would mostly idle.  Once at most 128 remain
    // (checked every kLockRounds rounds), the wave gathers them into a list
    // in LDS (its erosion-list space, unused until the erosion), finishes
    // them two to a lane, and each owner reads its walks' final states back
    // (bit kWalkExit: the walk left the tile).
    for (;;) {
      for (int r = 0; r < kLockRounds && act; ++r)
        walk_round<kStrip>(wk, act, exitm, rc, clw, &s_all);
      const int na = __popc(act);
      const int incl = wave_inclusive_scan(na);
      const int total = __builtin_amdgcn_readlane(incl, 63);
      if (total == 0) break;
      if (total > 2 * 64) continue;
      uint32_t* lst = (uint32_t*)wl;
      int p = incl - na;
#pragma unroll
      for (int t = 0; t < kStrip; ++t)
        if ((act >> t) & 1u) lst[p++] = wk[t];
      __builtin_amdgcn_wave_barrier();
      uint32_t tw[2] = {0u, 0u}, tact = 0, texit = 0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int e = lane + 64 * j;
        if (e < total) {
          tw[j] = lst[e];
          tact |= 1u << j;
        }
      }
      while (tact) walk_round<2>(tw, tact, texit, rc, clw, &s_all);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int e = lane + 64 * j;
        if (e < total) lst[e] = tw[j] | (((texit >> j) & 1u) ? kWalkExit : 0u);
      }
      __builtin_amdgcn_wave_barrier();
      p = incl - na;
#pragma unroll
      for (int t = 0; t < kStrip; ++t)
        if ((act >> t) & 1u) {
          const uint32_t v = lst[p++];
          wk[t] = v;
          exitm |= (uint32_t)((v & kWalkExit) != 0u) << t;
        }
      break;
    }
    uint64_t deps = 0;
    uint32_t roots[kStrip / 2];
#pragma unroll
    for (int t = 0; t < kStrip; ++t) {
      const int v = (int)(wk[t] & 0xFFFFu);
      // Outward directions of a border cell: 0-2 (top row), 5-7 (bottom
      // row), 0, 3, 5 (left column), 2, 4, 7 (right column).
      const int sy = sy0 + t;
      const uint32_t out = (sy == 0 ? 0x07u : 0u) | (sy == kTH - 1 ? 0xE0u : 0u) |
                           (tx == 0 ? 0x29u : 0u) | (tx == kTW - 1 ? 0x94u : 0u);
      if (((exitm >> t) & 1u) || (((dms >> (8 * t)) & out) != 0)) xr[v] = 1;
      deps |= (uint64_t)(wk[t] >> 24) << (8 * t);
      if (t & 1)
        roots[t >> 1] |= (uint32_t)v << 16;
      else
        roots[t >> 1] = (uint32_t)v;
    }
    __syncthreads();
    if (clock) tk[3] = wall_clock64();

    // Cells of trees that stay in the tile ("clean") and their deepest
    // level; the roots of the other trees are counted and their queue slots
    // reserved now (the atomic's reply is first needed at write-back).
    const uint32_t all_ok = s_all ? 0u : 0xFFu;
    uint32_t clean = 0, my_max = 0, root_bits = 0;
#pragma unroll
    for (int t = 0; t < kStrip; ++t) {
      const int r = (roots[t >> 1] >> (16 * (t & 1))) & 0xFFFF;
      const uint32_t code = (codes >> (4 * t)) & 15u;
      const uint32_t ok = (uint32_t)(code != kNone) & (uint32_t)(xr[r] == 0) & all_ok;
      clean |= ok << t;
      const uint32_t d = (uint32_t)((deps >> (8 * t)) & 0xFFu);
      my_max = max(my_max, ok ? d : 0u);
      root_bits |= (uint32_t)(!ok && code >= kSink && code != kNone) << t;
    }
    // Wave totals: lane 63 of the inclusive scans.
    const int wave_clean = __builtin_amdgcn_readlane(wave_inclusive_scan(__popc(clean)), 63);
    const int wave_max = __builtin_amdgcn_readlane((int)wave_inclusive_max(my_max), 63);
    if (lane == 0) {
      atomicMax(&s_cmax, wave_max);
      atomicAdd(&s_clean, wave_clean);
    }
    // Roots go to the grid's own queue slice for the per-grid level pass, to
    // the one shared queue otherwise (the chunk stage takes them from there).
    const bool pergrid_roots = a.pergrid && !a.chunked;
    int nroots_tile;
    const int root_pre = block_exclusive_scan<kTileThreads>(__popc(root_bits), wsum, &nroots_tile);
    int root_base = 0;
    if (tid == 0 && nroots_tile)
      root_base = atomicAdd(pergrid_roots ? &w.gcnt[gi] : &w.lcnt[0], nroots_tile);
    // Donor masks of the tile, row-major in the crossing flags' LDS (free
    // now), so that no register holds them through the erosion and rows can
    // be stored 8 bytes at a time at write-back.
    const bool wide_masks = inner && ((off + x0) & 7) == 0 && (nx & 7) == 0;
#pragma unroll
    for (int t = 0; t < kStrip; ++t) xr[(sy0 + t) * kTW + tx] = (uint8_t)((dms >> (8 * t)) & 0xFFu);
    if (clock) tk[4] = wall_clock64();

    // Steps 6-7 for clean trees, level by level from the roots outward.
    // Interior roots are only uplifted (at write-back: their level-1 donors
    // add the uplift to the root's height themselves, and nothing else reads
    // a root's new height).  Each wave compacts its cells of the level into
    // a list in LDS and spreads it over its 64 lanes.  F comes from the
    // grid's table staged in LDS (scalar K, n = 1, counts below kAmTab) or
    // from eroded_height_general.
    const bool table_f = !a.Kf && !G.newton;
    const bool need_c = a.Kf || a.Uf || !table_f;
    const int cmax = s_cmax;
    // Read once here: the loop below contains a call, which keeps the
    // compiler from hoisting these loads out of it.
    const double g_dt = G.dt, g_udt = G.udt;
    for (int l = 1; l <= cmax; ++l) {
      // The levels pass through an empty asm so that their bytes are not
      // extracted once before the loop and held (spilled) through it.
      uint64_t dl = deps;
      asm volatile("" : "+v"(dl));
      uint32_t at = 0;
#pragma unroll
      for (int t = 0; t < kStrip; ++t)
        at |= (uint32_t)(((dl >> (8 * t)) & 0xFFu) == (uint64_t)l) << t;
      at &= clean;
      const int cnt = __popc(at);
      const int incl = wave_inclusive_scan(cnt);
      const int total = __builtin_amdgcn_readlane(incl, 63);
      int pos = incl - cnt;
      // List entries: the cell's LDS index (bits 0-12) and its code (13-15).
      while (at) {
        const int t = __ffs(at) - 1;
        at &= at - 1;
        wl[pos++] = (uint16_t)((li0 + t * kSW) | (((codes >> (4 * t)) & 7u) << 13));
      }
      __builtin_amdgcn_wave_barrier();
      // New height of the cell of list entry e.
      auto erode = [&](uint32_t e) -> double {
        const int li = (int)(e & 0x1FFFu);
        const int code = (int)(e >> 13);
        const int u = li + lds_off(code);
        int64_t c = 0;
        if (need_c) {
          const int row = li / kSW;
          c = off + (int64_t)(y0 + row - 2) * nx + (x0 + (li - row * kSW) - 2);
        }
        double hr = hs[u];
        if (l == 1 && rc[u] == kSink)  // the receiver is an interior root: add its uplift
          hr = hr + (a.Uf ? a.Uf[c + neighbour_offset(code, nx)] * g_dt : g_udt);
        const uint32_t count = (clw[li >> 1] >> ((li & 1) * 16)) & 0xFFFFu;
        const double udt = a.Uf ? a.Uf[c] * g_dt : g_udt;
        const double h0 = hs[li] + udt;
        if (table_f && count < (uint32_t)kAmTab) {
          const double f = ftl[code_class(code) * kAmTab + count];
          if (a.project) return f > 0.0 ? hr + udt / f : h0;
          const double g = 1.0 + f;
          return (h0 + f * hr) / g;
        }
        return eroded_height_general(a.grids, gi, a.Kf, w.amtab, count, code, c, h0, hr,
                                     a.project, udt);
      };
      for (int j = lane; j < total; j += 64) {
        const uint32_t e0 = wl[j];
        hs[e0 & 0x1FFFu] = erode(e0);
      }
      __syncthreads();
    }
    if (clock) tk[5] = wall_clock64();

    // Write the tile back (heights of crossing trees unchanged here: the
    // crossing-tree passes read their starting heights from the output
    // buffer, so that a cell's read and its later write share one cache
    // line, and overwrite them); queue the roots of crossing trees.
    // Addresses are formed here, from a column index the compiler cannot
    // trace back (an empty asm), so that they are not computed early and
    // kept through the erosion.
    int gx_wb = gx, li0_wb = li0;
    asm volatile("" : "+v"(gx_wb), "+v"(li0_wb));
    const int64_t cw = off + (int64_t)(y0 + sy0) * nx + gx_wb;
#pragma unroll
    for (int t = 0; t < kStrip; ++t) {
      const int li = li0_wb + t * kSW;
      const uint32_t code = rc[li];
      if (code == kNone) continue;
      const int64_t c = cw + (int64_t)t * nx;
      const bool cl = (clean >> t) & 1u;
      double hv = hs[li];
      if (cl && code == kSink) hv = hv + (a.Uf ? a.Uf[c] * g_dt : g_udt);
      a.h_out[c] = hv;
      if (!wide_masks) w.dmask[c] = xr[(sy0 + t) * kTW + tx];
      if (a.export_routing) {
        if (cl) {
          w.dep_g[c] = (int32_t)((deps >> (8 * t)) & 0xFFu);
          w.cnt_g[c] = (clw[li >> 1] >> ((li & 1) * 16)) & 0xFFFFu;
        }
        if (!a.fixed) w.rcode[c] = (uint8_t)code;
      }
    }
    if (tid == 0) s_base = root_base;
    __syncthreads();
    if (wide_masks) {
      static_assert(kTH * kTW == 8 * kTileThreads, "eight mask bytes per thread");
      const int r = tid / (kTW / 8), cb = (tid % (kTW / 8)) * 8;
      *(uint64_t*)(w.dmask + off + (int64_t)(y0 + r) * nx + x0 + cb) =
          *(const uint64_t*)(xr + r * kTW + cb);
    }
    int pos = (pergrid_roots ? (int)off : 0) + s_base + root_pre;
    while (root_bits) {
      const int t = __ffs(root_bits) - 1;
      root_bits &= root_bits - 1;
      w.q[pos] = (int32_t)(cw + (int64_t)t * nx);
      w.gq[pos] = (uint16_t)gi;
      w.par[pos] = -1;
      w.kq[pos] = rc[li0_wb + t * kSW];
      ++pos;
    }
    if (tid == 0 && s_clean) {
      atomicAdd(&w.ctrl->clean, s_clean);
      atomicMax(&w.ctrl->clean_maxdepth, s_cmax);
    }
    if (clock) {
      tk[6] = wall_clock64();
      for (int k = 0; k < kTilePhases; ++k)
        atomicAdd((unsigned long long*)&w.ctrl->tile_ticks[k],
                  (unsigned long long)(tk[k + 1] - tk[k]));
      atomicAdd((unsigned long long*)&w.ctrl->tile_wgs, 1ull);
    }
  }
}

// ---------------------------------------------------------------------------
// Crossing trees: Steps 4 to 7 over the whole grid in one cooperative launch.

// Grid-wide barrier: arrival counter plus generation word on separate cache
// lines, agent-scope release on arrival and acquire on departure.  The wait
// is bounded; a timeout raises LEM_E_HIP on the device instead of hanging.
__device__ __forceinline__ void grid_barrier(Ctrl* ct) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t g0 = __hip_atomic_load(&ct->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(&ct->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(&ct->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ct->bar_gen, g0 + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&ct->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins == kSpinLimit) {
          atomicMax(&ct->status, 6);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// Breadth-first expansion of queue positions [lo, hi) (level L) by
// workgroups wg of nwg: the donors of each position are appended after hi,
// in the order of the positions (block_scan_items), so cells that are
// neighbours in one level have their donors next to each other in the next
// and the gathers of later levels stay local.
template <int ITEMS>
__device__ void expand_level(const StepArgs& a, int32_t lo, int32_t hi, int32_t L, int wg,
                             int nwg, uint64_t* wsum64, int* s_base) {
  const Work& w = a.w;
  const int tid = threadIdx.x;
  constexpr int W = ITEMS / 4, CHUNK = kBlock * ITEMS;
  for (int64_t base = lo + (int64_t)wg * CHUNK; base < hi; base += (int64_t)nwg * CHUNK) {
    uint32_t mk[W] = {};  // donor masks, four to a word
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + (int64_t)j * kBlock + tid;
      if (i < hi) {
        const uint32_t m = w.dmask[w.q[i]];
        mk[j >> 2] |= m << (8 * (j & 3));
      }
    }
    uint64_t v[W], pre[W], tot[W];
#pragma unroll
    for (int g = 0; g < W; ++g) v[g] = counts_of_masks(mk[g]);
    block_scan_items<kBlock, W>(v, wsum64, pre, tot);
    const int total = items_total<W>(tot);
    if (tid == 0) *s_base = total ? atomicAdd(&w.lcnt[L + 1], total) : 0;
    __syncthreads();
    int32_t run = hi + *s_base;
    // Groups of four items, not unrolled: keeps the re-reads below from being
    // hoisted (register pressure); the selects avoid indexing registers at run time.
#pragma unroll 1
    for (int g = 0; g < W; ++g) {
      uint64_t pg = pre[0], tg = tot[0];
      uint32_t mg = mk[0];
#pragma unroll
      for (int k = 1; k < W; ++k)
        if (g == k) pg = pre[k], tg = tot[k], mg = mk[k];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = base + (int64_t)(4 * g + e) * kBlock + tid;
        int32_t pos = run + item_field(pg, e);
        run += item_field(tg, e);
        if (i < hi) {
          uint32_t m = (mg >> (8 * e)) & 0xFFu;
          w.mq[i] = (uint8_t)m;
          w.fc[i] = pos;
          if (m) {
            const uint32_t gi = w.gq[i];
            const int nx = a.grids[gi].nx;
            const int32_t c = w.q[i];  // re-read: cheaper than keeping every item's cell live
            while (m) {
              const int b = __ffs(m) - 1;
              m &= m - 1;
              w.q[pos] = (int32_t)(c + neighbour_offset(b, nx));
              w.gq[pos] = (uint16_t)gi;
              w.par[pos] = (int32_t)i;
              w.kq[pos] = (uint8_t)(7 - b);
              ++pos;
            }
          }
        }
      }
    }
  }
}

// Step 5 for queue positions [a0, a1): count = 1 + the donors' counts.  A
// thread takes two positions at a time (a level of a deep grid has a few
// thousand cells and one workgroup): their loads are in flight together.
template <int NT = kBlock>
__device__ __forceinline__ void accumulate_level(const Work& w, int32_t a0, int32_t a1, int wg,
                                                 int nwg) {
  const int64_t stride = (int64_t)nwg * NT;
  for (int64_t i0 = a0 + (int64_t)wg * NT + threadIdx.x; i0 < a1; i0 += 2 * stride) {
    const int64_t ii[2] = {i0, i0 + stride};
    uint32_t m[2] = {0u, 0u};
    int32_t f[2] = {0, 0};
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ii[e] < a1) {
        m[e] = w.mq[ii[e]];
        f[e] = w.fc[ii[e]];
      }
    uint32_t s[2] = {1u, 1u};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = __popc(m[e]);
      for (int j = 0; j < k; ++j) s[e] += w.cnt[f[e] + j];
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ii[e] < a1) w.cnt[ii[e]] = s[e];
  }
}

// Steps 6-7 for queue positions [a0, a1) of a level >= 1.
template <int NT = kBlock>
__device__ __forceinline__ void erode_level(const StepArgs& a, int32_t a0, int32_t a1, int wg,
                                            int nwg) {
  const Work& w = a.w;
  for (int64_t i = a0 + (int64_t)wg * NT + threadIdx.x; i < a1;
       i += (int64_t)nwg * NT) {
    const int32_t c = w.q[i];
    const int gi = w.gq[i];
    const GridDev& G = a.grids[gi];
    const double hr = w.hq[w.par[i]];
    double f, g;
    erosion_factor(a, G, gi, w.cnt[i], w.kq[i], c, &f, &g);
    const double udt = a.Uf ? a.Uf[c] * G.dt : G.udt;
    const double h0 = a.h_out[c] + udt;
    const double hn = new_height(G, a.project != 0, h0, hr, f, g, udt);
    w.hq[i] = hn;
    a.h_out[c] = hn;
  }
}

// End of a step's crossing-tree work (one thread): the step's level count
// and statistics from the tile pass, the chunk stage (when it ran) and the
// level pass that ran last (`cross_total` cells in `nl_cross` levels, of
// which `glob_total` sit in the global queue for the routing export), then
// the per-step counters are cleared for the next step.
__device__ void finish_step(const StepArgs& a, Ctrl* ct, int64_t cross_total, int32_t nl_cross,
                            int32_t glob_total) {
  const Work& w = a.w;
  int64_t total = cross_total;
  if (a.chunked) {
    total += ct->chunk_total;
    nl_cross = nl_cross > ct->chunk_nl ? nl_cross : ct->chunk_nl;
  }
  const int32_t clean = ct->clean;
  const int32_t nl_clean = clean ? ct->clean_maxdepth + 1 : 0;
  const int32_t nl = nl_clean > nl_cross ? nl_clean : nl_cross;
  ct->nlevels = nl;
  ct->dirty_total = (int32_t)total;
  ct->glob_total = glob_total;
  ct->crossing_run += total;
  if (nl > ct->max_nlevels) ct->max_nlevels = nl;
  if (a.step < kHistCap) w.hist[a.step] = nl;
  ct->steps = a.step + 1;
  if ((int64_t)clean + total != (int64_t)a.n) atomicMax(&ct->status, 5);
  ct->clean = 0;
  ct->clean_maxdepth = 0;
  ct->chunk_total = 0;
  ct->chunk_nl = 0;
  ct->chunk_next = 0;
  ct->ovf_count = 0;
  w.lcnt[0] = 0;
  w.lcnt[1] = 0;
}

__global__ __launch_bounds__(kBlock) void k_global_levels(StepArgs a) {
  __shared__ uint64_t wsum64[4 * kBlock / 64 + 4];
  __shared__ int s_base;
  const Work w = a.w;
  Ctrl* ct = w.ctrl;
  const int tid = threadIdx.x;
  const int wg = blockIdx.x, nwg = gridDim.x;
  const bool lead = (wg == 0 && tid == 0);
  uint64_t t0 = 0, t1 = 0, t2 = 0;
  if (lead && a.timers) t0 = wall_clock64();

  // Breadth-first levels.  Cells appended to level L+1 are counted in
  // lcnt[L+1]; the workgroup-0 lead clears lcnt[L+2] while level L runs
  // (nobody else touches it then) and records lev[L+1].
  int32_t lo = 0, hi = load_acquire(&w.lcnt[0]), L = 0;
  if (a.chunked) {
    // The chunk stage finished most trees; the roots of the chunks it could
    // not hold were staged behind the chunk roots.  Move them to the front.
    const int32_t novf = ct->ovf_count;
    if (novf == 0) {
      if (lead) {
        ct->dirty_nlevels = 0;
        finish_step(a, ct, 0, 0, 0);
      }
      return;
    }
    for (int64_t j = (int64_t)wg * kBlock + tid; j < novf; j += (int64_t)nwg * kBlock) {
      w.q[j] = w.q[hi + j];
      w.gq[j] = w.gq[hi + j];
      w.kq[j] = w.kq[hi + j];
      w.par[j] = -1;
    }
    grid_barrier(ct);
    hi = novf;
  }
  bool done = false;
  if (lead) w.lev[0] = 0;
  while (!done) {
    if (hi - lo >= a.tail_level) {
      if (lead) {
        w.lev[L + 1] = hi;
        w.lcnt[L + 2] = 0;
      }
      expand_level<kExpandItems>(a, lo, hi, L, wg, nwg, wsum64, &s_base);
      grid_barrier(ct);
      const int32_t added = load_acquire(&w.lcnt[L + 1]);
      if (added == 0) {
        done = true;
      } else {
        lo = hi;
        hi += added;
        ++L;
      }
    } else {
      // Small levels: workgroup 0 continues alone until a level grows past
      // the threshold again or the queue ends.
      if (wg == 0) {
        int32_t tlo = lo, thi = hi, tL = L;
        bool tdone = false;
        while (true) {
          if (tid == 0) {
            w.lev[tL + 1] = thi;
            w.lcnt[tL + 2] = 0;
          }
          expand_level<kExpandItems>(a, tlo, thi, tL, 0, 1, wsum64, &s_base);
          __syncthreads();
          const int32_t added = load_acquire(&w.lcnt[tL + 1]);
          __syncthreads();
          if (added == 0) {
            tdone = true;
            break;
          }
          tlo = thi;
          thi += added;
          ++tL;
          if (thi - tlo >= a.tail_level) break;
        }
        if (tid == 0) {
          ct->tail_lo = tlo;
          ct->tail_hi = thi;
          ct->tail_L = tL;
          ct->tail_done = tdone ? 1 : 0;
        }
      }
      grid_barrier(ct);
      lo = __hip_atomic_load(&ct->tail_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hi = __hip_atomic_load(&ct->tail_hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      L = __hip_atomic_load(&ct->tail_L, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      done = __hip_atomic_load(&ct->tail_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
  }
  const int32_t nlevels = L + 1;
  const int32_t total = hi;
  if (lead && a.timers) t1 = wall_clock64();

  // Step 5: counts, deepest level first, down to level 1.
  for (int32_t l = nlevels - 1; l >= 1;) {
    if (w.lev[l + 1] - w.lev[l] >= a.tail_level) {
      accumulate_level(w, w.lev[l], w.lev[l + 1], wg, nwg);
      grid_barrier(ct);
      --l;
    } else {
      int32_t l2 = l;
      while (l2 >= 1 && w.lev[l2 + 1] - w.lev[l2] < a.tail_level) --l2;
      if (wg == 0) {
        for (int32_t k = l; k > l2; --k) {
          accumulate_level(w, w.lev[k], w.lev[k + 1], 0, 1);
          __syncthreads();
        }
      }
      grid_barrier(ct);
      l = l2;
    }
  }
  // Level 0: counts of the roots, and uplift of the interior roots.
  {
    const int32_t a1 = w.lev[1];
    accumulate_level(w, 0, a1, wg, nwg);
    for (int64_t i = (int64_t)wg * kBlock + tid; i < a1; i += (int64_t)nwg * kBlock) {
      const int32_t c = w.q[i];
      double hv = a.h_out[c];
      if (w.kq[i] == kSink) {
        const GridDev& G = a.grids[w.gq[i]];
        hv = hv + (a.Uf ? a.Uf[c] * G.dt : G.udt);
      }
      a.h_out[c] = hv;
      w.hq[i] = hv;
    }
  }
  if (lead && a.timers) t2 = wall_clock64();

  // Steps 6-7, levels 1 and up, from the roots outward.
  for (int32_t l = 1; l < nlevels;) {
    grid_barrier(ct);
    if (w.lev[l + 1] - w.lev[l] >= a.tail_level) {
      erode_level(a, w.lev[l], w.lev[l + 1], wg, nwg);
      ++l;
    } else {
      int32_t l2 = l;
      while (l2 < nlevels && w.lev[l2 + 1] - w.lev[l2] < a.tail_level) ++l2;
      if (wg == 0) {
        for (int32_t k = l; k < l2; ++k) {
          erode_level(a, w.lev[k], w.lev[k + 1], 0, 1);
          __syncthreads();
        }
      }
      l = l2;
    }
  }

  if (lead) {
    const int32_t nl_cross = total ? nlevels : 0;
    ct->dirty_nlevels = nl_cross;
    finish_step(a, ct, total, nl_cross, total);
    if (a.timers) {
      const uint64_t t3 = wall_clock64();
      ct->ticks[1] += t1 - t0;
      ct->ticks[2] += t2 - t1;
      ct->ticks[3] += t3 - t2;
    }
  }
}

// ---------------------------------------------------------------------------
// Crossing trees of a batch, one workgroup per grid.  Each grid's roots sit
// in its own region of the queue ([offset, offset + cells), appended by the
// tile pass), and its levels are separated by workgroup barriers only, so
// grids proceed independently and no device-wide barrier is needed.  Level
// offsets go to lev[offset + 2*grid ...] (at most cells + 1 of them).

// Breadth-first expansion of positions [lo, hi) by one workgroup: donors are
// appended at *s_next, which advances.
template <int NT>
__device__ void expand_level_wg(const StepArgs& a, int32_t lo, int32_t hi, int* wsum,
                                int32_t* s_next) {
  const Work& w = a.w;
  const int tid = threadIdx.x;
  for (int64_t base = lo; base < hi; base += (int64_t)NT * kItems) {
    int32_t cs[kItems];
    uint32_t ms[kItems];
    int cntv = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t i = base + (int64_t)j * NT + tid;
      cs[j] = 0;
      ms[j] = 0;
      if (i < hi) {
        cs[j] = w.q[i];
        const uint32_t m = w.dmask[cs[j]];
        ms[j] = m | ((uint32_t)w.gq[i] << 8);
        cntv += __popc(m);
      }
    }
    int tot;
    const int pre = block_exclusive_scan<NT>(cntv, wsum, &tot);
    const int32_t start = *s_next;
    int32_t pos = start + pre;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t i = base + (int64_t)j * NT + tid;
      if (i < hi) {
        uint32_t m = ms[j] & 0xFFu;
        const uint32_t gi = ms[j] >> 8;
        w.mq[i] = (uint8_t)m;
        w.fc[i] = pos;
        if (m) {
          const int nx = a.grids[gi].nx;
          while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1;
            w.q[pos] = (int32_t)(cs[j] + neighbour_offset(b, nx));
            w.gq[pos] = (uint16_t)gi;
            w.par[pos] = (int32_t)i;
            w.kq[pos] = (uint8_t)(7 - b);
            ++pos;
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0) *s_next = start + tot;
    __syncthreads();
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_grid_levels(StepArgs a) {
  __shared__ int wsum[NT / 64];
  __shared__ int32_t s_next;
  __shared__ uint64_t s_tk[3];
  const Work w = a.w;
  const int gi = blockIdx.x;
  const int tid = threadIdx.x;
  const GridDev& G = a.grids[gi];
  const int32_t nroots = w.gcnt[gi];
  if (nroots == 0) {
    if (tid == 0) {
      w.gnl[gi] = 0;
      w.gtot[gi] = 0;
    }
    return;
  }
  const int32_t base = (int32_t)G.offset;
  int32_t* lev = w.lev + G.offset + 2 * (int64_t)gi;
  // Phase clocks (LEM_F_PHASE_TIMERS) live in LDS, not in registers.
  const bool clock = a.timers && tid == 0;
  if (clock) s_tk[0] = wall_clock64();
  if (a.chunked) {
    // Roots of the chunks the chunk stage could not hold, staged in fc/mq.
    for (int32_t j = tid; j < nroots; j += NT) {
      w.q[base + j] = w.fc[base + j];
      w.kq[base + j] = w.mq[base + j];
      w.gq[base + j] = (uint16_t)gi;
      w.par[base + j] = -1;
    }
    __syncthreads();
  }
  int32_t lo = base, hi = base + nroots, L = 0;
  if (tid == 0) {
    lev[0] = lo;
    s_next = hi;
  }
  __syncthreads();
  // Step 4: levels from the roots outward.
  while (true) {
    if (tid == 0) lev[L + 1] = hi;
    expand_level_wg<NT>(a, lo, hi, wsum, &s_next);
    const int32_t nh = s_next;
    if (nh == hi) break;
    lo = hi;
    hi = nh;
    ++L;
  }
  __syncthreads();
  if (clock) s_tk[1] = wall_clock64();
  // Step 5: counts, deepest level first.
  for (int32_t l = L; l >= 0; --l) {
    accumulate_level<NT>(w, lev[l], lev[l + 1], 0, 1);
    __syncthreads();
  }
  if (clock) s_tk[2] = wall_clock64();
  // Level 0: uplift of the interior roots (perimeter roots keep their height).
  for (int32_t i = lev[0] + tid; i < lev[1]; i += NT) {
    const int32_t c = w.q[i];
    double hv = a.h_out[c];
    if (w.kq[i] == kSink) hv = hv + (a.Uf ? a.Uf[c] * G.dt : G.udt);
    a.h_out[c] = hv;
    w.hq[i] = hv;
  }
  __syncthreads();
  // Steps 6-7, levels 1 and up.
  for (int32_t l = 1; l <= L; ++l) {
    erode_level<NT>(a, lev[l], lev[l + 1], 0, 1);
    __syncthreads();
  }
  if (a.export_routing) {
    for (int32_t l = 0; l <= L; ++l)
      for (int32_t i = lev[l] + tid; i < lev[l + 1]; i += NT) {
        const int32_t c = w.q[i];
        w.dep_g[c] = l;
        w.cnt_g[c] = w.cnt[i];
      }
  }
  if (tid == 0) {
    w.gcnt[gi] = 0;
    w.gnl[gi] = L + 1;
    w.gtot[gi] = hi - base;
  }
  if (clock) {
    const uint64_t tk3 = wall_clock64();
    Ctrl* ct = w.ctrl;
    atomicMax((unsigned long long*)&ct->grid_phase_max[0], (unsigned long long)(s_tk[1] - s_tk[0]));
    atomicMax((unsigned long long*)&ct->grid_phase_max[1], (unsigned long long)(s_tk[2] - s_tk[1]));
    atomicMax((unsigned long long*)&ct->grid_phase_max[2], (unsigned long long)(tk3 - s_tk[2]));
  }
}

// After the per-grid level pass: the step's statistics (as the global pass
// records them) from the per-grid results.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_grid_levels_finish(StepArgs a) {
  __shared__ int32_t smax[1024];
  __shared__ long long ssum[1024];
  const Work w = a.w;
  int32_t mx = 0;
  long long sum = 0;
  for (int g = threadIdx.x; g < a.ngrids; g += 1024) {
    mx = max(mx, w.gnl[g]);
    sum += w.gtot[g];
  }
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = sum;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + s]);
      ssum[threadIdx.x] += ssum[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Ctrl* ct = w.ctrl;
    ct->dirty_nlevels = smax[0];
    finish_step(a, ct, ssum[0], smax[0], 0);
    if (a.timers)
      for (int k = 0; k < 3; ++k) {
        ct->ticks[k + 1] += ct->grid_phase_max[k];
        ct->grid_phase_max[k] = 0;
      }
  }
}


// ---------------------------------------------------------------------------
// Crossing trees, chunk stage.  The tile pass queued the root of every tree
// that crosses a tile edge (q[0, lcnt[0]), tile by tile).  Such trees are
// small on the paper's workloads (about a dozen cells on average), so a
// workgroup takes a chunk of consecutive roots from a device work counter
// and carries out Steps 4-7 for their whole trees in LDS: breadth-first
// levels (Algorithm 3; each level's cells gather their donor masks and
// starting heights from HBM), counts from the deepest level up
// (Algorithm 4; each cell adds its count to its receiver's), then uplift
// and the implicit update from the roots outward (Algorithms 5-6).  Only
// workgroup barriers separate levels, so chunks proceed independently.  A
// chunk whose trees need more than kChunkCap cells or kChunkLevCap levels
// writes nothing; its roots are staged for the level pass that follows
// (the global pass: behind the chunk roots in q/gq/kq; the per-grid pass:
// in the grid's slice of fc/mq), which orders those trees as before.
template <bool kMulti>
__global__ __launch_bounds__(kChunkThreads, 4) void k_chunk_trees(StepArgs a) {
  constexpr int NT = kChunkThreads;
  __shared__ int32_t s_cell[kChunkCap];      // cell of each entry, level-major
  __shared__ double s_h[kChunkCap];          // uplifted start height, then new height
  __shared__ uint16_t s_par[kChunkCap];      // entry of the receiver
  __shared__ uint16_t s_grid[kMulti ? kChunkCap : 1];  // grid of the entry (batches)
  __shared__ uint32_t s_cnt[kChunkCap / 2];  // upstream counts, two 16-bit halves a word
  __shared__ uint8_t s_k[kChunkCap];         // receiver code (roots: kSink or kBase)
  __shared__ uint16_t s_lev[kChunkLevCap + 2];
  __shared__ int wsum[NT / 64];
  __shared__ int s_chunk, s_slot;
  static_assert(kChunkCap < 65536, "16-bit entries and counts");

  const Work w = a.w;
  Ctrl* ct = w.ctrl;
  const int tid = threadIdx.x;
  const int32_t nroots = w.lcnt[0];  // final: written by the tile pass
  const int R = a.chunk_roots;
  constexpr bool multi = kMulti;  // a batch: entries carry their grid
  int64_t my_total = 0;
  int32_t my_nl = 0;
  uint64_t tk[3] = {0, 0, 0};
  const bool clock = a.timers && blockIdx.x == 0 && tid == 0;
  // One grid: its descriptor fields read once (inside the loops below, which
  // contain a call, the compiler would reload them for every entry).
  const GridDev& G0 = a.grids[0];
  const double g0_dt = G0.dt, g0_udt = G0.udt;
  const int g0_nx = G0.nx;
  const bool g0_newton = G0.newton != 0;

  for (;;) {
    if (tid == 0) s_chunk = atomicAdd(&ct->chunk_next, 1);
    __syncthreads();
    const int64_t r0 = (int64_t)s_chunk * R;
    if (r0 >= nroots) break;
    const int nr = (int)(nroots - r0 < R ? nroots - r0 : R);
    uint64_t t0 = clock ? wall_clock64() : 0;

    // Level 0: the chunk's roots.  Every count starts at 1 (the cell itself).
    for (int j = tid; j < kChunkCap / 2; j += NT) s_cnt[j] = 0x00010001u;
    for (int j = tid; j < nr; j += NT) {
      s_cell[j] = w.q[r0 + j];
      s_k[j] = w.kq[r0 + j];
      if (multi) s_grid[j] = w.gq[r0 + j];
    }
    if (tid == 0) {
      s_lev[0] = 0;
      s_lev[1] = (uint16_t)nr;
    }
    __syncthreads();

    // Step 4: breadth-first levels.  Each entry of level L gathers its donor
    // mask and its height (uplifted unless it is a perimeter root) and
    // appends its donors, in the order of the entries.
    int lo = 0, hi = nr, next = nr, L = 0;
    bool ovf = false;
    for (;;) {
      for (int base = lo; base < hi; base += NT) {
        const int i = base + tid;
        uint32_t m = 0;
        int32_t c = 0;
        int g = 0;
        if (i < hi) {
          c = s_cell[i];
          g = multi ? s_grid[i] : 0;
          m = w.dmask[c];
          double hv = a.h_out[c];
          if (s_k[i] != kBase)
            hv = hv + (a.Uf ? a.Uf[c] * (multi ? a.grids[g].dt : g0_dt)
                            : (multi ? a.grids[g].udt : g0_udt));
          s_h[i] = hv;
        }
        int tot;
        const int pre = block_exclusive_scan<NT>(__popc(m), wsum, &tot);
        if (next + tot > kChunkCap) {  // tot is the same in every thread
          ovf = true;
          break;
        }
        if (m) {
          const int nx = multi ? a.grids[g].nx : g0_nx;
          int pos = next + pre;
          while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1;
            s_cell[pos] = (int32_t)(c + neighbour_offset(b, nx));
            s_par[pos] = (uint16_t)i;
            if (multi) s_grid[pos] = (uint16_t)g;
            s_k[pos] = (uint8_t)(7 - b);
            ++pos;
          }
        }
        next += tot;
      }
      if (ovf) break;
      __syncthreads();
      if (next == hi) break;
      if (L + 1 >= kChunkLevCap) {
        ovf = true;
        break;
      }
      ++L;
      lo = hi;
      hi = next;
      if (tid == 0) s_lev[L + 1] = (uint16_t)hi;
    }
    uint64_t t1 = clock ? wall_clock64() : 0;

    if (ovf) {
      // Hand the chunk's roots to the level pass; nothing of it was written.
      if (a.pergrid) {
        for (int j = tid; j < nr; j += NT) {
          const int gi = multi ? w.gq[r0 + j] : 0;
          const int64_t o = a.grids[gi].offset;
          const int32_t k = atomicAdd(&w.gcnt[gi], 1);
          w.fc[o + k] = w.q[r0 + j];
          w.mq[o + k] = w.kq[r0 + j];
        }
      } else {
        if (tid == 0) s_slot = atomicAdd(&ct->ovf_count, nr);
        __syncthreads();
        const int64_t dst = (int64_t)nroots + s_slot;
        for (int j = tid; j < nr; j += NT) {
          w.q[dst + j] = w.q[r0 + j];
          w.gq[dst + j] = multi ? w.gq[r0 + j] : 0;
          w.kq[dst + j] = w.kq[r0 + j];
        }
      }
      __syncthreads();
      continue;
    }

    // Step 5: counts, deepest level first (a cell's donors are one level deeper).
    for (int l = L; l >= 1; --l) {
      for (int i = s_lev[l] + tid; i < s_lev[l + 1]; i += NT) {
        const uint32_t v = (s_cnt[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu;
        const int p = s_par[i];
        atomicAdd(&s_cnt[p >> 1], v << ((p & 1) * 16));
      }
      __syncthreads();
    }
    uint64_t t2 = clock ? wall_clock64() : 0;

    // Steps 6-7: roots keep their (uplifted) height; every other level takes
    // the implicit update towards its receiver's new height.
    for (int l = 0; l <= L; ++l) {
      for (int i = s_lev[l] + tid; i < s_lev[l + 1]; i += NT) {
        const int32_t c = s_cell[i];
        const uint32_t count = (s_cnt[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu;
        double hn = s_h[i];
        if (l > 0) {
          const int gi = multi ? s_grid[i] : 0;
          const GridDev& G = a.grids[gi];
          const int k = s_k[i];
          const double hr = s_h[s_par[i]];
          const double udt = a.Uf ? a.Uf[c] * (multi ? G.dt : g0_dt) : (multi ? G.udt : g0_udt);
          if (!a.Kf && !(multi ? G.newton != 0 : g0_newton) && count < (uint32_t)kAmTab) {
            // F from the grid's table (scalar K, n = 1, small counts).
            const double f = w.ftab[(gi * 3 + code_class(k)) * kAmTab + count];
            if (a.project) {
              hn = f > 0.0 ? hr + udt / f : hn;
            } else {
              const double g = 1.0 + f;
              hn = (hn + f * hr) / g;
            }
          } else {
            hn = eroded_height_general(a.grids, gi, a.Kf, w.amtab, count, k, c, hn, hr, a.project,
                                       udt);
          }
          s_h[i] = hn;
        }
        a.h_out[c] = hn;
        if (a.export_routing) {
          w.dep_g[c] = l;
          w.cnt_g[c] = count;
        }
      }
      __syncthreads();
    }
    my_total += next;
    my_nl = my_nl > L + 1 ? my_nl : L + 1;
    if (clock) {
      const uint64_t t3 = wall_clock64();
      tk[0] += t1 - t0;
      tk[1] += t2 - t1;
      tk[2] += t3 - t2;
    }
  }
  if (tid == 0) {
    if (my_total) atomicAdd((unsigned long long*)&ct->chunk_total, (unsigned long long)my_total);
    if (my_nl) atomicMax(&ct->chunk_nl, my_nl);
    if (clock)
      for (int k = 0; k < 3; ++k) ct->ticks[k + 1] += tk[k];
  }
}

// ---------------------------------------------------------------------------
// Multiple flow directions (section "Multiple Flow Directions"): every
// strictly lower neighbour is a receiver and gets the share
// S^p / sum_j S_j^p of the flow (S = slope to it); a cell is processed only
// after all of its receivers, so its level is the longest path to a root.
// Single grid, global memory, level-synchronous.  Levels use the donor masks
// and one counter byte per cell, four to a word in par's space (receivers
// not yet ordered); areas
// gather each donor's height, weight sum and area from one 32-byte MfdCell
// (grid order), about four cache lines per 3x3 neighbourhood instead of
// three per field; erosion reads the dense old and new heights of its
// receivers and its own weight sum and area from its record.

__device__ __forceinline__ double slope_pow(double s, double p) { return p == 1.0 ? s : pow(s, p); }

__device__ __forceinline__ double class_dist(const GridDev& G, int k) {
  const int cls = code_class(k);
  return cls == 0 ? G.dy : (cls == 1 ? G.dx : G.ddiag);
}

// Receivers, weight sums and counters; roots (no receiver) queued as level 0.
// Each block takes kRouteItems cells per thread between two appends to the
// queue counter (a same-address atomic serialises at about 11.5 ns).
constexpr int kRouteItems = 16;
constexpr int kRouteChunk = 256 * kRouteItems;

__global__ __launch_bounds__(256) void k_mfd_route(StepArgs a) {
  __shared__ int wsum[256 / 64];
  __shared__ int s_base;
  const Work w = a.w;
  const GridDev& G = a.grids[0];
  const int ny = G.ny, nx = G.nx;
  const int64_t n = (int64_t)ny * nx;
  for (int64_t base = (int64_t)blockIdx.x * kRouteChunk; base < n;
       base += (int64_t)gridDim.x * kRouteChunk) {
    uint32_t roots = 0;  // bit j: cell base + j * 256 + threadIdx.x is a root
#pragma unroll 4
    for (int j = 0; j < kRouteItems; ++j) {
      const int64_t c = base + (int64_t)j * 256 + threadIdx.x;
      if (c >= n) break;
      const int y = (int)(c / nx), x = (int)(c % nx);
      double wsum_c = 0.0;
      int nrec = 0;
      uint32_t recs = 0;    // receivers: neighbours below this interior cell
      uint32_t donors = 0;  // interior neighbours above this cell
      const double hc = a.h_in[c];
      if (y > 0 && x > 0 && y < ny - 1 && x < nx - 1) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const double hr = a.h_in[c + neighbour_offset(k, nx)];
          if (hc - hr > 0.0) {
            wsum_c += slope_pow((hc - hr) / class_dist(G, k), a.mfd_p);
            ++nrec;
            recs |= 1u << k;
          }
          const int yy = y + code_dy(k), xx = x + code_dx(k);
          if (yy > 0 && xx > 0 && yy < ny - 1 && xx < nx - 1 && hr - hc > 0.0) donors |= 1u << k;
        }
      } else {
        for (int k = 0; k < 8; ++k) {
          const int yy = y + code_dy(k), xx = x + code_dx(k);
          if (yy > 0 && xx > 0 && yy < ny - 1 && xx < nx - 1 &&
              a.h_in[c + neighbour_offset(k, nx)] - hc > 0.0)
            donors |= 1u << k;
        }
      }
      ((uint8_t*)w.par)[c] = (uint8_t)nrec;  // one byte per cell, four to a word
      w.mq[c] = (uint8_t)donors;
      w.kq[c] = (uint8_t)recs;
      MfdCell& mc = w.mc[c];
      mc.h = hc;
      mc.wsum = wsum_c;
      if (nrec == 0) {
        roots |= 1u << j;
        w.dep_g[c] = 0;
      }
    }
    int tot;
    const int pre = block_exclusive_scan<256>(__popc(roots), wsum, &tot);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(&w.lcnt[0], tot) : 0;
    __syncthreads();
    int32_t pos = s_base + pre;
    while (roots) {
      const int j = __ffs(roots) - 1;
      roots &= roots - 1;
      w.q[pos++] = (int32_t)(base + (int64_t)j * 256 + threadIdx.x);
    }
    __syncthreads();
  }
}

// Level L -> L+1: every processed cell releases its donors; a donor whose
// last receiver this was joins the next level.
template <int ITEMS>
__device__ void mfd_expand(const StepArgs& a, int32_t lo, int32_t hi, int32_t L, int wg, int nwg,
                           uint64_t* wsum64, int* s_base) {
  const Work& w = a.w;
  const GridDev& G = a.grids[0];
  const int nx = G.nx;
  const int tid = threadIdx.x;
  constexpr int W = ITEMS / 4, CHUNK = kBlock * ITEMS;
  for (int64_t base = lo + (int64_t)wg * CHUNK; base < hi; base += (int64_t)nwg * CHUNK) {
    uint32_t ready[ITEMS];
    int32_t cs[ITEMS];
    uint64_t v[W] = {};
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + (int64_t)j * kBlock + tid;
      ready[j] = 0;
      cs[j] = 0;
      if (i < hi) {
        const int32_t c = w.q[i];
        cs[j] = c;
        // Donors: the interior neighbours above the cell (mask from the routing).
        for (uint32_t m = w.mq[c]; m; m &= m - 1) {
          const int k = __ffs(m) - 1;
          const int32_t d = c + (int32_t)neighbour_offset(k, nx);
          const int sh = 8 * (d & 3);
          const uint32_t was = atomicSub((uint32_t*)w.par + (d >> 2), 1u << sh);
          if (((was >> sh) & 0xFFu) == 1u) ready[j] |= 1u << k;
        }
        v[j >> 2] += (uint64_t)__popc(ready[j]) << (16 * (j & 3));
      }
    }
    uint64_t pre[W], tot[W];
    block_scan_items<kBlock, W>(v, wsum64, pre, tot);
    const int total = items_total<W>(tot);
    if (tid == 0) *s_base = total ? atomicAdd(&w.lcnt[L + 1], total) : 0;
    __syncthreads();
    int32_t run = hi + *s_base;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      int32_t pos = run + item_field(pre[j >> 2], j & 3);
      run += item_field(tot[j >> 2], j & 3);
      uint32_t m = ready[j];
      while (m) {
        const int k = __ffs(m) - 1;
        m &= m - 1;
        const int32_t d = cs[j] + (int32_t)neighbour_offset(k, nx);
        w.q[pos++] = d;
        w.dep_g[d] = L + 1;
      }
    }
    __syncthreads();
  }
}

// Step 5: drainage area of the cells of one level, pulled from their donors
// in neighbour order.
__device__ void mfd_area_level(const StepArgs& a, int32_t a0, int32_t a1, int wg, int nwg) {
  const Work& w = a.w;
  // The grid's fields in registers before the loop: the loop calls pow, and
  // the compiler would otherwise load them again for every donor.
  const GridDev& G = a.grids[0];
  const int nx = G.nx;
  const double dist[3] = {G.dy, G.dx, G.ddiag};
  const double dxdy = G.dxdy, p = a.mfd_p;
  for (int64_t i = a0 + (int64_t)wg * kBlock + threadIdx.x; i < a1; i += (int64_t)nwg * kBlock) {
    const int32_t c = w.q[i];
    const double hc = w.mc[c].h;
    double acc = dxdy;
    // Donors in neighbour order (mask from the routing: interior neighbours above c).
    for (uint32_t m = w.mq[c]; m; m &= m - 1) {
      const int k = __ffs(m) - 1;
      const MfdCell& md = w.mc[c + (int32_t)neighbour_offset(k, nx)];
      const double hd = md.h;
      const int cls = code_class(k);
      const double dk = cls == 0 ? dist[0] : (cls == 1 ? dist[1] : dist[2]);
      const double share = slope_pow((hd - hc) / dk, p) / md.wsum;
      acc += share * md.area;
    }
    w.mc[c].area = acc;
  }
}

// Steps 6-7 for the cells of one level: uplift, then the implicit update
// with all receivers, h' = (h0 + sum F_k h_k') / (1 + sum F_k).
__device__ void mfd_erode_level(const StepArgs& a, int32_t a0, int32_t a1, int wg, int nwg) {
  const Work& w = a.w;
  // The grid's fields in registers before the loop (it calls pow and the
  // area power).
  const GridDev& G = a.grids[0];
  const int ny = G.ny, nx = G.nx;
  const double dist[3] = {G.dy, G.dx, G.ddiag};
  const double g_dt = G.dt, g_udt = G.udt, g_K = G.K, g_m = G.m, p = a.mfd_p;
  const int use_sqrt = G.use_sqrt;
  const double* const Uf = a.Uf;
  const double* const Kf = a.Kf;
  for (int64_t i = a0 + (int64_t)wg * kBlock + threadIdx.x; i < a1; i += (int64_t)nwg * kBlock) {
    const int32_t c = w.q[i];
    const int y = c / nx, x = c % nx;
    const double hc = a.h_in[c];
    if (y == 0 || x == 0 || y == ny - 1 || x == nx - 1) {
      a.h_out[c] = hc;
      continue;
    }
    const MfdCell& mc = w.mc[c];
    const double hup = hc + (Uf ? Uf[c] * g_dt : g_udt);
    const double wc = mc.wsum;
    const double ac = mc.area;
    const double kdt = (Kf ? Kf[c] : g_K) * g_dt;
    double sumf = 0.0, sumfh = 0.0;
    // Receivers in neighbour order (mask from the routing).
    const uint32_t recs = w.kq[c];
    for (uint32_t m = recs; m; m &= m - 1) {
      const int k = __ffs(m) - 1;
      const int32_t r = c + (int32_t)neighbour_offset(k, nx);
      const double hr = a.h_in[r];
      const int cls = code_class(k);
      const double dk = cls == 0 ? dist[0] : (cls == 1 ? dist[1] : dist[2]);
      const double share = slope_pow((hc - hr) / dk, p) / wc;
      const double f = (kdt * area_power_call(share * ac, use_sqrt, g_m)) / dk;
      sumf += f;
      sumfh += f * a.h_out[r];
    }
    a.h_out[c] = recs ? (hup + sumfh) / (1.0 + sumf) : hup;
  }
}

// The cells of each level in grid order: a counting sort by level over
// contiguous grid-order ranges, one per workgroup (per-range level
// histograms, their scan per level, then the scatter).  Level-order gathers
// then touch neighbouring rows close together in time and share cache lines;
// the order inside a level changes no result.  Counts and starts live in
// w.fc (level-major, nl * nwg entries).
constexpr int kMfdSortLevels = 1024;

__device__ void mfd_sort_by_level(const StepArgs& a, int32_t nl, int wg, int nwg, int32_t* hist,
                                  int* wsum, Ctrl* ct) {
  const Work& w = a.w;
  const int64_t n = a.n;
  const int64_t per = (n + nwg - 1) / nwg;
  const int64_t c0 = min((int64_t)wg * per, n), c1 = min(c0 + per, n);
  int32_t* cnt = w.fc;
  for (int l = threadIdx.x; l < nl; l += kBlock) hist[l] = 0;
  __syncthreads();
  for (int64_t c = c0 + threadIdx.x; c < c1; c += kBlock) {
    const int32_t l = w.dep_g[c];
    if ((uint32_t)l < (uint32_t)nl) atomicAdd(&hist[l], 1);
  }
  __syncthreads();
  for (int l = threadIdx.x; l < nl; l += kBlock) cnt[(int64_t)l * nwg + wg] = hist[l];
  grid_barrier(ct);
  for (int l = wg; l < nl; l += nwg) {  // nwg <= kBlock: one range per thread
    const int v = threadIdx.x < nwg ? cnt[(int64_t)l * nwg + threadIdx.x] : 0;
    int tot;
    const int pre = block_exclusive_scan<kBlock>(v, wsum, &tot);
    if (threadIdx.x < nwg) cnt[(int64_t)l * nwg + threadIdx.x] = w.lev[l] + pre;
  }
  grid_barrier(ct);
  for (int l = threadIdx.x; l < nl; l += kBlock) hist[l] = cnt[(int64_t)l * nwg + wg];
  __syncthreads();
  for (int64_t c = c0 + threadIdx.x; c < c1; c += kBlock) {
    const int32_t l = w.dep_g[c];
    if ((uint32_t)l < (uint32_t)nl) w.q[atomicAdd(&hist[l], 1)] = (int32_t)c;
  }
  grid_barrier(ct);
}

// Drainage areas of the last step out of the per-cell records.
__global__ __launch_bounds__(256) void k_mfd_export_area(StepArgs a, double* d_area) {
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < a.n;
       c += (int64_t)gridDim.x * 256)
    d_area[c] = a.w.mc[c].area;
}

__global__ __launch_bounds__(kBlock) void k_mfd_levels(StepArgs a) {
  __shared__ uint64_t wsum64[4 * kBlock / 64 + 4];
  __shared__ int wsum[kBlock / 64];
  __shared__ int32_t hist[kMfdSortLevels];
  __shared__ int s_base;
  const Work w = a.w;
  Ctrl* ct = w.ctrl;
  const int wg = blockIdx.x, nwg = gridDim.x;
  const bool lead = (wg == 0 && threadIdx.x == 0);
  int32_t lo = 0, hi = load_acquire(&w.lcnt[0]), L = 0;
  uint64_t t0 = 0, t1 = 0, t2 = 0;
  if (lead && a.timers) t0 = wall_clock64();
  if (lead) w.lev[0] = 0;
  while (true) {
    if (lead) {
      w.lev[L + 1] = hi;
      w.lcnt[L + 2] = 0;
    }
    mfd_expand<kExpandItems>(a, lo, hi, L, wg, nwg, wsum64, &s_base);
    grid_barrier(ct);
    const int32_t added = load_acquire(&w.lcnt[L + 1]);
    if (added == 0) break;
    lo = hi;
    hi += added;
    ++L;
  }
  // Every cell reached (else the step reports an error below) and a level
  // table that fits: put each level's cells in grid order.
  if (hi == a.n && L + 1 <= kMfdSortLevels && (int64_t)(L + 1) * nwg <= (int64_t)a.n &&
      nwg <= kBlock)
    mfd_sort_by_level(a, L + 1, wg, nwg, hist, wsum, ct);
  if (lead && a.timers) t1 = wall_clock64();
  for (int32_t l = L; l >= 0; --l) {
    mfd_area_level(a, w.lev[l], w.lev[l + 1], wg, nwg);
    grid_barrier(ct);
  }
  if (lead && a.timers) t2 = wall_clock64();
  for (int32_t l = 0; l <= L; ++l) {
    mfd_erode_level(a, w.lev[l], w.lev[l + 1], wg, nwg);
    if (l < L) grid_barrier(ct);
  }
  if (lead && a.timers) {
    // The last erosion level has no closing barrier: this is workgroup 0's end.
    const uint64_t t3 = wall_clock64();
    ct->ticks[1] += t1 - t0;
    ct->ticks[2] += t2 - t1;
    ct->ticks[3] += t3 - t2;
  }
  if (lead) {
    const int32_t nl = L + 1;
    ct->nlevels = nl;
    ct->dirty_total = hi;
    ct->dirty_nlevels = nl;
    ct->crossing_run += hi;
    if (nl > ct->max_nlevels) ct->max_nlevels = nl;
    if (a.step < kHistCap) w.hist[a.step] = nl;
    ct->steps = a.step + 1;
    if ((int64_t)hi != (int64_t)a.n) atomicMax(&ct->status, 5);
    w.lcnt[0] = 0;
    w.lcnt[1] = 0;
  }
}

// Start of a run: tabulate A^m, F and 1 + F per grid (block g does grid g)
// and reset the control block.
__global__ void k_begin_run(StepArgs a) {
  const int i = threadIdx.x, gi = blockIdx.x;
  const GridDev& G = a.grids[gi];
  if (i < kAmTab) {
    const double am = area_power((double)i * G.dxdy, G.use_sqrt, G.m);
    a.w.amtab[gi * kAmTab + i] = am;
    for (int c = 0; c < 3; ++c) {
      const double f = ((G.K * G.dt) * am) / G.dn[c];
      a.w.ftab[(gi * 3 + c) * kAmTab + i] = f;
      a.w.gtab[(gi * 3 + c) * kAmTab + i] = 1.0 + f;
    }
  }
  if (i == 0) a.w.gcnt[gi] = 0;
  if (i == 0 && gi == 0) {
    Ctrl* ct = a.w.ctrl;
    ct->max_nlevels = 0;
    ct->steps = 0;
    ct->clean = 0;
    ct->clean_maxdepth = 0;
    ct->crossing_run = 0;
    for (int k = 0; k < kTilePhases; ++k) ct->tile_ticks[k] = 0;
    ct->tile_wgs = 0;
    ct->chunk_total = 0;
    ct->chunk_next = 0;
    ct->ovf_count = 0;
    ct->chunk_nl = 0;
    for (int k = 0; k < 4; ++k) ct->ticks[k] = 0;
    a.w.lcnt[0] = 0;
    a.w.lcnt[1] = 0;
  }
}

// Fixed routing: copy caller codes, checking that each stays in the grid and
// that perimeter cells have none.  Bad codes raise LEM_E_ARG on the device
// and are treated as "no receiver".
__global__ __launch_bounds__(256) void k_fixed_routing(StepArgs a, const uint8_t* user) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  const GridDev& G = a.grids[0];
  const int y = (int)(c / G.nx), x = (int)(c % G.nx);
  const uint8_t u = user[c];
  const bool perim = (y == 0 || x == 0 || y == G.ny - 1 || x == G.nx - 1);
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

// Routing export, part 1: levels and counts of the crossing trees.
__global__ __launch_bounds__(256) void k_export_cross(StepArgs a) {
  const Work w = a.w;
  const int32_t nlev = w.ctrl->dirty_nlevels;
  // The per-grid level pass writes levels and counts itself.
  const int32_t total = a.pergrid ? 0 : w.ctrl->glob_total;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int32_t lo = 0, hi = nlev;  // largest l with lev[l] <= i
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (w.lev[mid] <= i) lo = mid; else hi = mid;
    }
    const int32_t c = w.q[i];
    w.dep_g[c] = lo;
    w.cnt_g[c] = w.cnt[i];
  }
  // Clear the level histogram for part 2.
  const int32_t nl = w.ctrl->nlevels;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nl + 2; i += stride)
    w.dhist[i] = 0;
}

// Routing export, part 2: per-cell receiver, level and count of grid g
// (cells [off, off + cells)) for the caller, and its level histogram.
__global__ __launch_bounds__(256) void k_export_cells(StepArgs a, int gi, int64_t off,
                                                      int64_t cells, int32_t* rec,
                                                      int32_t* depth, uint32_t* count) {
  // Level histogram: per block in LDS for the first kExportBins levels (one
  // device atomic per non-empty bin and block), deeper levels directly.
  constexpr int kExportBins = 2048;
  __shared__ int32_t bins[kExportBins];
  const Work w = a.w;
  const int nx = a.grids[gi].nx;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t nl = w.ctrl->nlevels;
  for (int b = threadIdx.x; b < kExportBins; b += blockDim.x) bins[b] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
    if (rec) {
      const uint8_t k = w.rcode[off + i];
      rec[i] = (k >= kSink) ? (int32_t)i : (int32_t)(i + neighbour_offset(k, nx));
    }
    const int32_t d = w.dep_g[off + i];
    if (depth) depth[i] = d;
    if (count) count[i] = w.cnt_g[off + i];
    if (d >= 0 && d < nl) {
      if (d < kExportBins)
        atomicAdd(&bins[d], 1);
      else
        atomicAdd(&w.dhist[d + 1], 1);
    }
  }
  __syncthreads();
  const int top = nl < kExportBins ? nl : kExportBins;
  for (int b = threadIdx.x; b < top; b += blockDim.x)
    if (bins[b]) atomicAdd(&w.dhist[b + 1], bins[b]);
}

// Per grid (blockIdx.y): the largest |h_out - h_in| and the largest |h_out|
// of the step just taken.  Non-negative doubles order like their bit
// patterns, so an unsigned atomic maximum on the bits is exact.
__global__ __launch_bounds__(256) void k_change(StepArgs a) {
  const GridDev& G = a.grids[blockIdx.y];
  const int64_t cells = (int64_t)G.ny * G.nx;
  // Maxima that keep a NaN (fmax would drop it): a grid whose heights are
  // no longer finite must not look steady; the host reports it.
  double dmax = 0.0, hmax = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double hn = a.h_out[G.offset + i];
    const double dh = fabs(hn - a.h_in[G.offset + i]), ah = fabs(hn);
    dmax = (dh > dmax || dh != dh) && dmax == dmax ? dh : dmax;
    hmax = (ah > hmax || ah != ah) && hmax == hmax ? ah : hmax;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const double od = __shfl_xor(dmax, d, 64), oh = __shfl_xor(hmax, d, 64);
    dmax = (od > dmax || od != od) && dmax == dmax ? od : dmax;
    hmax = (oh > hmax || oh != oh) && hmax == hmax ? oh : hmax;
  }
  if ((threadIdx.x & 63) == 0) {
    unsigned long long* cv = (unsigned long long*)a.w.conv;
    atomicMax(&cv[2 * blockIdx.y], (unsigned long long)__double_as_longlong(dmax));
    atomicMax(&cv[2 * blockIdx.y + 1], (unsigned long long)__double_as_longlong(hmax));
  }
}

__global__ void k_zero_u32(uint32_t* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0u;
}

__global__ void k_zero_f64(double* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_validate(const double* x, int64_t n, int32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    bad |= !isfinite(x[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

static int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

size_t workspace_bytes(int64_t n, int64_t ngrids, int64_t ntiles, bool mfd) {
  Work w;
  carve(nullptr, n, ngrids, ntiles, &w, mfd);
  return (size_t)(uintptr_t)w.scratch + (size_t)align256(4 * kScratchInts);
}

void carve(void* base, int64_t n, int64_t ngrids, int64_t ntiles, Work* w, bool mfd) {
  char* p = (char*)base;
  auto take = [&](int64_t bytes) { char* r = p; p += align256(bytes); return (void*)r; };
  w->h2 = (double*)take(8 * n);
  w->rcode = (uint8_t*)take(n);
  w->dmask = (uint8_t*)take(n);
  w->grids = (GridDev*)take((int64_t)sizeof(GridDev) * ngrids);
  w->tiles = (int32_t*)take(4 * ntiles);
  w->tgrid = (int32_t*)take(4 * ntiles);
  w->conv = (double*)take(8 * 2 * ngrids);
  w->q = (int32_t*)take(4 * n);
  w->gq = (uint16_t*)take(2 * n);
  w->par = (int32_t*)take(4 * n);
  w->fc = (int32_t*)take(4 * n);
  w->mq = (uint8_t*)take(n);
  w->kq = (uint8_t*)take(n);
  w->cnt = (uint32_t*)take(4 * n);
  w->hq = (double*)take(8 * n);
  w->lcnt = (int32_t*)take(4 * (n + 2));
  w->lev = (int32_t*)take(4 * (n + 2 * ngrids + 2));
  w->dep_g = (int32_t*)take(4 * n);
  w->cnt_g = (uint32_t*)take(4 * n);
  w->dhist = (int32_t*)take(4 * (n + 2));
  w->amtab = (double*)take(8 * kAmTab * ngrids);
  w->ftab = (double*)take(8 * 3 * kAmTab * ngrids);
  w->gtab = (double*)take(8 * 3 * kAmTab * ngrids);
  w->hist = (int32_t*)take(4 * kHistCap);
  w->gcnt = (int32_t*)take(4 * ngrids);
  w->gnl = (int32_t*)take(4 * ngrids);
  w->gtot = (int32_t*)take(4 * ngrids);
  w->mc = mfd ? (MfdCell*)take((int64_t)sizeof(MfdCell) * n) : nullptr;
  w->ctrl = (Ctrl*)take(sizeof(Ctrl));
  w->scratch = (int32_t*)take(4 * kScratchInts);
}

hipError_t launch_begin_run(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_begin_run, dim3((unsigned)a.ngrids), dim3(kAmTab), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fixed_routing(const StepArgs& a, const uint8_t* user, hipStream_t s) {
  hipLaunchKernelGGL(k_fixed_routing, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a,
                     user);
  return hipGetLastError();
}

hipError_t launch_tile_step(const StepArgs& a, int grid, hipStream_t s) {
  (void)grid;
  if (a.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_step, dim3((unsigned)a.ntiles), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t tile_kernel_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)k_tile_step,
                                                      kTileThreads, 0);
}

hipError_t launch_grid_levels(const StepArgs& a, int threads, hipStream_t s) {
  if (threads == 256)
    hipLaunchKernelGGL(k_grid_levels<256>, dim3((unsigned)a.ngrids), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_grid_levels<kBlock>, dim3((unsigned)a.ngrids), dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grid_levels_finish, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_chunk_trees(const StepArgs& a, int grid, hipStream_t s) {
  if (a.ngrids > 1)
    hipLaunchKernelGGL(k_chunk_trees<true>, dim3((unsigned)grid), dim3(kChunkThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_chunk_trees<false>, dim3((unsigned)grid), dim3(kChunkThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t chunk_kernel_occupancy(bool batch, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, batch ? (const void*)k_chunk_trees<true> : (const void*)k_chunk_trees<false>,
      kChunkThreads, 0);
}

hipError_t launch_mfd_route(const StepArgs& a, hipStream_t s) {
  const int64_t n = a.n;
  const int64_t chunks = (n + kRouteChunk - 1) / kRouteChunk;
  const unsigned blocks = (unsigned)(chunks < 4096 ? chunks : 4096);
  hipLaunchKernelGGL(k_mfd_route, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mfd_levels(const StepArgs& a, int grid, hipStream_t s) {
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_mfd_levels, dim3(grid), dim3(kBlock), args, 0,
                                    s);
}

hipError_t launch_mfd_export_area(const StepArgs& a, double* d_area, hipStream_t s) {
  const int64_t n = a.n;
  const unsigned blocks = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_mfd_export_area, dim3(blocks), dim3(256), 0, s, a, d_area);
  return hipGetLastError();
}

hipError_t mfd_kernel_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)k_mfd_levels,
                                                      kBlock, 0);
}

hipError_t launch_global_levels(const StepArgs& a, int grid, hipStream_t s) {
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_global_levels, dim3(grid), dim3(kBlock), args,
                                    0, s);
}

hipError_t launch_export(const StepArgs& a, int g, int64_t offset, int64_t cells, int32_t* rec,
                         int32_t* depth, uint32_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_export_cross, dim3(1024), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_export_cells, dim3(2048), dim3(256), 0, s, a, g, offset, cells, rec, depth,
                     count);
  return hipGetLastError();
}

hipError_t launch_change(const StepArgs& a, int64_t total_cells, hipStream_t s) {
  (void)total_cells;
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, s, a.w.conv, (int64_t)2 * a.ngrids);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_change, dim3(16, (unsigned)a.ngrids), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s) {
  if (words <= 0) return hipSuccess;
  const int64_t blocks = (words + 255) / 256;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s,
                     (uint32_t*)p, words);
  return hipGetLastError();
}

hipError_t launch_validate(const double* x, int64_t n, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(2048), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

hipError_t global_kernel_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                      (const void*)k_global_levels, kBlock, 0);
}

}  // namespace lem
