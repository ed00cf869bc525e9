// lem_internal.h -- declarations shared by the HIP kernels and the C-ABI host
// code of the GPU library.  Not part of the public ABI (that is include/lem.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lem {

// Receiver codes (Step 2).  0..7: the receiver is the neighbour at offset
// (dy,dx) = (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1), i.e. in
// ascending cell index; the opposite of code k is 7-k.  kSink: an interior
// cell with no strictly lower neighbour (a root that is uplifted); kBase: a
// perimeter cell (a root at base level that never changes); kNone: a
// position outside the grid (only inside a tile's halo).
constexpr uint8_t kSink = 8;
constexpr uint8_t kBase = 9;
constexpr uint8_t kNone = 10;

// Tiles of the local pass: kTH x kTW cells per workgroup of kTileThreads.
constexpr int kTH = 64;
constexpr int kTW = 64;
constexpr int kTileThreads = 512;
// Levels a tile resolves on its own before it hands all its trees to the
// global pass.
constexpr int kLocalDepthCap = 255;
// A^m is tabulated for upstream counts below kAmTab (same function, same
// inputs as computing it in place).
constexpr int kAmTab = 256;

// Threads per workgroup of the global level kernel, the queue entries each
// thread takes per chunk, the most workgroups it uses (a grid-wide barrier
// costs about 45 ns per participating workgroup on this part), and the
// level size below which one workgroup handles a level on its own.
constexpr int kBlock = 1024;
constexpr int kItems = 16;
constexpr int kChunk = kBlock * kItems;
// Queue positions per thread in a breadth-first expansion step (4, 8 or 16):
// levels of the crossing pass hold about 10^6 positions at 10^8 cells, so
// small chunks keep every workgroup busy.
constexpr int kExpandItems = 4;
constexpr int kGlobalMaxWGs = 192;
constexpr int kTailLevel = 8192;  // default; lem_set_tuning changes it per context

// Crossing trees, first stage: workgroups of kChunkThreads take chunks of
// consecutive crossing roots from a device work counter and finish their
// trees in LDS (at most kChunkCap cells and kChunkLevCap levels per chunk;
// a chunk that needs more is handed to the level pass).  Roots per chunk:
// 1..kChunkMaxRoots (kChunkMaxRoots <= kChunkLevCap and <= kChunkCap / 2,
// so the roots handed on fit in the queue behind the chunk roots).
constexpr int kChunkThreads = 256;
constexpr int kChunkCap = 2048;
constexpr int kChunkLevCap = 256;
constexpr int kChunkMaxRoots = 256;
constexpr int kChunkRootsDefault = 128;
static_assert(kChunkMaxRoots <= kChunkLevCap && 2 * kChunkMaxRoots <= kChunkCap,
              "roots handed on must fit behind the chunk roots");

// Phases of the tile pass timed with LEM_F_PHASE_TIMERS.
constexpr int kTilePhases = 6;

// Device-side control block (one per context, in the workspace).
struct Ctrl {
  int32_t status;          // lem_status of device-detected errors (0 = OK)
  int32_t nlevels;         // levels of the most recent step (whole grid)
  int32_t dirty_total;     // cells the global pass ordered in the most recent step
  int32_t dirty_nlevels;   // levels of the global pass in the most recent step
  int32_t max_nlevels;
  int32_t clean;           // cells resolved inside their tile (current step)
  int32_t clean_maxdepth;  // deepest level among them (current step)
  int32_t pad0;
  int64_t steps;           // steps recorded in the level history of the current run
  uint64_t ticks[4];       // device wall-clock ticks per phase (accumulated)
  int32_t tail_lo, tail_hi, tail_L, tail_done;  // state handed back by a one-workgroup run
  int64_t crossing_run;    // crossing-tree cells summed over the current run
  int64_t chunk_total;     // cells finished by the chunk stage (current step)
  int32_t chunk_next;      // work counter of the chunk stage (current step)
  int32_t ovf_count;       // roots the chunk stage handed to the level pass
  int32_t chunk_nl;        // deepest chunk's levels (current step)
  int32_t glob_total;      // cells ordered by the global level pass (current step)
  uint64_t tile_ticks[kTilePhases];  // tile pass: device clock per phase, summed over workgroups
  uint64_t tile_wgs;       // tile-pass workgroups timed
  uint64_t grid_phase_max[3];  // per-grid level pass: longest workgroup per phase (current step)
  int32_t pad[12];
  // Grid-wide barrier of the global level kernel (own cache lines).
  uint32_t bar_count;
  uint32_t pad1[31];
  uint32_t bar_gen;
  uint32_t pad2[31];
};
static_assert(sizeof(Ctrl) % 4 == 0, "cleared as 32-bit words");

// One grid of a batch (a single-grid context is a batch of one).  Grids
// are stored one after another in the batch arrays; tiles are numbered
// across the whole batch.
struct GridDev {
  int64_t offset;          // first cell of this grid in the batch arrays
  int32_t ny, nx;
  int32_t tiles_x, tile_base;  // tiles [tile_base, tile_base + tiles_x * tiles_y)
  int32_t use_sqrt;        // m == 0.5: A^m computed as sqrt(A)
  int32_t square;          // dx == dy
  double dx, dy, ddiag, dxdy;
  double dt, m, K, udt;
  double inv_dx, inv_dy, inv_dd;
  double dn[3];            // dist^n for the classes (dy, dx, diagonal); = dist for n = 1
  double nexp, eps;        // slope exponent n and the Newton tolerance (n != 1)
  int32_t newton;          // n != 1: the Newton-Raphson loop of Algorithm 6
  int32_t max_newton;      // iteration limit of that loop
};

// One cell of a multiple-flow-direction step as the area phase gathers it
// (grid order): height, weight sum and drainage area in one record.
struct MfdCell {
  double h;        // height at the start of the step
  double wsum;     // sum of the flow weights S^p over the receivers
  double area;     // drainage area (m^2)
  double pad;
};
static_assert(sizeof(MfdCell) == 32, "four cells per 128-byte line");

// Pointers into the workspace.
struct Work {
  double* h2;        // [N] second height buffer (steps alternate between h and h2)
  uint8_t* rcode;    // [N] receiver codes (fixed routing; export step)
  uint8_t* dmask;    // [N] donor mask per cell: bit k set <=> neighbour k drains here
  GridDev* grids;    // [ngrids] grid descriptors
  int32_t* tiles;    // [ntiles] tiles to process (all, or those of unfinished grids)
  int32_t* tgrid;    // [ntiles] grid of each entry of tiles
  double* conv;      // [2*ngrids] per grid: largest |change| and largest |h| of a step
  int32_t* q;        // [N] global queue: cell per position, level-major
  uint16_t* gq;      // [N] grid of each queue position
  int32_t* par;      // [N] queue position of the receiver (-1 at level 0); multiple
                     //     flow directions: receivers of each cell not yet ordered
  int32_t* fc;       // [N] queue position of the first donor
  uint8_t* mq;       // [N] donor mask in queue order
  uint8_t* kq;       // [N] receiver code in queue order
  uint32_t* cnt;     // [N] upstream cell count in queue order
  double* hq;        // [N] new heights in queue order
  int32_t* lcnt;     // [N+2] cells appended per level
  int32_t* lev;      // [N+2] level offsets into the queue
  int32_t* dep_g;    // [N] level per cell (export step)
  uint32_t* cnt_g;   // [N] upstream count per cell (export step)
  int32_t* dhist;    // [N+2] level histogram (export)
  double* amtab;     // [ngrids*kAmTab] A^m for small counts
  double* ftab;      // [ngrids*3*kAmTab] F = K*dt*A^m/d per distance class (scalar K)
  double* gtab;      // [ngrids*3*kAmTab] 1 + F
  int32_t* hist;     // [kHistCap] level count per step of the current run
  int32_t* gcnt;     // [ngrids] per-grid level pass: crossing roots queued per grid
  int32_t* gnl;      // [ngrids] per-grid level pass: levels of the crossing trees
  int32_t* gtot;     // [ngrids] per-grid level pass: cells of the crossing trees
  MfdCell* mc;       // [N] multiple flow directions: per-cell records (null otherwise)
  Ctrl* ctrl;
  int32_t* scratch;  // [kScratchInts] reductions (validation)
};

constexpr int64_t kHistCap = 1 << 16;
constexpr int64_t kScratchInts = 1024;

// Everything one time step needs, passed by value to the kernels.
struct StepArgs {
  const GridDev* grids;  // device copy of the grid descriptors
  int32_t ngrids;
  int32_t ntiles;        // entries of w.tiles to process
  int32_t n;             // cells of all grids
  int32_t timers;        // record per-phase ticks
  const double* Kf;      // nullable per-cell K (single-grid contexts only)
  const double* Uf;      // nullable per-cell U (single-grid contexts only)
  const double* h_in;    // heights at the start of the step
  double* h_out;         // heights at the end of the step
  Work w;
  int64_t step;          // index of this step within the run
  int32_t fixed;         // receivers come from w.rcode (fixed routing)
  int32_t export_routing;  // write per-cell codes, levels and counts
  int32_t tail_level;    // levels smaller than this run in one workgroup
  int32_t pergrid;       // crossing trees: one workgroup per grid (else the global pass)
  int32_t mfd;           // multiple flow directions (single grid)
  int32_t chunked;       // crossing trees go through the chunk stage first
  int32_t chunk_roots;   // roots per chunk of that stage
  int32_t project;       // steady-state projection instead of the implicit update
  int32_t tile_clocks;   // per-phase device clocks in every tile workgroup
  double mfd_p;          // exponent of the slope in the flow shares
};

size_t workspace_bytes(int64_t n, int64_t ngrids, int64_t ntiles, bool mfd = false);
void carve(void* base, int64_t n, int64_t ngrids, int64_t ntiles, Work* w, bool mfd = false);

hipError_t launch_begin_run(const StepArgs& a, hipStream_t s);
hipError_t launch_fixed_routing(const StepArgs& a, const uint8_t* user_rcode, hipStream_t s);
// Tile pass on at most `grid` persistent workgroups (a multiple of 8).
hipError_t launch_tile_step(const StepArgs& a, int grid, hipStream_t s);
hipError_t tile_kernel_occupancy(int* blocks_per_cu);
hipError_t launch_global_levels(const StepArgs& a, int grid, hipStream_t s);
hipError_t launch_grid_levels(const StepArgs& a, int threads, hipStream_t s);
// Chunk stage of the crossing trees (before the level pass) on `grid` workgroups.
hipError_t launch_chunk_trees(const StepArgs& a, int grid, hipStream_t s);
hipError_t chunk_kernel_occupancy(bool batch, int* blocks_per_cu);
// Multiple flow directions: routing (weight sums, receiver counters, roots),
// then levels, areas and heights in one cooperative launch of `grid`
// workgroups.
hipError_t launch_mfd_route(const StepArgs& a, hipStream_t s);
hipError_t launch_mfd_levels(const StepArgs& a, int grid, hipStream_t s);
// Copies the last step's drainage areas (m^2, grid order) to d_area.
hipError_t launch_mfd_export_area(const StepArgs& a, double* d_area, hipStream_t s);
hipError_t mfd_kernel_occupancy(int* blocks_per_cu);
// Routing export of grid g (its cells [offset, offset + ny*nx)).
hipError_t launch_export(const StepArgs& a, int g, int64_t offset, int64_t cells, int32_t* rec,
                         int32_t* depth, uint32_t* count, hipStream_t s);
// Per grid: largest |h_out - h_in| and largest |h_out| (into w.conv).
hipError_t launch_change(const StepArgs& a, int64_t total_cells, hipStream_t s);
hipError_t launch_validate(const double* x, int64_t n, int32_t* flag, hipStream_t s);
// Sets `words` 32-bit words at p to zero (a kernel, not hipMemsetAsync).
hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s);
hipError_t global_kernel_occupancy(int* blocks_per_cu);

}  // namespace lem
