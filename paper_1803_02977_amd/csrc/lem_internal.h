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
// perimeter cell (a root at base level that never changes).
constexpr uint8_t kSink = 8;
constexpr uint8_t kBase = 9;

// Threads per workgroup of the ordering/accumulation/erosion kernel and the
// number of queue entries each thread takes per chunk.
constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kChunk = kBlock * kItems;

// Device-side control block (one per context, in the workspace).
struct Ctrl {
  int32_t status;     // lem_status of device-detected errors (0 = OK)
  int32_t nlevels;    // levels of the most recent step
  int32_t total;      // cells enqueued by the most recent step
  int32_t max_nlevels;
  int64_t steps;      // steps recorded in the level history of the current run
  uint64_t ticks[4];  // device wall-clock ticks per phase (accumulated)
  int32_t pad[48];
};

// Pointers into the workspace.
struct Work {
  uint8_t* rcode;    // [N] receiver code per cell (grid order)
  uint8_t* dmask;    // [N] donor mask per cell: bit k set <=> neighbour k drains here
  int32_t* q;        // [N] queue: cell index per position, level-major
  int32_t* par;      // [N] queue position of the receiver (-1 at level 0)
  int32_t* fc;       // [N] queue position of the first donor
  uint8_t* mq;       // [N] donor mask in queue order
  uint8_t* kq;       // [N] receiver code in queue order
  uint32_t* cnt;     // [N] upstream cell count in queue order
  double* hq;        // [N] new heights in queue order
  int32_t* lcnt;     // [N+2] number of cells per level (built while ordering)
  int32_t* lev;      // [N+2] level offsets into the queue
  int32_t* hist;     // [kHistCap] level count per step of the current run
  Ctrl* ctrl;
  int32_t* scratch;  // [kScratchInts] reductions (validation)
};

constexpr int64_t kHistCap = 1 << 16;
constexpr int64_t kScratchInts = 1024;

// Everything one time step needs, passed by value to the kernels.
struct StepArgs {
  int32_t ny, nx;
  int32_t n;         // ny*nx
  int32_t use_sqrt;  // m == 0.5: A^m computed as sqrt(A)
  double dx, dy, ddiag, dxdy;
  double dt, m, K, udt;
  const double* Kf;  // nullable per-cell K
  const double* Uf;  // nullable per-cell U
  double* h;
  Work w;
  int64_t step;      // index of this step within the run
  int32_t timers;    // record per-phase ticks
};

size_t workspace_bytes(int64_t n);
void carve(void* base, int64_t n, Work* w);

hipError_t launch_route(const StepArgs& a, hipStream_t s);
hipError_t launch_fixed_routing(const StepArgs& a, const uint8_t* user_rcode, hipStream_t s);
hipError_t launch_order_accum_erode(const StepArgs& a, int grid, hipStream_t s);
hipError_t launch_begin_run(const StepArgs& a, hipStream_t s);
hipError_t launch_export(const StepArgs& a, int32_t* rec, int32_t* depth, uint32_t* count,
                         hipStream_t s);
hipError_t launch_validate(const double* x, int64_t n, int32_t* flag, hipStream_t s);
hipError_t order_kernel_occupancy(int* blocks_per_cu);

}  // namespace lem
