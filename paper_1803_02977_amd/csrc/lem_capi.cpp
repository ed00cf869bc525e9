// lem_capi.cpp -- the C ABI (include/lem.h): argument checking, workspace
// carving, per-context state and error strings.  Everything the method
// computes runs in the kernels of lem_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lem.h"
#include "lem_internal.h"

struct lem_ctx {
  uint32_t flags;
  bool batch;                       // created by lem_batch_create
  bool mfd;                         // created by lem_mfd_create (multiple flow directions)
  double mfd_p;                     // exponent of the slope in the flow shares
  std::vector<lem::GridDev> grids;  // host copy of the grid descriptors
  std::vector<int32_t> tiles;       // all tiles, in order
  std::vector<int32_t> active;      // tiles of unfinished grids (steady-state driver)
  std::vector<int32_t> tgrid_host;  // grid of each uploaded tile (kept until the copy ends)
  int64_t cells;                    // cells of all grids
  int32_t ntiles;
  hipStream_t stream;
  lem::Work w;
  int grid;                         // workgroups of the cooperative level kernel
  int grid_max;                     // most that stay resident on this device
  int tail_level;
  int level_pass;                   // LEM_LEVELS_* as set (0 = automatic)
  bool pergrid;                     // level pass in use: one workgroup per grid
  int level_threads;                // threads per workgroup of that pass (0 = automatic)
  bool chunked;                     // chunk stage before the level pass
  int chunk_roots;                  // roots per chunk of that stage
  int chunk_grid;                   // workgroups of that stage (resident on the device)
  int tile_grid;                    // persistent workgroups of the tile pass
  int device;
  double tick_khz;                  // device wall-clock rate
  int64_t steps_done;
  int64_t last_run_steps;
  bool has_routing;
  double route_ms;                  // accumulated with LEM_F_PHASE_TIMERS
  double order_ms;
  double chunk_ms;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;  // PHASE_TIMERS only
  std::string err;
};

namespace {

lem_status fail(lem_ctx* ctx, lem_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

lem_status hip_fail(lem_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, LEM_E_HIP, m);
}

// Checks one grid's problem statement.
lem_status check_grid(int32_t ny, int32_t nx, double dx, double dy, double dt, double m, double n,
                      double U, double K, double eps, int32_t max_newton, std::string* why) {
  if (ny < 3 || nx < 3) { *why = "ny and nx must be >= 3"; return LEM_E_SIZE; }
  if ((int64_t)ny * (int64_t)nx > (int64_t)INT32_MAX - 2) {
    *why = "ny*nx must be below 2^31-2";
    return LEM_E_SIZE;
  }
  if (!(dx > 0.0) || !(dy > 0.0) || !std::isfinite(dx) || !std::isfinite(dy)) {
    *why = "dx and dy must be finite and > 0";
    return LEM_E_ARG;
  }
  if (!(dt > 0.0) || !std::isfinite(dt)) { *why = "dt must be finite and > 0"; return LEM_E_ARG; }
  if (!(m >= 0.0) || !std::isfinite(m)) { *why = "m must be finite and >= 0"; return LEM_E_ARG; }
  if (!(n > 0.0) || !std::isfinite(n)) { *why = "n must be finite and > 0"; return LEM_E_ARG; }
  if (n != 1.0 && (!(eps > 0.0) || !std::isfinite(eps) || max_newton < 1)) {
    *why = "n != 1 needs a finite eps > 0 and max_newton >= 1";
    return LEM_E_ARG;
  }
  if (!std::isfinite(U)) { *why = "U must be finite"; return LEM_E_ARG; }
  if (!(K >= 0.0) || !std::isfinite(K)) { *why = "K must be finite and >= 0"; return LEM_E_ARG; }
  return LEM_OK;
}

lem_status check_params(const lem_params* p, std::string* why) {
  if (!p) { *why = "params is NULL"; return LEM_E_ARG; }
  lem_status st = check_grid(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->n, p->U, p->K, p->eps,
                             p->max_newton, why);
  if (st != LEM_OK) return st;
  if (p->flags & ~(LEM_F_VALIDATE | LEM_F_PHASE_TIMERS | LEM_F_TILE_CLOCKS)) {
    *why = "unknown flag bits";
    return LEM_E_ARG;
  }
  return LEM_OK;
}

lem::GridDev make_grid(int32_t ny, int32_t nx, double dx, double dy, double dt, double m, double U,
                       double K, double n, double eps, int32_t max_newton, int64_t offset,
                       int32_t tile_base) {
  lem::GridDev g{};
  g.offset = offset;
  g.ny = ny;
  g.nx = nx;
  g.tiles_x = (nx + lem::kTW - 1) / lem::kTW;
  g.tile_base = tile_base;
  g.use_sqrt = (m == 0.5) ? 1 : 0;
  g.square = (dx == dy) ? 1 : 0;
  g.dx = dx;
  g.dy = dy;
  g.ddiag = std::sqrt(dx * dx + dy * dy);
  g.dxdy = dx * dy;
  g.dt = dt;
  g.m = m;
  g.K = K;
  g.udt = U * dt;
  g.inv_dx = 1.0 / dx;
  g.inv_dy = 1.0 / dy;
  g.inv_dd = 1.0 / g.ddiag;
  const double d[3] = {dy, dx, g.ddiag};
  g.newton = (n != 1.0) ? 1 : 0;
  for (int c = 0; c < 3; ++c) g.dn[c] = g.newton ? std::pow(d[c], n) : d[c];
  g.nexp = n;
  g.eps = eps;
  g.max_newton = max_newton;
  return g;
}

int32_t grid_tiles(const lem::GridDev& g) {
  return g.tiles_x * ((g.ny + lem::kTH - 1) / lem::kTH);
}

// Builds the descriptors of a batch; grids are laid out back to back in the
// order given (offsets must match that layout).
lem_status build_batch(const lem_grid* gs, int32_t count, std::vector<lem::GridDev>* out,
                       int64_t* cells, int32_t* ntiles, std::string* why) {
  if (!gs || count < 1) { *why = "a batch needs at least one grid"; return LEM_E_ARG; }
  if (count > 65535) { *why = "at most 65535 grids per batch"; return LEM_E_SIZE; }
  out->clear();
  int64_t off = 0, tiles = 0;
  for (int32_t i = 0; i < count; ++i) {
    const lem_grid& g = gs[i];
    lem_status st = check_grid(g.ny, g.nx, g.dx, g.dy, g.dt, g.m, g.n, g.U, g.K, g.eps,
                               g.max_newton, why);
    if (st != LEM_OK) return st;
    if (g.offset != off) { *why = "grid offsets must follow the grids back to back"; return LEM_E_ARG; }
    lem::GridDev d = make_grid(g.ny, g.nx, g.dx, g.dy, g.dt, g.m, g.U, g.K, g.n, g.eps,
                               g.max_newton, off, (int32_t)tiles);
    tiles += grid_tiles(d);
    off += (int64_t)g.ny * g.nx;
    if (off > (int64_t)INT32_MAX - 2) { *why = "a batch holds fewer than 2^31-2 cells"; return LEM_E_SIZE; }
    out->push_back(d);
  }
  *cells = off;
  *ntiles = (int32_t)tiles;
  return LEM_OK;
}

lem::StepArgs make_args(const lem_ctx* ctx, const double* d_K, const double* d_U) {
  lem::StepArgs a{};
  a.grids = ctx->w.grids;
  a.ngrids = (int32_t)ctx->grids.size();
  a.ntiles = ctx->ntiles;
  a.n = (int32_t)ctx->cells;
  a.timers = (ctx->flags & LEM_F_PHASE_TIMERS) ? 1 : 0;
  a.tile_clocks = (ctx->flags & LEM_F_TILE_CLOCKS) ? 1 : 0;
  a.Kf = d_K;
  a.Uf = d_U;
  a.w = ctx->w;
  a.tail_level = ctx->tail_level;
  a.pergrid = ctx->pergrid ? 1 : 0;
  a.chunked = (ctx->chunked && !ctx->mfd) ? 1 : 0;
  a.chunk_roots = ctx->chunk_roots;
  a.mfd = ctx->mfd ? 1 : 0;
  a.mfd_p = ctx->mfd_p;
  return a;
}

lem_status validate_inputs(lem_ctx* ctx, const double* d_h, const double* d_K, const double* d_U) {
  const int64_t n = ctx->cells;
  int32_t* flag = ctx->w.scratch;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemsetAsync");
  const double* arrs[3] = {d_h, d_K, d_U};
  for (const double* x : arrs) {
    if (!x) continue;
    e = lem::launch_validate(x, n, flag, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "validate launch");
  }
  int32_t host = 0;
  e = hipMemcpyAsync(&host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "validate readback");
  if (host) return fail(ctx, LEM_E_NONFINITE, "an input holds a NaN or an infinity");
  return LEM_OK;
}

// Automatic choice of the level pass: one workgroup per grid pays off when
// there are several grids to run side by side and none is so large that its
// one workgroup would dominate the step.
bool auto_pergrid(const lem_ctx* ctx) {
  if (ctx->grids.size() < 2) return false;
  for (const lem::GridDev& g : ctx->grids)
    if ((int64_t)g.ny * g.nx > (int64_t(1) << 21)) return false;
  return true;
}

// Threads per workgroup of the per-grid level pass.  1024 by default: even
// for 256 x 256 grids the levels of evolved landscapes are wide enough that
// more loads in flight beat the cheaper barriers of smaller workgroups
// (measured on MI355X: 100 grids to steady state, 24 s with 1024 threads,
// 29 s with 256).
int pergrid_threads(const lem_ctx* ctx) {
  return ctx->level_threads ? ctx->level_threads : lem::kBlock;
}

// One step: the tile pass, then the global level pass for crossing trees
// (multiple flow directions: routing, then the level kernel).
lem_status step(lem_ctx* ctx, lem::StepArgs& a, bool timers) {
  if (timers) (void)hipEventRecord(ctx->ev0, ctx->stream);
  hipError_t e = ctx->mfd ? lem::launch_mfd_route(a, ctx->stream)
                          : lem::launch_tile_step(a, ctx->tile_grid, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, ctx->mfd ? "routing launch" : "tile launch");
  if (timers) (void)hipEventRecord(ctx->ev1, ctx->stream);
  if (a.chunked) {
    e = lem::launch_chunk_trees(a, ctx->chunk_grid, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "chunk-stage launch");
  }
  if (timers) (void)hipEventRecord(ctx->ev2, ctx->stream);
  e = ctx->mfd      ? lem::launch_mfd_levels(a, ctx->grid, ctx->stream)
      : ctx->pergrid ? lem::launch_grid_levels(a, pergrid_threads(ctx), ctx->stream)
                     : lem::launch_global_levels(a, ctx->grid, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "level-pass launch");
  if (timers) {
    (void)hipEventRecord(ctx->ev3, ctx->stream);
    e = hipEventSynchronize(ctx->ev3);
    if (e != hipSuccess) return hip_fail(ctx, e, "timer event");
    float ms0 = 0.f, ms1 = 0.f, ms2 = 0.f;
    (void)hipEventElapsedTime(&ms0, ctx->ev0, ctx->ev1);
    (void)hipEventElapsedTime(&ms1, ctx->ev1, ctx->ev3);
    (void)hipEventElapsedTime(&ms2, ctx->ev1, ctx->ev2);
    ctx->route_ms += ms0;
    ctx->order_ms += ms1;
    ctx->chunk_ms += ms2;
  }
  return LEM_OK;
}

// The grid of every tile in `tiles` (grids hold consecutive tile ranges).
std::vector<int32_t> tile_grids(const lem_ctx* ctx, const std::vector<int32_t>& tiles) {
  std::vector<int32_t> g(tiles.size());
  for (size_t i = 0; i < tiles.size(); ++i) {
    int32_t lo = 0, hi = (int32_t)ctx->grids.size();
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) / 2;
      if (ctx->grids[mid].tile_base <= tiles[i]) lo = mid; else hi = mid;
    }
    g[i] = lo;
  }
  return g;
}

lem_status upload_tiles(lem_ctx* ctx, const std::vector<int32_t>& tiles) {
  if (tiles.empty()) return LEM_OK;
  ctx->tgrid_host = tile_grids(ctx, tiles);
  hipError_t e = hipMemcpyAsync(ctx->w.tiles, tiles.data(), sizeof(int32_t) * tiles.size(),
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->w.tgrid, ctx->tgrid_host.data(), sizeof(int32_t) * tiles.size(),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "tile list upload");
  return LEM_OK;
}

lem_status run_impl(lem_ctx* ctx, double* d_h, const uint8_t* d_rcode, const double* d_K,
                    const double* d_U, int64_t steps) {
  if (!ctx) return LEM_E_ARG;
  if (!d_h) return fail(ctx, LEM_E_ARG, "d_h is NULL");
  if (steps < 0) return fail(ctx, LEM_E_ARG, "steps must be >= 0");
  if (steps == 0) return LEM_OK;
  if (ctx->mfd && d_rcode)
    return fail(ctx, LEM_E_ARG, "fixed routing needs a D8 context");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (ctx->flags & LEM_F_VALIDATE) {
    lem_status st = validate_inputs(ctx, d_h, d_K, d_U);
    if (st != LEM_OK) return st;
  }
  lem::StepArgs a = make_args(ctx, d_K, d_U);
  a.fixed = d_rcode ? 1 : 0;
  e = lem::launch_begin_run(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "begin-run launch");
  if (d_rcode) {
    e = lem::launch_fixed_routing(a, d_rcode, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "fixed-routing launch");
  }
  const bool timers = (ctx->flags & LEM_F_PHASE_TIMERS) != 0;
  ctx->route_ms = 0.0;
  ctx->order_ms = 0.0;
  ctx->chunk_ms = 0.0;
  // Steps alternate between the caller's buffer and the workspace copy, so a
  // tile never reads a neighbour's already-updated halo.
  for (int64_t s = 0; s < steps; ++s) {
    a.step = s;
    a.h_in = (s & 1) ? ctx->w.h2 : d_h;
    a.h_out = (s & 1) ? d_h : ctx->w.h2;
    a.export_routing = (s == steps - 1) ? 1 : 0;
    lem_status st = step(ctx, a, timers);
    if (st != LEM_OK) return st;
  }
  if (steps & 1) {
    e = hipMemcpyAsync(d_h, ctx->w.h2, sizeof(double) * (size_t)ctx->cells,
                       hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "final copy");
  }
  ctx->steps_done += steps;
  ctx->last_run_steps = steps;
  ctx->has_routing = true;
  return LEM_OK;
}

lem_status create_impl(lem_ctx* ctx, void* d_workspace, size_t ws_bytes, void* hip_stream) {
  const int64_t ng = (int64_t)ctx->grids.size();
  if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0) return LEM_E_WORKSPACE;
  if (ws_bytes < lem::workspace_bytes(ctx->cells, ng, ctx->ntiles, ctx->mfd)) return LEM_E_WORKSPACE;
  ctx->stream = (hipStream_t)hip_stream;
  lem::carve(d_workspace, ctx->cells, ng, ctx->ntiles, &ctx->w, ctx->mfd);
  ctx->tiles.resize(ctx->ntiles);
  for (int32_t t = 0; t < ctx->ntiles; ++t) ctx->tiles[t] = t;
  hipError_t e = hipGetDevice(&ctx->device);
  int cus = 0, per_cu = 0, rate = 0, per_cu_chunk = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  if (e == hipSuccess) e = lem::global_kernel_occupancy(&per_cu);
  if (e == hipSuccess) e = lem::chunk_kernel_occupancy(ng > 1, &per_cu_chunk);
  int per_cu_tile = 0;
  if (e == hipSuccess) e = lem::tile_kernel_occupancy(&per_cu_tile);
  if (e == hipSuccess && ctx->mfd) {
    int per_cu_mfd = 0;
    e = lem::mfd_kernel_occupancy(&per_cu_mfd);
    if (per_cu_mfd < per_cu) per_cu = per_cu_mfd;
  }
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, ctx->device);
  if (ctx->flags & LEM_F_PHASE_TIMERS) {
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev0);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev1);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev2);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev3);
  }
  if (e != hipSuccess || per_cu < 1 || per_cu_chunk < 1 || per_cu_tile < 1) return LEM_E_HIP;
  ctx->tile_grid = cus * per_cu_tile;
  if (ctx->tile_grid >= 8) ctx->tile_grid &= ~7;
  // Chunk stage: every resident workgroup, but no more than one per 4096
  // cells (small grids have few crossing roots).
  {
    const int64_t cap = (int64_t)cus * per_cu_chunk;
    const int64_t want = (ctx->cells + 4095) / 4096;
    ctx->chunk_grid = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
  }
  ctx->chunked = !ctx->mfd;
  ctx->chunk_roots = lem::kChunkRootsDefault;
  // The global level kernel uses at most kGlobalMaxWGs resident workgroups:
  // a grid-wide barrier's cost grows with the number of participants.
  ctx->grid_max = cus * per_cu;
  ctx->grid = ctx->grid_max < lem::kGlobalMaxWGs ? ctx->grid_max : lem::kGlobalMaxWGs;
  ctx->tail_level = lem::kTailLevel;
  ctx->level_pass = LEM_LEVELS_AUTO;
  ctx->pergrid = auto_pergrid(ctx);
  ctx->level_threads = 0;
  ctx->tick_khz = (double)rate;
  e = lem::launch_zero_words(ctx->w.ctrl, sizeof(lem::Ctrl) / 4, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->w.grids, ctx->grids.data(), sizeof(lem::GridDev) * ng,
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return LEM_E_HIP;
  if (upload_tiles(ctx, ctx->tiles) != LEM_OK) return LEM_E_HIP;
  return LEM_OK;
}

lem_status routing_impl(lem_ctx* ctx, int32_t g, int32_t* d_rec, int32_t* d_depth,
                        uint32_t* d_count, int64_t* h_level_offsets, int64_t cap,
                        int64_t* h_nlevels) {
  if (!ctx) return LEM_E_ARG;
  if (ctx->mfd) return fail(ctx, LEM_E_ARG, "multiple-flow-direction routing: use lem_mfd_export");
  if (!ctx->has_routing) return fail(ctx, LEM_E_STATE, "no lem_run/lem_batch_run step yet");
  if (cap < 0) return fail(ctx, LEM_E_ARG, "cap must be >= 0");
  if (g < 0 || g >= (int32_t)ctx->grids.size()) return fail(ctx, LEM_E_ARG, "no such grid");
  const lem::GridDev& G = ctx->grids[g];
  lem::StepArgs a = make_args(ctx, nullptr, nullptr);
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess)
    e = lem::launch_export(a, g, G.offset, (int64_t)G.ny * G.nx, d_rec, d_depth, d_count,
                           ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "export launch");
  lem::Ctrl ct;
  e = hipMemcpyAsync(&ct, ctx->w.ctrl, sizeof(ct), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "routing readback");
  // The histogram spans the batch's deepest level; this grid's levels end
  // at its last non-empty bin.
  std::vector<int32_t> tmp((size_t)ct.nlevels + 1);
  e = hipMemcpy(tmp.data(), ctx->w.dhist, sizeof(int32_t) * tmp.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "level histogram readback");
  int64_t nl = ct.nlevels;
  while (nl > 1 && tmp[nl] == 0) --nl;
  if (h_nlevels) *h_nlevels = nl;
  if (h_level_offsets && cap >= nl + 1) {
    int64_t acc = 0;
    for (int64_t l = 0; l <= nl; ++l) {
      acc += (l == 0) ? 0 : tmp[l];
      h_level_offsets[l] = acc;
    }
  }
  return LEM_OK;
}

lem_status steady_impl(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                       double rtol, int64_t check_every, int64_t max_steps, int64_t* h_steps,
                       bool project);

}  // namespace

extern "C" {

size_t lem_workspace_bytes(const lem_params* p) {
  std::string why;
  if (check_params(p, &why) != LEM_OK) return 0;
  lem::GridDev g = make_grid(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->U, p->K, p->n, p->eps,
                               p->max_newton, 0, 0);
  return lem::workspace_bytes((int64_t)p->ny * p->nx, 1, grid_tiles(g));
}

lem_status lem_create(const lem_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream,
                      lem_ctx** out) {
  if (!out) return LEM_E_ARG;
  *out = nullptr;
  std::string why;
  lem_status st = check_params(p, &why);
  if (st != LEM_OK) return st;
  if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0) return LEM_E_WORKSPACE;
  if (ws_bytes < lem_workspace_bytes(p)) return LEM_E_WORKSPACE;
  lem_ctx* ctx = new (std::nothrow) lem_ctx();
  if (!ctx) return LEM_E_ARG;
  ctx->flags = p->flags;
  ctx->batch = false;
  ctx->grids.push_back(make_grid(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->U, p->K, p->n, p->eps,
                               p->max_newton, 0, 0));
  ctx->cells = (int64_t)p->ny * p->nx;
  ctx->ntiles = grid_tiles(ctx->grids[0]);
  st = create_impl(ctx, d_workspace, ws_bytes, hip_stream);
  if (st != LEM_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return LEM_OK;
}

size_t lem_batch_workspace_bytes(const lem_grid* grids, int32_t count) {
  std::vector<lem::GridDev> g;
  int64_t cells = 0;
  int32_t ntiles = 0;
  std::string why;
  if (build_batch(grids, count, &g, &cells, &ntiles, &why) != LEM_OK) return 0;
  return lem::workspace_bytes(cells, count, ntiles);
}

lem_status lem_batch_create(const lem_grid* grids, int32_t count, uint32_t flags,
                            void* d_workspace, size_t ws_bytes, void* hip_stream, lem_ctx** out) {
  if (!out) return LEM_E_ARG;
  *out = nullptr;
  if (flags & ~(LEM_F_VALIDATE | LEM_F_PHASE_TIMERS | LEM_F_TILE_CLOCKS)) return LEM_E_ARG;
  lem_ctx* ctx = new (std::nothrow) lem_ctx();
  if (!ctx) return LEM_E_ARG;
  std::string why;
  lem_status st = build_batch(grids, count, &ctx->grids, &ctx->cells, &ctx->ntiles, &why);
  if (st == LEM_OK) {
    ctx->flags = flags;
    ctx->batch = true;
    st = create_impl(ctx, d_workspace, ws_bytes, hip_stream);
  }
  if (st != LEM_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return LEM_OK;
}

lem_status lem_run(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                   int64_t steps) {
  return run_impl(ctx, d_h, nullptr, d_K, d_U, steps);
}

lem_status lem_batch_run(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                         int64_t steps) {
  return run_impl(ctx, d_h, nullptr, d_K, d_U, steps);
}

lem_status lem_batch_run_to_steady(lem_ctx* ctx, double* d_h, const double* d_K,
                                   const double* d_U, double rtol, int64_t check_every,
                                   int64_t max_steps, int64_t* h_steps) {
  return steady_impl(ctx, d_h, d_K, d_U, rtol, check_every, max_steps, h_steps, false);
}

lem_status lem_batch_project_to_steady(lem_ctx* ctx, double* d_h, const double* d_K,
                                       const double* d_U, double rtol, int64_t check_every,
                                       int64_t max_iters, int64_t* h_iters) {
  if (ctx && ctx->mfd) return fail(ctx, LEM_E_ARG, "projection needs a D8 context");
  return steady_impl(ctx, d_h, d_K, d_U, rtol, check_every, max_iters, h_iters, true);
}

}  // extern "C"

namespace {

// Runs to steady state: time steps of the method, or (project) steady-state
// projections, until each grid changes by at most rtol of its largest height.
lem_status steady_impl(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                       double rtol, int64_t check_every, int64_t max_steps, int64_t* h_steps,
                       bool project) {
  if (!ctx) return LEM_E_ARG;
  if (!d_h || !h_steps) return fail(ctx, LEM_E_ARG, "d_h and h_steps must not be NULL");
  if (!(rtol > 0.0) || check_every < 1 || max_steps < 1)
    return fail(ctx, LEM_E_ARG, "rtol must be > 0, check_every and max_steps >= 1");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (ctx->flags & LEM_F_VALIDATE) {
    lem_status st = validate_inputs(ctx, d_h, d_K, d_U);
    if (st != LEM_OK) return st;
  }
  const int32_t ng = (int32_t)ctx->grids.size();
  std::vector<char> done(ng, 0);
  int64_t active_cells = ctx->cells;
  for (int32_t g = 0; g < ng; ++g) {
    if (h_steps[g] >= 0) {  // steady on entry: not stepped, entry kept
      done[g] = 1;
      active_cells -= (int64_t)ctx->grids[g].ny * ctx->grids[g].nx;
    } else {
      h_steps[g] = -1;
    }
  }
  lem::StepArgs a = make_args(ctx, d_K, d_U);
  a.project = project ? 1 : 0;
  e = lem::launch_begin_run(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "begin-run launch");
  const bool timers = (ctx->flags & LEM_F_PHASE_TIMERS) != 0;
  ctx->route_ms = ctx->order_ms = ctx->chunk_ms = 0.0;
  std::vector<double> conv(2 * (size_t)ng);
  int64_t s = 0;
  double* cur = d_h;  // buffer holding the latest heights
  double* other = ctx->w.h2;
  lem_status st = LEM_OK;
  if (active_cells < ctx->cells) {
    // Both buffers hold the heights of the grids that are already steady.
    e = hipMemcpyAsync(other, d_h, sizeof(double) * (size_t)ctx->cells, hipMemcpyDeviceToDevice,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "initial copy");
    ctx->active.clear();
    for (int32_t g = 0; g < ng; ++g) {
      if (done[g]) continue;
      const lem::GridDev& G = ctx->grids[g];
      for (int32_t t = 0; t < grid_tiles(G); ++t) ctx->active.push_back(G.tile_base + t);
    }
    if (active_cells > 0) {
      st = upload_tiles(ctx, ctx->active);
      a.ntiles = (int32_t)ctx->active.size();
      a.n = (int32_t)active_cells;
    }
  }
  while (s < max_steps && active_cells > 0 && st == LEM_OK) {
    const int64_t k = (max_steps - s) < check_every ? (max_steps - s) : check_every;
    for (int64_t j = 0; j < k; ++j, ++s) {
      a.step = s;
      a.h_in = cur;
      a.h_out = other;
      a.export_routing = 0;
      st = step(ctx, a, timers);
      if (st != LEM_OK) break;
      double* t = cur;
      cur = other;
      other = t;
    }
    if (st != LEM_OK) break;
    // Relative change of the last step, per grid: max|dh| <= rtol * max|h|.
    lem::StepArgs c = a;
    c.h_in = other;
    c.h_out = cur;
    e = lem::launch_change(c, ctx->cells, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(conv.data(), ctx->w.conv, sizeof(double) * conv.size(),
                         hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "convergence check");
    bool changed = false;
    for (int32_t g = 0; g < ng; ++g) {
      if (!done[g] && !(std::isfinite(conv[2 * g]) && std::isfinite(conv[2 * g + 1]))) {
        st = fail(ctx, LEM_E_NONFINITE, "grid " + std::to_string(g) +
                                            ": heights are no longer finite after step " +
                                            std::to_string(s));
        break;
      }
      if (done[g] || !(conv[2 * g] <= rtol * conv[2 * g + 1])) continue;
      done[g] = 1;
      h_steps[g] = s;
      changed = true;
      // Both height buffers hold the grid's final heights from now on.
      const lem::GridDev& G = ctx->grids[g];
      e = hipMemcpyAsync(other + G.offset, cur + G.offset, sizeof(double) * G.ny * G.nx,
                         hipMemcpyDeviceToDevice, ctx->stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "freeze copy");
      active_cells -= (int64_t)G.ny * G.nx;
    }
    if (st != LEM_OK) break;
    if (changed && active_cells > 0) {
      ctx->active.clear();
      for (int32_t g = 0; g < ng; ++g) {
        if (done[g]) continue;
        const lem::GridDev& G = ctx->grids[g];
        for (int32_t t = 0; t < grid_tiles(G); ++t) ctx->active.push_back(G.tile_base + t);
      }
      st = upload_tiles(ctx, ctx->active);
      a.ntiles = (int32_t)ctx->active.size();
      a.n = (int32_t)active_cells;
    }
  }
  // Restore the full tile list for later runs.
  const lem_status st2 = upload_tiles(ctx, ctx->tiles);
  if (st == LEM_OK) st = st2;
  if (st != LEM_OK) return st;
  if (cur != d_h) {
    e = hipMemcpyAsync(d_h, cur, sizeof(double) * (size_t)ctx->cells, hipMemcpyDeviceToDevice,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "final copy");
  }
  ctx->steps_done += s;
  ctx->last_run_steps = s;
  return LEM_OK;
}

}  // namespace

extern "C" {

lem_status lem_run_fixed_routing(lem_ctx* ctx, double* d_h, const uint8_t* d_rcode,
                                 const double* d_K, const double* d_U, int64_t steps) {
  if (!ctx) return LEM_E_ARG;
  if (ctx->batch) return fail(ctx, LEM_E_ARG, "fixed routing needs a single-grid context");
  if (!d_rcode) return fail(ctx, LEM_E_ARG, "d_rcode is NULL");
  return run_impl(ctx, d_h, d_rcode, d_K, d_U, steps);
}

lem_status lem_sync(lem_ctx* ctx) {
  if (!ctx) return LEM_E_ARG;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  int32_t status = 0;
  e = hipMemcpy(&status, &ctx->w.ctrl->status, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "status readback");
  if (status != 0) {
    int32_t zero = 0;
    (void)hipMemcpy(&ctx->w.ctrl->status, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
    if (status == LEM_E_CYCLE)
      return fail(ctx, LEM_E_CYCLE, "receivers form a cycle or leave cells unreachable");
    if (status == LEM_E_HIP)
      return fail(ctx, LEM_E_HIP, "a device-wide barrier timed out");
    return fail(ctx, (lem_status)status, "fixed routing holds an invalid receiver code");
  }
  return LEM_OK;
}

lem_status lem_routing(lem_ctx* ctx, int32_t* d_rec, int32_t* d_depth, uint32_t* d_count,
                       int64_t* h_level_offsets, int64_t cap, int64_t* h_nlevels) {
  return routing_impl(ctx, 0, d_rec, d_depth, d_count, h_level_offsets, cap, h_nlevels);
}

lem_status lem_batch_routing(lem_ctx* ctx, int32_t grid, int32_t* d_rec, int32_t* d_depth,
                             uint32_t* d_count, int64_t* h_level_offsets, int64_t cap,
                             int64_t* h_nlevels) {
  return routing_impl(ctx, grid, d_rec, d_depth, d_count, h_level_offsets, cap, h_nlevels);
}

size_t lem_mfd_workspace_bytes(const lem_params* p) {
  std::string why;
  if (check_params(p, &why) != LEM_OK || p->n != 1.0) return 0;
  lem::GridDev g = make_grid(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->U, p->K, p->n, p->eps,
                             p->max_newton, 0, 0);
  return lem::workspace_bytes((int64_t)p->ny * p->nx, 1, grid_tiles(g), true);
}

lem_status lem_mfd_create(const lem_params* p, double exponent, void* d_workspace,
                          size_t ws_bytes, void* hip_stream, lem_ctx** out) {
  if (!out) return LEM_E_ARG;
  *out = nullptr;
  std::string why;
  lem_status st = check_params(p, &why);
  if (st != LEM_OK) return st;
  if (p->n != 1.0) return LEM_E_ARG;
  if (!(exponent > 0.0) || !std::isfinite(exponent)) return LEM_E_ARG;
  if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0) return LEM_E_WORKSPACE;
  if (ws_bytes < lem_mfd_workspace_bytes(p)) return LEM_E_WORKSPACE;
  lem_ctx* ctx = new (std::nothrow) lem_ctx();
  if (!ctx) return LEM_E_ARG;
  ctx->flags = p->flags;
  ctx->batch = false;
  ctx->mfd = true;
  ctx->mfd_p = exponent;
  ctx->grids.push_back(make_grid(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->U, p->K, p->n,
                                 p->eps, p->max_newton, 0, 0));
  ctx->cells = (int64_t)p->ny * p->nx;
  ctx->ntiles = grid_tiles(ctx->grids[0]);
  st = create_impl(ctx, d_workspace, ws_bytes, hip_stream);
  if (st != LEM_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return LEM_OK;
}

lem_status lem_mfd_export(lem_ctx* ctx, double* d_area, int32_t* d_level, int64_t* h_nlevels) {
  if (!ctx) return LEM_E_ARG;
  if (!ctx->mfd) return fail(ctx, LEM_E_ARG, "not a multiple-flow-direction context");
  if (!ctx->has_routing) return fail(ctx, LEM_E_STATE, "no lem_run step yet");
  hipError_t e = hipSetDevice(ctx->device);
  const size_t n = (size_t)ctx->cells;
  if (e == hipSuccess && d_area) {
    const lem::StepArgs a = make_args(ctx, nullptr, nullptr);
    e = lem::launch_mfd_export_area(a, d_area, ctx->stream);
  }
  if (e == hipSuccess && d_level)
    e = hipMemcpyAsync(d_level, ctx->w.dep_g, sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                       ctx->stream);
  lem::Ctrl ct;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&ct, ctx->w.ctrl, sizeof(ct), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "export");
  if (h_nlevels) *h_nlevels = ct.nlevels;
  return LEM_OK;
}

lem_status lem_level_history(lem_ctx* ctx, int32_t* h_levels, int64_t cap, int64_t* h_n) {
  if (!ctx || !h_n || (cap > 0 && !h_levels)) return LEM_E_ARG;
  lem::Ctrl ct;
  hipError_t e = hipMemcpyAsync(&ct, ctx->w.ctrl, sizeof(ct), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "history readback");
  int64_t n = ct.steps < lem::kHistCap ? ct.steps : lem::kHistCap;
  *h_n = n;
  if (cap < n) n = cap;
  if (n > 0) {
    e = hipMemcpy(h_levels, ctx->w.hist, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "history copy");
  }
  return LEM_OK;
}

lem_status lem_stats(lem_ctx* ctx, lem_stats_t* out) {
  if (!ctx || !out) return LEM_E_ARG;
  lem::Ctrl ct;
  hipError_t e = hipMemcpyAsync(&ct, ctx->w.ctrl, sizeof(ct), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "stats readback");
  std::memset(out, 0, sizeof(*out));
  out->steps_done = ctx->steps_done;
  out->last_nlevels = ct.nlevels;
  out->max_nlevels = ct.max_nlevels;
  out->last_run_steps = ctx->last_run_steps;
  out->phase_ms[0] = ctx->route_ms;
  out->kernel_ms[0] = ctx->route_ms;
  out->kernel_ms[1] = ctx->order_ms;
  out->kernel_ms[2] = ctx->chunk_ms;
  out->crossing_last = ct.dirty_total;
  out->crossing_run = ct.crossing_run;
  for (int k = 1; k < 4; ++k)
    out->phase_ms[k] = ctx->tick_khz > 0 ? (double)ct.ticks[k] / ctx->tick_khz : 0.0;
  for (int k = 0; k < lem::kTilePhases; ++k)
    out->tile_phase_ms[k] = ctx->tick_khz > 0 && ct.tile_wgs
                                ? (double)ct.tile_ticks[k] / ctx->tick_khz / (double)ct.tile_wgs *
                                      (double)ct.steps
                                : 0.0;
  return LEM_OK;
}

lem_status lem_set_tuning(lem_ctx* ctx, const lem_tuning* t) {
  if (!ctx || !t) return LEM_E_ARG;
  if (t->global_workgroups < 0 || t->tail_level < 0 || t->level_pass < 0 || t->level_pass > 2 ||
      (t->level_threads != 0 && t->level_threads != 256 && t->level_threads != lem::kBlock) ||
      t->chunk_pass < 0 || t->chunk_pass > 2 || t->chunk_roots < 0 ||
      t->chunk_roots > lem::kChunkMaxRoots)
    return fail(ctx, LEM_E_ARG,
                "tuning fields must be >= 0 (level_pass 0, 1 or 2; level_threads 0, 256 or 1024; "
                "chunk_pass 0, 1 or 2; chunk_roots at most 256)");
  ctx->chunked = !ctx->mfd && t->chunk_pass != LEM_CHUNKS_OFF;
  ctx->chunk_roots = t->chunk_roots ? t->chunk_roots : lem::kChunkRootsDefault;
  ctx->level_threads = t->level_threads;
  int g = t->global_workgroups ? t->global_workgroups : lem::kGlobalMaxWGs;
  ctx->grid = g < ctx->grid_max ? g : ctx->grid_max;
  ctx->tail_level = t->tail_level ? t->tail_level : lem::kTailLevel;
  ctx->level_pass = t->level_pass;
  ctx->pergrid = t->level_pass == LEM_LEVELS_PER_GRID ||
                 (t->level_pass == LEM_LEVELS_AUTO && auto_pergrid(ctx));
  return LEM_OK;
}

lem_status lem_get_tuning(const lem_ctx* ctx, lem_tuning* out) {
  if (!ctx || !out) return LEM_E_ARG;
  out->global_workgroups = ctx->grid;
  out->tail_level = ctx->tail_level;
  out->level_pass = ctx->pergrid ? LEM_LEVELS_PER_GRID : LEM_LEVELS_GLOBAL;
  out->level_threads = pergrid_threads(ctx);
  out->chunk_pass = ctx->chunked ? LEM_CHUNKS_ON : LEM_CHUNKS_OFF;
  out->chunk_roots = ctx->chunk_roots;
  return LEM_OK;
}

lem_status lem_destroy(lem_ctx* ctx) {
  if (!ctx) return LEM_OK;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
  if (ctx->ev3) (void)hipEventDestroy(ctx->ev3);
  delete ctx;
  return LEM_OK;
}

const char* lem_status_str(lem_status s) {
  switch (s) {
    case LEM_OK: return "LEM_OK";
    case LEM_E_ARG: return "LEM_E_ARG: invalid argument";
    case LEM_E_SIZE: return "LEM_E_SIZE: grid size out of range";
    case LEM_E_WORKSPACE: return "LEM_E_WORKSPACE: workspace missing, misaligned or too small";
    case LEM_E_NONFINITE: return "LEM_E_NONFINITE: non-finite input";
    case LEM_E_CYCLE: return "LEM_E_CYCLE: receivers form a cycle";
    case LEM_E_HIP: return "LEM_E_HIP: HIP runtime error";
    case LEM_E_STATE: return "LEM_E_STATE: context not ready";
  }
  return "unknown lem_status";
}

const char* lem_last_error(const lem_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"
