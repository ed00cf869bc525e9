// lem_capi.cpp -- the C ABI (include/lem.h): argument checking, workspace
// carving, per-context state and error strings.  Everything the method
// computes runs in the kernels of lem_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lem.h"
#include "lem_internal.h"

struct lem_ctx {
  lem_params p;
  hipStream_t stream;
  lem::Work w;
  int grid;              // workgroups of the cooperative level kernel
  int grid_max;          // most that stay resident on this device
  int tail_level;
  int device;
  double tick_khz;       // device wall-clock rate
  int64_t steps_done;
  int64_t last_run_steps;
  bool has_routing;
  double route_ms;       // accumulated with LEM_F_PHASE_TIMERS
  double order_ms;
  hipEvent_t ev0, ev1, ev2;
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

lem_status check_params(const lem_params* p, std::string* why) {
  if (!p) { *why = "params is NULL"; return LEM_E_ARG; }
  if (p->ny < 3 || p->nx < 3) { *why = "ny and nx must be >= 3"; return LEM_E_SIZE; }
  if ((int64_t)p->ny * (int64_t)p->nx > (int64_t)INT32_MAX - 2) {
    *why = "ny*nx must be below 2^31-2";
    return LEM_E_SIZE;
  }
  if (!(p->dx > 0.0) || !(p->dy > 0.0) || !std::isfinite(p->dx) || !std::isfinite(p->dy)) {
    *why = "dx and dy must be finite and > 0";
    return LEM_E_ARG;
  }
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) { *why = "dt must be finite and > 0"; return LEM_E_ARG; }
  if (!(p->m >= 0.0) || !std::isfinite(p->m)) { *why = "m must be finite and >= 0"; return LEM_E_ARG; }
  if (p->n != 1.0) { *why = "only the slope exponent n = 1 is supported"; return LEM_E_ARG; }
  if (!std::isfinite(p->U)) { *why = "U must be finite"; return LEM_E_ARG; }
  if (!(p->K >= 0.0) || !std::isfinite(p->K)) { *why = "K must be finite and >= 0"; return LEM_E_ARG; }
  if (p->flags & ~(LEM_F_VALIDATE | LEM_F_PHASE_TIMERS)) { *why = "unknown flag bits"; return LEM_E_ARG; }
  return LEM_OK;
}

lem::StepArgs make_args(const lem_ctx* ctx, const double* d_K, const double* d_U) {
  lem::StepArgs a{};
  const lem_params& p = ctx->p;
  a.ny = p.ny;
  a.nx = p.nx;
  a.n = p.ny * p.nx;
  a.use_sqrt = (p.m == 0.5) ? 1 : 0;
  a.dx = p.dx;
  a.dy = p.dy;
  a.ddiag = std::sqrt(p.dx * p.dx + p.dy * p.dy);
  a.dxdy = p.dx * p.dy;
  a.dt = p.dt;
  a.m = p.m;
  a.K = p.K;
  a.udt = p.U * p.dt;
  a.Kf = d_K;
  a.Uf = d_U;
  a.w = ctx->w;
  a.step = 0;
  a.timers = (p.flags & LEM_F_PHASE_TIMERS) ? 1 : 0;
  a.tiles_x = (p.nx + lem::kTW - 1) / lem::kTW;
  a.tiles_y = (p.ny + lem::kTH - 1) / lem::kTH;
  a.tail_level = ctx->tail_level;
  return a;
}

lem_status validate_inputs(lem_ctx* ctx, const double* d_h, const double* d_K, const double* d_U) {
  const int64_t n = (int64_t)ctx->p.ny * ctx->p.nx;
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

lem_status run_impl(lem_ctx* ctx, double* d_h, const uint8_t* d_rcode, const double* d_K,
                    const double* d_U, int64_t steps) {
  if (!ctx) return LEM_E_ARG;
  if (!d_h) return fail(ctx, LEM_E_ARG, "d_h is NULL");
  if (steps < 0) return fail(ctx, LEM_E_ARG, "steps must be >= 0");
  if (steps == 0) return LEM_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (ctx->p.flags & LEM_F_VALIDATE) {
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
  const bool timers = (ctx->p.flags & LEM_F_PHASE_TIMERS) != 0;
  ctx->route_ms = 0.0;
  ctx->order_ms = 0.0;
  // Steps alternate between the caller's buffer and the workspace copy, so a
  // tile never reads a neighbour's already-updated halo.
  for (int64_t s = 0; s < steps; ++s) {
    a.step = s;
    a.h_in = (s & 1) ? ctx->w.h2 : d_h;
    a.h_out = (s & 1) ? d_h : ctx->w.h2;
    a.export_routing = (s == steps - 1) ? 1 : 0;
    if (timers) (void)hipEventRecord(ctx->ev0, ctx->stream);
    e = lem::launch_tile_step(a, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "tile launch");
    if (timers) (void)hipEventRecord(ctx->ev1, ctx->stream);
    e = lem::launch_global_levels(a, ctx->grid, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "global-level launch");
    if (timers) {
      (void)hipEventRecord(ctx->ev2, ctx->stream);
      e = hipEventSynchronize(ctx->ev2);
      if (e != hipSuccess) return hip_fail(ctx, e, "timer event");
      float ms0 = 0.f, ms1 = 0.f;
      (void)hipEventElapsedTime(&ms0, ctx->ev0, ctx->ev1);
      (void)hipEventElapsedTime(&ms1, ctx->ev1, ctx->ev2);
      ctx->route_ms += ms0;
      ctx->order_ms += ms1;
    }
  }
  if (steps & 1) {
    e = hipMemcpyAsync(d_h, ctx->w.h2, sizeof(double) * (size_t)a.n, hipMemcpyDeviceToDevice,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "final copy");
  }
  ctx->steps_done += steps;
  ctx->last_run_steps = steps;
  ctx->has_routing = true;
  return LEM_OK;
}

}  // namespace

extern "C" {

size_t lem_workspace_bytes(const lem_params* p) {
  std::string why;
  if (check_params(p, &why) != LEM_OK) return 0;
  return lem::workspace_bytes((int64_t)p->ny * p->nx);
}

lem_status lem_create(const lem_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream,
                      lem_ctx** out) {
  if (!out) return LEM_E_ARG;
  *out = nullptr;
  std::string why;
  lem_status st = check_params(p, &why);
  if (st != LEM_OK) return st;
  const int64_t n = (int64_t)p->ny * p->nx;
  if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0) return LEM_E_WORKSPACE;
  if (ws_bytes < lem::workspace_bytes(n)) return LEM_E_WORKSPACE;
  lem_ctx* ctx = new (std::nothrow) lem_ctx();
  if (!ctx) return LEM_E_ARG;
  ctx->p = *p;
  ctx->stream = (hipStream_t)hip_stream;
  lem::carve(d_workspace, n, &ctx->w);
  hipError_t e = hipGetDevice(&ctx->device);
  int cus = 0, per_cu = 0, rate = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  if (e == hipSuccess) e = lem::global_kernel_occupancy(&per_cu);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, ctx->device);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev0);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev1);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev2);
  if (e != hipSuccess || per_cu < 1) {
    delete ctx;
    return LEM_E_HIP;
  }
  // The global level kernel uses at most kGlobalMaxWGs resident workgroups:
  // a grid-wide barrier's cost grows with the number of participants.
  ctx->grid_max = cus * per_cu;
  ctx->grid = ctx->grid_max < lem::kGlobalMaxWGs ? ctx->grid_max : lem::kGlobalMaxWGs;
  ctx->tail_level = lem::kTailLevel;
  ctx->tick_khz = (double)rate;
  e = hipMemsetAsync(ctx->w.ctrl, 0, sizeof(lem::Ctrl), ctx->stream);
  if (e != hipSuccess) {
    delete ctx;
    return LEM_E_HIP;
  }
  *out = ctx;
  return LEM_OK;
}

lem_status lem_run(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                   int64_t steps) {
  return run_impl(ctx, d_h, nullptr, d_K, d_U, steps);
}

lem_status lem_run_fixed_routing(lem_ctx* ctx, double* d_h, const uint8_t* d_rcode,
                                 const double* d_K, const double* d_U, int64_t steps) {
  if (!ctx) return LEM_E_ARG;
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
    return fail(ctx, (lem_status)status, "fixed routing holds an invalid receiver code");
  }
  return LEM_OK;
}

lem_status lem_routing(lem_ctx* ctx, int32_t* d_rec, int32_t* d_depth, uint32_t* d_count,
                       int64_t* h_level_offsets, int64_t cap, int64_t* h_nlevels) {
  if (!ctx) return LEM_E_ARG;
  if (!ctx->has_routing) return fail(ctx, LEM_E_STATE, "no step has run on this context");
  if (cap < 0) return fail(ctx, LEM_E_ARG, "cap must be >= 0");
  lem::StepArgs a = make_args(ctx, nullptr, nullptr);
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = lem::launch_export(a, d_rec, d_depth, d_count, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "export launch");
  lem::Ctrl ct;
  e = hipMemcpyAsync(&ct, ctx->w.ctrl, sizeof(ct), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "routing readback");
  const int64_t nl = ct.nlevels;
  if (h_nlevels) *h_nlevels = nl;
  if (h_level_offsets && cap >= nl + 1) {
    int32_t* tmp = new (std::nothrow) int32_t[nl + 1];
    if (!tmp) return fail(ctx, LEM_E_ARG, "host allocation failed");
    e = hipMemcpy(tmp, ctx->w.dhist, sizeof(int32_t) * (nl + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
      int64_t acc = 0;
      for (int64_t l = 0; l <= nl; ++l) {
        acc += (l == 0) ? 0 : tmp[l];
        h_level_offsets[l] = acc;
      }
    }
    delete[] tmp;
    if (e != hipSuccess) return hip_fail(ctx, e, "level histogram readback");
  }
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
  out->crossing_last = ct.dirty_total;
  out->crossing_run = ct.crossing_run;
  for (int k = 1; k < 4; ++k)
    out->phase_ms[k] = ctx->tick_khz > 0 ? (double)ct.ticks[k] / ctx->tick_khz : 0.0;
  return LEM_OK;
}

lem_status lem_set_tuning(lem_ctx* ctx, const lem_tuning* t) {
  if (!ctx || !t) return LEM_E_ARG;
  if (t->global_workgroups < 0 || t->tail_level < 0)
    return fail(ctx, LEM_E_ARG, "tuning fields must be >= 0");
  int g = t->global_workgroups ? t->global_workgroups : lem::kGlobalMaxWGs;
  ctx->grid = g < ctx->grid_max ? g : ctx->grid_max;
  ctx->tail_level = t->tail_level ? t->tail_level : lem::kTailLevel;
  return LEM_OK;
}

lem_status lem_get_tuning(const lem_ctx* ctx, lem_tuning* out) {
  if (!ctx || !out) return LEM_E_ARG;
  out->global_workgroups = ctx->grid;
  out->tail_level = ctx->tail_level;
  return LEM_OK;
}

lem_status lem_destroy(lem_ctx* ctx) {
  if (!ctx) return LEM_OK;
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipEventDestroy(ctx->ev0);
  (void)hipEventDestroy(ctx->ev1);
  (void)hipEventDestroy(ctx->ev2);
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
