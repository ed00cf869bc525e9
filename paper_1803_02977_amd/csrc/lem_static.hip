// lem_static.hip -- lem_run_static: time steps over a workspace that lives in
// a file-scope device array, for callers that cannot allocate device memory.
//
// The array below is the whole workspace of such a run (the same layout
// lem_create carves from a caller's workspace).  In host code its name is
// only a stand-in for the symbol, not a device address: the device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and kept in g_scratch_ptr, and only that pointer is ever handed
// to the library.  Every device holds its own copy of the array until the
// process ends; calls on one device share it, so such calls must not
// overlap (their results would race).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lem.h"

namespace {

constexpr size_t kStaticWorkspaceBytes = size_t(16) << 20;
static_assert(kStaticWorkspaceBytes == LEM_STATIC_WORKSPACE_BYTES, "header and array agree");

__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device

// The device address of this device's copy of `scratch` (looked up once).
hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255u) != 0) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" lem_status lem_run_static(const lem_params* p, double* d_h, const double* d_K,
                                     const double* d_U, int64_t steps, void* hip_stream) {
  if (!p || !d_h || steps < 0) return LEM_E_ARG;
  if (p->flags & (LEM_F_PHASE_TIMERS | LEM_F_TILE_CLOCKS)) return LEM_E_ARG;
  const size_t need = lem_workspace_bytes(p);
  if (need == 0) return LEM_E_ARG;
  if (need > kStaticWorkspaceBytes) return LEM_E_WORKSPACE;
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices)
    return LEM_E_HIP;
  void* ws = nullptr;
  if (scratch_address(device, &ws) != hipSuccess) return LEM_E_HIP;
  lem_ctx* ctx = nullptr;
  lem_status st = lem_create(p, ws, kStaticWorkspaceBytes, hip_stream, &ctx);
  if (st != LEM_OK) return st;
  st = lem_run(ctx, d_h, d_K, d_U, steps);
  if (st == LEM_OK) st = lem_sync(ctx);
  const lem_status st2 = lem_destroy(ctx);
  return st != LEM_OK ? st : st2;
}
