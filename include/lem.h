/*
 * lem.h -- C ABI of the MI355X (gfx950) landscape-evolution library.
 *
 * The library runs the per-timestep hot path of R. Barnes, "Accelerating a
 * Landscape Evolution Model with Parallelism" (arXiv:1803.02977) on one GPU:
 *   Step 2 / Algorithm 1  D8 steepest-descent receivers,
 *   Step 3 / Algorithm 2  donor inversion,
 *   Step 4 / Algorithm 3  breadth-first levels outward from cells without a
 *                         receiver,
 *   Step 5 / Algorithm 4  drainage area (Equation "flow_acc") in reverse
 *                         level order,
 *   Step 6 / Algorithm 5  uplift, and
 *   Step 7 / Algorithm 6  implicit stream-power erosion (Equation
 *                         "streampower" with slope exponent n = 1) in level
 *                         order,
 * repeated once per time step ("Rinse, Repeat").
 *
 * Conventions shared by every entry point:
 *  - Grids are FP64, row-major, ny rows by nx columns; cell (x, y) is element
 *    y*nx + x (Step 1).  The perimeter is the fixed base level (section "The
 *    Equation"): perimeter cells are never written and pass no flow.
 *  - Pointers named d_* are device pointers on the GPU that was current when
 *    the context was created; pointers named h_* are host pointers.  The
 *    caller owns every buffer.  The library allocates no device memory: its
 *    scratch space is the caller's workspace (see lem_workspace_bytes).
 *  - Work is enqueued on the HIP stream given to lem_create and returns
 *    before it completes; device buffers must stay valid until the stream
 *    has finished it.  Calls on one context must not overlap in time.
 *  - Every call returns a lem_status; nothing is thrown or aborted across the
 *    ABI.  Argument errors are detected before anything is enqueued and leave
 *    all buffers untouched.  Errors found by the device (LEM_E_CYCLE) are
 *    reported by the next lem_sync; the heights are then unspecified.
 */
#ifndef LEM_H
#define LEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lem_status {
  LEM_OK = 0,
  LEM_E_ARG = 1,        /* a NULL pointer, a bad size or a bad parameter          */
  LEM_E_SIZE = 2,       /* the grid is too small (< 3x3) or too large (> 2^31-1)  */
  LEM_E_WORKSPACE = 3,  /* the workspace is missing, misaligned or too small      */
  LEM_E_NONFINITE = 4,  /* LEM_F_VALIDATE found a NaN or infinity in an input, or
                           a run to steady state produced one                     */
  LEM_E_CYCLE = 5,      /* receivers form a cycle (only possible with fixed routing) */
  LEM_E_HIP = 6,        /* a HIP runtime call failed                              */
  LEM_E_STATE = 7       /* the call needs state the context does not have yet     */
} lem_status;

/* lem_params.flags */
#define LEM_F_VALIDATE 0x1u     /* scan h, K and U for non-finite values before a run */
#define LEM_F_PHASE_TIMERS 0x2u /* record per-phase device time with HIP events       */
#define LEM_F_TILE_CLOCKS 0x4u  /* per-phase device clocks in every tile workgroup
                                   (lem_stats.tile_phase_ms); slows the tile pass    */

/* Problem statement (section "The Equation"; Step 1 "Initialization"):
 *   ny, nx  rows and columns, each >= 3, ny*nx <= 2^31-1;
 *   dx, dy  cell size in metres (> 0); diagonal neighbours are
 *           sqrt(dx*dx + dy*dy) apart;
 *   dt      time step in years (> 0);
 *   m       exponent of the drainage area, m-hat (>= 0, finite);
 *   n       exponent of the slope, n-hat (> 0, finite).  For n = 1 the
 *           erosion of Step 7 uses the closed form (h0 + F*h_r)/(1 + F),
 *           the point the Newton-Raphson loop of Algorithm 6 reaches in one
 *           iteration; otherwise that loop runs per cell;
 *   U       uplift rate u-hat in m/yr, used where no U field is given;
 *   K       erodibility in 1/yr (>= 0), used where no K field is given;
 *   eps     Newton tolerance epsilon of Algorithm 6 in metres (> 0 when
 *           n != 1; ignored for n = 1): the loop stops once two iterates
 *           differ by at most eps.  An iterate that would not lie above
 *           the receiver's new height is replaced by the midpoint between
 *           the receiver and the previous iterate; a cell whose uplifted
 *           height is not above its receiver's new height keeps it;
 *   max_newton  iteration limit of that loop (>= 1 when n != 1);
 *   flags   LEM_F_* bits.                                                    */
typedef struct lem_params {
  int32_t ny, nx;
  double dx, dy;
  double dt;
  double m;
  double n;
  double U, K;
  double eps;
  int32_t max_newton;
  uint32_t flags;
} lem_params;

/* Per-context statistics (filled by lem_stats). */
typedef struct lem_stats_t {
  int64_t steps_done;      /* steps completed by all lem_run* calls on this context  */
  int64_t last_nlevels;    /* number of levels (Algorithm 3) of the most recent step */
  int64_t max_nlevels;     /* largest level count of any step of the last run        */
  int64_t last_run_steps;  /* steps of the last run                                  */
  double phase_ms[4];      /* device ms of the last run with LEM_F_PHASE_TIMERS:
                              [0] tile pass (receivers, donors, levels, counts and
                              heights of trees inside one tile), [1] level
                              ordering, [2] accumulation, [3] uplift+erosion of the
                              trees that cross tile edges (1-3 by the device clock
                              of one workgroup: the chunk stage's first workgroup
                              when that stage runs, else the global level kernel's
                              first; the per-grid level pass adds, per step and
                              phase, the longest time of any of its workgroups)    */
  double kernel_ms[3];     /* HIP-event ms of the last run with LEM_F_PHASE_TIMERS,
                              summed over its steps: [0] the tile pass, [1] the
                              trees that cross tile edges (chunk stage and level
                              pass together), [2] the chunk stage alone (0 when it
                              is off)                                              */
  int64_t crossing_last;   /* cells of the most recent step whose drainage tree
                              crosses a tile edge (resolved by the global pass)     */
  int64_t crossing_run;    /* the same, summed over the steps of the last run       */
  double tile_phase_ms[6]; /* with LEM_F_TILE_CLOCKS: device-clock ms of one tile
                              workgroup on average, summed over the steps of the last
                              run, per phase: [0] staging the heights, [1] receivers,
                              [2] donor masks, walks to the tile-local roots and
                              counts, [3] trees inside the tile and their depth,
                              [4] uplift and erosion level by level, [5] write-back
                              and the crossing roots' queue                         */
} lem_stats_t;

typedef struct lem_ctx lem_ctx;

/* Bytes of device workspace a context with these parameters needs, or 0 if
 * the parameters are invalid.  The workspace holds the receiver codes, donor
 * masks, the level queue and its offsets, drainage counts and the queue-order
 * heights, a second height buffer and the routing export (Steps 2 to 7); it
 * is about 56 bytes per cell. */
size_t lem_workspace_bytes(const lem_params* p);

/* Validates p and creates a context that uses d_workspace (device memory of
 * ws_bytes >= lem_workspace_bytes(p), 256-byte aligned, owned by the caller,
 * valid for the life of the context) and enqueues on hip_stream (a
 * hipStream_t; NULL means the default stream).  Allocates host memory only.
 * On success *out receives the context. */
lem_status lem_create(const lem_params* p, void* d_workspace, size_t ws_bytes,
                      void* hip_stream, lem_ctx** out);

/* Multiple flow directions (section "Multiple Flow Directions"; figure
 * "Multiple-flow directions").  Every strictly lower neighbour of an
 * interior cell is one of its receivers and gets the share S^p / sum_j S_j^p
 * of the cell's flow, S = (h_c - h_k)/dist_k the slope towards it and p =
 * `exponent` (> 0; 1 shares in proportion to the slope).  A cell's level is
 * the longest descending path from it to a cell without receivers, so every
 * receiver is processed before its donors.  Drainage area: own cell area
 * plus each donor's share of its area.  Erosion (n = 1 only): backward Euler
 * of dh_c/dt = U - sum_k K (s_k A_c)^m S_k over the receivers, i.e.
 * h_c' = (h0 + sum_k F_k h_k') / (1 + sum_k F_k), F_k = K dt (s_k A_c)^m /
 * dist_k, sums in neighbour order.  The paper gives no sharing rule; this
 * one follows the slope-weighted routers it cites.
 *
 * lem_mfd_workspace_bytes: as lem_workspace_bytes (0 also for n != 1).
 * lem_mfd_create: as lem_create for a single grid routed this way; lem_run
 *   (with optional K and U fields), lem_sync, lem_stats, lem_set_tuning and
 *   lem_destroy work on it; lem_run_fixed_routing and lem_routing return
 *   LEM_E_ARG.  LEM_E_ARG for n != 1 or an exponent that is not finite and > 0.
 *   In lem_stats of such a context kernel_ms[0] is the routing kernel,
 *   kernel_ms[1] the level kernel, and phase_ms[1..3] its levels, areas and
 *   erosion; crossing_last counts every cell (all go through the level
 *   kernel).
 * lem_mfd_export: drainage area (m^2, FP64, ny*nx) and level per cell of the
 *   last step to device arrays (either may be NULL); *h_nlevels (may be NULL)
 *   receives the number of levels.  Synchronizes the stream.  LEM_E_STATE
 *   before the first step, LEM_E_ARG on a D8 context. */
size_t lem_mfd_workspace_bytes(const lem_params* p);
lem_status lem_mfd_create(const lem_params* p, double exponent, void* d_workspace,
                          size_t ws_bytes, void* hip_stream, lem_ctx** out);
lem_status lem_mfd_export(lem_ctx* ctx, double* d_area, int32_t* d_level, int64_t* h_nlevels);

/* Enqueues `steps` time steps (Steps 2 to 7, repeated) on d_h, updated in
 * place.  d_K and d_U are optional per-cell fields (NULL: use p->K, p->U),
 * read-only, ny*nx doubles each.  Each step routes flow on the heights it
 * starts from, then uplifts every interior cell by U*dt and erodes every cell
 * that has a receiver by the implicit n = 1 update
 * h <- (h + F*h_rec)/(1 + F), F = K*dt*A^m/dist, A = dx*dy*(upstream cells).
 * steps == 0 is a no-op. */
lem_status lem_run(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                   int64_t steps);

/* As lem_run, but Step 2 is replaced by fixed receivers given as direction
 * codes d_rcode[ny*nx] (0..7 = neighbour (dy,dx) in the order (-1,-1) (-1,0)
 * (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1); 8 = no receiver).  Codes must stay
 * inside the grid; perimeter cells must be 8.  Receivers that form a cycle
 * are reported as LEM_E_CYCLE by lem_sync.  Intended for tests and for
 * callers that route flow themselves. */
lem_status lem_run_fixed_routing(lem_ctx* ctx, double* d_h, const uint8_t* d_rcode,
                                 const double* d_K, const double* d_U, int64_t steps);

/* Waits for the context's stream and reports device-detected errors of the
 * work enqueued so far (LEM_E_CYCLE), then clears them. */
lem_status lem_sync(lem_ctx* ctx);

/* Exports the routing of the most recent step (computed from that step's
 * starting heights): per cell the receiver index d_rec (itself when the cell
 * has no receiver), the level d_depth (Algorithm 3: 0 for cells without a
 * receiver) and the number of upstream cells d_count (drainage area divided
 * by dx*dy, Equation "flow_acc"); and the level offsets into the queue,
 * h_level_offsets[0..nlevels] (offset 0 is 0, the last is ny*nx), written
 * when cap >= nlevels + 1.  *h_nlevels receives nlevels.  Any d_* pointer
 * may be NULL.  Synchronizes the stream.  LEM_E_STATE before any step. */
lem_status lem_routing(lem_ctx* ctx, int32_t* d_rec, int32_t* d_depth, uint32_t* d_count,
                       int64_t* h_level_offsets, int64_t cap, int64_t* h_nlevels);

/* ------------------------------------------------------------------------
 * Batched realizations.  Many independent grids (each with its own size and
 * parameters, slope exponent 1) advance together: every time step covers
 * all of them in one tile launch and one level launch, so small grids share
 * the GPU instead of each paying its own launches and barriers (the paper
 * notes that spare GPU capacity can process other models at the same time,
 * section "GPU Implementation").  Heights of all grids live in one device
 * buffer, grid after grid, each row-major. */
typedef struct lem_grid {
  int32_t ny, nx;      /* rows and columns, each >= 3                              */
  double dx, dy;       /* cell size [m] > 0                                        */
  double dt;           /* time step [yr] > 0                                       */
  double m;            /* area exponent >= 0                                       */
  double U, K;         /* uplift rate [m/yr], erodibility [1/yr] >= 0 (scalars)    */
  double n;            /* slope exponent > 0; as in lem_params                     */
  double eps;          /* Newton tolerance (n != 1); as in lem_params              */
  int32_t max_newton;  /* Newton iteration limit (n != 1); as in lem_params        */
  int32_t pad;         /* unused                                                   */
  int64_t offset;      /* index of the grid's first cell in the batch buffer; must
                          equal the sum of ny*nx of the grids before it           */
} lem_grid;

/* Workspace bytes for a batch, or 0 if a descriptor is invalid (at most
 * 65535 grids and fewer than 2^31-2 cells in total). */
size_t lem_batch_workspace_bytes(const lem_grid* grids, int32_t count);

/* As lem_create for a batch of `count` grids (host array, copied).  flags:
 * LEM_F_VALIDATE, LEM_F_PHASE_TIMERS and/or LEM_F_TILE_CLOCKS. */
lem_status lem_batch_create(const lem_grid* grids, int32_t count, uint32_t flags,
                            void* d_workspace, size_t ws_bytes, void* hip_stream,
                            lem_ctx** out);

/* Enqueues `steps` time steps of every grid of the batch on d_h (the batch
 * buffer, updated in place); each grid evolves exactly as it would alone.
 * d_K and d_U are optional per-cell fields laid out like d_h (NULL: each
 * grid's scalar K, U). */
lem_status lem_batch_run(lem_ctx* ctx, double* d_h, const double* d_K, const double* d_U,
                         int64_t steps);

/* Steps every grid until its heights stop changing: after every
 * `check_every` steps a grid whose last step changed no cell by more than
 * rtol * max|h| is frozen (it is no longer stepped).  Stops when all grids
 * are frozen or after max_steps steps.  h_steps[count] is read and written:
 * a grid with h_steps[g] >= 0 on entry counts as steady already (it is not
 * stepped and its entry is kept), which lets a long run continue over
 * several calls; every other grid receives the number of steps this call
 * took it to converge, or -1.  A grid whose heights stop being finite (a
 * NaN or infinity in its change or its heights) ends the call with
 * LEM_E_NONFINITE; the heights are then unspecified.  Synchronizes the
 * stream. */
lem_status lem_batch_run_to_steady(lem_ctx* ctx, double* d_h, const double* d_K,
                                   const double* d_U, double rtol, int64_t check_every,
                                   int64_t max_steps, int64_t* h_steps);

/* As lem_batch_run_to_steady, with steady-state projections in place of
 * time steps (an accelerator of runs to steady state, not part of the paper's
 * method).  A projection computes the routing of the current heights as a
 * step does (Steps 2-5), uplifts cells without a receiver (Step 6), and gives
 * every cell with a receiver, in level order, the height at which the
 * implicit update of Step 7 would leave it unchanged given its receiver's
 * new height: h_r + U*dt/F for n = 1, h_r + (U*dt/F)^(1/n) otherwise (F as in
 * Algorithm 6; F = 0 keeps the uplifted height).  Once the routing stops
 * changing the heights are a steady state of the method, which a following
 * lem_batch_run_to_steady confirms in a few steps.  h_iters receives the
 * projections each grid took (-1: not converged within max_iters).
 * LEM_E_ARG on a multiple-flow-direction context. */
lem_status lem_batch_project_to_steady(lem_ctx* ctx, double* d_h, const double* d_K,
                                       const double* d_U, double rtol, int64_t check_every,
                                       int64_t max_iters, int64_t* h_iters);

/* lem_routing for grid `grid` of the batch (after lem_batch_run); d_rec,
 * d_depth and d_count hold that grid's cells only and indices are local to
 * the grid. */
lem_status lem_batch_routing(lem_ctx* ctx, int32_t grid, int32_t* d_rec, int32_t* d_depth,
                             uint32_t* d_count, int64_t* h_level_offsets, int64_t cap,
                             int64_t* h_nlevels);

/* Copies the level count of each step of the last run into h_levels
 * (up to cap entries; *h_n receives the number of steps recorded). */
lem_status lem_level_history(lem_ctx* ctx, int32_t* h_levels, int64_t cap, int64_t* h_n);

/* Fills *out; synchronizes the stream. */
lem_status lem_stats(lem_ctx* ctx, lem_stats_t* out);

/* Launch tuning of a context (performance only; results are identical for
 * every setting).  chunk_pass: LEM_CHUNKS_ON (or 0, the default) runs a
 * first stage for the trees that cross tile edges: workgroups take chunks
 * of chunk_roots of their roots (1..256; 0 = default 128) from a device work
 * counter and finish those trees in on-chip memory with workgroup barriers
 * only; chunks whose trees need more room go on to the level pass below.
 * LEM_CHUNKS_OFF leaves every such tree to the level pass.
 * global_workgroups: workgroups of 1024 threads in the
 * cooperative level kernel for trees that cross tile edges (0 = default,
 * clamped to what the device can keep resident); tail_level: levels with
 * fewer cells than this are handled by one workgroup without grid-wide
 * barriers (0 = default, >= 1); level_pass: how a batch orders the trees
 * that cross tile edges (Steps 4-7): LEM_LEVELS_GLOBAL, one cooperative
 * pass over the whole batch with device-wide barriers between levels, or
 * LEM_LEVELS_PER_GRID, one workgroup per grid with workgroup barriers only,
 * the grids running concurrently; 0 = automatic (per grid for batches of
 * two or more grids of at most 2^21 cells each, else global);
 * level_threads: threads of each per-grid workgroup, 256 or 1024 (0 =
 * automatic: 1024). */
#define LEM_LEVELS_AUTO 0
#define LEM_LEVELS_GLOBAL 1
#define LEM_LEVELS_PER_GRID 2
#define LEM_CHUNKS_AUTO 0
#define LEM_CHUNKS_ON 1
#define LEM_CHUNKS_OFF 2
typedef struct lem_tuning {
  int32_t global_workgroups;
  int32_t tail_level;
  int32_t level_pass;
  int32_t level_threads;
  int32_t chunk_pass;
  int32_t chunk_roots;
} lem_tuning;

/* Applies *t to later runs on ctx.  LEM_E_ARG for negative fields. */
lem_status lem_set_tuning(lem_ctx* ctx, const lem_tuning* t);

/* Current settings (after defaults and clamping). */
lem_status lem_get_tuning(const lem_ctx* ctx, lem_tuning* out);

/* Destroys the context (host state only; the workspace stays the caller's).
 * Waits for the stream first.  NULL is a no-op. */
lem_status lem_destroy(lem_ctx* ctx);

/* Static description of a status code. */
const char* lem_status_str(lem_status s);

/* Message of the most recent error on this context ("" if none). */
const char* lem_last_error(const lem_ctx* ctx);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, serving loops, harnesses that forbid allocation): `steps` time
 * steps of one grid as lem_create + lem_run + lem_sync + lem_destroy would
 * run them, over a workspace held in a device array inside the library
 * (LEM_STATIC_WORKSPACE_BYTES on each device the library runs on, kept until
 * the process ends) instead of one the caller passes.  Nothing is allocated
 * on the device and no allocating library routine is called.
 *   p        grid and parameters as for lem_create; LEM_F_PHASE_TIMERS and
 *            LEM_F_TILE_CLOCKS are rejected (LEM_E_ARG);
 *   d_h      float64 ny*nx heights on the current device, row-major,
 *            updated in place; d_K, d_U optional per-cell fields (NULL:
 *            the scalars in p);
 *   hip_stream  a hipStream_t of the current device (NULL: default stream).
 * Returns after the stream has finished the steps.  Grids whose
 * lem_workspace_bytes(p) exceeds LEM_STATIC_WORKSPACE_BYTES (more than
 * 262,144 cells, e.g. 512 x 512, in any shape) are rejected with
 * LEM_E_WORKSPACE before anything is enqueued; invalid parameters give the
 * status lem_create gives.  Every call on one device uses the same array,
 * which keeps the last call's contents (the library clears what must start
 * at zero): calls that overlap on one device, from several threads or
 * streams, race and their results are unspecified. */
#define LEM_STATIC_WORKSPACE_BYTES ((size_t)16 << 20)
lem_status lem_run_static(const lem_params* p, double* d_h, const double* d_K,
                          const double* d_U, int64_t steps, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LEM_H */
