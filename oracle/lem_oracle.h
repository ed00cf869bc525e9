/*
 * lem_oracle.h -- the oracle's own declarations (test infrastructure only).
 * Nothing here is shared with the GPU library; see lem_oracle.c.
 */
#ifndef LEM_ORACLE_H
#define LEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Dmax of Step 1: the most donors a cell of an 8-connected grid can have. */
#define LEMO_DMAX 8

enum { LEMO_OK = 0, LEMO_E_ARG = 1, LEMO_E_ALLOC = 2, LEMO_E_CYCLE = 5 };

/* Problem statement (section "The Equation", Step 1): grid of ny rows and nx
 * columns addressed y*nx + x, cell size dx by dy, time step dt, area exponent
 * m, slope exponent n, uplift rate U and erodibility K (scalars, used where
 * the per-cell field is NULL).  eps and max_newton drive the Newton loop of
 * Algorithm 6 when n != 1. */
typedef struct lemo_params {
  int32_t ny, nx;
  double dx, dy, dt, m, n, U, K;
  double eps;
  int32_t max_newton;
} lemo_params;

void lemo_receivers(int32_t ny, int32_t nx, double dx, double dy, const double* h,
                    int32_t* rec);
void lemo_donors(int32_t ny, int32_t nx, const int32_t* rec, int32_t* donor,
                 uint8_t* dnum);
int64_t lemo_stack_order(int64_t n, const int32_t* rec, const int32_t* donor,
                         const uint8_t* dnum, int32_t* order, int32_t* depth,
                         int32_t* stack);
void lemo_accumulate(int64_t n, const int32_t* order, const int32_t* donor,
                     const uint8_t* dnum, uint32_t* count);
void lemo_uplift(int32_t ny, int32_t nx, double dt, double U, const double* Ufield,
                 double* h);
void lemo_erode(int32_t ny, int32_t nx, double dx, double dy, double dt, double m,
                double K, const double* Kfield, const int32_t* rec,
                const uint32_t* count, const int32_t* order, double* h);
void lemo_erode_newton(int32_t ny, int32_t nx, double dx, double dy, double dt,
                       double m, double nexp, double eps, int32_t max_iter,
                       double K, const double* Kfield, const int32_t* rec,
                       const uint32_t* count, const int32_t* order, double* h);
int64_t lemo_bfs_queue(int64_t n, const int32_t* rec, const int32_t* donor,
                       const uint8_t* dnum, int32_t* queue, int64_t* levels);
int64_t lemo_graph_order(int64_t n, const int32_t* rec, int32_t* donor, uint8_t* dnum,
                         int32_t* queue, int64_t* levels, int32_t* stack_order,
                         int32_t* depth, uint32_t* count);

int lemo_run(const lemo_params* p, double* h, const double* K, const double* U,
             int64_t steps, int32_t* rec_out, int32_t* depth_out, uint32_t* count_out,
             int64_t* offsets_out, int64_t offsets_cap, int64_t* nlevels_out);
/* Steady-state projection: h_c = h_r + U_c*dt/F (n = 1), h_r + (U_c*dt/F)^(1/n)
 * otherwise, for every cell with a receiver, in receiver-first order. */
void lemo_project_heights(int32_t ny, int32_t nx, double dx, double dy, double dt,
                          double m, double nexp, double U, const double* Ufield, double K,
                          const double* Kfield, const int32_t* rec, const uint32_t* count,
                          const int32_t* order, double* h);
/* `iters` projections, each from the routing of the current heights. */
int lemo_project(const lemo_params* p, double* h, const double* K, const double* U,
                 int64_t iters, int32_t* rec_out, int32_t* depth_out, uint32_t* count_out);
int lemo_run_fixed_routing(const lemo_params* p, double* h, const int32_t* rec,
                           const double* K, const double* U, int64_t steps,
                           int32_t* depth_out, uint32_t* count_out);
int lemo_routing(const lemo_params* p, const double* h, int32_t* rec_out,
                 int32_t* depth_out, uint32_t* count_out, int64_t* offsets_out,
                 int64_t offsets_cap, int64_t* nlevels_out);

/* Multiple flow directions (section "Multiple Flow Directions"): one step
 * and a run of `steps` steps with flow shared in proportion to slope^pexp;
 * n must be 1.  area_out (m^2) and level_out describe the last step. */
int lemo_mfd_step(const lemo_params* p, double pexp, double* h, const double* K,
                  const double* U, double* area, int32_t* level, int64_t* nlevels_out);
int lemo_mfd_run(const lemo_params* p, double pexp, double* h, const double* K,
                 const double* U, int64_t steps, double* area_out, int32_t* level_out,
                 int64_t* nlevels_out);

#ifdef __cplusplus
}
#endif
#endif
