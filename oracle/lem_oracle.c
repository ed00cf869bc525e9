/*
 * lem_oracle.c -- serial CPU oracle for the per-timestep hot path of the
 * parallel landscape-evolution method of R. Barnes, "Accelerating a Landscape
 * Evolution Model with Parallelism" (arXiv:1803.02977).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it; the product path never calls, links or executes it.  It shares no
 * header, source file, table or helper with the GPU library: it has its own
 * parameter struct, its own neighbour tables and its own loader.
 *
 * It is deliberately plain and slow: one host thread, FP64, IEEE
 * round-to-nearest, built with -O2 -ffp-contract=off and without fast-math,
 * no blocking, no fusion.  Each function names the passage of the paper it
 * follows.  Processing order is the depth-first "stack" order of the earlier
 * serial method (section "Step 4: Generate Queue", figure "Stack vs. queue",
 * panel (a)); the breadth-first queue of Algorithm 3 ("Generate Queue") is
 * also provided for the graph-level worked example (Table 1).
 *
 * Readings of passages that are silent or ambiguous (each is listed in the
 * design notes as well):
 *  - NoFlow is represented by a cell being its own receiver (rec[c] == c).
 *  - Neighbour order (which decides ties under the strict ">" of Algorithm 1)
 *    is row-major: offsets (dy,dx) = (-1,-1) (-1,0) (-1,+1) (0,-1) (0,+1)
 *    (+1,-1) (+1,0) (+1,+1), which is also ascending cell index.
 *  - dist(c,n) of Algorithm 1 is the distance between cell centres:
 *    dx, dy or sqrt(dx*dx + dy*dy).
 *  - Algorithm 2 ("Determine donors") loops over the interior only; the
 *    perimeter cells are the base level, so their donors must be found too.
 *    The donor loop here covers every cell.
 *  - Drainage area (Equation "flow_acc") with w(c) = dx*dy and alpha = 1 is
 *    dx*dy times the number of cells in the upstream subtree; the oracle
 *    accumulates that integer count and multiplies by dx*dy once.
 *  - For the slope exponent n = 1 the Newton-Raphson loop of Algorithm 6
 *    ("Calculate erosion") has the closed-form root
 *    h = (h0 + F*h_rec) / (1 + F); the oracle uses that closed form.  The
 *    literal Newton loop is kept separately for general n.
 *  - Within a step: receivers are found from the pre-uplift heights, then
 *    donors, order, accumulation, uplift of every interior cell (pits
 *    included) and erosion of every cell that has a receiver, as in the
 *    paper's step sequence (Steps 2 to 7, then "Rinse, Repeat").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "lem_oracle.h"

/* Neighbour offsets in the oracle's canonical (row-major) order. */
static const int LEMO_DY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
static const int LEMO_DX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};

/* Distance from a cell to its k-th neighbour (cell-centre distance). */
static void lemo_distances(double dx, double dy, double dist[8]) {
  const double ddiag = sqrt(dx * dx + dy * dy);
  for (int k = 0; k < 8; ++k) {
    if (LEMO_DY[k] != 0 && LEMO_DX[k] != 0)
      dist[k] = ddiag;
    else if (LEMO_DY[k] != 0)
      dist[k] = dy;
    else
      dist[k] = dx;
  }
}

static int lemo_is_perimeter(int32_t ny, int32_t nx, int32_t y, int32_t x) {
  return y == 0 || x == 0 || y == ny - 1 || x == nx - 1;
}

/* Step 2, Algorithm 1 ("Determine Receivers"): each interior cell sends its
 * flow to the neighbour of greatest downhill slope (h_c - h_n)/dist, strictly
 * greater than zero, the first such neighbour winning ties; otherwise it has
 * no receiver.  Perimeter cells transfer no flow. */
void lemo_receivers(int32_t ny, int32_t nx, double dx, double dy,
                    const double* h, int32_t* rec) {
  double dist[8];
  lemo_distances(dx, dy, dist);
  for (int32_t y = 0; y < ny; ++y) {
    for (int32_t x = 0; x < nx; ++x) {
      const int64_t c = (int64_t)y * nx + x;
      rec[c] = (int32_t)c; /* NoFlow */
      if (lemo_is_perimeter(ny, nx, y, x)) continue;
      double smax = 0.0;
      int64_t nmax = c;
      for (int k = 0; k < 8; ++k) {
        const int64_t n = (int64_t)(y + LEMO_DY[k]) * nx + (x + LEMO_DX[k]);
        const double s = (h[c] - h[n]) / dist[k];
        if (s > smax) {
          smax = s;
          nmax = n;
        }
      }
      rec[c] = (int32_t)nmax;
    }
  }
}

/* Step 3, Algorithm 2 ("Determine donors"): each cell lists the neighbours
 * whose receiver it is, in neighbour order, in slots Dmax*c + k.  Every cell
 * is visited, the perimeter included. */
void lemo_donors(int32_t ny, int32_t nx, const int32_t* rec, int32_t* donor,
                 uint8_t* dnum) {
  for (int32_t y = 0; y < ny; ++y) {
    for (int32_t x = 0; x < nx; ++x) {
      const int64_t c = (int64_t)y * nx + x;
      dnum[c] = 0;
      for (int k = 0; k < 8; ++k) {
        const int32_t yy = y + LEMO_DY[k], xx = x + LEMO_DX[k];
        if (yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
        const int64_t n = (int64_t)yy * nx + xx;
        if (rec[n] == c) {
          donor[LEMO_DMAX * c + dnum[c]] = (int32_t)n;
          dnum[c] = (uint8_t)(dnum[c] + 1);
        }
      }
    }
  }
}

/* Depth-first "stack" order of the earlier serial method (figure "Stack vs.
 * queue", panel (a)): every cell without a receiver starts a traversal, in
 * ascending cell order; a cell is emitted when popped and its donors are
 * pushed so that they are visited in donor order.  depth[] is the number of
 * receiver hops to the tree's root, i.e. the level of the breadth-first queue
 * that the cell belongs to.  Returns the number of cells emitted (fewer than
 * n only if the receivers contain a cycle). */
int64_t lemo_stack_order(int64_t n, const int32_t* rec, const int32_t* donor,
                         const uint8_t* dnum, int32_t* order, int32_t* depth,
                         int32_t* stack) {
  int64_t emitted = 0;
  for (int64_t r = 0; r < n; ++r) {
    if (rec[r] != r) continue;
    int64_t top = 0;
    stack[top++] = (int32_t)r;
    depth[r] = 0;
    while (top > 0) {
      const int32_t c = stack[--top];
      order[emitted++] = c;
      for (int k = (int)dnum[c] - 1; k >= 0; --k) {
        const int32_t d = donor[LEMO_DMAX * (int64_t)c + k];
        depth[d] = depth[c] + 1;
        stack[top++] = d;
      }
    }
  }
  return emitted;
}

/* Equation "flow_acc" with w(c) = 1 cell and alpha(n,c) = 1 for the single
 * receiver of D8 routing: count(c) = 1 + sum of count over the donors of c.
 * Evaluated in reverse stack order, so every donor is final before its
 * receiver (the pull form of Algorithm 4, "Flow Accumulation"). */
void lemo_accumulate(int64_t n, const int32_t* order, const int32_t* donor,
                     const uint8_t* dnum, uint32_t* count) {
  for (int64_t i = n - 1; i >= 0; --i) {
    const int32_t c = order[i];
    uint32_t a = 1u;
    for (int k = 0; k < dnum[c]; ++k) a += count[donor[LEMO_DMAX * (int64_t)c + k]];
    count[c] = a;
  }
}

/* Step 6, Algorithm 5 ("Uplift"): every interior cell rises by U*dt; U may
 * vary from cell to cell.  Perimeter cells stay at base level. */
void lemo_uplift(int32_t ny, int32_t nx, double dt, double U, const double* Ufield,
                 double* h) {
  const double udt = U * dt;
  for (int32_t y = 1; y < ny - 1; ++y) {
    for (int32_t x = 1; x < nx - 1; ++x) {
      const int64_t c = (int64_t)y * nx + x;
      h[c] = h[c] + (Ufield ? Ufield[c] * dt : udt);
    }
  }
}

/* Step 7, Algorithm 6 ("Calculate erosion") for slope exponent n = 1.  The
 * implicit (backward Euler) step of Equation "streampower" for cell c with
 * receiver r, F = K*dt*A^m/dist(c,r), has the unique root
 * h_c <- (h_c + F*h_r)/(1 + F), where h_c already includes uplift and h_r is
 * the receiver's new height.  Cells are visited in stack order, so every
 * receiver is updated before its donors.  Cells without a receiver do not
 * erode. */
void lemo_erode(int32_t ny, int32_t nx, double dx, double dy, double dt, double m,
                double K, const double* Kfield, const int32_t* rec,
                const uint32_t* count, const int32_t* order, double* h) {
  const int64_t n = (int64_t)ny * nx;
  const double ddiag = sqrt(dx * dx + dy * dy);
  const double dxdy = dx * dy;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = order[i];
    const int32_t r = rec[c];
    if (r == c) continue;
    const int32_t cy = c / nx, cx = c % nx, ry = r / nx, rx = r % nx;
    const double d = (cy != ry && cx != rx) ? ddiag : (cy != ry ? dy : dx);
    const double area = (double)count[c] * dxdy;
    const double am = (m == 0.5) ? sqrt(area) : pow(area, m);
    const double kc = Kfield ? Kfield[c] : K;
    const double f = ((kc * dt) * am) / d;
    h[c] = (h[c] + f * h[r]) / (1.0 + f);
  }
}

/* Algorithm 6 ("Calculate erosion") with its Newton-Raphson loop, for a
 * general slope exponent n > 0: starting from the uplifted height h0,
 * h <- h - (h - h0 + F*(h - h_r)^n) / (1 + F*n*(h - h_r)^(n-1)) until the
 * change is at most eps or max_iter iterations have run, with
 * F = K*dt*A^m/dist^n.  The equation h - h0 + F*(h - h_r)^n = 0 has exactly
 * one root in (h_r, h0] when h0 > h_r; a Newton iterate that does not lie
 * above the receiver (possible for n < 1, where the residual is concave) is
 * replaced by the midpoint between the receiver and the previous iterate.
 * A cell whose uplifted height is not above its receiver's new height keeps
 * h0 (no positive slope, no erosion). */
void lemo_erode_newton(int32_t ny, int32_t nx, double dx, double dy, double dt,
                       double m, double nexp, double eps, int32_t max_iter,
                       double K, const double* Kfield, const int32_t* rec,
                       const uint32_t* count, const int32_t* order, double* h) {
  const int64_t n = (int64_t)ny * nx;
  const double ddiag = sqrt(dx * dx + dy * dy);
  const double dxdy = dx * dy;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = order[i];
    const int32_t r = rec[c];
    if (r == c) continue;
    const int32_t cy = c / nx, cx = c % nx, ry = r / nx, rx = r % nx;
    const double d = (cy != ry && cx != rx) ? ddiag : (cy != ry ? dy : dx);
    const double area = (double)count[c] * dxdy;
    const double kc = Kfield ? Kfield[c] : K;
    const double f = ((kc * dt) * pow(area, m)) / pow(d, nexp);
    const double h0 = h[c];
    const double hn = h[r];
    double hnew = h0, delta = 2.0 * eps;
    int32_t it = 0;
    if (h0 - hn > 0.0) {
      while (fabs(delta) > eps && it < max_iter) {
        const double g = hnew - hn;
        double next = hnew - (hnew - h0 + f * pow(g, nexp)) / (1.0 + f * nexp * pow(g, nexp - 1.0));
        if (!(next - hn > 0.0)) next = 0.5 * (hnew + hn);
        delta = next - hnew;
        hnew = next;
        ++it;
      }
    }
    h[c] = hnew;
  }
}

/* Steady-state projection (an accelerator of runs to steady state, not a
 * step of the paper's method): with the receivers, counts and stack order of
 * the step, every cell with a receiver takes the height at which one step of
 * Algorithm 6 would leave it unchanged given its receiver's new height,
 * F*(h_c - h_r)^n = U_c*dt, i.e. h_c = h_r + U_c*dt/F for n = 1 and
 * h_r + (U_c*dt/F)^(1/n) otherwise (F as in Algorithm 6).  Cells without a
 * receiver keep their uplifted height (interior sinks rise by U*dt, as in a
 * step).  F = 0 (K = 0) leaves the uplifted height. */
void lemo_project_heights(int32_t ny, int32_t nx, double dx, double dy, double dt,
                          double m, double nexp, double U, const double* Ufield, double K,
                          const double* Kfield, const int32_t* rec, const uint32_t* count,
                          const int32_t* order, double* h) {
  const int64_t n = (int64_t)ny * nx;
  const double ddiag = sqrt(dx * dx + dy * dy);
  const double dxdy = dx * dy;
  const double udt = U * dt;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = order[i];
    const int32_t r = rec[c];
    if (r == c) continue;
    const int32_t cy = c / nx, cx = c % nx, ry = r / nx, rx = r % nx;
    const double d = (cy != ry && cx != rx) ? ddiag : (cy != ry ? dy : dx);
    const double area = (double)count[c] * dxdy;
    const double kc = Kfield ? Kfield[c] : K;
    const double uc = Ufield ? Ufield[c] * dt : udt;
    if (nexp == 1.0) {
      const double am = (m == 0.5) ? sqrt(area) : pow(area, m);
      const double f = ((kc * dt) * am) / d;
      if (f > 0.0) h[c] = h[r] + uc / f;
    } else {
      const double f = ((kc * dt) * pow(area, m)) / pow(d, nexp);
      if (f > 0.0) h[c] = h[r] + pow(uc / f, 1.0 / nexp);
    }
  }
}

/* Step 4, Algorithm 3 ("Generate Queue") for a general forest given by rec[]
 * (rec[c] == c marks a cell without receiver) and donor lists: the cells
 * without receiver form the first level; then the donors of each level, in
 * queue order and donor order, form the next.  Levels[] holds the start of
 * each level and ends with n; empty levels are not recorded.  Returns the
 * number of levels. */
int64_t lemo_bfs_queue(int64_t n, const int32_t* rec, const int32_t* donor,
                       const uint8_t* dnum, int32_t* queue, int64_t* levels) {
  int64_t nqueue = 0;
  int64_t ls = 0;
  for (int64_t c = 0; c < n; ++c)
    if (rec[c] == c) queue[nqueue++] = (int32_t)c;
  levels[ls++] = 0;
  int64_t lo = 0, hi = nqueue;
  while (lo < hi) {
    levels[ls++] = hi;
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t c = queue[i];
      for (int k = 0; k < dnum[c]; ++k) queue[nqueue++] = donor[LEMO_DMAX * (int64_t)c + k];
    }
    lo = hi;
    hi = nqueue;
  }
  return ls - 1;
}

/* Graph-level form of Steps 3 to 5 for an arbitrary forest (the worked
 * example of Table 1): donors of c are the nodes whose receiver is c, in
 * ascending node order; then the breadth-first queue and its levels
 * (Algorithm 3), the depth-first stack order (figure "Stack vs. queue" (a)),
 * the depth of every node and the flow accumulation with unit area per node
 * (Equation "flow_acc", Algorithm 4).  Returns the number of levels, or -1
 * if the receivers contain a cycle or a node has more than Dmax donors. */
int64_t lemo_graph_order(int64_t n, const int32_t* rec, int32_t* donor, uint8_t* dnum,
                         int32_t* queue, int64_t* levels, int32_t* stack_order,
                         int32_t* depth, uint32_t* count) {
  for (int64_t c = 0; c < n; ++c) dnum[c] = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t r = rec[v];
    if (r == v) continue;
    if (dnum[r] >= LEMO_DMAX) return -1;
    donor[LEMO_DMAX * (int64_t)r + dnum[r]] = (int32_t)v;
    dnum[r] = (uint8_t)(dnum[r] + 1);
  }
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!stack) return -1;
  const int64_t emitted = lemo_stack_order(n, rec, donor, dnum, stack_order, depth, stack);
  free(stack);
  if (emitted != n) return -1;
  lemo_accumulate(n, stack_order, donor, dnum, count);
  return lemo_bfs_queue(n, rec, donor, dnum, queue, levels);
}

/* ------------------------------------------------------------------------- */
/* Whole time loop ("Rinse, Repeat"). */

struct lemo_work {
  int32_t* rec;
  int32_t* donor;
  uint8_t* dnum;
  int32_t* order;
  int32_t* depth;
  int32_t* stack;
  uint32_t* count;
};

static void lemo_work_free(struct lemo_work* w) {
  free(w->rec);
  free(w->donor);
  free(w->dnum);
  free(w->order);
  free(w->depth);
  free(w->stack);
  free(w->count);
}

static int lemo_work_alloc(struct lemo_work* w, int64_t n) {
  memset(w, 0, sizeof(*w));
  w->rec = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  w->donor = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * LEMO_DMAX);
  w->dnum = (uint8_t*)malloc((size_t)n);
  w->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  w->depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  w->stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  w->count = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
  if (!w->rec || !w->donor || !w->dnum || !w->order || !w->depth || !w->stack ||
      !w->count) {
    lemo_work_free(w);
    return LEMO_E_ALLOC;
  }
  return LEMO_OK;
}

static int lemo_check(const lemo_params* p) {
  if (!p) return LEMO_E_ARG;
  if (p->ny < 3 || p->nx < 3) return LEMO_E_ARG;
  if ((int64_t)p->ny * p->nx > INT32_MAX) return LEMO_E_ARG;
  if (!(p->dx > 0.0) || !(p->dy > 0.0) || !(p->dt > 0.0) || !(p->m >= 0.0))
    return LEMO_E_ARG;
  if (!(p->n > 0.0) || !isfinite(p->n)) return LEMO_E_ARG;
  return LEMO_OK;
}

static void lemo_export(int64_t n, const struct lemo_work* w, int32_t* rec_out,
                        int32_t* depth_out, uint32_t* count_out, int64_t* offsets_out,
                        int64_t offsets_cap, int64_t* nlevels_out) {
  if (rec_out) memcpy(rec_out, w->rec, sizeof(int32_t) * (size_t)n);
  if (depth_out) memcpy(depth_out, w->depth, sizeof(int32_t) * (size_t)n);
  if (count_out) memcpy(count_out, w->count, sizeof(uint32_t) * (size_t)n);
  int32_t maxd = 0;
  for (int64_t c = 0; c < n; ++c)
    if (w->depth[c] > maxd) maxd = w->depth[c];
  const int64_t nlevels = (int64_t)maxd + 1;
  if (nlevels_out) *nlevels_out = nlevels;
  if (offsets_out && offsets_cap >= nlevels + 1) {
    for (int64_t l = 0; l <= nlevels; ++l) offsets_out[l] = 0;
    for (int64_t c = 0; c < n; ++c) offsets_out[w->depth[c] + 1] += 1;
    for (int64_t l = 1; l <= nlevels; ++l) offsets_out[l] += offsets_out[l - 1];
  }
}

/* One step of the method with the given receivers already in w->rec:
 * donors, order, accumulation, uplift, erosion. */
static int lemo_step_from_rec(const lemo_params* p, double* h, const double* K,
                              const double* U, struct lemo_work* w) {
  const int64_t n = (int64_t)p->ny * p->nx;
  lemo_donors(p->ny, p->nx, w->rec, w->donor, w->dnum);
  if (lemo_stack_order(n, w->rec, w->donor, w->dnum, w->order, w->depth, w->stack) != n)
    return LEMO_E_CYCLE;
  lemo_accumulate(n, w->order, w->donor, w->dnum, w->count);
  lemo_uplift(p->ny, p->nx, p->dt, p->U, U, h);
  if (p->n == 1.0)
    lemo_erode(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->K, K, w->rec, w->count,
               w->order, h);
  else
    lemo_erode_newton(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->n, p->eps,
                      p->max_newton, p->K, K, w->rec, w->count, w->order, h);
  return LEMO_OK;
}

int lemo_run(const lemo_params* p, double* h, const double* K, const double* U,
             int64_t steps, int32_t* rec_out, int32_t* depth_out, uint32_t* count_out,
             int64_t* offsets_out, int64_t offsets_cap, int64_t* nlevels_out) {
  int st = lemo_check(p);
  if (st != LEMO_OK) return st;
  if (!h || steps < 0) return LEMO_E_ARG;
  const int64_t n = (int64_t)p->ny * p->nx;
  struct lemo_work w;
  if (lemo_work_alloc(&w, n) != LEMO_OK) return LEMO_E_ALLOC;
  for (int64_t s = 0; s < steps && st == LEMO_OK; ++s) {
    lemo_receivers(p->ny, p->nx, p->dx, p->dy, h, w.rec);
    st = lemo_step_from_rec(p, h, K, U, &w);
  }
  if (st == LEMO_OK && steps > 0)
    lemo_export(n, &w, rec_out, depth_out, count_out, offsets_out, offsets_cap,
                nlevels_out);
  lemo_work_free(&w);
  return st;
}

/* `iters` steady-state projections: receivers from the current heights,
 * donors, order and counts as in a step, uplift, then lemo_project_heights.
 * Routing of the last one is exported as by lemo_run. */
int lemo_project(const lemo_params* p, double* h, const double* K, const double* U,
                 int64_t iters, int32_t* rec_out, int32_t* depth_out, uint32_t* count_out) {
  int st = lemo_check(p);
  if (st != LEMO_OK) return st;
  if (!h || iters < 0) return LEMO_E_ARG;
  const int64_t n = (int64_t)p->ny * p->nx;
  struct lemo_work w;
  if (lemo_work_alloc(&w, n) != LEMO_OK) return LEMO_E_ALLOC;
  for (int64_t s = 0; s < iters && st == LEMO_OK; ++s) {
    lemo_receivers(p->ny, p->nx, p->dx, p->dy, h, w.rec);
    lemo_donors(p->ny, p->nx, w.rec, w.donor, w.dnum);
    if (lemo_stack_order(n, w.rec, w.donor, w.dnum, w.order, w.depth, w.stack) != n) {
      st = LEMO_E_CYCLE;
      break;
    }
    lemo_accumulate(n, w.order, w.donor, w.dnum, w.count);
    lemo_uplift(p->ny, p->nx, p->dt, p->U, U, h);
    lemo_project_heights(p->ny, p->nx, p->dx, p->dy, p->dt, p->m, p->n, p->U, U, p->K, K,
                         w.rec, w.count, w.order, h);
  }
  if (st == LEMO_OK && iters > 0)
    lemo_export(n, &w, rec_out, depth_out, count_out, NULL, 0, NULL);
  lemo_work_free(&w);
  return st;
}

int lemo_run_fixed_routing(const lemo_params* p, double* h, const int32_t* rec,
                           const double* K, const double* U, int64_t steps,
                           int32_t* depth_out, uint32_t* count_out) {
  int st = lemo_check(p);
  if (st != LEMO_OK) return st;
  if (!h || !rec || steps < 0) return LEMO_E_ARG;
  const int64_t n = (int64_t)p->ny * p->nx;
  struct lemo_work w;
  if (lemo_work_alloc(&w, n) != LEMO_OK) return LEMO_E_ALLOC;
  memcpy(w.rec, rec, sizeof(int32_t) * (size_t)n);
  for (int64_t s = 0; s < steps && st == LEMO_OK; ++s) st = lemo_step_from_rec(p, h, K, U, &w);
  if (st == LEMO_OK && steps > 0)
    lemo_export(n, &w, NULL, depth_out, count_out, NULL, 0, NULL);
  lemo_work_free(&w);
  return st;
}

/* Routing of the given heights only (Steps 2 to 5, no height change). */
int lemo_routing(const lemo_params* p, const double* h, int32_t* rec_out,
                 int32_t* depth_out, uint32_t* count_out, int64_t* offsets_out,
                 int64_t offsets_cap, int64_t* nlevels_out) {
  int st = lemo_check(p);
  if (st != LEMO_OK) return st;
  if (!h) return LEMO_E_ARG;
  const int64_t n = (int64_t)p->ny * p->nx;
  struct lemo_work w;
  if (lemo_work_alloc(&w, n) != LEMO_OK) return LEMO_E_ALLOC;
  lemo_receivers(p->ny, p->nx, p->dx, p->dy, h, w.rec);
  lemo_donors(p->ny, p->nx, w.rec, w.donor, w.dnum);
  if (lemo_stack_order(n, w.rec, w.donor, w.dnum, w.order, w.depth, w.stack) != n) {
    lemo_work_free(&w);
    return LEMO_E_CYCLE;
  }
  lemo_accumulate(n, w.order, w.donor, w.dnum, w.count);
  lemo_export(n, &w, rec_out, depth_out, count_out, offsets_out, offsets_cap, nlevels_out);
  lemo_work_free(&w);
  return LEMO_OK;
}

/* ------------------------------------------------------------------------
 * Multiple flow directions (section "Multiple Flow Directions", figure
 * "Multiple-flow directions").  Every strictly lower neighbour of an
 * interior cell is one of its receivers, and a cell can be processed only
 * after all of its receivers.  The paper gives no rule for sharing the flow
 * and keeps the multiple-receiver form of the stream power law out of its
 * printed text; the readings taken here (also in the design notes):
 *  - receiver k of cell c gets the share s_k = S_k^p / sum_j S_j^p of the
 *    flow, S_k = (h_c - h_k)/dist_k (p = 1: in proportion to the slope);
 *  - the drainage area of c is its own cell area plus, from every donor d,
 *    d's share towards c times d's drainage area;
 *  - erosion for n = 1 is backward Euler of dh_c/dt = U - sum_k K (s_k A_c)^m
 *    S_k over the receivers, i.e. h_c' = (h0 + sum_k F_k h_k') /
 *    (1 + sum_k F_k) with F_k = K dt (s_k A_c)^m / dist_k, the sums taken in
 *    neighbour order;
 *  - the level of a cell is 0 without receivers and otherwise one more than
 *    the deepest level among its receivers (the longest path to a root), so
 *    that every receiver lies on an earlier level.
 * Flow only descends, so the oracle simply takes the cells in order of
 * height: ascending puts every receiver before its donors, descending every
 * donor before its receivers.
 */
static const double* lemo_sort_h;

static int lemo_cmp_height(const void* a, const void* b) {
  const int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
  const double hi = lemo_sort_h[i], hj = lemo_sort_h[j];
  if (hi < hj) return -1;
  if (hi > hj) return 1;
  return (i > j) - (i < j);
}

static double lemo_slope_pow(double s, double pexp) { return pexp == 1.0 ? s : pow(s, pexp); }

static double lemo_area_pow(double a, double m) {
  return m == 0.5 ? sqrt(a) : (m == 1.0 ? a : pow(a, m));
}

int lemo_mfd_step(const lemo_params* p, double pexp, double* h, const double* K,
                  const double* U, double* area, int32_t* level, int64_t* nlevels_out) {
  const int32_t ny = p->ny, nx = p->nx;
  const int64_t n = (int64_t)ny * nx;
  double dist[8];
  lemo_distances(p->dx, p->dy, dist);
  const double dxdy = p->dx * p->dy;
  double* h0 = (double*)malloc(sizeof(double) * (size_t)n);
  double* wsum = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t* nrec = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* ord = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!h0 || !wsum || !nrec || !ord) {
    free(h0); free(wsum); free(nrec); free(ord);
    return LEMO_E_ALLOC;
  }
  memcpy(h0, h, sizeof(double) * (size_t)n);
  /* Receivers and the sum of their weights, from the step's starting heights. */
  for (int32_t y = 0; y < ny; ++y)
    for (int32_t x = 0; x < nx; ++x) {
      const int64_t c = (int64_t)y * nx + x;
      wsum[c] = 0.0;
      nrec[c] = 0;
      if (lemo_is_perimeter(ny, nx, y, x)) continue;
      for (int k = 0; k < 8; ++k) {
        const int64_t r = (int64_t)(y + LEMO_DY[k]) * nx + (x + LEMO_DX[k]);
        if (h0[c] - h0[r] > 0.0) {
          wsum[c] += lemo_slope_pow((h0[c] - h0[r]) / dist[k], pexp);
          nrec[c] += 1;
        }
      }
    }
  for (int64_t i = 0; i < n; ++i) ord[i] = (int32_t)i;
  lemo_sort_h = h0;
  qsort(ord, (size_t)n, sizeof(int32_t), lemo_cmp_height);
  /* Levels, ascending height. */
  int32_t deepest = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = ord[i], y = c / nx, x = c % nx;
    int32_t l = 0;
    if (nrec[c] > 0)
      for (int k = 0; k < 8; ++k) {
        const int64_t r = (int64_t)(y + LEMO_DY[k]) * nx + (x + LEMO_DX[k]);
        if (h0[c] - h0[r] > 0.0 && level[r] + 1 > l) l = level[r] + 1;
      }
    level[c] = l;
    if (l > deepest) deepest = l;
  }
  /* Drainage areas, descending height: each cell pulls from its donors. */
  for (int64_t i = n - 1; i >= 0; --i) {
    const int32_t c = ord[i], y = c / nx, x = c % nx;
    double acc = dxdy;
    for (int k = 0; k < 8; ++k) {
      const int32_t yy = y + LEMO_DY[k], xx = x + LEMO_DX[k];
      if (yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
      if (lemo_is_perimeter(ny, nx, yy, xx)) continue;
      const int64_t d = (int64_t)yy * nx + xx;
      if (h0[d] - h0[c] > 0.0) {
        const double share = lemo_slope_pow((h0[d] - h0[c]) / dist[k], pexp) / wsum[d];
        acc += share * area[d];
      }
    }
    area[c] = acc;
  }
  /* Uplift and erosion, ascending height (receivers first). */
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = ord[i], y = c / nx, x = c % nx;
    if (lemo_is_perimeter(ny, nx, y, x)) continue;
    const double hup = h0[c] + (U ? U[c] * p->dt : p->U * p->dt);
    if (nrec[c] == 0) {
      h[c] = hup;
      continue;
    }
    const double kc = K ? K[c] : p->K;
    double sumf = 0.0, sumfh = 0.0;
    for (int k = 0; k < 8; ++k) {
      const int64_t r = (int64_t)(y + LEMO_DY[k]) * nx + (x + LEMO_DX[k]);
      if (h0[c] - h0[r] > 0.0) {
        const double share = lemo_slope_pow((h0[c] - h0[r]) / dist[k], pexp) / wsum[c];
        const double f = ((kc * p->dt) * lemo_area_pow(share * area[c], p->m)) / dist[k];
        sumf += f;
        sumfh += f * h[r];
      }
    }
    h[c] = (hup + sumfh) / (1.0 + sumf);
  }
  if (nlevels_out) *nlevels_out = (int64_t)deepest + 1;
  free(h0); free(wsum); free(nrec); free(ord);
  return LEMO_OK;
}

int lemo_mfd_run(const lemo_params* p, double pexp, double* h, const double* K,
                 const double* U, int64_t steps, double* area_out, int32_t* level_out,
                 int64_t* nlevels_out) {
  int st = lemo_check(p);
  if (st != LEMO_OK) return st;
  if (!h || steps < 0 || !(pexp > 0.0) || !isfinite(pexp) || p->n != 1.0) return LEMO_E_ARG;
  const int64_t n = (int64_t)p->ny * p->nx;
  double* area = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t* level = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!area || !level) {
    free(area); free(level);
    return LEMO_E_ALLOC;
  }
  int64_t nl = 0;
  for (int64_t s = 0; s < steps && st == LEMO_OK; ++s)
    st = lemo_mfd_step(p, pexp, h, K, U, area, level, &nl);
  if (st == LEMO_OK && steps > 0) {
    if (area_out) memcpy(area_out, area, sizeof(double) * (size_t)n);
    if (level_out) memcpy(level_out, level, sizeof(int32_t) * (size_t)n);
    if (nlevels_out) *nlevels_out = nl;
  }
  free(area); free(level);
  return st;
}
