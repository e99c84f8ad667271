/*
 * qtensor_planner.h -- host-only planning entry points: elimination orders
 * and the step-dependent slicing search that produce the qt_plan_desc
 * consumed by qt_load_plan (qtensor_hip.h).  No GPU is touched.
 *
 * The line graph of a network (Section IV-B) has one vertex per variable
 * and a clique per tensor.  Eliminating a vertex connects its neighbours and
 * removes it; the contraction width c of an order is the largest neighbour
 * count met at elimination (Section IV-B).  Degrees never count self-loops.
 */
#ifndef QTENSOR_PLANNER_H
#define QTENSOR_PLANNER_H

#include <stdint.h>

#include "qtensor_hip.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QT_ORDER_MIN_DEGREE = 0, /* greedy: lowest neighbour count first (Section V-A1); ties: smallest id */
  QT_ORDER_MIN_FILL = 1,   /* greedy: fewest fill-in edges; ties: lowest degree, then smallest id */
  QT_ORDER_RGREEDY = 2     /* randomised greedy (Section V-A2): vertex v drawn with weight
                              exp(-N(v)/tau), `repeats` runs, the narrowest kept */
} qt_order_algo;

/* Greedy elimination order of every variable of `net` except the `n_exclude`
 * ids in `exclude` (which are deleted from the graph first, without fill --
 * the graph of a sliced expression, Section VI-C).
 *   order_out   capacity n_vars of the network desc; receives *n_order_out ids
 *   width_out   contraction width of the order
 *   tau, repeats, seed   used by QT_ORDER_RGREEDY only (repeats >= 1)
 * Errors: QT_EINVAL on null pointers, unknown algo, ids out of range. */
qt_status qt_order_greedy(const qt_network* net, int32_t algo,
                          const int32_t* exclude, int32_t n_exclude,
                          double tau, int32_t repeats, uint64_t seed,
                          int32_t* order_out, int32_t* n_order_out, int32_t* width_out);

#define QT_MAX_SLICE_GROUPS 16

typedef struct {
  int32_t algo;            /* qt_order_algo used for every ordering run */
  int32_t n_slice_vars;    /* n: variables sliced in total */
  int32_t max_candidates;  /* 0 = every step up to the peak; else that many, evenly spaced */
  int32_t threads;         /* host threads for the candidate sweep (0 = hardware concurrency, capped at 16) */
  double tau;              /* rgreedy temperature */
  int32_t repeats;         /* rgreedy runs per ordering */
  uint64_t seed;
  int32_t group_size;      /* r of Section VI-D: variables sliced per group (0 or >= n: one group, r = n) */
  const int32_t* exclude;  /* variables held out of the search (open outputs): deleted without fill first */
  int32_t n_exclude;
} qt_slicing_opts;

typedef struct {
  int32_t step;            /* s: buckets eliminated before the first group is sliced */
  int32_t width;           /* max(prefix_width, slice_width) */
  int32_t prefix_width;    /* widest step before the last group's step */
  int32_t slice_width;     /* widest step after it */
  int32_t unsliced_width;  /* width of the initial full order */
  int32_t peak_step;       /* first step at which the initial order reaches its width */
  double cost;             /* sum over steps of 2^(N+1), each times the number of slices it runs for */
  int32_t n_groups;        /* slice groups (ceil(n / r)) */
  int32_t group_step[QT_MAX_SLICE_GROUPS];  /* order position at which group g is sliced (non-decreasing) */
  int32_t group_len[QT_MAX_SLICE_GROUPS];   /* its number of variables */
} qt_slicing_result;

/* Step-dependent slicing search (Section VI-C "late parallelization",
 * Section VI-D):
 *   1. order the full graph; the peak is the first step reaching its width;
 *   2. for every candidate step s up to the peak: eliminate the first s
 *      vertices of that order, delete the r vertices of highest degree one
 *      at a time (degrees recomputed after each deletion, ties to the
 *      smallest id), and order the rest afresh;
 *   3. keep the step with the smallest width; ties go to the smaller cost,
 *      then the smaller step;
 *   4. with r < n, repeat 1-3 on the expression left after that step and
 *      those deletions, until n variables are sliced (each group at its own
 *      best step).
 * Outputs: order_out (capacity n_vars): every group's prefix order in turn,
 * then the order of the fully sliced expression; slice_vars_out (capacity
 * n_slice_vars) group by group in deletion order (first = most significant
 * slice-id bit); result->group_step/group_len give the groups;
 * width_by_step (optional, capacity n_vars + 1): the width reached at each
 * candidate step of the first group, -1 where not evaluated. */
qt_status qt_plan_slicing(const qt_network* net, const qt_slicing_opts* opts,
                          int32_t* order_out, int32_t* n_order_out,
                          int32_t* slice_vars_out, qt_slicing_result* result,
                          int32_t* width_by_step);

#ifdef __cplusplus
}
#endif

#endif /* QTENSOR_PLANNER_H */
