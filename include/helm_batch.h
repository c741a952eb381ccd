/*
 * Batched solves of independent problems (one call, many grids).
 *
 * Every problem is its own Helmholtz system: grid, squared slowness m,
 * frequency, global PML width, layer count and a set of point sources.  Its
 * layers are factored (Algorithm 1) and its sources solved (Algorithm 2)
 * exactly as by helm_factorize + helm_solve_points with the same options;
 * this call only schedules the problems on one device:
 *
 *  - Problems are admitted in the given order while the planned device
 *    memory of the admitted ones (factor_bytes + min(n_rhs, slots) *
 *    lane_bytes_per_rhs from helm_plan / helm_plan_lane) fits the budget and
 *    at most max_resident are resident.  A problem whose plan does not fit
 *    an empty device ends with HELM_ENOMEM and the others proceed.  The
 *    factorization also needs a transient frontal workspace; when that does
 *    not fit beside the resident problems, the problem waits for one of them
 *    to finish and is factored again (its factor_ms counts every attempt).
 *  - An admitted problem is factored on its own stream by the calling
 *    thread while the problems admitted before it keep solving, then served
 *    by a lane of the request server (include/helm_serve.h): its columns run
 *    through the lane's slots with continuous batching and every layer-set
 *    solve is replayed from a captured HIP graph.  Lanes of resident
 *    problems run concurrently.
 *  - When a problem's last column is done, its lane and factors are freed
 *    and the next problem is admitted.
 *
 * The arithmetic of a problem does not depend on the other problems: each
 * result equals the one helm_solve_points would give for that problem with
 * the same options (up to the rounding order of the GEMM tile widths, which
 * does not change a column's sums either).
 */
#ifndef HELM_BATCH_H
#define HELM_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "helm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  helm_grid grid;
  const double* m;          /* host, nx*ny*nz squared slowness 1/c^2 */
  double omega;
  int pml_width;            /* global PML points per face */
  int n_layers;
  int n_rhs;
  const int64_t* node_index; /* host, n_rhs linear node indices (x fastest) */
  const double* amplitude;  /* host, 2*n_rhs doubles (complex amplitudes) */
  double* u;                /* host or device, n_rhs volumes of nx*ny*nz complex128 */
} helm_problem;

typedef struct {
  helm_options opt;         /* options of every problem (precision, tolerances,
                               flags such as HELM_FLAG_AUTOTUNE); opt.device
                               selects the device */
  size_t hbm_budget_bytes;  /* 0: 90% of the device memory free at the call */
  int slots;                /* column slots per problem lane (default 64) */
  int max_resident;         /* problems resident at once; 0: memory decides */
} helm_batch_options;

typedef struct {
  int status;               /* HELM_OK, HELM_ENOCONV, HELM_ENOMEM, HELM_EZEROPIVOT,
                               HELM_EINVAL, HELM_EHIP */
  int slots;
  size_t planned_bytes;     /* factors + lane workspace admitted */
  double t_admit_ms;        /* times since the call started */
  double t_factored_ms;
  double t_done_ms;
  double factor_ms;
  int ir_steps_max;
  double rel_residual_max, est_error_max;
} helm_problem_info;

typedef struct {
  double wall_s;            /* whole call */
  double factor_s;          /* sum of the factorization times */
  long long columns;        /* right-hand sides solved */
  double rhs_per_s;         /* columns / wall_s */
  int max_resident;         /* most problems resident at once */
  size_t peak_planned_bytes;
} helm_batch_summary;

void helm_batch_default_options(helm_batch_options* o);

/* Solve n independent problems.  info (n records) and summary may be NULL.
 * Returns HELM_OK when every problem ended with HELM_OK, else the first
 * failing problem's status (each problem's own status is in info);
 * HELM_EINVAL for a null problem array or a problem with null or mis-sized
 * arguments (checked before anything runs). */
int helm_solve_batch(int n, const helm_problem* problems, const helm_batch_options* opt,
                     helm_problem_info* info, helm_batch_summary* summary);

#ifdef __cplusplus
}
#endif

#endif /* HELM_BATCH_H */
