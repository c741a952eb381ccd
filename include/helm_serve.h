/*
 * Request server over resident factorizations (continuous batching).
 *
 * The paper's online stage reuses one factorization for many right-hand
 * sides and pipelines right-hand sides that are at different stages of
 * their solve through the layers (Section 4, pipelining of the sweeps).
 * This interface serves requests against several resident factorizations
 * (one per model and frequency), with these rules:
 *
 *  - Every model has a lane: a fixed number of column slots, its own HIP
 *    stream and a host thread.  Lanes of different models run concurrently
 *    on the device.  A lane launches its kernels one by one (no HIP graph
 *    capture on the lane's thread), so the caller may allocate, compute and
 *    synchronize the device from its own threads while requests run.
 *  - A request is a set of point sources for one model.  Its columns wait
 *    in the model's FIFO queue and enter free slots of the lane between
 *    refinement steps, while the columns already in the lane continue;
 *    all slots of a lane share every layer-solve launch.
 *  - Each step applies one polarized solve to every occupied slot
 *    (Algorithm 2, complex64 factors for HELM_MIXED handles) and then the
 *    FP64 residual r = f - H u.  Occupied slots are kept at the front of the
 *    lane and a step runs at the narrowest width of 1, 2, 4, ... up to the
 *    slot count that covers them, so a lightly loaded lane does not pay for
 *    its empty slots.  A column leaves its slot, and its volume is copied to the
 *    request's output, when its relative residual reaches ir_tol or its
 *    estimated error reaches half of err_target, or after ir_max_steps
 *    steps (request status HELM_ENOCONV).  The first step of a column uses
 *    the handle's inner_tol, later steps inner_tol_refine, and a step taken
 *    when the estimate is within err_target but not within half of it
 *    inner_tol_final; for an FP64 handle one step with gmres_tol solves the
 *    column.
 *  - The arithmetic of a column does not depend on the other columns of its
 *    lane, so a request's result is the same alone and in a mix (up to the
 *    rounding order of the GEMM tiles, which does not depend on the
 *    neighbouring columns either).
 *  - Memory admission: a model is admitted with the largest slot count (at
 *    most `slots`) whose workspace (that of the full width plus the
 *    interface vectors of the narrower widths), with the factors, fits the
 *    server's budget; a model that does not fit with one slot is refused
 *    with HELM_ENOMEM.
 *
 * Thread safety: all calls may be made from any host thread.  A handle
 * given to a server must not be used through any other call, nor freed,
 * until helm_server_free has returned.
 */
#ifndef HELM_SERVE_H
#define HELM_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "helm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helm_server helm_server;

typedef struct {
  size_t hbm_budget_bytes; /* device bytes for the factors + lane workspace of
                              all models; 0: a model's lane workspace must fit
                              in 90% of the device memory free when it is
                              added (its factors are already resident) */
  int slots;               /* column slots per model lane (default 32) */
  int device;              /* HIP device ordinal */
} helm_server_options;

typedef struct {
  int status;              /* HELM_OK, HELM_ENOCONV (some column did not reach
                              the tolerance), HELM_EHIP or HELM_EINVAL */
  int n_rhs;
  int model;
  int ir_steps_max;        /* refinement steps of the slowest column */
  double rel_residual_max; /* final FP64 relative residual, max over columns */
  double est_error_max;    /* estimated relative error, max over columns */
  double t_submit_ms;      /* times since the server was created */
  double t_first_ms;       /* first column entered a slot */
  double t_done_ms;        /* last column copied out */
  double latency_ms;       /* t_done - t_submit */
} helm_request_info;

typedef struct {
  long long requests_done, columns_done, steps;
  double p50_ms, p99_ms, mean_ms; /* request latency over completed requests */
  double mean_active_slots;       /* occupancy averaged over steps */
  double elapsed_s;               /* first submit to last completion */
  double columns_per_s;           /* columns_done / elapsed_s */
  size_t bytes_reserved;          /* factors + lane workspace admitted */
} helm_server_summary;

void helm_server_default_options(helm_server_options* o);

/* Create a server.  Returns HELM_EINVAL for a null `out`. */
int helm_server_create(const helm_server_options* opt, helm_server** out);

/* Admit a factorization (borrowed, see above) as model `*model_id`, with the
 * lane's slot count reduced until factors + workspace fit the budget
 * (`*slots_out`, nullable).  HELM_ENOMEM when not even one slot fits. */
int helm_server_add_model(helm_server* s, helm_handle* h, int* model_id, int* slots_out);

/* Stop serving a model: blocks until its queued and active columns have
 * completed, then ends its lane and releases the lane's memory (the handle
 * itself is not freed and may be freed by the caller afterwards).  Further
 * submissions to the model fail with HELM_EINVAL. */
int helm_server_remove_model(helm_server* s, int model_id);

/* Queue a request of n_rhs point sources: node_index[c] is the linear index
 * (x fastest) of source c, amplitude[2c], amplitude[2c+1] its complex
 * amplitude (f = amplitude / h^3 at the node).  The solutions are written to
 * u (host or device memory, RHS-major, n_rhs * nx * ny * nz complex128),
 * which must stay valid until the request completes.  Inputs are copied
 * before the call returns.  HELM_EINVAL for an unknown model, a node
 * outside the grid, a non-finite amplitude or a null pointer. */
int helm_server_submit(helm_server* s, int model_id, int n_rhs, const int64_t* node_index,
                       const double* amplitude, double* u, int64_t* request_id);

/* Block until the request has completed; returns its status and fills
 * `info` (nullable).  A request can be waited for once. */
int helm_server_wait(helm_server* s, int64_t request_id, helm_request_info* info);

/* Non-blocking: *done = 1 once the request has completed. */
int helm_server_poll(helm_server* s, int64_t request_id, int* done);

int helm_server_get_stats(helm_server* s, helm_server_summary* out);

/* Stop the lanes after their current step; queued and active requests that
 * have not completed end with HELM_EINVAL.  Handles are not freed. */
int helm_server_free(helm_server* s);

#ifdef __cplusplus
}
#endif

#endif /* HELM_SERVE_H */
