/*
 * helm.h -- C ABI of the MI355X (gfx950) solver for the 3D constant-density
 * Helmholtz equation by the method of polarized traces.
 *
 * Problem (Eq. "Helmholtz" and Eq. "discrete_Helmholtz" of the paper):
 *     Laplacian(u) + omega^2 m(x) u = f_s,  s = 1..R,  m = 1/c^2,
 * discretised with second-order 7-point finite differences on a regular grid
 * (Section "Formulation"), with absorbing layers made by complex coordinate
 * stretching beta = 1/(1 + i sigma/omega), sigma = (C/delta)(d/delta)^2
 * (Eq. "appendix:eq:def_alpha").  The grid is decomposed into L layers in z;
 * every internal side of a layer is padded with `pml_local` extra absorbing
 * planes (Fig. "DDM_sketch_PML").
 *
 * Offline stage (Algorithm 1, "Factorization(m, omega)"): helm_factorize
 * builds and factors every local layer operator H^l and keeps the factors
 * resident in device memory.  Online stage (Algorithm 2, "Helmholtz
 * solver(f)"): helm_solve* returns u = H^{-1} f for a batch of right-hand
 * sides by GMRES on the preconditioned polarized interface system (Eqs.
 * "polarized_SIE", "preconditioner_GS", "precond_polarized_SIE") followed by
 * the local reconstruction.
 *
 * Conventions shared by every entry point:
 *   - grid nodes (i, j, k), 0 <= i < nx, ..., at (i h, j h, k h); the grid
 *     INCLUDES the global absorbing layer of `pml_width` nodes per face;
 *   - volume arrays are plane-major: index i + nx*(j + ny*k) ("x fastest");
 *   - batches of volumes are RHS-major: column r starts at r*nx*ny*nz;
 *   - complex numbers are interleaved (re, im) pairs of double;
 *   - the operator is assembled in the complex-symmetric form (H = H^T);
 *     a unit point source is f = 1/h^3 at one node.
 * All entry points return a status code (HELM_OK on success) and never throw.
 * helm_last_error() gives a human-readable description of the last failure
 * on the calling thread.
 * The solve entry points capture their launch sequences into HIP graphs on
 * the calling thread (on a private stream) the first time a layer set meets
 * a batch width: another thread that synchronizes the whole device while
 * such a capture lasts gets an error from HIP (HELM_FLAG_NO_GRAPHS avoids
 * captures; the request server's lanes never capture).
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define HELM_OK          0
#define HELM_EINVAL      1  /* null pointer, bad size, non-finite input      */
#define HELM_ENOMEM      2  /* plan exceeds the memory budget / alloc failed */
#define HELM_EZEROPIVOT  3  /* exact zero or non-finite pivot in a front      */
#define HELM_ENOCONV     4  /* GMRES / refinement hit its iteration limit     */
#define HELM_EHIP        5  /* HIP runtime error                              */

/* ---- option flags ------------------------------------------------------ */
#define HELM_FLAG_PROFILE 1  /* time every substitution / sweep kernel launch with
                                HIP events on the handle's stream            */
#define HELM_FLAG_NO_GRAPHS 2 /* launch the substitution kernels one by one
                                instead of replaying captured HIP graphs     */
#define HELM_FLAG_AUTOTUNE 4  /* on the first solve of a layer set at a batch
                                width, time every column-tile width of the
                                substitution GEMMs per depth of the front
                                trees and keep the fastest (default: widths
                                from the batch width alone)                  */
#define HELM_FLAG_FULL_KRYLOV 16 /* GMRES on the whole polarized system rather
                                 than on its up-going block (the operator is
                                 block triangular; same stopping test)      */
#define HELM_FLAG_PROFILE_FWD 8 /* time only the forward substitution GEMM
                                launches, each with start and stop events
                                that the launch itself records; the other
                                kernels run without events between them     */
#define HELM_FLAG_BICGSTAB 64  /* Bi-CGSTAB instead of GMRES on the preconditioned
                                polarized system (the memory-lean Krylov method
                                named in Section "Method of Polarized traces":
                                six work vectors per column, two operator
                                applications per iteration)                   */
#define HELM_FLAG_UNPOLARIZED 128 /* GMRES on the unpolarized SIE (Eq. "SIE",
                                Algorithms 2-3, sign made consistent: (I - GJ) u
                                = v) without preconditioner: every iteration
                                is one batched solve of all layers at once    */
#define HELM_FLAG_NO_PRUNE 256 /* the sweep solves of the GMRES iterations run
                                every front of the layer; by default they skip
                                the fronts that neither their interface sources
                                nor their interface read-outs reach (Section
                                "Local Solves: Parallel Multi-frontal Methods":
                                sources supported on the interfaces, only the
                                boundary values needed)                       */
#define HELM_FLAG_GEMM_4M 512 /* complex64 substitution GEMMs form each complex
                                product from four real matrix-core products;
                                by default they take three (Pr Qr, Pi Qi and
                                (Pr + Pi)(Qr + Qi)), whose rounding error is
                                bounded in norm rather than per component.
                                No effect on HELM_FP64 handles               */
#define HELM_FLAG_FACTOR_4M 1024 /* the complex64 factorization's sweep GEMM
                                forms each complex product from four real
                                products (default: three, as the
                                substitutions).  No effect on HELM_FP64
                                handles                                      */
#define HELM_FLAG_NO_NARROW 2048 /* every refinement step and every GMRES
                                iteration runs at the batch's full width.  By
                                default (mixed) a column that meets the target
                                leaves the refinement, and a later step whose
                                remaining columns fit in half the width or
                                less runs them, gathered, at the narrowest
                                power-of-two width that holds them; and (both
                                precisions) a GMRES iteration whose running
                                columns fit in half the width applies the
                                operator to those columns only, gathered the
                                same way                                      */
#define HELM_FLAG_TEST_ZERO_FRONT 32 /* test hook of the zero-pivot status:
                                the factorization leaves one leaf front of
                                layer 0 unassembled, so its pivots are exactly
                                zero; the kernels run to the end (a zero pivot
                                is replaced by one) and helm_factorize returns
                                HELM_EZEROPIVOT                              */

/* ---- precision of the local factors ----------------------------------- */
#define HELM_FP64   0   /* complex128 fronts and substitutions              */
#define HELM_MIXED  1   /* complex64 fronts on MFMA + FP64 refinement       */

typedef struct helm_handle helm_handle;   /* opaque */

typedef struct {
  int nx, ny, nz;   /* nodes per axis, absorbing layer included */
  double h;         /* grid spacing */
} helm_grid;

typedef struct {
  int    pml_local;        /* absorbing planes added at internal sides (>=1) */
  double pml_C;            /* PML strength C; <= 0 selects 20 * max(c)       */
  int    precision;        /* HELM_FP64 or HELM_MIXED                        */
  double gmres_tol;        /* stop on |P(f - M x)| <= tol |P f|              */
  int    gmres_max_iter;   /* max GMRES iterations over all restart cycles  */
  double ir_tol;           /* mixed: stop refinement at |f-Hu| <= ir_tol |f| */
  int    ir_max_steps;     /* mixed: max refinement steps                    */
  double inner_tol;        /* mixed: GMRES tolerance of the first solve      */
  double inner_tol_refine; /* mixed: GMRES tolerance of later refinement steps
                              (<= 0: same as inner_tol)                      */
  double err_target;       /* mixed: a column also stops once its estimated
                              error is at most a quarter of this after the
                              second solve (the estimate then rests on one
                              measured contraction) or at most half of it
                              from the third on (a factor 4 / 2 margin
                              against the estimate; <= 0: off)              */
  size_t hbm_budget_bytes; /* 0 = 90% of free device memory                  */
  int    device;           /* HIP device ordinal                             */
  void*  stream;           /* hipStream_t for the *_dev entry points (NULL = default) */
  int    max_rhs;          /* widest RHS batch one internal launch carries   */
  int    leaf_size;        /* nested-dissection leaf size (DOFs), 0 = default */
  int    flags;            /* HELM_FLAG_* bits, 0 by default */
  int    gmres_restart;    /* GMRES restart length (basis vectors kept); 0 =
                              as many as device memory allows, at most 60.
                              A smaller value is honoured, and the memory
                              bound still caps it                           */
  double inner_tol_final;  /* mixed: GMRES tolerance of a step taken when a
                              column's estimated error is already within
                              err_target but not within the part of it that
                              stops the column (<= 0: inner_tol_refine)     */
} helm_options;

typedef struct {
  int    n_rhs;
  int    gmres_iters;        /* total GMRES iterations (max over columns)   */
  int    ir_steps;           /* refinement steps taken (1 for FP64)          */
  double rel_residual_max;   /* max over columns of |f - H u| / |f| (FP64)   */
  double t_setup_ms;         /* local solves of the partitioned source       */
  double t_gmres_ms;         /* GMRES on the interface system                */
  double t_reconstruct_ms;   /* final local solves                           */
  double t_residual_ms;      /* FP64 residual / refinement updates           */
  double t_total_ms;
  long long layer_solves;    /* number of single-layer multi-RHS solves      */
  double factor_bytes_read;  /* factor bytes streamed by the substitutions   */
  double ir_residual[8];     /* max over columns of |f - H u| / |f| after each
                                refinement step (first 8 steps)              */
  double est_error_max;      /* mixed: max over columns of the estimated
                                relative error |u - H^-1 f| / |u| when the
                                column stopped: |d_k|/|u| * q/(1-q) with d_k
                                the last correction and q the larger of the
                                last two measured contractions |d_k|/|d_{k-1}|
                                (one after the second step) and of 4 times
                                the relative residual the step's GMRES
                                reached; 1 (unknown) after a single step or
                                when q > 1/2                                 */
  int    ir_gmres_iters[8];  /* GMRES iterations of each refinement step     */
  /* Per right-hand side: arrays of n_rhs entries owned by the caller, each
   * may be NULL; set them before the call (they survive the call's reset of
   * the other fields) and the solve fills them. */
  double* rhs_rel_residual;  /* final FP64 |f - H u| / |f| of each column    */
  double* rhs_est_error;     /* mixed: estimated relative error of each
                                column (as est_error_max); 0 for FP64         */
  int*    rhs_ir_steps;      /* refinement step at which the column first met
                                ir_tol or err_target (the steps taken if it
                                never did; 1 for FP64)                        */
  int*    rhs_gmres_iters;   /* GMRES iterations in which the column was
                                still active, summed over refinement steps   */
  double krylov_bytes;       /* device bytes of the Krylov vectors (basis or
                                Bi-CGSTAB work vectors) the solve held       */
  int    ir_width[8];        /* columns each refinement step ran at (first 8
                                steps; the widest over the internal batches) */
  int    narrow_products;    /* GMRES operator products applied to the
                                running columns at a narrower width          */
} helm_solve_info;

/* Fill `opt` with defaults: pml_local 4, pml_C 0 (auto), HELM_MIXED,
 * gmres_tol 1e-10, gmres_max_iter 40, ir_tol 1e-9, ir_max_steps 6,
 * inner_tol 5e-4, inner_tol_refine 2e-4, err_target 0 (off), hbm_budget 0
 * (auto), device 0, stream NULL, max_rhs 64, leaf_size 64, flags 0,
 * gmres_restart 0 (memory-bound, at most 60), inner_tol_final 1e-1. */
void helm_default_options(helm_options* opt);

/* Planner (no device memory is touched).  Exact sizes from the symbolic
 * nested-dissection analysis of all layers:
 *   factor_bytes  -- resident factors for the chosen precision;
 *   bytes_per_rhs -- device memory one more RHS column costs in helm_solve;
 *   max_front     -- largest frontal matrix dimension s + b.
 * Any output pointer may be NULL.  Returns HELM_EINVAL for impossible
 * geometries (layers thinner than one plane, pml_width too large). */
int helm_plan(const helm_grid* g, int pml_width, int n_layers,
              const helm_options* opt, size_t* factor_bytes,
              size_t* bytes_per_rhs, size_t* max_front);

/* Device memory one more column slot costs in a lane of the request server
 * or of a batched problem (include/helm_serve.h, include/helm_batch.h): the
 * bytes_per_rhs of helm_plan plus the Krylov and sweep vectors of the lane's
 * narrower step widths.  A lane of K slots reserves factor_bytes +
 * K * lane_bytes_per_rhs.  Same arguments and errors as helm_plan. */
int helm_plan_lane(const helm_grid* g, int pml_width, int n_layers,
                   const helm_options* opt, size_t* lane_bytes_per_rhs);

/* Offline stage (Algorithm 1).  `m` is the squared slowness 1/c^2 on the
 * full grid (host pointer, nx*ny*nz doubles, copied).  `omega` > 0 is the
 * angular frequency, `pml_width` the global absorbing nodes per face,
 * `n_layers` >= 1 the number of layers L.  On success *out owns the device
 * factors until helm_free.  opt == NULL selects the defaults. */
int helm_factorize(const helm_grid* g, const double* m, double omega,
                   int pml_width, int n_layers, const helm_options* opt,
                   helm_handle** out);

/* Same with `m_dev` a device pointer (read during the call only). */
int helm_factorize_dev(const helm_grid* g, const double* m_dev, double omega,
                       int pml_width, int n_layers, const helm_options* opt,
                       helm_handle** out);

/* Online stage (Algorithm 2) for host arrays: f and u hold n_rhs volumes
 * of complex doubles (2*nx*ny*nz*n_rhs doubles, RHS-major).  u is written,
 * f is not modified.  info may be NULL.  Returns HELM_ENOCONV (u then holds
 * the last iterate and info is filled) when a tolerance was not met. */
int helm_solve(helm_handle* h, int n_rhs, const double* f, double* u,
               helm_solve_info* info);

/* Same with device pointers; work is enqueued on opt->stream of the handle
 * and the call returns after the stream has completed. */
int helm_solve_dev(helm_handle* h, int n_rhs, const double* f_dev,
                   double* u_dev, helm_solve_info* info);

/* Point sources: column r is amplitude[r] / h^3 at node node_index[r]
 * (index i + nx*(j + ny*k)); arrays are host pointers of length n_rhs
 * (amplitude: 2*n_rhs doubles, complex).  The 1/h^3 scale is the numerical
 * Dirac delta of the classical finite-difference discretization (Section
 * "Formulation", definition of the delta at a fixed depth), taken at a single
 * node.  u_dev is a device array of n_rhs volumes.  Errors: HELM_EINVAL for
 * a node outside the grid or a non-finite amplitude (nothing is solved). */
int helm_solve_points(helm_handle* h, int n_rhs, const int64_t* node_index,
                      const double* amplitude, double* u_dev,
                      helm_solve_info* info);

/* Per-kernel-class launch statistics gathered while HELM_FLAG_PROFILE is set:
 * launch count, summed event-timed duration, and the algorithmic flops and
 * HBM bytes of those launches (complex work counted as 8 real flops per
 * multiply-add; bytes = factor blocks read once plus the right-hand-side
 * rows read and written).  Writes up to `max` records, the number of
 * classes to *count; `reset` != 0 clears the counters afterwards. */
typedef struct {
  char      name[32];
  long long launches;
  double    total_ms;
  double    flops;
  double    bytes;
} helm_kernel_stat;

int helm_kernel_stats(helm_handle* h, helm_kernel_stat* out, int max, int* count,
                      int reset);

/* Column-tile choices of the substitution GEMMs: one record per (layer set,
 * batch width k, depth of the front trees), for the sets used so far.  A
 * layer set is described by its number of layers.  fwd_bn / bwd_bn are the
 * tile kinds in use: 16, 32 or 64 for MFMA tiles of that many columns, 1
 * for the vector path (default up to 2 columns, a candidate up to 4); when
 * the choice was measured (HELM_FLAG_AUTOTUNE), t_fwd_us / t_bwd_us hold the
 * timed launch of each kind in the order 1, 16, 32, 64 (0 where a kind was
 * not tried).  Writes up to `max` records and the total to *count. */
typedef struct {
  int    set_layers, k, depth, fronts;
  double mean_s, mean_b;   /* mean pivot / boundary size of the depth's fronts */
  int    fwd_bn, bwd_bn, bwd_bm, tuned;
  double t_fwd_us[4], t_bwd_us[4];
  double fwd_elems;        /* sum of (s + b) s over the forward list: the
                              forward product's complex multiply-adds per
                              column */
  double bwd_elems;        /* sum of b s over the backward list (the same
                              for the backward product) */
} helm_tile_choice;

int helm_tile_choices(helm_handle* h, helm_tile_choice* out, int max, int* count);

/* Calibration: the attainable rates of the device, measured with the
 * instruction shapes and access widths the solver uses.  Matrix cores:
 * back-to-back v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 on 8
 * independent accumulators per wave, 8 workgroups of 4 waves per compute
 * unit (TFLOP/s).  HBM: a streaming 16-byte read of 2 GiB and a copy of
 * 2 GiB (bytes read + written per second, GB/s).  Best of three runs each.
 * Any output pointer may be NULL.  Allocates 4 GiB of device memory for the
 * duration of the call. */
int helm_device_peaks(int device, double* mfma_f32_tflops, double* mfma_f64_tflops,
                      double* hbm_read_gbps, double* hbm_copy_gbps);

/* Change the online-stage options of a factorized handle (gmres_tol,
 * gmres_max_iter, gmres_restart, ir_tol, ir_max_steps, inner_tol,
 * inner_tol_refine, inner_tol_final, err_target, max_rhs, flags); the
 * geometry, precision,
 * device and stream fields are ignored. */
int helm_set_solve_options(helm_handle* h, const helm_options* opt);

/* Record of the offline stage (Algorithm 1) of a factorized handle.
 *   lu_flops     -- algorithmic real flops: an LU of every front,
 *                   sum 4 (2/3 s^3 + 2 s^2 b + 2 s b^2) over fronts with s
 *                   pivots and b boundary variables;
 *   gj_flops     -- real flops the blocked Gauss-Jordan sweep executes (it
 *                   also forms F11^-1, so that the substitutions are plain
 *                   products);
 *   pivot_min / pivot_max -- smallest and largest |pivot| chosen by the
 *                   partial pivoting within the fully summed rows of each
 *                   front;
 *   diag_max     -- largest |diagonal entry| of the assembled operators;
 *                   pivot_max / diag_max is the pivot growth;
 *   factor_bytes -- resident factors; n_fronts, max_front -- over layers;
 *   seconds      -- wall time of the numeric factorization (assembly and
 *                   elimination of every front);
 *   symbolic_seconds -- the layers' nested-dissection plans and PML
 *                   profiles (host);
 *   setup_seconds -- device allocation and upload of the model, the plans
 *                   and the front tables;
 *   lists_seconds -- launch lists of the single-layer solves.
 * The four times add up to the wall time of helm_factorize(_dev) apart
 * from the model's copy and checks. */
typedef struct {
  double seconds;
  double lu_flops, gj_flops;
  double pivot_min, pivot_max, diag_max;
  size_t factor_bytes;
  long long n_fronts, max_front;
  double symbolic_seconds, setup_seconds, lists_seconds;
} helm_factor_info;

int helm_get_factor_info(const helm_handle* h, helm_factor_info* out);

/* Release the factors and all device memory owned by the handle. */
int helm_free(helm_handle* h);

/* Static description of a status code; thread-local detail of the last
 * failure. */
const char* helm_strerror(int status);
const char* helm_last_error(void);

/* ---- inspection entry points (used by the tests) ------------------------
 * They expose single steps of the online stage so that each can be
 * compared with an independent implementation. */

/* Number of layers and the plane range of layer l: bulk [s, e] and the
 * extended range [lo, hi] (global plane indices). */
int helm_layer_info(const helm_handle* h, int l, int* s, int* e, int* lo,
                    int* hi);

/* One multi-RHS local solve w = (H^l)^{-1} r of Eq. "discrete_local_Helmholtz"
 * (the forward and backward substitutions over the layer's front tree).
 * r_dev, w_dev: device arrays of k local volumes, RHS-major, natural order
 * (i + nx*(j + ny*(z - lo))), complex double.  In HELM_MIXED the substitution
 * runs in complex64. */
int helm_layer_solve_dev(helm_handle* h, int l, int k, const double* r_dev,
                         double* w_dev);

/* Allocation-free variant of helm_layer_solve_dev, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, layout and result as
 * helm_layer_solve_dev (and the same kernels), but the solve's workspace --
 * the solve vector, the forward results, the update buffers and the split-K
 * partial products of layer l for k columns, plus the kernels' layer table --
 * lives in a static device array of HELM_NOALLOC_SCRATCH_BYTES per GPU (held
 * until the process ends) instead of the handle's allocations; it calls no
 * hipMalloc, hipFree or other allocating routine and never replays a graph.
 * Errors: HELM_EINVAL for bad arguments, HELM_ENOMEM (nothing launched) when
 * the workspace of k columns of this layer exceeds the array.  Every call on
 * one GPU uses that GPU's single array: calls that overlap on one GPU (other
 * handles or streams, other threads) race and must be serialized by the
 * caller.  Nothing in the array needs to start at zero: each call writes
 * every byte it reads. */
#define HELM_NOALLOC_SCRATCH_BYTES (128ull << 20)
int helm_layer_solve_noalloc_dev(helm_handle* h, int l, int k, const double* r_dev,
                                 double* w_dev);

/* FP64 residual r = f - H u of the global 7-point operator (device arrays of
 * k volumes, RHS-major).  With f_dev == NULL it returns H u. */
int helm_apply_operator_dev(helm_handle* h, int k, const double* f_dev,
                            const double* u_dev, double* r_dev);

/* Polarized interface operators on pair vectors.  A pair vector holds, for
 * interfaces j = 0..L-2, the two planes (u(e_j), u(e_j + 1)); layout
 * [j][plane 0/1][y][x][column], complex double, device memory.
 *   op 0: the preconditioner P applied to (x_down, x_up)  (Algs. 4-6),
 *   op 1: P M x = x + P (U x_up, 0)                        (Alg. 7 + P),
 *         with the local solves of U folded into the sweeps,
 *   op 2: U x_up                                            (Alg. 10),
 *   op 3: the polarized right-hand side (f_down, f_up) of a volume source
 *         (the first steps of Alg. 2); `in_dev` is then k volumes
 *         (RHS-major),
 *   op 4: P (f_down, f_up) of a volume source in one folded sweep pair (the
 *         right-hand side GMRES works on); `in_dev` is k volumes.
 * For ops 0-1 `in_dev`/`out_dev` hold [x_down | x_up], each a pair vector;
 * for ops 3-4 `out_dev` holds [down | up]. */
int helm_polarized_op_dev(helm_handle* h, int op, int k, const double* in_dev,
                          double* out_dev);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
