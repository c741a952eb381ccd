// Host-side declarations of the kernel launchers (definitions in *.hip).
#pragma once

#include "helm_internal.h"

namespace helm {
namespace kern {

// out(a|b) = sx * R(X)(a|b) + sum_i (ca_i in_i(a), cb_i in_i(b))
// Only the planes of `planes` are written (bit 0: a, bit 1: b).
struct ReadTerms {
  const double2* in[3];
  double ca[3], cb[3];
  int planes;
};

// --- factorization (kernels_factor.hip) -------------------------------------
// Device record of a factorization: flag set on an exact-zero or non-finite
// pivot; smallest and largest |pivot|^2 and largest |diagonal entry|^2 of
// the assembled operator, as the bit patterns of non-negative doubles (which
// order like the numbers, so integer atomics min / max them).
struct FactorStatus {
  int flag;
  int pad;
  unsigned long long pmin, pmax, dmax;
};
template <typename T>
void launch_extend_add(const FrontDev* fronts, const int* ids, int n_ids,
                       const int2* tmap, int total, const LayerDev* layers,
                       void* ws0, void* ws1, hipStream_t st);
// skip_front >= 0: that front is left unassembled (its pivots are then
// exactly zero), a hook that lets tests reach the zero-pivot status
template <typename T>
void launch_orig_entries(const FrontDev* fronts, const int* ids, int n_ids,
                         const int2* tmap, int total, const LayerDev* layers,
                         void* ws0, void* ws1, const GridDev& g, int skip_front,
                         FactorStatus* status, hipStream_t st);
template <typename T>
void launch_panel(const FrontDev* fronts, const int* ids, int n_active, int max_rows,
                  int k, int nb, void* ws0, void* ws1, void* panel,
                  const long long* panel_off, void* D, int* ipiv, int* perm,
                  const long long* perm_off, FactorStatus* status, hipStream_t st);
template <typename T>
void launch_swap_JO(const FrontDev* fronts, const int* ids, int n_active,
                    const int2* tmap, int total, int k, int nb, void* ws0,
                    void* ws1, const void* D, const int* ipiv,
                    const long long* panel_off, const long long* perm_off,
                    hipStream_t st);
template <typename T>
// m3: three real products per complex product (complex64 only)
void launch_sweep_gemm(const FrontDev* fronts, const int* ids, int n_active,
                       const int2* tmap, int total, int k, int nb, void* ws0,
                       void* ws1, bool m3, hipStream_t st);
template <typename T>
void launch_update_OJ(const FrontDev* fronts, const int* ids, int n_active,
                      const int2* tmap, int total, int k, int nb, void* ws0,
                      void* ws1, const void* D, const long long* panel_off,
                      hipStream_t st);
template <typename T>
void launch_store_factor(const FrontDev* fronts, const int* ids, int n_ids,
                         const int2* tmap, int total, const LayerDev* layers,
                         void* ws0, void* ws1, const int* perm,
                         const long long* perm_off, hipStream_t st);

// --- substitutions (kernels_solve.hip) --------------------------------------
template <typename T>
void launch_fwd_gather(const FrontDev* fr, const int* ids, int n, const int2* tmap,
                       int total, const LayerDev* layers, int k, hipStream_t st);
template <typename T>
// t0 / t1 non-null: the launch records its own start and stop in them
// (timing of the kernel alone, without event commands around it).
// m3: three real products per complex product (complex64 only; ignored for
// complex128).
void launch_fwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bn, bool m3, hipStream_t st, hipEvent_t t0 = nullptr,
                     hipEvent_t t1 = nullptr);
// vector path of the substitutions for k <= 4 columns (same tiles and
// scratch layout as launch_fwd_gemm / launch_bwd_gemm with 64-row tiles)
template <typename T>
void launch_fwd_gemv(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, hipStream_t st, hipEvent_t t0 = nullptr,
                     hipEvent_t t1 = nullptr);
template <typename T>
void launch_bwd_gemv(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bm, hipStream_t st, hipEvent_t t0 = nullptr,
                     hipEvent_t t1 = nullptr);
template <typename T>
void launch_fwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int2* tmap, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st);
template <typename T>
void launch_bwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bm, int bn, bool m3, hipStream_t st,
                     hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
template <typename T>
void launch_bwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int2* tmap, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st);

// --- volumes, traces, Krylov (kernels_volume.hip) ---------------------------
template <typename T>
void launch_scatter_source(const LayerDev& L, const double2* f, int nx, int ny,
                           long long N, int k, hipStream_t st);
template <typename T>
void launch_gather_volume(const LayerDev& L, double2* u, int nx, int ny,
                          long long N, int k, hipStream_t st);
template <typename T>
void launch_local_to_X(const LayerDev& L, const double2* r, int k, hipStream_t st);
template <typename T>
void launch_X_to_local(const LayerDev& L, double2* w, int k, hipStream_t st);
// Interface source sum c0 in0 + c1 in1 + c2 in2 of pair vectors (null
// entries skipped).
struct JumpTerms {
  const double2* in[3];
  double c[3];
};
template <typename T>
void launch_jump(const LayerDev& L, const JumpTerms& t, const double2* B, int bottom, int nx,
                 int ny, int k, hipStream_t st);
template <typename T>
void launch_readout(const LayerDev& L, int bottom, double sx, const ReadTerms& terms,
                    double2* out, int nx, int ny, int k, hipStream_t st);

void launch_dot(const double2* x, const double2* y, long long V, int k,
                double2* partial, double2* out, hipStream_t st);
void launch_axpy_cols(double2* y, const double2* x, const double2* alpha,
                      double sign, long long V, int k, hipStream_t st);
// Column selection of a batch of k interleaved columns (element e of column
// c at e k + c), at most kMaxGatherCols columns.
constexpr int kMaxGatherCols = 64;
struct ColMap {
  int col[kMaxGatherCols];
};
// out[e w + j] = in[e k + map.col[j]] for j < m, zero for m <= j < w
void launch_gather_cols(double2* out, const double2* in, long long V, int k, int w, int m,
                        const ColMap& map, hipStream_t st);
// out[e k + c] = in[e w + slot.col[c]] where slot.col[c] >= 0, else zero
void launch_scatter_cols(double2* out, const double2* in, long long V, int k, int w,
                         const ColMap& slot, hipStream_t st);
void launch_scale_cols(double2* y, const double2* x, const double* s, long long V,
                       int k, hipStream_t st);
void launch_add(double2* y, const double2* x, const double2* z, long long n,
                hipStream_t st);
// y = z - y in place (elementwise)
void launch_rsub(double2* y, const double2* z, long long n, hipStream_t st);
// y[v, c] = x[v, c] + alpha[c] y[v, c]   (alpha per column, complex)
void launch_xpay_cols(double2* y, const double2* x, const double2* alpha, long long V, int k,
                      hipStream_t st);
void launch_residual(const GridDev& g, const double2* f, const double2* u,
                     double2* r, int k, hipStream_t st);
void launch_point_sources(double2* f, const long long* node, const double2* amp,
                          double inv_h3, long long N, int k, hipStream_t st);
void launch_accumulate(double2* u, const double2* d, long long n, hipStream_t st);
void launch_volume_norm2(const double2* x, long long N, int k, double* partial,
                         double* out, hipStream_t st);

constexpr int DOT_PARTIAL_BLOCKS = 256;   // partial buffer: k * 256 double2
constexpr int NORM_PARTIAL_BLOCKS = 128;  // partial buffer: k * 128 double

}  // namespace kern
}  // namespace helm
