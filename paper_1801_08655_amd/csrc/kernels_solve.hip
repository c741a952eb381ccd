// Multi-RHS substitutions over a layer's front tree (online stage: every
// local solve (H^l)^-1 of Algorithms 2-10).
//
// With the stored blocks [F11^-1; -F21 F11^-1] of every front:
//   forward (leaves -> root):  w = [X(S) + children; children] (extend-add of
//     the children's updates), X(S) <- F11^-1 w_S, update_B <- w_B - F21 F11^-1 w_S
//   backward (root -> leaves): X(S) <- X(S) + (-F21 F11^-1)^T X(B)
// Both passes are dense complex GEMMs with the RHS columns as N; the solve
// vector X is stored in nested-dissection order with the columns fastest.
#include "kernels.h"
#include "kernels_common.h"

namespace helm {
namespace kern {

namespace {

template <typename T>
__device__ __forceinline__ C_t<T>* ub_ptr(const LayerDev& L, int parity) {
  return reinterpret_cast<C_t<T>*>(L.Ub[parity]);
}

// forward, step 1: gather the pivots' right-hand side plus the children's
// updates into Wt (pivot rows) and Ub (boundary rows).
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_gather(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_ids, const int* __restrict__ prefix,
             const LayerDev* __restrict__ layers, int k) {
  using C = C_t<T>;
  const int a = find_segment(prefix, n_ids, blockIdx.x);
  const FrontDev f = fronts[ids[a]];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int r0 = (blockIdx.x - prefix[a]) * GT;
  const C* X = reinterpret_cast<const C*>(L.X);
  C* Wt = reinterpret_cast<C*>(L.Wt);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  const C* Uc = ub_ptr<T>(L, f.ub_parity ^ 1);
  long long cub[2] = {0, 0};
  const int* inv[2] = {nullptr, nullptr};
  for (int slot = 0; slot < 2; ++slot)
    if (f.child[slot] >= 0) {
      cub[slot] = fronts[f.child[slot]].ub;
      inv[slot] = L.inv + f.inv[slot];
    }
  const int rows = (n - r0) < GT ? (n - r0) : GT;
  for (int e = threadIdx.x; e < rows * k; e += 256) {
    const int rr = r0 + e / k, c = e % k;
    C v = rr < f.s ? X[(long long)(f.off + rr) * k + c] : czero<C>();
#pragma unroll
    for (int slot = 0; slot < 2; ++slot)
      if (inv[slot]) {
        int q = inv[slot][rr];
        if (q >= 0) v = cadd(v, Uc[(cub[slot] + q) * k + c]);
      }
    if (rr < f.s) Wt[(f.wt + rr) * k + c] = v;
    else Uo[(f.ub + rr - f.s) * k + c] = v;
  }
}

// forward, step 2: [X(S); Ub] = [F11^-1 w_S; Ub - F21 F11^-1 w_S], the K
// (pivot) dimension optionally split into chunks (partials to scratch).
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int* __restrict__ prefix,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  __shared__ GemmSmem<T> sm;
  const int ntn = (k + GT - 1) / GT;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int a = find_segment(prefix, n_ids, mt);
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = mt - prefix[a];
  const int chunk = local % tk.nch_f;
  const int m0 = (local / tk.nch_f) * GT, n0 = nt * GT;
  const int kb = chunk * tk.kc_f;
  const int ke = min(f.s, kb + tk.kc_f);
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  // P = FT (col-major, rows m), Q = Wt (rows = pivots, columns = RHS)
  View<T> pv{FT, 1, (long long)n, n, f.s};
  View<T> qv{reinterpret_cast<const C*>(L.Wt) + f.wt * k, 1, (long long)k, k, f.s};
  WaveAcc<T> acc;
  gemm_tile<T, true, true>(sm, acc, pv, qv, m0, n0, kb, ke);
  C* X = reinterpret_cast<C*>(L.X);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  C* S = reinterpret_cast<C*>(scratch);
  for_each_acc<T>(acc, [&](int r, int c, C z) {
    const int gm = m0 + r, gc = n0 + c;
    if (gm >= n || gc >= k) return;
    if (tk.nch_f > 1) {
      S[(tk.scr_f + (long long)chunk * n + gm) * k + gc] = z;
    } else if (gm < f.s) {
      X[(long long)(f.off + gm) * k + gc] = z;
    } else {
      C& u = Uo[(f.ub + gm - f.s) * k + gc];
      u = cadd(u, z);
    }
  });
}

// forward, step 3 (split fronts only): sum the chunk partials in order
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_reduce(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             const SolveTask* __restrict__ tasks, int n_ids, const int* __restrict__ prefix,
             const LayerDev* __restrict__ layers, int k, const void* scratch) {
  using C = C_t<T>;
  const int a = find_segment(prefix, n_ids, blockIdx.x);
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int r0 = (blockIdx.x - prefix[a]) * GT;
  const int rows = min(GT, n - r0);
  const C* S = reinterpret_cast<const C*>(scratch);
  C* X = reinterpret_cast<C*>(L.X);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  for (int e = threadIdx.x; e < rows * k; e += 256) {
    const int gm = r0 + e / k, gc = e % k;
    C z = czero<C>();
    for (int ch = 0; ch < tk.nch_f; ++ch)
      z = cadd(z, S[(tk.scr_f + (long long)ch * n + gm) * k + gc]);
    if (gm < f.s) {
      X[(long long)(f.off + gm) * k + gc] = z;
    } else {
      C& u = Uo[(f.ub + gm - f.s) * k + gc];
      u = cadd(u, z);
    }
  }
}

// backward: X(S) += (-F21 F11^-1)^T X(B); X(B) is read in place through the
// front's boundary index list, the K (boundary) dimension optionally split.
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int* __restrict__ prefix,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  __shared__ GemmSmem<T> sm;
  const int ntn = (k + GT - 1) / GT;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int a = find_segment(prefix, n_ids, mt);
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = mt - prefix[a];
  const int chunk = local % tk.nch_b;
  const int m0 = (local / tk.nch_b) * GT, n0 = nt * GT;
  const int kb = chunk * tk.kc_b;
  const int ke = min(f.b, kb + tk.kc_b);
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  C* X = reinterpret_cast<C*>(L.X);
  // P(m, q) = FT[(s + q) + m n]  (transposed lower block, contiguous in q)
  View<T> pv{FT + f.s, (long long)n, 1, f.s, f.b};
  // Q(c, q) = X[B[q] k + c]
  View<T> qv{X, 1, (long long)k, k, f.b, L.bidx + f.bidx};
  WaveAcc<T> acc;
  gemm_tile<T, false, true>(sm, acc, pv, qv, m0, n0, kb, ke);
  C* S = reinterpret_cast<C*>(scratch);
  for_each_acc<T>(acc, [&](int r, int c, C z) {
    const int gm = m0 + r, gc = n0 + c;
    if (gm >= f.s || gc >= k) return;
    if (tk.nch_b > 1) {
      S[(tk.scr_b + (long long)chunk * f.s + gm) * k + gc] = z;
    } else {
      C& x = X[(long long)(f.off + gm) * k + gc];
      x = cadd(x, z);
    }
  });
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_reduce(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             const SolveTask* __restrict__ tasks, int n_ids, const int* __restrict__ prefix,
             const LayerDev* __restrict__ layers, int k, const void* scratch) {
  using C = C_t<T>;
  const int a = find_segment(prefix, n_ids, blockIdx.x);
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int r0 = (blockIdx.x - prefix[a]) * GT;
  const int rows = min(GT, f.s - r0);
  const C* S = reinterpret_cast<const C*>(scratch);
  C* X = reinterpret_cast<C*>(L.X);
  for (int e = threadIdx.x; e < rows * k; e += 256) {
    const int gm = r0 + e / k, gc = e % k;
    C z = czero<C>();
    for (int ch = 0; ch < tk.nch_b; ++ch)
      z = cadd(z, S[(tk.scr_b + (long long)ch * f.s + gm) * k + gc]);
    C& x = X[(long long)(f.off + gm) * k + gc];
    x = cadd(x, z);
  }
}

}  // namespace

template <typename T>
void launch_fwd_gather(const FrontDev* fr, const int* ids, int n, const int* prefix,
                       int total, const LayerDev* layers, int k, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_fwd_gather<T>, dim3(total), dim3(256), 0, st, fr, ids, n,
                     prefix, layers, k);
}
template <typename T>
void launch_fwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int* prefix, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, hipStream_t st) {
  if (total_tiles <= 0) return;
  const int ntn = (k + GT - 1) / GT;
  hipLaunchKernelGGL(k_fwd_gemm<T>, dim3(total_tiles * ntn), dim3(256), 0, st, fr, ids,
                     tasks, n, prefix, layers, k, scratch);
}
template <typename T>
void launch_fwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int* prefix, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_fwd_reduce<T>, dim3(total), dim3(256), 0, st, fr, ids, tasks, n,
                     prefix, layers, k, scratch);
}
template <typename T>
void launch_bwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int* prefix, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, hipStream_t st) {
  if (total_tiles <= 0) return;
  const int ntn = (k + GT - 1) / GT;
  hipLaunchKernelGGL(k_bwd_gemm<T>, dim3(total_tiles * ntn), dim3(256), 0, st, fr, ids,
                     tasks, n, prefix, layers, k, scratch);
}
template <typename T>
void launch_bwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int* prefix, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_bwd_reduce<T>, dim3(total), dim3(256), 0, st, fr, ids, tasks, n,
                     prefix, layers, k, scratch);
}

#define HELM_INST_SOLVE(T)                                                           \
  template void launch_fwd_gather<T>(const FrontDev*, const int*, int, const int*,   \
                                     int, const LayerDev*, int, hipStream_t);        \
  template void launch_fwd_gemm<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int*, int, const LayerDev*, int,       \
                                   void*, hipStream_t);                              \
  template void launch_fwd_reduce<T>(const FrontDev*, const int*, const SolveTask*,  \
                                     int, const int*, int, const LayerDev*, int,     \
                                     const void*, hipStream_t);                      \
  template void launch_bwd_gemm<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int*, int, const LayerDev*, int,       \
                                   void*, hipStream_t);                              \
  template void launch_bwd_reduce<T>(const FrontDev*, const int*, const SolveTask*,  \
                                     int, const int*, int, const LayerDev*, int,     \
                                     const void*, hipStream_t);
HELM_INST_SOLVE(float)
HELM_INST_SOLVE(double)

}  // namespace kern
}  // namespace helm
