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

// forward, step 2: [X(S); Ub] = [F11^-1 w_S; Ub - F21 F11^-1 w_S]
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           int n_ids, const int* __restrict__ prefix,
           const LayerDev* __restrict__ layers, int k) {
  using C = C_t<T>;
  __shared__ GemmSmem<T> sm;
  const int ntn = (k + GT - 1) / GT;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int a = find_segment(prefix, n_ids, mt);
  const FrontDev f = fronts[ids[a]];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int m0 = (mt - prefix[a]) * GT, n0 = nt * GT;
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  // P = FT (col-major, rows m), Q = Wt (rows = pivots, columns = RHS)
  View<T> pv{FT, 1, (long long)n, n, f.s};
  View<T> qv{reinterpret_cast<const C*>(L.Wt) + f.wt * k, 1, (long long)k, k, f.s};
  WaveAcc<T> acc;
  gemm_tile<T, true, true>(sm, acc, pv, qv, m0, n0, f.s);
  C* X = reinterpret_cast<C*>(L.X);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  for_each_acc<T>(acc, [&](int r, int c, C z) {
    const int gm = m0 + r, gc = n0 + c;
    if (gm >= n || gc >= k) return;
    if (gm < f.s) {
      X[(long long)(f.off + gm) * k + gc] = z;
    } else {
      C& u = Uo[(f.ub + gm - f.s) * k + gc];
      u = cadd(u, z);
    }
  });
}

// backward, step 1: gather X at the boundary variables into Ub
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_gather(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_ids, const int* __restrict__ prefix,
             const LayerDev* __restrict__ layers, int k) {
  using C = C_t<T>;
  const int a = find_segment(prefix, n_ids, blockIdx.x);
  const FrontDev f = fronts[ids[a]];
  const LayerDev& L = layers[f.layer];
  const int r0 = (blockIdx.x - prefix[a]) * GT;
  const C* X = reinterpret_cast<const C*>(L.X);
  C* Ub = ub_ptr<T>(L, f.ub_parity);
  const int* B = L.bidx + f.bidx;
  const int rows = (f.b - r0) < GT ? (f.b - r0) : GT;
  for (int e = threadIdx.x; e < rows * k; e += 256) {
    const int rr = r0 + e / k, c = e % k;
    Ub[(f.ub + rr) * k + c] = X[(long long)B[rr] * k + c];
  }
}

// backward, step 2: X(S) += (-F21 F11^-1)^T X(B)
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           int n_ids, const int* __restrict__ prefix,
           const LayerDev* __restrict__ layers, int k) {
  using C = C_t<T>;
  __shared__ GemmSmem<T> sm;
  const int ntn = (k + GT - 1) / GT;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int a = find_segment(prefix, n_ids, mt);
  const FrontDev f = fronts[ids[a]];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int m0 = (mt - prefix[a]) * GT, n0 = nt * GT;
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  // P(m, q) = FT[(s + q) + m n]  (transposed lower block, contiguous in q)
  View<T> pv{FT + f.s, (long long)n, 1, f.s, f.b};
  View<T> qv{ub_ptr<T>(L, f.ub_parity) + f.ub * k, 1, (long long)k, k, f.b};
  WaveAcc<T> acc;
  gemm_tile<T, false, true>(sm, acc, pv, qv, m0, n0, f.b);
  C* X = reinterpret_cast<C*>(L.X);
  for_each_acc<T>(acc, [&](int r, int c, C z) {
    const int gm = m0 + r, gc = n0 + c;
    if (gm >= f.s || gc >= k) return;
    C& x = X[(long long)(f.off + gm) * k + gc];
    x = cadd(x, z);
  });
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
void launch_fwd_gemm(const FrontDev* fr, const int* ids, int n, const int* prefix,
                     int total_mtiles, const LayerDev* layers, int k, hipStream_t st) {
  if (total_mtiles <= 0) return;
  const int ntn = (k + GT - 1) / GT;
  hipLaunchKernelGGL(k_fwd_gemm<T>, dim3(total_mtiles * ntn), dim3(256), 0, st, fr,
                     ids, n, prefix, layers, k);
}
template <typename T>
void launch_bwd_gather(const FrontDev* fr, const int* ids, int n, const int* prefix,
                       int total, const LayerDev* layers, int k, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_bwd_gather<T>, dim3(total), dim3(256), 0, st, fr, ids, n,
                     prefix, layers, k);
}
template <typename T>
void launch_bwd_gemm(const FrontDev* fr, const int* ids, int n, const int* prefix,
                     int total_mtiles, const LayerDev* layers, int k, hipStream_t st) {
  if (total_mtiles <= 0) return;
  const int ntn = (k + GT - 1) / GT;
  hipLaunchKernelGGL(k_bwd_gemm<T>, dim3(total_mtiles * ntn), dim3(256), 0, st, fr,
                     ids, n, prefix, layers, k);
}

#define HELM_INST_SOLVE(T)                                                         \
  template void launch_fwd_gather<T>(const FrontDev*, const int*, int, const int*, \
                                     int, const LayerDev*, int, hipStream_t);      \
  template void launch_fwd_gemm<T>(const FrontDev*, const int*, int, const int*,   \
                                   int, const LayerDev*, int, hipStream_t);        \
  template void launch_bwd_gather<T>(const FrontDev*, const int*, int, const int*, \
                                     int, const LayerDev*, int, hipStream_t);      \
  template void launch_bwd_gemm<T>(const FrontDev*, const int*, int, const int*,   \
                                   int, const LayerDev*, int, hipStream_t);
HELM_INST_SOLVE(float)
HELM_INST_SOLVE(double)

}  // namespace kern
}  // namespace helm
