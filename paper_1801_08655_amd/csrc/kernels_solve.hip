// Multi-RHS substitutions over a layer's front tree (online stage: every
// local solve (H^l)^-1 of Algorithms 2-10).
//
// With the stored blocks [F11^-1; -F21 F11^-1] of every front:
//   forward (leaves -> root): X(S) += children's updates (extend-add, in
//     place; leaves have none), Z(S) <- F11^-1 X(S),
//     update_B <- children's updates - F21 F11^-1 X(S)
//   backward (root -> leaves): X(S) <- Z(S) + (-F21 F11^-1)^T X(B)
// Both passes are dense complex GEMMs with the RHS columns as N.  X (the
// solve vector) and Z are stored in nested-dissection order with the columns
// fastest; update_B lives in a per-depth-parity buffer.
#include "kernels.h"
#include "kernels_common.h"

namespace helm {
namespace kern {

namespace {

template <typename T>
__device__ __forceinline__ C_t<T>* ub_ptr(const LayerDev& L, int parity) {
  return reinterpret_cast<C_t<T>*>(L.Ub[parity]);
}

// Sum of the children's updates landing on front row `row` (extend-add in
// pull form through the front-row -> child-boundary maps).
template <typename T> struct ChildSum {
  const C_t<T>* Uc;
  long long cub[2];
  const int* inv[2];
  __device__ ChildSum(const FrontDev* fronts, const FrontDev& f, const LayerDev& L) {
    Uc = reinterpret_cast<const C_t<T>*>(L.Ub[f.ub_parity ^ 1]);
    for (int slot = 0; slot < 2; ++slot) {
      cub[slot] = 0;
      inv[slot] = nullptr;
      if (f.child[slot] >= 0) {
        cub[slot] = fronts[f.child[slot]].ub;
        inv[slot] = L.inv + f.inv[slot];
      }
    }
  }
  __device__ __forceinline__ C_t<T> operator()(int row, int col, int k) const {
    C_t<T> v = czero<C_t<T>>();
#pragma unroll
    for (int slot = 0; slot < 2; ++slot)
      if (inv[slot]) {
        const int q = inv[slot][row];
        if (q >= 0) v = cadd(v, Uc[(cub[slot] + q) * k + col]);
      }
    return v;
  }
};

// forward, step 1 (fronts with children): X(S) += children's updates on the
// pivot rows, in place.  The boundary rows are summed in the GEMM epilogue.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_gather(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, int k) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const LayerDev& L = layers[f.layer];
  const int r0 = tm.y * RT;
  C* X = reinterpret_cast<C*>(L.X);
  const ChildSum<T> cs(fronts, f, L);
  const int rows = (f.s - r0) < RT ? (f.s - r0) : RT;
  const int ty = threadIdx.x / GT, tx = threadIdx.x % GT;
  for (int rr = r0 + ty; rr < r0 + rows; rr += 256 / GT)
    for (int c = tx; c < k; c += GT) {
      C& x = X[(long long)(f.off + rr) * k + c];
      x = cadd(x, cs(rr, c, k));
    }
}

// forward, step 2: [X(S); Ub] = [F11^-1 w_S; Ub - F21 F11^-1 w_S], the K
// (pivot) dimension optionally split into chunks (partials to scratch).
template <typename T, int BN>
__global__ void __launch_bounds__(256)
k_fwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  constexpr int BM = FWD_BM;
  __shared__ GemmSmem<T, BM, BN> sm;
  const int ntn = (k + BN - 1) / BN;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = tm.y;
  const int chunk = local % tk.nch_f;
  const int m0 = (local / tk.nch_f) * BM, n0 = nt * BN;
  const int kb = chunk * tk.kc_f;
  const int ke = min(f.s, kb + tk.kc_f);
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  // P = FT (col-major, rows m), Q = X(S) (rows = pivots, columns = RHS)
  const C* X = reinterpret_cast<const C*>(L.X);
  View<T> pv{FT, 1, (long long)n, n, f.s};
  View<T> qv{X + (long long)f.off * k, 1, (long long)k, k, f.s};
  WaveAcc<T, BM, BN> acc;
  gemm_tile<T, BM, true, true>(sm, acc, pv, qv, m0, n0, kb, ke);
  C* Z = reinterpret_cast<C*>(L.Wt);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  C* S = reinterpret_cast<C*>(scratch);
  const ChildSum<T> cs(fronts, f, L);
  for_each_acc<T, BM>(acc, [&](int r, int c, C z) {
    const int gm = m0 + r, gc = n0 + c;
    if (gm >= n || gc >= k) return;
    if (tk.nch_f > 1) {
      S[(tk.scr_f + (long long)chunk * n + gm) * k + gc] = z;
    } else if (gm < f.s) {
      Z[(long long)(f.off + gm) * k + gc] = z;
    } else {
      Uo[(f.ub + gm - f.s) * k + gc] = cadd(z, cs(gm, gc, k));
    }
  });
}

// forward, step 3 (split fronts only): sum the chunk partials in order
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_reduce(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, int k, const void* scratch) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int r0 = tm.y * RT;
  const int rows = min(RT, n - r0);
  const C* S = reinterpret_cast<const C*>(scratch);
  C* Z = reinterpret_cast<C*>(L.Wt);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  const ChildSum<T> cs(fronts, f, L);
  for (int e = threadIdx.x; e < rows * k; e += 256) {
    const int gm = r0 + e / k, gc = e % k;
    C z = czero<C>();
    for (int ch = 0; ch < tk.nch_f; ++ch)
      z = cadd(z, S[(tk.scr_f + (long long)ch * n + gm) * k + gc]);
    if (gm < f.s) Z[(long long)(f.off + gm) * k + gc] = z;
    else Uo[(f.ub + gm - f.s) * k + gc] = cadd(z, cs(gm, gc, k));
  }
}

// backward: X(S) = Z(S) + (-F21 F11^-1)^T X(B); X(B) is read in place
// through the front's boundary index list, the K (boundary) dimension
// optionally split.  Fronts without boundary (roots) just copy Z(S).
template <typename T, int BM, int BN>
__global__ void __launch_bounds__(256)
k_bwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  __shared__ GemmSmem<T, BM, BN> sm;
  const int ntn = (k + BN - 1) / BN;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = tm.y;
  const int chunk = local % tk.nch_b;
  const int m0 = (local / tk.nch_b) * BM, n0 = nt * BN;
  const int kb = chunk * tk.kc_b;
  const int ke = min(f.b, kb + tk.kc_b);
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  C* X = reinterpret_cast<C*>(L.X);
  // P(m, q) = FT[(s + q) + m n]  (transposed lower block, contiguous in q)
  View<T> pv{FT + f.s, (long long)n, 1, f.s, f.b};
  // Q(c, q) = X[B[q] k + c]
  View<T> qv{X, 1, (long long)k, k, f.b, L.bidx + f.bidx};
  WaveAcc<T, BM, BN> acc;
  gemm_tile<T, BM, false, true>(sm, acc, pv, qv, m0, n0, kb, ke);
  C* S = reinterpret_cast<C*>(scratch);
  const C* Z = reinterpret_cast<const C*>(L.Wt);
  for_each_acc<T, BM>(acc, [&](int r, int c, C z) {
    const int gm = m0 + r, gc = n0 + c;
    if (gm >= f.s || gc >= k) return;
    const long long idx = (long long)(f.off + gm) * k + gc;
    if (tk.nch_b > 1) S[(tk.scr_b + (long long)chunk * f.s + gm) * k + gc] = z;
    else X[idx] = cadd(Z[idx], z);
  });
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_reduce(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, int k, const void* scratch) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int r0 = tm.y * RT;
  const int rows = min(RT, f.s - r0);
  const C* S = reinterpret_cast<const C*>(scratch);
  C* X = reinterpret_cast<C*>(L.X);
  const C* Z = reinterpret_cast<const C*>(L.Wt);
  for (int e = threadIdx.x; e < rows * k; e += 256) {
    const int gm = r0 + e / k, gc = e % k;
    const long long idx = (long long)(f.off + gm) * k + gc;
    C z = Z[idx];
    for (int ch = 0; ch < tk.nch_b; ++ch)
      z = cadd(z, S[(tk.scr_b + (long long)ch * f.s + gm) * k + gc]);
    X[idx] = z;
  }
}

// ---------------------------------------------------------------------------
// Vector path for batches of KC <= KV columns (a template argument): the GEMMs above would pad
// the columns to a 16-wide MFMA tile, so at k <= 4 the substitutions are
// done with plain FMAs while streaming the factor blocks once, which makes
// them bound by HBM bandwidth.  The tile and K-chunk decomposition (and the
// scratch layout of split fronts) is the one of the MFMA kernels, so the
// reduction kernels are shared.
// ---------------------------------------------------------------------------
constexpr int KV = 4;

// forward: one 64-row tile of one front and one K chunk per block; wave w
// takes the pivot columns kb + w, kb + w + 4, ... and the 4 partial sums of
// a row are added in LDS in fixed order.
template <typename T, int KC>
__global__ void __launch_bounds__(256)
k_fwd_gemv(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  __shared__ C red[3][64][KC];
  const int mt = blockIdx.x;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = tm.y;
  const int chunk = local % tk.nch_f;
  const int m0 = (local / tk.nch_f) * 64;
  const int kb = chunk * tk.kc_f;
  const int ke = min(f.s, kb + tk.kc_f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = m0 + lane;
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  const C* X = reinterpret_cast<const C*>(L.X) + (long long)f.off * KC;
  C acc[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) acc[c] = czero<C>();
  // q is the same for the whole wave: the right-hand-side values are
  // loaded once per wave (scalar loads), the factor column by every lane
  const int q0 = __builtin_amdgcn_readfirstlane(kb + w);
  if (m < n) {
#pragma unroll 4
    for (int q = q0; q < ke; q += 4) {
      const C fa = FT[m + (long long)q * n];
      const C* xq = X + (long long)q * KC;
#pragma unroll
      for (int c = 0; c < KC; ++c) cfma(acc[c], fa, xq[c]);
    }
  }
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < KC; ++c) red[w - 1][lane][c] = acc[c];
  }
  __syncthreads();
  if (w != 0 || m >= n) return;
  C* Z = reinterpret_cast<C*>(L.Wt);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  C* S = reinterpret_cast<C*>(scratch);
  const ChildSum<T> cs(fronts, f, L);
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const C z = cadd(cadd(acc[c], red[0][lane][c]), cadd(red[1][lane][c], red[2][lane][c]));
    if (tk.nch_f > 1) S[(tk.scr_f + (long long)chunk * n + m) * KC + c] = z;
    else if (m < f.s) Z[(long long)(f.off + m) * KC + c] = z;
    else Uo[(f.ub + m - f.s) * KC + c] = cadd(z, cs(m, c, KC));
  }
}

template <typename T> __device__ __forceinline__ T shfl_xor_t(T v, int mask) {
  return __shfl_xor(v, mask, 64);
}

// backward: one BM-row tile (BM = 32 or 64) and one K chunk per block; each
// 16-lane quarter of a wave takes one row at a time (BM/16 rows per
// quarter), its lanes walk the boundary index q (contiguous in the stored
// block) and a butterfly over the quarter sums the row.
template <typename T, int KC>
__global__ void __launch_bounds__(256)
k_bwd_gemv(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch, int bm) {
  using C = C_t<T>;
  const int mt = blockIdx.x;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = tm.y;
  const int chunk = local % tk.nch_b;
  const int m0 = (local / tk.nch_b) * bm;
  const int kb = chunk * tk.kc_b;
  const int ke = min(f.b, kb + tk.kc_b);
  const int g = threadIdx.x >> 4, gl = threadIdx.x & 15;   // 16 groups of 16 lanes
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  C* X = reinterpret_cast<C*>(L.X);
  const C* Z = reinterpret_cast<const C*>(L.Wt);
  C* S = reinterpret_cast<C*>(scratch);
  const int* B = L.bidx + f.bidx;
  for (int m = m0 + g; m < m0 + bm && m < f.s; m += 16) {
    C acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = czero<C>();
    const C* col = FT + f.s + (long long)m * n;
#pragma unroll 4
    for (int q = kb + gl; q < ke; q += 16) {
      const C fa = col[q];
      const C* xb = X + (long long)B[q] * KC;
#pragma unroll
      for (int c = 0; c < KC; ++c) cfma(acc[c], fa, xb[c]);
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        acc[c].x += shfl_xor_t(acc[c].x, off);
        acc[c].y += shfl_xor_t(acc[c].y, off);
      }
    }
    if (gl < KC) {
      C z = acc[0];
#pragma unroll
      for (int c = 1; c < KC; ++c)
        if (gl == c) z = acc[c];
      const long long idx = (long long)(f.off + m) * KC + gl;
      if (tk.nch_b > 1) S[(tk.scr_b + (long long)chunk * f.s + m) * KC + gl] = z;
      else X[idx] = cadd(Z[idx], z);
    }
  }
}

}  // namespace

template <typename T>
void launch_fwd_gemv(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, hipStream_t st) {
  if (total_tiles <= 0) return;
#define HELM_FWDV(KC_)                                                                     \
  hipLaunchKernelGGL((k_fwd_gemv<T, KC_>), dim3(total_tiles), dim3(256), 0, st, fr, ids,   \
                     tasks, n, tmap, layers, k, scratch)
  switch (k) {
    case 1: HELM_FWDV(1); break;
    case 2: HELM_FWDV(2); break;
    case 3: HELM_FWDV(3); break;
    default: HELM_FWDV(4); break;
  }
#undef HELM_FWDV
}
template <typename T>
void launch_bwd_gemv(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bm, hipStream_t st) {
  if (total_tiles <= 0) return;
#define HELM_BWDV(KC_)                                                                     \
  hipLaunchKernelGGL((k_bwd_gemv<T, KC_>), dim3(total_tiles), dim3(256), 0, st, fr, ids,   \
                     tasks, n, tmap, layers, k, scratch, bm)
  switch (k) {
    case 1: HELM_BWDV(1); break;
    case 2: HELM_BWDV(2); break;
    case 3: HELM_BWDV(3); break;
    default: HELM_BWDV(4); break;
  }
#undef HELM_BWDV
}

template <typename T>
void launch_fwd_gather(const FrontDev* fr, const int* ids, int n, const int2* tmap,
                       int total, const LayerDev* layers, int k, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_fwd_gather<T>, dim3(total), dim3(256), 0, st, fr, ids, n,
                     tmap, layers, k);
}
template <typename T>
void launch_fwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bn, hipStream_t st) {
  if (total_tiles <= 0) return;
  const int ntn = (k + bn - 1) / bn;
  const dim3 grid(total_tiles * ntn);
  if (bn == 16)
    hipLaunchKernelGGL((k_fwd_gemm<T, 16>), grid, dim3(256), 0, st, fr, ids, tasks, n,
                       tmap, layers, k, scratch);
  else if (bn == 32)
    hipLaunchKernelGGL((k_fwd_gemm<T, 32>), grid, dim3(256), 0, st, fr, ids, tasks, n,
                       tmap, layers, k, scratch);
  else
    hipLaunchKernelGGL((k_fwd_gemm<T, 64>), grid, dim3(256), 0, st, fr, ids, tasks, n,
                       tmap, layers, k, scratch);
}
template <typename T>
void launch_fwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int2* tmap, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_fwd_reduce<T>, dim3(total), dim3(256), 0, st, fr, ids, tasks, n,
                     tmap, layers, k, scratch);
}
template <typename T>
void launch_bwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bm, int bn, hipStream_t st) {
  if (total_tiles <= 0) return;
  // a 32 x 16 tile has fewer MFMA blocks than waves: use 32 columns there
  if (bm == 32 && bn == 16) bn = 32;
  const int ntn = (k + bn - 1) / bn;
  const dim3 grid(total_tiles * ntn);
#define HELM_BWD(BM_, BN_)                                                              \
  hipLaunchKernelGGL((k_bwd_gemm<T, BM_, BN_>), grid, dim3(256), 0, st, fr, ids, tasks, \
                     n, tmap, layers, k, scratch)
  if (bm == 32) {
    if (bn == 32) HELM_BWD(32, 32); else HELM_BWD(32, 64);
  } else {
    if (bn == 16) HELM_BWD(64, 16); else if (bn == 32) HELM_BWD(64, 32); else HELM_BWD(64, 64);
  }
#undef HELM_BWD
}
template <typename T>
void launch_bwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int2* tmap, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_bwd_reduce<T>, dim3(total), dim3(256), 0, st, fr, ids, tasks, n,
                     tmap, layers, k, scratch);
}

#define HELM_INST_SOLVE(T)                                                           \
  template void launch_fwd_gather<T>(const FrontDev*, const int*, int, const int2*,   \
                                     int, const LayerDev*, int, hipStream_t);        \
  template void launch_fwd_gemm<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, int, hipStream_t);                         \
  template void launch_fwd_reduce<T>(const FrontDev*, const int*, const SolveTask*,  \
                                     int, const int2*, int, const LayerDev*, int,     \
                                     const void*, hipStream_t);                      \
  template void launch_bwd_gemm<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, int, int, hipStream_t);                    \
  template void launch_bwd_reduce<T>(const FrontDev*, const int*, const SolveTask*,  \
                                     int, const int2*, int, const LayerDev*, int,     \
                                     const void*, hipStream_t);
HELM_INST_SOLVE(float)
HELM_INST_SOLVE(double)

#define HELM_INST_GEMV(T)                                                            \
  template void launch_fwd_gemv<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, hipStream_t);                              \
  template void launch_bwd_gemv<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, int, hipStream_t);
HELM_INST_GEMV(float)
HELM_INST_GEMV(double)


}  // namespace kern
}  // namespace helm
