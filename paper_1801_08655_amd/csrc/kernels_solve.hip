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
#include <hip/hip_ext.h>

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
  // raw: the list entry of the front (flags kSkipChild0/1 drop a child)
  __device__ ChildSum(const FrontDev* fronts, const FrontDev& f, const LayerDev& L, int raw) {
    Uc = reinterpret_cast<const C_t<T>*>(L.Ub[f.ub_parity ^ 1]);
    for (int slot = 0; slot < 2; ++slot) {
      cub[slot] = 0;
      inv[slot] = nullptr;
      if (f.child[slot] >= 0 && !(raw & (kSkipChild0 << slot))) {
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
        const int q = ld(inv[slot] + row);
        if (q >= 0) v = cadd(v, ld(Uc + (cub[slot] + q) * k + col));
      }
    return v;
  }
};

// forward, step 1 (fronts with children): X(S) += children's updates on the
// pivot rows, in place.  The boundary rows are summed in the GEMM epilogue.
template <typename T, int NT>
__global__ void __launch_bounds__(NT)
k_fwd_gather(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, int k) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
  const LayerDev& L = layers[f.layer];
  const int r0 = tm.y * RT;
  C* X = reinterpret_cast<C*>(L.X);
  const ChildSum<T> cs(fronts, f, L, raw);
  const int rows = (f.s - r0) < RT ? (f.s - r0) : RT;
  const int total = rows * k;
  // EPT elements (row, column) per thread and pass: child rows first, then
  // every value, then the stores (one latency per group of loads, not one
  // per element)
  constexpr int EPT = 4;
  for (int e0 = 0; e0 < total; e0 += NT * EPT) {
    int q[2][EPT], rr[EPT], cc[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = e0 + (int)threadIdx.x + j * NT;
      const bool ok = e < total;
      rr[j] = ok ? r0 + e / k : -1;
      cc[j] = ok ? e % k : 0;
#pragma unroll
      for (int sl = 0; sl < 2; ++sl)
        q[sl][j] = (ok && cs.inv[sl]) ? ld(cs.inv[sl] + rr[j]) : -1;
    }
    C v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      C u[2];
#pragma unroll
      for (int sl = 0; sl < 2; ++sl)
        u[sl] = ld_or_zero(q[sl][j] >= 0, cs.Uc + (cs.cub[sl] + q[sl][j]) * k + cc[j]);
      const C x = ld_or_zero(rr[j] >= 0, X + (long long)(f.off + rr[j]) * k + cc[j]);
      v[j] = cadd(x, cadd(cadd(czero<C>(), u[0]), u[1]));
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j)
      if (rr[j] >= 0) st(X + (long long)(f.off + rr[j]) * k + cc[j], v[j]);
  }
}

// Occupancy floor (waves per SIMD) asked of the compiler for the
// substitution GEMM tiles: 4 for the complex64 tiles, which then fit in 128
// registers without spilling (at its default the compiler spends up to
// ~160 on hoisting LDS reads and drops to 3 waves, which measured slower);
// 3 for the three-product 64 x 64 tile (2 at the compiler's default); no
// floor for the four-product 64 x 64 and the complex128 tiles, which would
// spill.
template <typename T, int BM, int BN, bool M3> constexpr int gemm_waves() {
  if (sizeof(T) != 4) return 1;
  if (BM == 64 && BN == 64) return M3 ? 3 : 1;
  return 4;
}

// Forward GEMM epilogue of an unsplit front: pivot rows to Z, boundary rows
// to the update buffer with the children's updates added.  The child rows of
// all of this lane's outputs are loaded first, then the child values, then
// the results are stored, so that the latencies of each group of loads
// overlap instead of following one another output by output.
template <typename T, int BM, int BN, bool M3>
__device__ __forceinline__ void fwd_epilogue(const WaveAcc<T, BM, BN, M3>& acc, const FrontDev& f,
                                             const ChildSum<T>& cs, C_t<T>* Z, C_t<T>* Uo,
                                             int m0, int n0, int k) {
  using C = C_t<T>;
  using O = LaneOut<T, BM, BN>;
  const O o;
  const int n = f.s + f.b;
  int q[2][O::NR];
#pragma unroll
  for (int i = 0; i < O::NR; ++i) {
    const int gm = m0 + o.r[i];
    const bool bnd = gm >= f.s && gm < n;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) q[sl][i] = (bnd && cs.inv[sl]) ? ld(cs.inv[sl] + gm) : -1;
  }
  C add[O::NR][O::NC];
#pragma unroll
  for (int i = 0; i < O::NR; ++i)
#pragma unroll
    for (int j = 0; j < O::NC; ++j) add[i][j] = czero<C>();
  if (cs.inv[0] || cs.inv[1]) {   // uniform: leaves have no children
#pragma unroll
    for (int i = 0; i < O::NR; ++i)
#pragma unroll
      for (int j = 0; j < O::NC; ++j) {
        const int gc = n0 + o.c[j];
        C u[2];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
          u[sl] = ld_or_zero(q[sl][i] >= 0 && gc < k, cs.Uc + (cs.cub[sl] + q[sl][i]) * k + gc);
        add[i][j] = cadd(cadd(add[i][j], u[0]), u[1]);
      }
  }
#pragma unroll
  for (int i = 0; i < O::NR; ++i)
#pragma unroll
    for (int j = 0; j < O::NC; ++j) {
      const int gm = m0 + o.r[i], gc = n0 + o.c[j];
      if (gm >= n || gc >= k) continue;
      const C z = acc_at(acc, i, j);
      if (gm < f.s) st(Z + (long long)(f.off + gm) * k + gc, z);
      else st(Uo + (f.ub + gm - f.s) * k + gc, cadd(z, add[i][j]));
    }
}

// forward, step 2: [X(S); Ub] = [F11^-1 w_S; Ub - F21 F11^-1 w_S], the K
// (pivot) dimension optionally split into chunks (partials to scratch).
// M3: the three-product complex form (complex64 only).
template <typename T, int BN, bool M3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves<T, FWD_BM, BN, M3>(), 8)))
k_fwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  constexpr int BM = FWD_BM;
  __shared__ GemmSmem<T, BM, BN, true, M3> sm;
  const int ntn = (k + BN - 1) / BN;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
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
  WaveAcc<T, BM, BN, M3> acc;
  gemm_tile<T, BM, true, true>(sm, acc, pv, qv, m0, n0, kb, ke);
  if (tk.nch_f > 1) {
    C* S = reinterpret_cast<C*>(scratch);
    for_each_acc<T, BM>(acc, [&](int r, int c, C z) {
      const int gm = m0 + r, gc = n0 + c;
      if (gm < n && gc < k) st(S + (tk.scr_f + (long long)chunk * n + gm) * k + gc, z);
    });
    return;
  }
  fwd_epilogue<T, BM, BN>(acc, f, ChildSum<T>(fronts, f, L, raw), reinterpret_cast<C*>(L.Wt),
                          ub_ptr<T>(L, f.ub_parity), m0, n0, k);
}

// elements per thread and pass of the split-K reductions
constexpr int RED_EPT = 4;

// forward, step 3 (split fronts only): sum the chunk partials in order
template <typename T, int NT>
__global__ void __launch_bounds__(NT)
k_fwd_reduce(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, int k, const void* scratch) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int r0 = tm.y * RT;
  const int rows = min(RT, n - r0);
  const C* S = reinterpret_cast<const C*>(scratch);
  C* Z = reinterpret_cast<C*>(L.Wt);
  C* Uo = ub_ptr<T>(L, f.ub_parity);
  const ChildSum<T> cs(fronts, f, L, raw);
  // RED_EPT elements per thread at a time: all their loads, then the stores
  for (int e0 = 0; e0 < rows * k; e0 += NT * RED_EPT) {
    C z[RED_EPT];
#pragma unroll
    for (int j = 0; j < RED_EPT; ++j) {
      const int e = e0 + (int)threadIdx.x + j * NT;
      z[j] = czero<C>();
      if (e >= rows * k) continue;
      const int gm = r0 + e / k, gc = e % k;
      for (int ch = 0; ch < tk.nch_f; ++ch)
        z[j] = cadd(z[j], ld(S + (tk.scr_f + (long long)ch * n + gm) * k + gc));
      if (gm >= f.s) z[j] = cadd(z[j], cs(gm, gc, k));
    }
#pragma unroll
    for (int j = 0; j < RED_EPT; ++j) {
      const int e = e0 + (int)threadIdx.x + j * NT;
      if (e >= rows * k) continue;
      const int gm = r0 + e / k, gc = e % k;
      if (gm < f.s) st(Z + (long long)(f.off + gm) * k + gc, z[j]);
      else st(Uo + (f.ub + gm - f.s) * k + gc, z[j]);
    }
  }
}

// backward: X(S) = Z(S) + (-F21 F11^-1)^T X(B); X(B) is read in place
// through the front's boundary index list, the K (boundary) dimension
// optionally split.  Fronts without boundary (roots) just copy Z(S).
template <typename T, int BM, int BN, bool M3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves<T, BM, BN, M3>(), 8)))
k_bwd_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  __shared__ GemmSmem<T, BM, BN, false, M3> sm;
  const int ntn = (k + BN - 1) / BN;
  const int mt = blockIdx.x / ntn, nt = blockIdx.x % ntn;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
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
  WaveAcc<T, BM, BN, M3> acc;
  gemm_tile<T, BM, false, true>(sm, acc, pv, qv, m0, n0, kb, ke);
  if (tk.nch_b > 1) {
    C* S = reinterpret_cast<C*>(scratch);
    for_each_acc<T, BM>(acc, [&](int r, int c, C z) {
      const int gm = m0 + r, gc = n0 + c;
      if (gm < f.s && gc < k) st(S + (tk.scr_b + (long long)chunk * f.s + gm) * k + gc, z);
    });
    return;
  }
  // X(S) = Z(S) + product: every Z value of the lane is loaded before the
  // first store (X and Z are distinct buffers, but the compiler cannot tell)
  using O = LaneOut<T, BM, BN>;
  const O o;
  const C* Z = reinterpret_cast<const C*>(L.Wt);
  C zv[O::NR][O::NC];
#pragma unroll
  for (int i = 0; i < O::NR; ++i)
#pragma unroll
    for (int j = 0; j < O::NC; ++j) {
      const int gm = m0 + o.r[i], gc = n0 + o.c[j];
      zv[i][j] = ld_or_zero(gm < f.s && gc < k && !(raw & kZeroZ),
                            Z + (long long)(f.off + gm) * k + gc);
    }
#pragma unroll
  for (int i = 0; i < O::NR; ++i)
#pragma unroll
    for (int j = 0; j < O::NC; ++j) {
      const int gm = m0 + o.r[i], gc = n0 + o.c[j];
      if (gm < f.s && gc < k)
        st(X + (long long)(f.off + gm) * k + gc, cadd(zv[i][j], acc_at(acc, i, j)));
    }
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT)
k_bwd_reduce(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, int k, const void* scratch) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int r0 = tm.y * RT;
  const int rows = min(RT, f.s - r0);
  const C* S = reinterpret_cast<const C*>(scratch);
  C* X = reinterpret_cast<C*>(L.X);
  const C* Z = reinterpret_cast<const C*>(L.Wt);
  for (int e0 = 0; e0 < rows * k; e0 += NT * RED_EPT) {
    C z[RED_EPT];
#pragma unroll
    for (int j = 0; j < RED_EPT; ++j) {
      const int e = e0 + (int)threadIdx.x + j * NT;
      z[j] = czero<C>();
      if (e >= rows * k) continue;
      const int gm = r0 + e / k, gc = e % k;
      z[j] = ld_or_zero(!(raw & kZeroZ), Z + (long long)(f.off + gm) * k + gc);
      for (int ch = 0; ch < tk.nch_b; ++ch)
        z[j] = cadd(z[j], ld(S + (tk.scr_b + (long long)ch * f.s + gm) * k + gc));
    }
#pragma unroll
    for (int j = 0; j < RED_EPT; ++j) {
      const int e = e0 + (int)threadIdx.x + j * NT;
      if (e >= rows * k) continue;
      const int gm = r0 + e / k, gc = e % k;
      st(X + (long long)(f.off + gm) * k + gc, z[j]);
    }
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
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
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
      const C fa = ld(FT + m + (long long)q * n);
      const C* xq = X + (long long)q * KC;
#pragma unroll
      for (int c = 0; c < KC; ++c) cfma(acc[c], fa, ld(xq + c));
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
  const ChildSum<T> cs(fronts, f, L, raw);
  C add[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) add[c] = czero<C>();
  if (tk.nch_f == 1 && m >= f.s) {
    // the row's children's updates, loaded before any store
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int q = cs.inv[sl] ? ld(cs.inv[sl] + m) : -1;
      if (q >= 0) {
#pragma unroll
        for (int c = 0; c < KC; ++c) add[c] = cadd(add[c], ld(cs.Uc + (cs.cub[sl] + q) * KC + c));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const C z = cadd(cadd(acc[c], red[0][lane][c]), cadd(red[1][lane][c], red[2][lane][c]));
    if (tk.nch_f > 1) st(S + (tk.scr_f + (long long)chunk * n + m) * KC + c, z);
    else if (m < f.s) st(Z + (long long)(f.off + m) * KC + c, z);
    else st(Uo + (f.ub + m - f.s) * KC + c, cadd(z, add[c]));
  }
}

template <typename T> __device__ __forceinline__ T shfl_xor_t(T v, int mask) {
  return __shfl_xor(v, mask, 64);
}

// backward: one BM-row tile (BM = 32 or 64) and one K chunk per block; the
// 256 threads form 256 / GW groups of GW lanes and group g takes the rows
// m0 + g, m0 + g + 256 / GW, ... (RPG of them) together: its lanes walk the
// boundary index q (contiguous in the stored block), load X(B[q]) once for
// all those rows and the factor entry of every row, so that several
// independent factor loads are in flight per lane; a butterfly over the
// group sums each row.
template <typename T, int KC, int RPG, int GW = 16>
__global__ void __launch_bounds__(256)
k_bwd_gemv(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           const SolveTask* __restrict__ tasks, int n_ids, const int2* __restrict__ tmap,
           const LayerDev* __restrict__ layers, int k, void* scratch) {
  using C = C_t<T>;
  constexpr int NG = 256 / GW;
  constexpr int bm = NG * RPG;   // row tile
  const int mt = blockIdx.x;
  const int2 tm = tmap[mt];
  const int a = tm.x;
  const int raw = ids[a];
  const FrontDev f = fronts[raw & kFrontIdMask];
  const SolveTask tk = tasks[a];
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  const int local = tm.y;
  const int chunk = local % tk.nch_b;
  const int m0 = (local / tk.nch_b) * bm;
  const int kb = chunk * tk.kc_b;
  const int ke = min(f.b, kb + tk.kc_b);
  const int g = threadIdx.x / GW, gl = threadIdx.x % GW;
  const C* FT = reinterpret_cast<const C*>(L.fac) + f.fac;
  C* X = reinterpret_cast<C*>(L.X);
  const C* Z = reinterpret_cast<const C*>(L.Wt);
  C* S = reinterpret_cast<C*>(scratch);
  const int* B = L.bidx + f.bidx;
  bool row_ok[RPG];
  const C* col[RPG];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int m = m0 + g + NG * r;
    row_ok[r] = m < f.s;
    col[r] = FT + f.s + (long long)(row_ok[r] ? m : 0) * n;
  }
  C acc[RPG][KC];
#pragma unroll
  for (int r = 0; r < RPG; ++r)
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[r][c] = czero<C>();
#pragma unroll 2
  for (int q = kb + gl; q < ke; q += GW) {
    const C* xb = X + (long long)ld(B + q) * KC;
    C fa[RPG], xv[KC];
#pragma unroll
    for (int r = 0; r < RPG; ++r) fa[r] = ld_or_zero(row_ok[r], col[r] + q);
#pragma unroll
    for (int c = 0; c < KC; ++c) xv[c] = ld(xb + c);
#pragma unroll
    for (int r = 0; r < RPG; ++r)
#pragma unroll
      for (int c = 0; c < KC; ++c) cfma(acc[r][c], fa[r], xv[c]);
  }
  // reduce-scatter over the group: each halving step trades half of the
  // lane's row sums with the partner lane (offset GW/2, GW/4, ...), so
  // that after log2(RPG) steps the lane holds one row's partial sum (the
  // row given by its high bits); a butterfly over the GW/RPG lanes that
  // share the row completes it (RPG = 8: 18 exchanges per column instead
  // of 80 for a butterfly per row)
  static_assert((RPG & (RPG - 1)) == 0 && RPG <= GW && KC <= GW / RPG, "group shape");
  int rsel = 0;
#pragma unroll
  for (int h = RPG / 2, off = GW / 2; h >= 1; h >>= 1, off >>= 1) {
    const bool up = (gl & off) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i)
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const C send = up ? acc[i][c] : acc[i + h][c];
        const C keep = up ? acc[i + h][c] : acc[i][c];
        acc[i][c].x = keep.x + shfl_xor_t(send.x, off);
        acc[i][c].y = keep.y + shfl_xor_t(send.y, off);
      }
    if (up) rsel += h;
  }
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int off = GW / (2 * RPG); off > 0; off >>= 1) {
      acc[0][c].x += shfl_xor_t(acc[0][c].x, off);
      acc[0][c].y += shfl_xor_t(acc[0][c].y, off);
    }
  const int lo = gl & (GW / RPG - 1);
  const int m = m0 + g + NG * rsel;
  if (m < f.s && lo < KC) {
    C z = acc[0][0];
#pragma unroll
    for (int c = 1; c < KC; ++c)
      if (lo == c) z = acc[0][c];
    const long long idx = (long long)(f.off + m) * KC + lo;
    if (tk.nch_b > 1) st(S + (tk.scr_b + (long long)chunk * f.s + m) * KC + lo, z);
    else st(X + idx, cadd(ld_or_zero(!(raw & kZeroZ), Z + idx), z));
  }
}

}  // namespace

template <typename T>
void launch_fwd_gemv(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (total_tiles <= 0) return;
#define HELM_FWDV(KC_)                                                                      \
  if (t0)                                                                                   \
    hipExtLaunchKernelGGL((k_fwd_gemv<T, KC_>), dim3(total_tiles), dim3(256), 0, st, t0, t1, \
                          0, fr, ids, tasks, n, tmap, layers, k, scratch);                  \
  else                                                                                      \
    hipLaunchKernelGGL((k_fwd_gemv<T, KC_>), dim3(total_tiles), dim3(256), 0, st, fr, ids,  \
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
                     void* scratch, int bm, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (total_tiles <= 0) return;
#define HELM_BWDV1(RPG_, KC_)                                                              \
  if (t0)                                                                                  \
    hipExtLaunchKernelGGL((k_bwd_gemv<T, KC_, RPG_, 32>), dim3(total_tiles), dim3(256), 0, \
                          st, t0, t1, 0, fr, ids, tasks, n, tmap, layers, k, scratch);     \
  else                                                                                     \
    hipLaunchKernelGGL((k_bwd_gemv<T, KC_, RPG_, 32>), dim3(total_tiles), dim3(256), 0,    \
                       st, fr, ids, tasks, n, tmap, layers, k, scratch)
#define HELM_BWDV(KC_)                                                                     \
  if (bm == 32) {                                                                          \
    HELM_BWDV1(4, KC_);                                                                    \
  } else {                                                                                 \
    HELM_BWDV1(8, KC_);                                                                    \
  }
  switch (k) {
    case 1: HELM_BWDV(1); break;
    case 2: HELM_BWDV(2); break;
    case 3: HELM_BWDV(3); break;
    default: HELM_BWDV(4); break;
  }
#undef HELM_BWDV
#undef HELM_BWDV1
}

template <typename T>
void launch_fwd_gather(const FrontDev* fr, const int* ids, int n, const int2* tmap,
                       int total, const LayerDev* layers, int k, hipStream_t st) {
  if (total <= 0) return;
  // a tile is RT rows x k columns: one wave per tile for few columns
  if (k <= 4)
    hipLaunchKernelGGL((k_fwd_gather<T, 64>), dim3(total), dim3(64), 0, st, fr, ids, n,
                       tmap, layers, k);
  else
    hipLaunchKernelGGL((k_fwd_gather<T, 256>), dim3(total), dim3(256), 0, st, fr, ids, n,
                       tmap, layers, k);
}
template <typename T>
void launch_fwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bn, bool m3, hipStream_t st, hipEvent_t t0,
                     hipEvent_t t1) {
  if (total_tiles <= 0) return;
  const int ntn = (k + bn - 1) / bn;
  const dim3 grid(total_tiles * ntn);
#define HELM_FWD(BN_, M3_)                                                                  \
  if (t0)                                                                                   \
    hipExtLaunchKernelGGL((k_fwd_gemm<T, BN_, M3_>), grid, dim3(256), 0, st, t0, t1, 0, fr, \
                          ids, tasks, n, tmap, layers, k, scratch);                         \
  else                                                                                      \
    hipLaunchKernelGGL((k_fwd_gemm<T, BN_, M3_>), grid, dim3(256), 0, st, fr, ids, tasks,   \
                       n, tmap, layers, k, scratch)
  constexpr bool C64 = sizeof(T) == 4;   // the three-product form is for complex64
  if (C64 && m3) {
    if (bn == 16) HELM_FWD(16, C64); else if (bn == 32) HELM_FWD(32, C64); else HELM_FWD(64, C64);
  } else {
    if (bn == 16) HELM_FWD(16, false); else if (bn == 32) HELM_FWD(32, false); else HELM_FWD(64, false);
  }
#undef HELM_FWD
}
template <typename T>
void launch_fwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int2* tmap, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st) {
  if (total <= 0) return;
  if (k <= 4)
    hipLaunchKernelGGL((k_fwd_reduce<T, 64>), dim3(total), dim3(64), 0, st, fr, ids, tasks,
                       n, tmap, layers, k, scratch);
  else
    hipLaunchKernelGGL((k_fwd_reduce<T, 256>), dim3(total), dim3(256), 0, st, fr, ids, tasks,
                       n, tmap, layers, k, scratch);
}
template <typename T>
void launch_bwd_gemm(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                     const int2* tmap, int total_tiles, const LayerDev* layers, int k,
                     void* scratch, int bm, int bn, bool m3, hipStream_t st, hipEvent_t t0,
                     hipEvent_t t1) {
  if (total_tiles <= 0) return;
  // a 32 x 16 tile has fewer MFMA blocks than waves: use 32 columns there
  if (bm == 32 && bn == 16) bn = 32;
  const int ntn = (k + bn - 1) / bn;
  const dim3 grid(total_tiles * ntn);
#define HELM_BWD(BM_, BN_, M3_)                                                              \
  if (t0)                                                                                    \
    hipExtLaunchKernelGGL((k_bwd_gemm<T, BM_, BN_, M3_>), grid, dim3(256), 0, st, t0, t1, 0, \
                          fr, ids, tasks, n, tmap, layers, k, scratch);                      \
  else                                                                                       \
    hipLaunchKernelGGL((k_bwd_gemm<T, BM_, BN_, M3_>), grid, dim3(256), 0, st, fr, ids,      \
                       tasks, n, tmap, layers, k, scratch)
#define HELM_BWD_ALL(M3_)                                                                   \
  if (bm == 32) {                                                                           \
    if (bn == 32) { HELM_BWD(32, 32, M3_); } else { HELM_BWD(32, 64, M3_); }                \
  } else {                                                                                  \
    if (bn == 16) { HELM_BWD(64, 16, M3_); }                                                \
    else if (bn == 32) { HELM_BWD(64, 32, M3_); }                                           \
    else { HELM_BWD(64, 64, M3_); }                                                         \
  }
  constexpr bool C64 = sizeof(T) == 4;   // the three-product form is for complex64
  if (C64 && m3) {
    HELM_BWD_ALL(C64)
  } else {
    HELM_BWD_ALL(false)
  }
#undef HELM_BWD_ALL
#undef HELM_BWD
}
template <typename T>
void launch_bwd_reduce(const FrontDev* fr, const int* ids, const SolveTask* tasks, int n,
                       const int2* tmap, int total, const LayerDev* layers, int k,
                       const void* scratch, hipStream_t st) {
  if (total <= 0) return;
  if (k <= 4)
    hipLaunchKernelGGL((k_bwd_reduce<T, 64>), dim3(total), dim3(64), 0, st, fr, ids, tasks,
                       n, tmap, layers, k, scratch);
  else
    hipLaunchKernelGGL((k_bwd_reduce<T, 256>), dim3(total), dim3(256), 0, st, fr, ids, tasks,
                       n, tmap, layers, k, scratch);
}

#define HELM_INST_SOLVE(T)                                                           \
  template void launch_fwd_gather<T>(const FrontDev*, const int*, int, const int2*,   \
                                     int, const LayerDev*, int, hipStream_t);        \
  template void launch_fwd_gemm<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, int, bool, hipStream_t, hipEvent_t,         \
                                   hipEvent_t);                                      \
  template void launch_fwd_reduce<T>(const FrontDev*, const int*, const SolveTask*,  \
                                     int, const int2*, int, const LayerDev*, int,     \
                                     const void*, hipStream_t);                      \
  template void launch_bwd_gemm<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, int, int, bool, hipStream_t, hipEvent_t,    \
                                   hipEvent_t);                                      \
  template void launch_bwd_reduce<T>(const FrontDev*, const int*, const SolveTask*,  \
                                     int, const int2*, int, const LayerDev*, int,     \
                                     const void*, hipStream_t);
HELM_INST_SOLVE(float)
HELM_INST_SOLVE(double)

#define HELM_INST_GEMV(T)                                                            \
  template void launch_fwd_gemv<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, hipStream_t, hipEvent_t, hipEvent_t);      \
  template void launch_bwd_gemv<T>(const FrontDev*, const int*, const SolveTask*,    \
                                   int, const int2*, int, const LayerDev*, int,       \
                                   void*, int, hipStream_t, hipEvent_t, hipEvent_t);
HELM_INST_GEMV(float)
HELM_INST_GEMV(double)


}  // namespace kern
}  // namespace helm
