// Device helpers shared by the HIP kernels: complex arithmetic, tile lookup
// and the 64x64 complex GEMM tile on CDNA matrix cores (MFMA).
#pragma once

#include <hip/hip_runtime.h>

#include "helm_internal.h"

namespace helm {
namespace kern {

template <typename T> using C_t = typename Cplx<T>::type;

template <typename C> __device__ __forceinline__ C cmake(double re, double im) {
  C z;
  z.x = re;
  z.y = im;
  return z;
}
template <typename C> __device__ __forceinline__ C czero() { return cmake<C>(0, 0); }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) {
  C z; z.x = a.x + b.x; z.y = a.y + b.y; return z;
}
template <typename C> __device__ __forceinline__ C csub(C a, C b) {
  C z; z.x = a.x - b.x; z.y = a.y - b.y; return z;
}
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C z;
  z.x = a.x * b.x - a.y * b.y;
  z.y = a.x * b.y + a.y * b.x;
  return z;
}
template <typename C> __device__ __forceinline__ C cneg(C a) {
  C z; z.x = -a.x; z.y = -a.y; return z;
}
// a += b * c
template <typename C> __device__ __forceinline__ void cfma(C& a, C b, C c) {
  a.x += b.x * c.x - b.y * c.y;
  a.y += b.x * c.y + b.y * c.x;
}
// a -= b * c
template <typename C> __device__ __forceinline__ void cfms(C& a, C b, C c) {
  a.x -= b.x * c.x - b.y * c.y;
  a.y -= b.x * c.y + b.y * c.x;
}
// a / b with scaling against overflow (Smith's method)
template <typename C> __device__ __forceinline__ C cdiv(C a, C b) {
  C z;
  if (fabs((double)b.x) >= fabs((double)b.y)) {
    auto r = b.y / b.x;
    auto d = b.x + b.y * r;
    z.x = (a.x + a.y * r) / d;
    z.y = (a.y - a.x * r) / d;
  } else {
    auto r = b.x / b.y;
    auto d = b.x * r + b.y;
    z.x = (a.x * r + a.y) / d;
    z.y = (a.y * r - a.x) / d;
  }
  return z;
}
template <typename C> __device__ __forceinline__ double cabs2(C a) {
  return (double)a.x * a.x + (double)a.y * a.y;
}

__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
template <typename C> __device__ __forceinline__ C from_d2(double2 a);
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }

// largest i in [0, n) with prefix[i] <= x  (prefix has n + 1 entries, prefix[0] = 0)
__device__ __forceinline__ int find_segment(const int* __restrict__ prefix, int n, int x) {
  int lo = 0, hi = n;  // invariant prefix[lo] <= x < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// MFMA 16x16x4 (one block).  Lane l supplies A[l%16][l/16] and B[l/16][l%16];
// element v of the result vector holds D[row(l, v)][l%16] with
// row = 4*(l/16) + v for the f32 instruction and 4*v + l/16 for the f64 one
// (both checked on the device).
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

constexpr int GT = 64;   // tile edge (complex elements)
constexpr int GK = 16;   // K step (complex elements)

// Shared-memory staging for one 64x64 complex GEMM tile.
//   P[r][k]: operand whose rows become the MFMA rows,
//   Q[k][c]: operand whose columns become the MFMA columns.
template <typename T> struct GemmSmem {
  C_t<T> P[GT][GK + 1];
  C_t<T> Q[GK][GT + 1];
};

// Operand view: element (r, k) at base[r * sr + kk * sk], valid for r < nr,
// k < nk, with kk = k, or kk = kmap[k] when a row map is given (indirect
// rows, e.g. the boundary variables of a front).
template <typename T> struct View {
  const C_t<T>* base;
  long long sr, sk;
  int nr, nk;
  const int* kmap = nullptr;
};

template <typename T>
__device__ __forceinline__ C_t<T> view_at(const View<T>& v, int r, int k) {
  C_t<T> val = czero<C_t<T>>();
  if (r < v.nr && k < v.nk) {
    const long long kk = v.kmap ? (long long)v.kmap[k] : (long long)k;
    val = v.base[(long long)r * v.sr + kk * v.sk];
  }
  return val;
}

constexpr int GLOADS = (GT * GK) / 256;   // elements per thread per operand tile

// Per-thread staging registers for one K step of both operands.
template <typename T> struct Stage {
  C_t<T> p[GLOADS], q[GLOADS];
};

// Global loads of the 64 x GK block of P (rows r0.., k0..) and the GK x 64
// block of Q (columns c0.., k0..).  FAST_R / FAST_C: consecutive threads walk
// the rows of P / the columns of Q (the contiguous dimension in memory).
template <typename T, bool FAST_R, bool FAST_C>
__device__ __forceinline__ void stage_load(Stage<T>& g, const View<T>& pv, const View<T>& qv,
                                           int r0, int c0, int k0, int kend) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < GLOADS; ++it) {
    const int e = t + it * 256;
    int r, k;
    if (FAST_R) { r = e % GT; k = e / GT; } else { k = e % GK; r = e / GK; }
    g.p[it] = (k0 + k < kend) ? view_at(pv, r0 + r, k0 + k) : czero<C_t<T>>();
    int c, kq;
    if (FAST_C) { c = e % GT; kq = e / GT; } else { kq = e % GK; c = e / GK; }
    g.q[it] = (k0 + kq < kend) ? view_at(qv, c0 + c, k0 + kq) : czero<C_t<T>>();
  }
}

template <typename T, bool FAST_R, bool FAST_C>
__device__ __forceinline__ void stage_store(GemmSmem<T>& sm, const Stage<T>& g) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < GLOADS; ++it) {
    const int e = t + it * 256;
    int r, k;
    if (FAST_R) { r = e % GT; k = e / GT; } else { k = e % GK; r = e / GK; }
    sm.P[r][k] = g.p[it];
    int c, kq;
    if (FAST_C) { c = e % GT; kq = e / GT; } else { kq = e % GK; c = e / GK; }
    sm.Q[kq][c] = g.q[it];
  }
}

// Accumulators of one wave: a 32x32 complex sub-tile as 2x2 MFMA blocks.
template <typename T> struct WaveAcc {
  typename Mfma<T>::v4 re[2][2], im[2][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) { re[a][b][v] = 0; im[a][b][v] = 0; }
  }
};

// One GK step of MFMAs for this wave.  Real form of the complex product:
// rows of P are read as [re, im, re, im] along k and columns of Q as
// [re, -im, ...] (real part) and [im, re, ...] (imaginary part).
template <typename T>
__device__ __forceinline__ void mfma_step_q(const GemmSmem<T>& sm, const C_t<T> (*Q)[GT + 1],
                                            WaveAcc<T>& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int p = 0; p < GK / 2; ++p) {
    const int kc = 2 * p + (lq >> 1);
    const bool imag_part = lq & 1;
    T a[2];
#pragma unroll
    for (int bm = 0; bm < 2; ++bm) {
      C_t<T> x = sm.P[wr * 32 + bm * 16 + li][kc];
      a[bm] = imag_part ? x.y : x.x;
    }
    T bre[2], bim[2];
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
      C_t<T> y = Q[kc][wc * 32 + bn * 16 + li];
      bre[bn] = imag_part ? -y.y : y.x;
      bim[bn] = imag_part ? y.x : y.y;
    }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) {
        acc.re[bm][bn] = Mfma<T>::op(a[bm], bre[bn], acc.re[bm][bn]);
        acc.im[bm][bn] = Mfma<T>::op(a[bm], bim[bn], acc.im[bm][bn]);
      }
  }
}

template <typename T>
__device__ __forceinline__ void mfma_step(const GemmSmem<T>& sm, WaveAcc<T>& acc,
                                          int wr, int wc, int lane) {
  mfma_step_q<T>(sm, sm.Q, acc, wr, wc, lane);
}

// K loop of a 64x64 tile over k in [kbeg, kend): rows of P from `pv`
// starting at r0, columns of Q from `qv` starting at c0.  The global loads
// of the next K step are issued before the matrix-core work of the current
// one, so their latency overlaps the MFMAs.
template <typename T, bool P_FAST_R, bool Q_FAST_C>
__device__ __forceinline__ void gemm_tile(GemmSmem<T>& sm, WaveAcc<T>& acc,
                                          const View<T>& pv, const View<T>& qv,
                                          int r0, int c0, int kbeg, int kend) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  acc.zero();
  if (kbeg >= kend) return;
  Stage<T> g;
  stage_load<T, P_FAST_R, Q_FAST_C>(g, pv, qv, r0, c0, kbeg, kend);
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    stage_store<T, P_FAST_R, Q_FAST_C>(sm, g);
    __syncthreads();
    if (k0 + GK < kend) stage_load<T, P_FAST_R, Q_FAST_C>(g, pv, qv, r0, c0, k0 + GK, kend);
    mfma_step<T>(sm, acc, wr, wc, lane);
    __syncthreads();
  }
}

// Visit this lane's outputs: f(r, c, value) with r, c the tile-local MFMA
// row / column (0..63).
template <typename T, class F>
__device__ __forceinline__ void for_each_acc(const WaveAcc<T>& acc, F&& f) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = wr * 32 + bm * 16 + Mfma<T>::row(lane, v);
        int c = wc * 32 + bn * 16 + (lane & 15);
        C_t<T> z;
        z.x = acc.re[bm][bn][v];
        z.y = acc.im[bm][bn][v];
        f(r, c, z);
      }
}

}  // namespace kern
}  // namespace helm
