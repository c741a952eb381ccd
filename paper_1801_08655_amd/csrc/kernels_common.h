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

// Global-memory loads and stores through address-space-1 pointers.  A
// pointer read from a device structure is generic to the compiler, which
// then emits FLAT instructions; those also count against the LDS wait
// counter, so the LDS waits of an MFMA loop would wait for every global
// prefetch in flight.  Through these helpers the compiler emits
// global_load / global_store.  Only for pointers into device memory.
#define HELM_AS1 __attribute__((address_space(1)))
template <typename C> __device__ __forceinline__ C ld(const C* p) {
  typedef typename C::value_type E;
  typedef E V __attribute__((ext_vector_type(2)));
  const V v = *(const HELM_AS1 V*)p;
  C r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
__device__ __forceinline__ int ld(const int* p) { return *(const HELM_AS1 int*)p; }

// A complex zero in device memory (room for complex128), the load address
// of the masked-off lanes of ld_or_zero.
static __device__ __align__(16) double kZeroC[2] = {0.0, 0.0};

// *p when ok, else zero, as one unconditional load (no branch), so that a
// run of such loads is issued back to back and waited for once.
template <typename C> __device__ __forceinline__ C ld_or_zero(bool ok, const C* p) {
  return ld(ok ? p : reinterpret_cast<const C*>(kZeroC));
}
template <typename C> __device__ __forceinline__ void st(C* p, C v) {
  typedef typename C::value_type E;
  typedef E V __attribute__((ext_vector_type(2)));
  V w;
  w.x = v.x;
  w.y = v.y;
  *(HELM_AS1 V*)p = w;
}
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

// Launches over variable-size items (fronts, their tiles and chunks) index
// their blocks through a tile map built on the host: entry t holds the item
// of block t and the block's index within that item, so a block finds its
// work with one load.

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
constexpr int FWD_BM = 64;   // row tile of the forward substitution GEMM
constexpr int RT = 16;       // row tile of the gather / split-K reduction kernels

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
    const long long kk = v.kmap ? (long long)ld(v.kmap + k) : (long long)k;
    val = ld(v.base + (long long)r * v.sr + kk * v.sk);
  }
  return val;
}

// Shared-memory staging of one K step of a BM x BN complex GEMM tile in the
// real form of the complex product:
//   P[r][2k + {0,1}] = (re, im) of the row operand,
//   Q1[2k][c] = re, Q1[2k+1][c] = -im   (column operand, real part of C),
//   Q2[2k][c] = im, Q2[2k+1][c] = re    (imaginary part of C),
// so that every MFMA reads its operands with one load and no arithmetic.
// BN (columns of the tile: right-hand sides in the substitutions) is 64, 32
// or 16; narrow tiles keep the matrix cores busy on useful columns when a
// batch has fewer than 64 columns.
//
// LDS layout and bank conflicts.  An MFMA operand read has lane l at
// (row base + l % 16, k 4p + l / 16) of P and at (k 4p + l / 16, column
// base + l % 16) of Q.  P is stored in one of two layouts, chosen by the
// order in which the global loads deliver it:
//  - k-major, P[2k + {0,1}][r], when consecutive threads hold consecutive
//    rows (the stored factor columns of the forward GEMM): the staging
//    stores then hit consecutive banks;
//  - row-major, P[r][2k + {0,1}], when consecutive threads hold consecutive
//    k (the transposed block of the backward GEMM).
// A k-major row of W elements is padded to 48 (W <= 32) or 80 (W = 64)
// elements: the four k rows of one read then start 16, 32 and 48 banks
// apart (mod 64), so the 64 lanes touch 64 distinct banks.  The row-major
// stride 2 GK + 2 puts the 16 rows of a read on even banks, offset by k.
constexpr int PSTR = 2 * GK + 2;
template <int W> constexpr int kmajor_stride() {
  static_assert(W == 16 || W == 32 || W == 64, "k-major rows are padded for 16, 32 or 64");
  return W == 64 ? 80 : 48;
}
//
// The three-product form (M3, complex64 substitutions): the complex product
// is formed from the real products Pr Qr, Pi Qi and (Pr + Pi)(Qr + Qi)
// (re = t1 - t2, im = t3 - t1 - t2), so a complex multiply-add costs three
// real ones on the matrix cores instead of four.  Each operand is staged as
// three real planes of GK rows (k-major P and Q: plane * GK + k; row-major
// P: r, plane * GK + k with stride 3 GK + 4, which puts the 16 rows of a read
// on distinct multiples of 4 banks, offset by k).  Its rounding error is
// bounded in norm, not element by element: an imaginary part much smaller
// than |P||Q| carries a larger relative error than in the four-product form.
constexpr int PSTR3 = 3 * GK + 4;
template <typename T, int BM, int BN = GT, bool PKM = false, bool M3 = false> struct GemmSmem {
  static constexpr int NPL = M3 ? 3 : 2;   // real rows per complex k
  T P[PKM ? NPL * GK : BM][PKM ? kmajor_stride<BM>() : (M3 ? PSTR3 : PSTR)];
  T Q1[NPL * GK][kmajor_stride<BN>()];
  T Q2[M3 ? 1 : 2 * GK][kmajor_stride<BN>()];
};

// The 4 waves of a block tile it as WR x WC sub-tiles of RW x CW, each made
// of MB x NB MFMA 16x16 blocks.
template <int BM, int BN> struct WaveGrid {
  static constexpr int WC = BN >= 32 ? 2 : 1;
  static constexpr int WR = 4 / WC;
  static constexpr int RW = BM / WR, CW = BN / WC;
  static constexpr int MB = RW / 16, NB = CW / 16;
  static_assert(RW >= 16 && CW >= 16 && RW % 16 == 0 && CW % 16 == 0,
                "wave sub-tile must be whole MFMA blocks");
};

// Per-thread staging registers for one K step of both operands, and the
// resolved K indices of this thread's Q elements for the step after it.
template <typename T, int BM, int BN = GT> struct Stage {
  static constexpr int NP = BM * GK / 256, NQ = BN * GK / 256;
  C_t<T> p[NP], q[NQ];
  int qk[NQ];
};

// K indices of this thread's Q elements for the step at k0 (through the row
// map of an indirect view), -1 past the valid range.  They are loaded one K
// step ahead of the values they address, so that the value loads of a step
// never wait for an index load.
template <typename T, int BM, int BN, bool FAST_C>
__device__ __forceinline__ void stage_index(Stage<T, BM, BN>& g, const View<T>& qv, int k0,
                                            int kend) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < Stage<T, BM, BN>::NQ; ++it) {
    const int e = t + it * 256;
    const int kq = FAST_C ? e / BN : e % GK;
    const int k = k0 + kq;
    int kk = -1;
    if (k < kend && k < qv.nk) kk = qv.kmap ? ld(qv.kmap + k) : k;
    g.qk[it] = kk;
  }
}

// Global loads of the BM x GK block of P (rows r0.., k0..) and the GK x BN
// block of Q (columns c0.., K indices from stage_index).  FAST_R / FAST_C:
// consecutive threads walk the rows of P / the columns of Q (the contiguous
// dimension in memory).
template <typename T, int BM, int BN, bool FAST_R, bool FAST_C>
__device__ __forceinline__ void stage_load(Stage<T, BM, BN>& g, const View<T>& pv,
                                           const View<T>& qv, int r0, int c0, int k0,
                                           int kend) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < Stage<T, BM, BN>::NP; ++it) {
    const int e = t + it * 256;
    int r, k;
    if (FAST_R) { r = e % BM; k = e / BM; } else { k = e % GK; r = e / GK; }
    g.p[it] = (k0 + k < kend) ? view_at(pv, r0 + r, k0 + k) : czero<C_t<T>>();
  }
#pragma unroll
  for (int it = 0; it < Stage<T, BM, BN>::NQ; ++it) {
    const int e = t + it * 256;
    const int c = FAST_C ? e % BN : e / GK;
    const int kk = g.qk[it];
    C_t<T> val = czero<C_t<T>>();
    if (kk >= 0 && c0 + c < qv.nr)
      val = ld(qv.base + (long long)(c0 + c) * qv.sr + (long long)kk * qv.sk);
    g.q[it] = val;
  }
}

template <typename T, int BM, int BN, bool FAST_R, bool FAST_C, bool M3 = false>
__device__ __forceinline__ void stage_store(GemmSmem<T, BM, BN, FAST_R, M3>& sm,
                                            const Stage<T, BM, BN>& g) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < Stage<T, BM, BN>::NP; ++it) {
    const int e = t + it * 256;
    int r, k;
    if (FAST_R) { r = e % BM; k = e / BM; } else { k = e % GK; r = e / GK; }
    const C_t<T> x = g.p[it];
    if constexpr (M3) {
      if (FAST_R) {
        sm.P[k][r] = x.x;
        sm.P[GK + k][r] = x.y;
        sm.P[2 * GK + k][r] = x.x + x.y;
      } else {
        sm.P[r][k] = x.x;
        sm.P[r][GK + k] = x.y;
        sm.P[r][2 * GK + k] = x.x + x.y;
      }
    } else if (FAST_R) {
      sm.P[2 * k][r] = x.x;
      sm.P[2 * k + 1][r] = x.y;
    } else {
      sm.P[r][2 * k] = x.x;
      sm.P[r][2 * k + 1] = x.y;
    }
  }
#pragma unroll
  for (int it = 0; it < Stage<T, BM, BN>::NQ; ++it) {
    const int e = t + it * 256;
    int c, kq;
    if (FAST_C) { c = e % BN; kq = e / BN; } else { kq = e % GK; c = e / GK; }
    const C_t<T> y = g.q[it];
    if constexpr (M3) {
      sm.Q1[kq][c] = y.x;
      sm.Q1[GK + kq][c] = y.y;
      sm.Q1[2 * GK + kq][c] = y.x + y.y;
    } else {
      sm.Q1[2 * kq][c] = y.x;
      sm.Q1[2 * kq + 1][c] = -y.y;
      sm.Q2[2 * kq][c] = y.y;
      sm.Q2[2 * kq + 1][c] = y.x;
    }
  }
}

// Accumulators of one wave: its RW x CW complex sub-tile as MB x NB MFMA
// 16x16 blocks (real and imaginary parts).
// In the three-product form re, t and im accumulate Pr Qr, Pi Qi and
// (Pr + Pi)(Qr + Qi) until finish() turns them into the real and imaginary
// parts.
template <typename T, int BM, int BN = GT, bool M3 = false> struct WaveAcc {
  using G = WaveGrid<BM, BN>;
  typename Mfma<T>::v4 re[G::MB][G::NB], im[G::MB][G::NB];
  typename Mfma<T>::v4 t[M3 ? G::MB : 1][M3 ? G::NB : 1];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < G::MB; ++a)
#pragma unroll
      for (int b = 0; b < G::NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          re[a][b][v] = 0;
          im[a][b][v] = 0;
          if (M3) t[M3 ? a : 0][M3 ? b : 0][v] = 0;
        }
  }
  __device__ void finish() {
    if constexpr (M3) {
#pragma unroll
      for (int a = 0; a < G::MB; ++a)
#pragma unroll
        for (int b = 0; b < G::NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T t1 = re[a][b][v], t2 = t[a][b][v];
            re[a][b][v] = t1 - t2;
            im[a][b][v] = im[a][b][v] - t1 - t2;
          }
    }
  }
};

// One sub-step (4 real K = 2 complex) of MFMAs for this wave: lane l
// supplies A'[l%16][l/16] and B'[l/16][l%16] of each 16x16x4 block (real form).
// Three-product sub-step: 4 complex K, lane l at complex k = kk (plane rows
// kk, GK + kk, 2 GK + kk).
template <typename T, int BM, int BN, bool PKM>
__device__ __forceinline__ void mfma_sub3(const GemmSmem<T, BM, BN, PKM, true>& sm,
                                          WaveAcc<T, BM, BN, true>& acc, int wr, int wc,
                                          int li, int kk) {
  using G = WaveGrid<BM, BN>;
  T a[3][G::MB], b[3][G::NB];
#pragma unroll
  for (int pl = 0; pl < 3; ++pl) {
#pragma unroll
    for (int bm = 0; bm < G::MB; ++bm) {
      const int r = wr * G::RW + bm * 16 + li;
      a[pl][bm] = PKM ? sm.P[pl * GK + kk][r] : sm.P[r][pl * GK + kk];
    }
#pragma unroll
    for (int bn = 0; bn < G::NB; ++bn) b[pl][bn] = sm.Q1[pl * GK + kk][wc * G::CW + bn * 16 + li];
  }
#pragma unroll
  for (int bm = 0; bm < G::MB; ++bm)
#pragma unroll
    for (int bn = 0; bn < G::NB; ++bn) {
      acc.re[bm][bn] = Mfma<T>::op(a[0][bm], b[0][bn], acc.re[bm][bn]);
      acc.t[bm][bn] = Mfma<T>::op(a[1][bm], b[1][bn], acc.t[bm][bn]);
      acc.im[bm][bn] = Mfma<T>::op(a[2][bm], b[2][bn], acc.im[bm][bn]);
    }
}

template <typename T, int BM, int BN, bool PKM>
__device__ __forceinline__ void mfma_sub(const GemmSmem<T, BM, BN, PKM>& sm,
                                         WaveAcc<T, BM, BN>& acc, int wr, int wc, int li,
                                         int kk) {
  using G = WaveGrid<BM, BN>;
  T a[G::MB], b1[G::NB], b2[G::NB];
#pragma unroll
  for (int bm = 0; bm < G::MB; ++bm) {
    const int r = wr * G::RW + bm * 16 + li;
    a[bm] = PKM ? sm.P[kk][r] : sm.P[r][kk];
  }
#pragma unroll
  for (int bn = 0; bn < G::NB; ++bn) {
    b1[bn] = sm.Q1[kk][wc * G::CW + bn * 16 + li];
    b2[bn] = sm.Q2[kk][wc * G::CW + bn * 16 + li];
  }
#pragma unroll
  for (int bm = 0; bm < G::MB; ++bm)
#pragma unroll
    for (int bn = 0; bn < G::NB; ++bn) {
      acc.re[bm][bn] = Mfma<T>::op(a[bm], b1[bn], acc.re[bm][bn]);
      acc.im[bm][bn] = Mfma<T>::op(a[bm], b2[bn], acc.im[bm][bn]);
    }
}

// One K step (GK complex = 2 GK real) of MFMAs for this wave.  A full
// complex64 step is straight-line code, so the compiler can issue the LDS
// reads of later sub-steps under the MFMAs of earlier ones (for complex128
// the extra registers cost more than that gains); otherwise the sub-steps
// past the valid complex columns of a partial last step (zero-filled in LDS)
// are skipped (kvalid is the same for the whole block).
template <typename T, int BM, int BN, bool PKM, bool M3>
__device__ __forceinline__ void mfma_step(const GemmSmem<T, BM, BN, PKM, M3>& sm,
                                          WaveAcc<T, BM, BN, M3>& acc, int wr, int wc, int lane,
                                          int kvalid) {
  const int li = lane & 15, lq = lane >> 4;
  if constexpr (M3) {
    if (kvalid >= GK) {
#pragma unroll
      for (int p = 0; p < GK / 4; ++p) mfma_sub3<T, BM, BN, PKM>(sm, acc, wr, wc, li, 4 * p + lq);
    } else {
#pragma unroll
      for (int p = 0; p < GK / 4; ++p) {
        if (4 * p >= kvalid) break;
        mfma_sub3<T, BM, BN, PKM>(sm, acc, wr, wc, li, 4 * p + lq);
      }
    }
  } else if (sizeof(T) == 4 && kvalid >= GK) {
#pragma unroll
    for (int p = 0; p < GK / 2; ++p) mfma_sub<T, BM, BN, PKM>(sm, acc, wr, wc, li, 4 * p + lq);
  } else {
#pragma unroll
    for (int p = 0; p < GK / 2; ++p) {
      if (2 * p >= kvalid) break;
      mfma_sub<T, BM, BN, PKM>(sm, acc, wr, wc, li, 4 * p + lq);
    }
  }
}

// K loop of a BM x BN tile over k in [kbeg, kend): rows of P from `pv`
// starting at r0, columns of Q from `qv` starting at c0.  The global loads
// of the next K step are issued before the matrix-core work of the current
// one, so their latency overlaps the MFMAs.
template <typename T, int BM, bool P_FAST_R, bool Q_FAST_C, int BN, bool M3 = false>
__device__ __forceinline__ void gemm_tile(GemmSmem<T, BM, BN, P_FAST_R, M3>& sm,
                                          WaveAcc<T, BM, BN, M3>& acc,
                                          const View<T>& pv, const View<T>& qv,
                                          int r0, int c0, int kbeg, int kend) {
  using G = WaveGrid<BM, BN>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave / G::WC, wc = wave % G::WC;
  acc.zero();
  if (kbeg >= kend) return;
  Stage<T, BM, BN> g;
  stage_index<T, BM, BN, Q_FAST_C>(g, qv, kbeg, kend);
  stage_load<T, BM, BN, P_FAST_R, Q_FAST_C>(g, pv, qv, r0, c0, kbeg, kend);
  stage_index<T, BM, BN, Q_FAST_C>(g, qv, kbeg + GK, kend);
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    stage_store<T, BM, BN, P_FAST_R, Q_FAST_C, M3>(sm, g);
    __syncthreads();
    if (k0 + GK < kend) {
      stage_load<T, BM, BN, P_FAST_R, Q_FAST_C>(g, pv, qv, r0, c0, k0 + GK, kend);
      stage_index<T, BM, BN, Q_FAST_C>(g, qv, k0 + 2 * GK, kend);
    }
    mfma_step<T, BM, BN, P_FAST_R, M3>(sm, acc, wr, wc, lane, kend - k0);
    __syncthreads();
  }
  acc.finish();
}

// Output rows and columns (tile offsets) of this lane's accumulators, in the
// order of WaveAcc: row i = 4 bm + v, column j = bn.
template <typename T, int BM, int BN> struct LaneOut {
  using G = WaveGrid<BM, BN>;
  static constexpr int NR = G::MB * 4, NC = G::NB;
  int r[NR], c[NC];
  __device__ __forceinline__ LaneOut() {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave / G::WC, wc = wave % G::WC;
#pragma unroll
    for (int bm = 0; bm < G::MB; ++bm)
#pragma unroll
      for (int v = 0; v < 4; ++v) r[bm * 4 + v] = wr * G::RW + bm * 16 + Mfma<T>::row(lane, v);
#pragma unroll
    for (int bn = 0; bn < G::NB; ++bn) c[bn] = wc * G::CW + bn * 16 + (lane & 15);
  }
};

template <typename T, int BM, int BN, bool M3>
__device__ __forceinline__ C_t<T> acc_at(const WaveAcc<T, BM, BN, M3>& acc, int i, int j) {
  C_t<T> z;
  z.x = acc.re[i / 4][j][i % 4];
  z.y = acc.im[i / 4][j][i % 4];
  return z;
}

// Visit this lane's outputs: f(r, c, value) with r (0..BM-1), c (0..BN-1) the
// tile-local MFMA row / column.
template <typename T, int BM, int BN, bool M3, class F>
__device__ __forceinline__ void for_each_acc(const WaveAcc<T, BM, BN, M3>& acc, F&& f) {
  using G = WaveGrid<BM, BN>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave / G::WC, wc = wave % G::WC;
#pragma unroll
  for (int bm = 0; bm < G::MB; ++bm)
#pragma unroll
    for (int bn = 0; bn < G::NB; ++bn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = wr * G::RW + bm * 16 + Mfma<T>::row(lane, v);
        int c = wc * G::CW + bn * 16 + (lane & 15);
        C_t<T> z;
        z.x = acc.re[bm][bn][v];
        z.y = acc.im[bm][bn][v];
        f(r, c, z);
      }
}

}  // namespace kern
}  // namespace helm
