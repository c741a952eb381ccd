// Multifrontal factorization kernels (offline stage, Algorithm 1).
//
// Every front holds an (s+b) x (s+b) column-major frontal matrix
//   F = [F11 F12; F21 F22]   (s pivots, b boundary variables).
// Instead of an LU with separate triangular solves, the s pivots are
// eliminated by a blocked Gauss-Jordan sweep with partial pivoting restricted
// to the rows of F11.  After the sweep the front holds
//   [F11^-1, F11^-1 F12; -F21 F11^-1, F22 - F21 F11^-1 F12],
// i.e. the inverse of the pivot block, the multipliers and the Schur
// complement passed to the parent.  Each block step of nb pivots is a small
// panel factorization (pivot choice), a row swap, and one rank-nb update of
// the whole front -- a dense complex GEMM that runs on the matrix cores.
// With the complex-symmetric operator (H = H^T) the stored left block
// [F11^-1; -F21 F11^-1] is all the substitutions need: the backward step uses
// the transpose of -F21 F11^-1 in place of F11^-1 F12.
#include "kernels.h"
#include "kernels_common.h"

namespace helm {
namespace kern {

namespace {

template <typename T>
__device__ __forceinline__ C_t<T>* front_ptr(void* ws0, void* ws1, const FrontDev& f) {
  C_t<T>* base = reinterpret_cast<C_t<T>*>(f.ws_parity ? ws1 : ws0);
  return base + f.ws;
}

// --------------------------------------------------------------------------
// front assembly: frontal matrix = extend-add of the children's Schur
// complements (pull form: every entry is written once) ...
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_extend_add(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_ids, const int2* __restrict__ tmap,
             const LayerDev* __restrict__ layers, void* ws0, void* ws1) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int nt = (n + GT - 1) / GT;
  const int tile = tm.y;
  const int i0 = (tile % nt) * GT, j0 = (tile / nt) * GT;
  __shared__ int inv_r[2][GT], inv_c[2][GT];
  const LayerDev& L = layers[f.layer];
  const int t = threadIdx.x;
  if (t < 2 * GT) {
    int slot = t / GT, q = t % GT;
    int vr = -1, vc = -1;
    if (f.inv[slot] >= 0) {
      if (i0 + q < n) vr = L.inv[f.inv[slot] + i0 + q];
      if (j0 + q < n) vc = L.inv[f.inv[slot] + j0 + q];
    }
    inv_r[slot][q] = vr;
    inv_c[slot][q] = vc;
  }
  __syncthreads();
  C* F = front_ptr<T>(ws0, ws1, f);
  const C* S[2] = {nullptr, nullptr};
  int ldc[2] = {0, 0}, sc[2] = {0, 0};
  for (int slot = 0; slot < 2; ++slot) {
    if (f.child[slot] >= 0) {
      const FrontDev c = fronts[f.child[slot]];
      S[slot] = front_ptr<T>(ws0, ws1, c);
      ldc[slot] = c.s + c.b;
      sc[slot] = c.s;
    }
  }
  const int i = t % GT;
  for (int jj = t / GT; jj < GT; jj += 256 / GT) {
    const int gi = i0 + i, gj = j0 + jj;
    if (gi >= n || gj >= n) continue;
    C v = czero<C>();
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      int ri = inv_r[slot][i], cj = inv_c[slot][jj];
      if (S[slot] && ri >= 0 && cj >= 0)
        v = cadd(v, S[slot][(long long)(sc[slot] + ri) +
                            (long long)(sc[slot] + cj) * ldc[slot]]);
    }
    F[(long long)gi + (long long)gj * n] = v;
  }
}

// ... plus the entries of H^l whose first-eliminated variable is a pivot of
// this front.  Discrete operator of Eq. discrete_local_Helmholtz in the
// complex-symmetric form: off-diagonal h^-2 beta_a(half) / (other two betas),
// diagonal minus their sum plus omega^2 m / (beta_x beta_y beta_z).
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) { return cdiv(a, b); }

template <typename T>
__global__ void __launch_bounds__(256)
k_orig_entries(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
               int n_ids, const int2* __restrict__ tmap,
               const LayerDev* __restrict__ layers, void* ws0, void* ws1,
               GridDev g) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int r = tm.y * 256 + threadIdx.x;
  if (r >= f.s) return;
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  C* F = front_ptr<T>(ws0, ws1, f);
  const int nd = f.off + r;
  const int nat = L.nd2nat[nd];
  const int nx = g.nx, ny = g.ny;
  const int x = nat % nx, y = (nat / nx) % ny, z = nat / (nx * ny);
  const double2 bx = g.bx[x], by = g.by[y], bz = L.bz[z];
  const double ih2 = 1.0 / (g.h * g.h);
  const double2 bxy = zmul(bx, by), bxz = zmul(bx, bz), byz = zmul(by, bz);
  // six couplings: -x, +x, -y, +y, -z, +z
  double2 cpl[6];
  cpl[0] = zdiv(g.bxh[x], byz);
  cpl[1] = zdiv(g.bxh[x + 1], byz);
  cpl[2] = zdiv(g.byh[y], bxz);
  cpl[3] = zdiv(g.byh[y + 1], bxz);
  cpl[4] = zdiv(L.bzh[z], bxy);
  cpl[5] = zdiv(L.bzh[z + 1], bxy);
  int zg = L.lo + z;
  zg = zg < L.s ? L.s : (zg > L.e ? L.e : zg);   // model copied into the local PML
  const double mm = g.m[(long long)x + (long long)nx * ((long long)y + (long long)ny * zg)];
  double2 dg = zdiv(make_double2(g.omega * g.omega * mm, 0.0), zmul(bxy, bz));
  for (int q = 0; q < 6; ++q) { dg.x -= cpl[q].x * ih2; dg.y -= cpl[q].y * ih2; }
  {
    C& d = F[(long long)r + (long long)r * n];
    d = cadd(d, from_d2<C>(dg));
  }
  const int dx[6] = {-1, 1, 0, 0, 0, 0}, dy[6] = {0, 0, -1, 1, 0, 0},
            dz[6] = {0, 0, 0, 0, -1, 1};
  const int* B = L.bidx + f.bidx;
  for (int q = 0; q < 6; ++q) {
    int xx = x + dx[q], yy = y + dy[q], zz = z + dz[q];
    if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= L.t) continue;
    int ndn = L.nat2nd[xx + nx * (yy + ny * zz)];
    if (ndn < f.off) continue;  // assembled in a descendant front
    C v = from_d2<C>(make_double2(cpl[q].x * ih2, cpl[q].y * ih2));
    if (ndn < f.off + f.s) {
      int col = ndn - f.off;
      C& e = F[(long long)r + (long long)col * n];
      e = cadd(e, v);
    } else {
      // boundary variable: binary search in the sorted boundary list
      int lo = 0, hi = f.b - 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (B[mid] < ndn) lo = mid + 1; else hi = mid;
      }
      if (f.b == 0 || B[lo] != ndn) continue;   // cannot happen for a valid plan
      int col = f.s + lo;
      C& e1 = F[(long long)r + (long long)col * n];
      e1 = cadd(e1, v);
      C& e2 = F[(long long)col + (long long)r * n];
      e2 = cadd(e2, v);
    }
  }
}

// --------------------------------------------------------------------------
// panel: LU with partial pivoting of rows [k, s) x columns [k, k+nbf) on a
// copy, to choose the nbf pivot rows; then D = (pivoted diagonal block)^-1.
// One 1024-thread workgroup per front.
// --------------------------------------------------------------------------
constexpr int PANEL_THREADS = 1024;
constexpr int NBMAX = 64;
constexpr int PB = 8;   // column block of the panel LU

template <typename T>
__global__ void __launch_bounds__(PANEL_THREADS)
k_panel(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
        int k, int nb, void* ws0, void* ws1, void* panel_base,
        const long long* __restrict__ panel_off, void* D_base, int* ipiv_base,
        int* perm_base, const long long* __restrict__ perm_off, int* status) {
  using C = C_t<T>;
  const int a = blockIdx.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int R = f.s - k;
  if (R <= 0) return;
  const int nbf = R < nb ? R : nb;
  const int t = threadIdx.x;
  C* F = front_ptr<T>(ws0, ws1, f);
  C* P = reinterpret_cast<C*>(panel_base) + panel_off[a];
  C* D = reinterpret_cast<C*>(D_base) + panel_off[a];
  int* ipiv = ipiv_base + perm_off[a];
  int* perm = perm_base + perm_off[a];
  if (k == 0)
    for (int i = t; i < f.s; i += PANEL_THREADS) perm[i] = i;
  for (long long e = t; e < (long long)R * nbf; e += PANEL_THREADS) {
    int r = e % R, c = e / R;
    P[r + (long long)c * R] = F[(long long)(k + r) + (long long)(k + c) * n];
  }
  __shared__ double red_v[PANEL_THREADS / 64];
  __shared__ int red_i[PANEL_THREADS / 64];
  __shared__ int piv_row;
  __syncthreads();
  // Blocked right-looking LU of the panel: columns in blocks of PB; inside
  // a block every column is pivoted, scaled and applied to the block's
  // remaining columns; then the block rows of the trailing columns are
  // solved with the block's unit lower triangle and the trailing columns
  // get one rank-PB update (one pass over them per block instead of one per
  // column).
  __shared__ C U12[PB][NBMAX];
  for (int c0 = 0; c0 < nbf; c0 += PB) {
    const int c1 = (c0 + PB < nbf) ? c0 + PB : nbf;
    for (int c = c0; c < c1; ++c) {
      // arg max |P[r][c]|, r >= c (ties: smallest row, so the choice is
      // reproducible)
      double best = -1.0;
      int bi = R;
      for (int r = c + t; r < R; r += PANEL_THREADS) {
        double v = cabs2(P[r + (long long)c * R]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_down(best, off);
        int oi = __shfl_down(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if ((t & 63) == 0) { red_v[t >> 6] = best; red_i[t >> 6] = bi; }
      __syncthreads();
      if (t == 0) {
        double bv = red_v[0];
        int bidx = red_i[0];
        for (int w = 1; w < PANEL_THREADS / 64; ++w)
          if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bidx)) {
            bv = red_v[w];
            bidx = red_i[w];
          }
        if (!(bv > 0.0) || !isfinite(bv)) {
          atomicExch(status, 1);   // zero or non-finite pivot
          bidx = c;
        }
        piv_row = bidx;
        ipiv[c] = bidx;
        if (bidx != c) {
          int tmp = perm[k + c];
          perm[k + c] = perm[k + bidx];
          perm[k + bidx] = tmp;
        }
      }
      __syncthreads();
      const int p = piv_row;
      if (p != c)
        for (int cc = t; cc < nbf; cc += PANEL_THREADS) {
          C x = P[c + (long long)cc * R];
          P[c + (long long)cc * R] = P[p + (long long)cc * R];
          P[p + (long long)cc * R] = x;
        }
      __syncthreads();
      C piv = P[c + (long long)c * R];
      if (cabs2(piv) == 0.0) piv = cmake<C>(1.0, 0.0);
      const C one = cmake<C>(1.0, 0.0);
      const C ipv = cdiv(one, piv);
      for (int r = c + 1 + t; r < R; r += PANEL_THREADS)
        P[r + (long long)c * R] = cmul(P[r + (long long)c * R], ipv);
      __syncthreads();
      // rank-1 update of the block's remaining columns
      const int rows = R - c - 1, cols = c1 - c - 1;
      for (long long e = t; e < (long long)rows * cols; e += PANEL_THREADS) {
        int r = c + 1 + (int)(e % rows), cc = c + 1 + (int)(e / rows);
        C& x = P[r + (long long)cc * R];
        cfms(x, P[r + (long long)c * R], P[c + (long long)cc * R]);
      }
      __syncthreads();
    }
    if (c1 >= nbf) break;
    const int W = nbf - c1, bw = c1 - c0;
    // block rows of the trailing columns: U12 = L11^-1 A12 (unit lower)
    for (int cc = t; cc < W; cc += PANEL_THREADS) {
      const long long col = (long long)(c1 + cc) * R;
      for (int i = 0; i < bw; ++i) {
        C x = P[c0 + i + col];
        for (int j = 0; j < i; ++j) cfms(x, P[c0 + i + (long long)(c0 + j) * R], U12[j][cc]);
        U12[i][cc] = x;
        P[c0 + i + col] = x;
      }
    }
    __syncthreads();
    // rank-bw update of the trailing columns below the block
    for (int r = c1 + t; r < R; r += PANEL_THREADS) {
      C l[PB];
#pragma unroll
      for (int j = 0; j < PB; ++j)
        l[j] = j < bw ? P[r + (long long)(c0 + j) * R] : czero<C>();
      for (int cc = 0; cc < W; ++cc) {
        C& x = P[r + (long long)(c1 + cc) * R];
        C y = x;
#pragma unroll
        for (int j = 0; j < PB; ++j)
          if (j < bw) cfms(y, l[j], U12[j][cc]);
        x = y;
      }
    }
    __syncthreads();
  }
  // D = U^-1 L^-1 of the leading nbf x nbf block, one column per thread
  __shared__ C LU[NBMAX][NBMAX + 1];
  for (int e = t; e < nbf * nbf; e += PANEL_THREADS) {
    int r = e % nbf, c = e / nbf;
    LU[r][c] = P[r + (long long)c * R];
  }
  __syncthreads();
  if (t < nbf) {
    const int j = t;
    // forward: L y = e_j (unit lower), y stored in D[:, j]
    for (int i = 0; i < nbf; ++i) {
      C y = cmake<C>(i == j ? 1.0 : 0.0, 0.0);
      for (int q = 0; q < i; ++q) cfms(y, LU[i][q], D[q + j * nb]);
      D[i + j * nb] = y;
    }
    // backward: U x = y
    for (int i = nbf - 1; i >= 0; --i) {
      C x = D[i + j * nb];
      for (int q = i + 1; q < nbf; ++q) cfms(x, LU[i][q], D[q + j * nb]);
      D[i + j * nb] = cdiv(x, LU[i][i]);
    }
  }
}

// --------------------------------------------------------------------------
// apply the nbf row swaps to every column, then rows J <- D * rows J for the
// columns outside J.  One workgroup per 64-column tile.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_swap_JO(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
          int n_active, const int2* __restrict__ tmap, int k, int nb,
          void* ws0, void* ws1, const void* D_base, const int* __restrict__ ipiv_base,
          const long long* __restrict__ panel_off, const long long* __restrict__ perm_off) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int nbf = (f.s - k) < nb ? (f.s - k) : nb;
  const int c0 = tm.y * GT;
  C* F = front_ptr<T>(ws0, ws1, f);
  const int* ipiv = ipiv_base + perm_off[a];
  const C* D = reinterpret_cast<const C*>(D_base) + panel_off[a];
  const int t = threadIdx.x;
  if (t < GT && c0 + t < n) {
    C* col = F + (long long)(c0 + t) * n;
    for (int jj = 0; jj < nbf; ++jj) {
      int r2 = k + ipiv[jj];
      if (r2 != k + jj) {
        C x = col[k + jj];
        col[k + jj] = col[r2];
        col[r2] = x;
      }
    }
  }
  __syncthreads();
  __shared__ C V[NBMAX][GT + 1];
  __shared__ C Ds[NBMAX][NBMAX + 1];
  for (int e = t; e < nbf * GT; e += 256) {
    int r = e % nbf, c = e / nbf;
    V[r][c] = (c0 + c < n) ? F[(long long)(k + r) + (long long)(c0 + c) * n] : czero<C>();
  }
  for (int e = t; e < nbf * nbf; e += 256) {
    int r = e % nbf, c = e / nbf;
    Ds[r][c] = D[r + c * nb];
  }
  __syncthreads();
  for (int e = t; e < nbf * GT; e += 256) {
    int r = e % nbf, c = e / nbf;
    int gc = c0 + c;
    if (gc >= n || (gc >= k && gc < k + nbf)) continue;
    C acc = czero<C>();
    for (int q = 0; q < nbf; ++q) cfma(acc, Ds[r][q], V[q][c]);
    F[(long long)(k + r) + (long long)gc * n] = acc;
  }
}

// --------------------------------------------------------------------------
// rank-nb update of every entry outside the pivot rows / columns J:
//   F(O, O) -= F(O, J) F(J, O)     (J rows already hold D * F(J, O))
// Computed as C^T = B^T A^T so that the MFMA column index walks the
// contiguous (row) dimension of the column-major front.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_sweep_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_active, const int2* __restrict__ tmap, int k, int nb,
             void* ws0, void* ws1) {
  using C = C_t<T>;
  __shared__ GemmSmem<T, 64, 64, false> sm;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int nbf = (f.s - k) < nb ? (f.s - k) : nb;
  const int nt = (n + GT - 1) / GT;
  const int tile = tm.y;
  const int i0 = (tile % nt) * GT;   // C rows
  const int j0 = (tile / nt) * GT;   // C columns
  C* F = front_ptr<T>(ws0, ws1, f);
  // P rows = C columns j: B^T(j, q) = F[(k+q) + j n]
  View<T> pv{F + k, (long long)n, 1, n, nbf};
  // Q columns = C rows i: A^T(q, i) = F[i + (k+q) n]
  View<T> qv{F + (long long)k * n, 1, (long long)n, n, nbf};
  WaveAcc<T, 64> acc;
  gemm_tile<T, 64, false, true>(sm, acc, pv, qv, j0, i0, 0, nbf);
  for_each_acc<T, 64, 64>(acc, [&](int r, int c, C z) {
    const int gi = i0 + c, gj = j0 + r;
    if (gi < n && gj < n && (gi < k || gi >= k + nbf) && (gj < k || gj >= k + nbf)) {
      C& e = F[(long long)gi + (long long)gj * n];
      e = csub(e, z);
    }
  });
}

// --------------------------------------------------------------------------
// columns J: rows outside J <- -F(O, J) D, rows J <- D.  One workgroup per
// 64-row tile.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_update_OJ(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
            int n_active, const int2* __restrict__ tmap, int k, int nb,
            void* ws0, void* ws1, const void* D_base,
            const long long* __restrict__ panel_off) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int nbf = (f.s - k) < nb ? (f.s - k) : nb;
  const int r0 = tm.y * GT;
  C* F = front_ptr<T>(ws0, ws1, f);
  const C* D = reinterpret_cast<const C*>(D_base) + panel_off[a];
  __shared__ C V[GT][NBMAX + 1];
  __shared__ C Ds[NBMAX][NBMAX + 1];
  const int t = threadIdx.x;
  for (int e = t; e < GT * nbf; e += 256) {
    int r = e % GT, c = e / GT;
    V[r][c] = (r0 + r < n) ? F[(long long)(r0 + r) + (long long)(k + c) * n] : czero<C>();
  }
  for (int e = t; e < nbf * nbf; e += 256) {
    int r = e % nbf, c = e / nbf;
    Ds[r][c] = D[r + c * nb];
  }
  __syncthreads();
  for (int e = t; e < GT * nbf; e += 256) {
    int r = e % GT, c = e / GT;
    int gr = r0 + r;
    if (gr >= n) continue;
    C out;
    if (gr >= k && gr < k + nbf) {
      out = Ds[gr - k][c];
    } else {
      C acc = czero<C>();
      for (int q = 0; q < nbf; ++q) cfma(acc, V[r][q], Ds[q][c]);
      out = cneg(acc);
    }
    F[(long long)gr + (long long)(k + c) * n] = out;
  }
}

// --------------------------------------------------------------------------
// copy the first s columns to the factor store, undoing the row pivoting of
// F11 (which permuted the columns of the swept inverse): true column perm[i]
// <- swept column i.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_store_factor(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
               int n_ids, const int2* __restrict__ tmap,
               const LayerDev* __restrict__ layers, void* ws0, void* ws1,
               const int* __restrict__ perm_base, const long long* __restrict__ perm_off) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int nrt = (n + GT - 1) / GT;
  const int tile = tm.y;
  const int i0 = (tile % nrt) * GT, j0 = (tile / nrt) * GT;
  const C* F = front_ptr<T>(ws0, ws1, f);
  C* FT = reinterpret_cast<C*>(layers[f.layer].fac) + f.fac;
  const int* perm = perm_base + perm_off[a];
  const int t = threadIdx.x;
  const int i = t % GT;
  for (int jj = t / GT; jj < GT; jj += 256 / GT) {
    int gi = i0 + i, gj = j0 + jj;
    if (gi >= n || gj >= f.s) continue;
    FT[(long long)gi + (long long)perm[gj] * n] = F[(long long)gi + (long long)gj * n];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_extend_add(const FrontDev* fronts, const int* ids, int n_ids,
                       const int2* tmap, int total, const LayerDev* layers,
                       void* ws0, void* ws1, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_extend_add<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_ids, tmap, layers, ws0, ws1);
}
template <typename T>
void launch_orig_entries(const FrontDev* fronts, const int* ids, int n_ids,
                         const int2* tmap, int total, const LayerDev* layers,
                         void* ws0, void* ws1, const GridDev& g, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_orig_entries<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_ids, tmap, layers, ws0, ws1, g);
}
template <typename T>
void launch_panel(const FrontDev* fronts, const int* ids, int n_active, int k,
                  int nb, void* ws0, void* ws1, void* panel,
                  const long long* panel_off, void* D, int* ipiv, int* perm,
                  const long long* perm_off, int* status, hipStream_t st) {
  if (n_active <= 0) return;
  hipLaunchKernelGGL(k_panel<T>, dim3(n_active), dim3(PANEL_THREADS), 0, st, fronts,
                     ids, k, nb, ws0, ws1, panel, panel_off, D, ipiv, perm,
                     perm_off, status);
}
template <typename T>
void launch_swap_JO(const FrontDev* fronts, const int* ids, int n_active,
                    const int2* tmap, int total, int k, int nb, void* ws0,
                    void* ws1, const void* D, const int* ipiv,
                    const long long* panel_off, const long long* perm_off,
                    hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_swap_JO<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_active, tmap, k, nb, ws0, ws1, D, ipiv, panel_off, perm_off);
}
template <typename T>
void launch_sweep_gemm(const FrontDev* fronts, const int* ids, int n_active,
                       const int2* tmap, int total, int k, int nb, void* ws0,
                       void* ws1, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_sweep_gemm<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_active, tmap, k, nb, ws0, ws1);
}
template <typename T>
void launch_update_OJ(const FrontDev* fronts, const int* ids, int n_active,
                      const int2* tmap, int total, int k, int nb, void* ws0,
                      void* ws1, const void* D, const long long* panel_off,
                      hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_update_OJ<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_active, tmap, k, nb, ws0, ws1, D, panel_off);
}
template <typename T>
void launch_store_factor(const FrontDev* fronts, const int* ids, int n_ids,
                         const int2* tmap, int total, const LayerDev* layers,
                         void* ws0, void* ws1, const int* perm,
                         const long long* perm_off, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_store_factor<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_ids, tmap, layers, ws0, ws1, perm, perm_off);
}

#define HELM_INST_FACTOR(T)                                                        \
  template void launch_extend_add<T>(const FrontDev*, const int*, int, const int2*, \
                                     int, const LayerDev*, void*, void*,           \
                                     hipStream_t);                                 \
  template void launch_orig_entries<T>(const FrontDev*, const int*, int,          \
                                       const int2*, int, const LayerDev*, void*,    \
                                       void*, const GridDev&, hipStream_t);        \
  template void launch_panel<T>(const FrontDev*, const int*, int, int, int, void*, \
                                void*, void*, const long long*, void*, int*, int*, \
                                const long long*, int*, hipStream_t);              \
  template void launch_swap_JO<T>(const FrontDev*, const int*, int, const int2*,    \
                                  int, int, int, void*, void*, const void*,        \
                                  const int*, const long long*, const long long*,  \
                                  hipStream_t);                                    \
  template void launch_sweep_gemm<T>(const FrontDev*, const int*, int, const int2*, \
                                     int, int, int, void*, void*, hipStream_t);    \
  template void launch_update_OJ<T>(const FrontDev*, const int*, int, const int2*,  \
                                    int, int, int, void*, void*, const void*,      \
                                    const long long*, hipStream_t);                \
  template void launch_store_factor<T>(const FrontDev*, const int*, int,          \
                                       const int2*, int, const LayerDev*, void*,    \
                                       void*, const int*, const long long*,        \
                                       hipStream_t);
HELM_INST_FACTOR(float)
HELM_INST_FACTOR(double)

}  // namespace kern
}  // namespace helm
