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
  // the lane's 16 entries are all gathered before the first store
  constexpr int NJ = GT / (256 / GT);
  const int i = t % GT, gi = i0 + i;
  C v[NJ];
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int jj = t / GT + u * (256 / GT), gj = j0 + jj;
    C acc = czero<C>();
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const int ri = inv_r[slot][i], cj = inv_c[slot][jj];
      const bool hit = gi < n && gj < n && S[slot] && ri >= 0 && cj >= 0;
      acc = cadd(acc, ld_or_zero(hit, S[slot] + (hit ? (long long)(sc[slot] + ri) +
                                                         (long long)(sc[slot] + cj) * ldc[slot]
                                                     : 0)));
    }
    v[u] = acc;
  }
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int gj = j0 + t / GT + u * (256 / GT);
    if (gi < n && gj < n) st(F + (long long)gi + (long long)gj * n, v[u]);
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
               GridDev g, int skip_front, FactorStatus* status) {
  using C = C_t<T>;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int r = tm.y * 256 + threadIdx.x;
  // a front left unassembled on request (exercises the zero-pivot status)
  const bool valid = r < f.s && ids[a] != skip_front;
  const LayerDev& L = layers[f.layer];
  const int n = f.s + f.b;
  C* F = front_ptr<T>(ws0, ws1, f);
  const int nx = g.nx, ny = g.ny;
  int x = 0, y = 0, z = 0;
  double2 cpl[6];
  double2 dg = make_double2(0.0, 0.0);
  const double ih2 = 1.0 / (g.h * g.h);
  if (valid) {
    const int nat = L.nd2nat[f.off + r];
    x = nat % nx; y = (nat / nx) % ny; z = nat / (nx * ny);
    const double2 bx = g.bx[x], by = g.by[y], bz = L.bz[z];
    const double2 bxy = zmul(bx, by), bxz = zmul(bx, bz), byz = zmul(by, bz);
    // six couplings: -x, +x, -y, +y, -z, +z
    cpl[0] = zdiv(g.bxh[x], byz);
    cpl[1] = zdiv(g.bxh[x + 1], byz);
    cpl[2] = zdiv(g.byh[y], bxz);
    cpl[3] = zdiv(g.byh[y + 1], bxz);
    cpl[4] = zdiv(L.bzh[z], bxy);
    cpl[5] = zdiv(L.bzh[z + 1], bxy);
    int zg = L.lo + z;
    zg = zg < L.s ? L.s : (zg > L.e ? L.e : zg);   // model copied into the local PML
    const double mm = g.m[(long long)x + (long long)nx * ((long long)y + (long long)ny * zg)];
    dg = zdiv(make_double2(g.omega * g.omega * mm, 0.0), zmul(bxy, bz));
    for (int q = 0; q < 6; ++q) { dg.x -= cpl[q].x * ih2; dg.y -= cpl[q].y * ih2; }
  }
  {
    // largest |diagonal entry|^2 of the operator: a wave-wide maximum, then
    // one atomic per wave (bit patterns of non-negative doubles order like
    // the numbers)
    double d2 = dg.x * dg.x + dg.y * dg.y;
    for (int off = 32; off > 0; off >>= 1) d2 = fmax(d2, __shfl_xor(d2, off));
    if ((threadIdx.x & 63) == 0 && d2 > 0.0)
      atomicMax(&status->dmax, (unsigned long long)__double_as_longlong(d2));
  }
  if (!valid) return;
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
// One workgroup of NT threads per front.  The copy lives in LDS (PR rows at
// most) when the launch's tallest panel fits, as every leaf front's does,
// else (PR = 0) in the global panel buffer; only D, the pivots and the
// permutation leave the kernel.
// --------------------------------------------------------------------------
constexpr int NBMAX = 64;
constexpr int PB = 8;   // column block of the panel LU
template <typename T> constexpr int panel_lds_rows() { return sizeof(T) == 4 ? 192 : 64; }

// D = U^-1 L^-1 of the leading nbf x nbf block of the factored panel P
// (R rows, column-major, in LDS when LDSP), in LDS: X = L^-1 by eliminating
// below each unit pivot, then D = U^-1 X from the last row up.  Every step
// updates all entries it touches in parallel.
template <typename T, int NT, bool LDSP>
__device__ __forceinline__ void panel_inverse(const C_t<T>* P, int R, int nbf, int nb,
                                              C_t<T>* D) {
  using C = C_t<T>;
  const int t = threadIdx.x;
  // (the factors are read in place when the panel is in LDS)
  __shared__ C LUs[LDSP ? 1 : NBMAX][LDSP ? 1 : NBMAX + 1];
  __shared__ C X[NBMAX][NBMAX + 1];
  __shared__ C uinv[NBMAX];
  auto LU = [&](int r, int c) -> C { return LDSP ? P[r + c * R] : LUs[r][c]; };
  if (!LDSP) {
    // the factors from the global panel, every load before the first store
    constexpr int PER = (NBMAX * NBMAX + NT - 1) / NT;
    C w[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + NT * i, r = e % NBMAX, c = e / NBMAX;
      const bool ok = r < nbf && c < nbf;
      w[i] = ld_or_zero(ok, P + (ok ? r + (long long)c * R : 0));
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + NT * i, r = e % NBMAX, c = e / NBMAX;
      if (r < nbf && c < nbf) LUs[r][c] = w[i];
    }
  }
  for (int e = t; e < nbf * nbf; e += NT) {
    int r = e % nbf, c = e / nbf;
    X[r][c] = cmake<C>(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (t < nbf) {
    C u = LU(t, t);
    if (cabs2(u) == 0.0) u = cmake<C>(1.0, 0.0);
    uinv[t] = cdiv(cmake<C>(1.0, 0.0), u);
  }
  __syncthreads();
  // X[i][j] -= L[i][q] X[q][j] for i > q, j <= q
  for (int q = 0; q + 1 < nbf; ++q) {
    const int rows = nbf - 1 - q, cols = q + 1;
    for (int e = t; e < rows * cols; e += NT) {
      const int i = q + 1 + e % rows, j = e / rows;
      cfms(X[i][j], LU(i, q), X[q][j]);
    }
    __syncthreads();
  }
  // X[i][j] -= U[i][q] / U[q][q] X[q][j] for i < q; rows scaled at the end
  for (int q = nbf - 1; q > 0; --q) {
    for (int e = t; e < q * nbf; e += NT) {
      const int i = e % q, j = e / q;
      cfms(X[i][j], cmul(LU(i, q), uinv[q]), X[q][j]);
    }
    __syncthreads();
  }
  for (int e = t; e < nbf * nbf; e += NT) {
    int r = e % nbf, c = e / nbf;
    st(D + r + c * nb, cmul(X[r][c], uinv[r]));
  }
}

template <typename T, int NT, int PR>
__global__ void __launch_bounds__(NT)
k_panel(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
        int k, int nb, void* ws0, void* ws1, void* panel_base,
        const long long* __restrict__ panel_off, void* D_base, int* ipiv_base,
        int* perm_base, const long long* __restrict__ perm_off, FactorStatus* status) {
  using C = C_t<T>;
  constexpr int NW = NT / 64;
  constexpr bool LDSP = PR > 0;
  __shared__ C Ps[LDSP ? PR * NBMAX : 1];
  const int a = blockIdx.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int R = f.s - k;
  if (R <= 0) return;
  const int nbf = R < nb ? R : nb;
  const int t = threadIdx.x;
  const C* F = front_ptr<T>(ws0, ws1, f);
  C* P = LDSP ? Ps : reinterpret_cast<C*>(panel_base) + panel_off[a];
  C* D = reinterpret_cast<C*>(D_base) + panel_off[a];
  int* ipiv = ipiv_base + perm_off[a];
  int* perm = perm_base + perm_off[a];
  if (k == 0)
    for (int i = t; i < f.s; i += NT) perm[i] = i;
  for (long long e = t; e < (long long)R * nbf; e += NT) {
    int r = e % R, c = e / R;
    P[r + (long long)c * R] = ld(F + (long long)(k + r) + (long long)(k + c) * n);
  }
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ int piv_row;
  // smallest and largest |pivot|^2 of this panel (thread 0)
  double pv_min = INFINITY, pv_max = 0.0;
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
      for (int r = c + t; r < R; r += NT) {
        double v = cabs2(P[r + (long long)c * R]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_down(best, off);
        int oi = __shfl_down(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (NW > 1) {
        if ((t & 63) == 0) { red_v[t >> 6] = best; red_i[t >> 6] = bi; }
        __syncthreads();
      }
      if (t == 0) {
        double bv = NW > 1 ? red_v[0] : best;
        int bidx = NW > 1 ? red_i[0] : bi;
        for (int w = 1; w < NW; ++w)
          if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bidx)) {
            bv = red_v[w];
            bidx = red_i[w];
          }
        if (!(bv > 0.0) || !isfinite(bv)) {
          atomicExch(&status->flag, 1);   // zero or non-finite pivot
          bidx = c;
        } else {
          pv_min = fmin(pv_min, bv);
          pv_max = fmax(pv_max, bv);
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
        for (int cc = t; cc < nbf; cc += NT) {
          C x = P[c + (long long)cc * R];
          P[c + (long long)cc * R] = P[p + (long long)cc * R];
          P[p + (long long)cc * R] = x;
        }
      __syncthreads();
      C piv = P[c + (long long)c * R];
      if (cabs2(piv) == 0.0) piv = cmake<C>(1.0, 0.0);
      const C one = cmake<C>(1.0, 0.0);
      const C ipv = cdiv(one, piv);
      for (int r = c + 1 + t; r < R; r += NT)
        P[r + (long long)c * R] = cmul(P[r + (long long)c * R], ipv);
      __syncthreads();
      // rank-1 update of the block's remaining columns
      const int rows = R - c - 1, cols = c1 - c - 1;
      for (long long e = t; e < (long long)rows * cols; e += NT) {
        int r = c + 1 + (int)(e % rows), cc = c + 1 + (int)(e / rows);
        C& x = P[r + (long long)cc * R];
        cfms(x, P[r + (long long)c * R], P[c + (long long)cc * R]);
      }
      __syncthreads();
    }
    if (c1 >= nbf) break;
    const int W = nbf - c1, bw = c1 - c0;
    // block rows of the trailing columns: U12 = L11^-1 A12 (unit lower)
    for (int cc = t; cc < W; cc += NT) {
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
    for (int r = c1 + t; r < R; r += NT) {
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
  if (t == 0 && pv_max > 0.0) {
    atomicMin(&status->pmin, (unsigned long long)__double_as_longlong(pv_min));
    atomicMax(&status->pmax, (unsigned long long)__double_as_longlong(pv_max));
  }
  panel_inverse<T, NT, LDSP>(P, R, nbf, nb, D);
}

// Panels of at most 64 NW rows, complex64: NW waves per front, thread r
// holding row r of the panel in registers.  Gauss-Jordan elimination with
// partial pivoting turns the panel into the inverse of its pivoted diagonal
// block in place: at column c the chosen row is scaled by the pivot's
// inverse and removed from every other row, and column c's slot, no longer
// needed, takes column c of the inverse (the eliminated unit column carried
// along).  Rows never leave their threads; each thread tracks the index its
// row would have if rows were exchanged as in the LU, which gives the pivot
// choice of the LU with partial pivoting (largest |entry| among the rows not
// yet chosen, ties to the smallest index), the same exchange record ipiv and
// the same permutation.  One wave broadcasts the pivot row with lane reads;
// several exchange the wave maxima and the pivot row through LDS (two
// barriers per column).
template <typename T, int NW>
__global__ void __launch_bounds__(64 * NW)
k_panel_regs(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int k, int nb, void* ws0, void* ws1, void* D_base, int* ipiv_base,
             int* perm_base, const long long* __restrict__ perm_off,
             const long long* __restrict__ panel_off, FactorStatus* status) {
  using C = C_t<T>;
  const int a = blockIdx.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int R = f.s - k;
  if (R <= 0) return;
  const int nbf = R < nb ? R : nb;
  const int t = threadIdx.x, lane = t & 63;
  const bool row = t < R;
  const C* F = front_ptr<T>(ws0, ws1, f);
  C* D = reinterpret_cast<C*>(D_base) + panel_off[a];
  int* ipiv = ipiv_base + perm_off[a];
  int* perm = perm_base + perm_off[a];
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ C prow[NW > 1 ? NBMAX : 1];
  C x[NBMAX];
#pragma unroll
  for (int j = 0; j < NBMAX; ++j)
    x[j] = ld_or_zero(row && j < nbf,
                      F + (long long)(k + (row ? t : 0)) + (long long)(k + (j < nbf ? j : 0)) * n);
  // the permutation entry of this thread's row, read before any is written
  const int pold = k == 0 ? t : (row ? ld(perm + k + t) : 0);
  int pos = t;           // the row's index were rows exchanged as in the LU
  bool chosen = false;   // the row is the pivot row of an earlier column
  double pv_min = INFINITY, pv_max = 0.0;
  for (int c = 0; c < nbf; ++c) {
    C xc = x[0];
#pragma unroll
    for (int j = 1; j < NBMAX; ++j)
      if (j == c) xc = x[j];
    // arg max over the rows not yet chosen, the key (|x|^2, smallest
    // index): within the wave, then over the waves' maxima
    const bool cand = row && !chosen;
    double v = cand ? cabs2(xc) : -1.0;
    int bi = cand ? pos : R;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > v || (ov == v && oi < bi)) { v = ov; bi = oi; }
    }
    double bv;
    int P;
    if (NW == 1) {
      bv = __shfl(v, 0, 64);
      P = __builtin_amdgcn_readfirstlane(bi);
    } else {
      if (lane == 0) { red_v[t >> 6] = v; red_i[t >> 6] = bi; }
      __syncthreads();
      bv = red_v[0];
      P = red_i[0];
#pragma unroll
      for (int w = 1; w < NW; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < P)) {
          bv = red_v[w];
          P = red_i[w];
        }
    }
    // a zero or non-finite maximum: flagged, the row at index c taken
    const bool bad = !(bv > 0.0) || !isfinite(bv);
    if (bad) {
      P = c;
      if (t == 0) atomicExch(&status->flag, 1);
    } else {
      pv_min = fmin(pv_min, bv);
      pv_max = fmax(pv_max, bv);
    }
    if (t == 0) ipiv[c] = P;
    const bool win = cand && pos == P;
    C w_c;   // the pivot row's entries come from its lane (one wave) or LDS
    int pl = 0;
    if (NW == 1) {
      pl = __builtin_amdgcn_readfirstlane(__ffsll((long long)__ballot(win)) - 1);
      w_c.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xc.x), pl));
      w_c.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xc.y), pl));
    } else {
      if (win)
#pragma unroll
        for (int j = 0; j < NBMAX; ++j)
          if (j < nbf) prow[j] = x[j];
      __syncthreads();
      w_c = xc;
#pragma unroll
      for (int j = 0; j < NBMAX; ++j)
        if (j == c) w_c = prow[j];
    }
    // exchange of indices c and P: the row at c moves to P, the pivot row to c
    if (pos == c) pos = P;
    if (win) {
      pos = c;
      chosen = true;
    }
    C piv = w_c;
    if (cabs2(piv) == 0.0) piv = cmake<C>(1.0, 0.0);
    const C ipv = cdiv(cmake<C>(1.0, 0.0), piv);
    // pivot row w (column c read as 1) scaled by ipv; every other row loses
    // g w' with g its column-c entry (that slot read as 0)
    const C g = win ? czero<C>() : xc;
#pragma unroll
    for (int j = 0; j < NBMAX; ++j) {
      if (j < nbf) {
        C w;
        if (NW == 1) {
          w.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[j].x), pl));
          w.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[j].y), pl));
        } else {
          w = prow[j];
        }
        if (j == c) w = cmake<C>(1.0, 0.0);
        const C ws = cmul(w, ipv);
        C y = win ? ws : (j == c ? czero<C>() : x[j]);
        cfms(y, g, ws);
        x[j] = y;
      }
    }
  }
  if (t == 0 && pv_max > 0.0) {
    atomicMin(&status->pmin, (unsigned long long)__double_as_longlong(pv_min));
    atomicMax(&status->pmax, (unsigned long long)__double_as_longlong(pv_max));
  }
  if (row) perm[k + pos] = pold;
  if (row && pos < nbf) {
#pragma unroll
    for (int j = 0; j < NBMAX; ++j)
      if (j < nbf) st(D + pos + (long long)j * nb, x[j]);
  }
}

// Tall panels (more rows than the LDS holds): the same blocked LU with
// partial pivoting, with the current column block of every row held in
// registers.  Thread t owns the rows t, t + NT, ... (RPT of them); a column
// step (pivot search, row exchange, scaling, rank-1 update of the block)
// works on registers and LDS only, so the panel copy in global memory is
// passed over once per block (the trailing update) instead of once per
// column.  Pivots, swaps and arithmetic are those of k_panel.
template <typename T, int NT, int RPT, int BW>
__global__ void __launch_bounds__(NT)
k_panel_rb(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
           int k, int nb, void* ws0, void* ws1, void* panel_base,
           const long long* __restrict__ panel_off, void* D_base, int* ipiv_base,
           int* perm_base, const long long* __restrict__ perm_off, FactorStatus* status) {
  using C = C_t<T>;
  constexpr int NW = NT / 64;
  const int a = blockIdx.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int R = f.s - k;
  if (R <= 0) return;
  const int nbf = R < nb ? R : nb;
  const int t = threadIdx.x;
  const C* F = front_ptr<T>(ws0, ws1, f);
  C* P = reinterpret_cast<C*>(panel_base) + panel_off[a];
  C* D = reinterpret_cast<C*>(D_base) + panel_off[a];
  int* ipiv = ipiv_base + perm_off[a];
  int* perm = perm_base + perm_off[a];
  if (k == 0)
    for (int i = t; i < f.s; i += NT) perm[i] = i;
  // the panel's columns past the first block to the global copy (each
  // thread its own rows, a group of columns' loads before their stores);
  // the first block goes straight to registers
  constexpr int CG = sizeof(T) == 4 ? BW : BW / 2;   // columns per load group
  for (int cg = BW; cg < nbf; cg += CG) {
    C v[RPT][CG];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = t + i * NT;
#pragma unroll
      for (int j = 0; j < CG; ++j)
        v[i][j] = ld_or_zero(r < R && cg + j < nbf,
                             F + (long long)(k + (r < R ? r : 0)) + (long long)(k + cg + j) * n);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = t + i * NT;
#pragma unroll
      for (int j = 0; j < CG; ++j)
        if (r < R && cg + j < nbf) P[r + (long long)(cg + j) * R] = v[i][j];
    }
  }
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ C xch[BW];      // row c's block values, for the pivot row's owner
  __shared__ C prow[BW];     // the pivot row's block values
  __shared__ int bsw[BW];    // the block's pivot rows (swap c0 + j <-> bsw[j])
  __shared__ int src[2 * BW], dst[2 * BW];   // the block's composed row moves
  __shared__ int nmove;
  __shared__ C mv[NBMAX][2 * BW];            // staged values of the moves
  __shared__ C L11[BW][BW];  // the block rows' factors (unit lower part used)
  __shared__ C U12[BW][NBMAX];
  double pv_min = INFINITY, pv_max = 0.0;
  C x[RPT][BW];
  for (int c0 = 0; c0 < nbf; c0 += BW) {
    const int c1 = (c0 + BW < nbf) ? c0 + BW : nbf;
    const int bw = c1 - c0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = t + i * NT;
#pragma unroll
      for (int j = 0; j < BW; ++j) {
        const bool ok = r < R && j < bw;
        x[i][j] = c0 == 0 ? ld_or_zero(ok, F + (long long)(k + (ok ? r : 0)) + (long long)(k + j) * n)
                          : (ok ? P[r + (long long)(c0 + j) * R] : czero<C>());
      }
    }
    if (c0 == 0) __syncthreads();   // the copy is complete before any row swap
#pragma unroll
    for (int jc = 0; jc < BW; ++jc) {
      if (jc >= bw) break;
      const int c = c0 + jc;
      // arg max |P[r][c]|, r >= c (ties: smallest row): wave maxima to LDS,
      // then every thread reduces them (no second barrier)
      double best = -1.0;
      int bi = R;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = t + i * NT;
        if (r >= c && r < R) {
          const double v = cabs2(x[i][jc]);
          if (v > best) { best = v; bi = r; }
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_down(best, off);
        int oi = __shfl_down(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if ((t & 63) == 0) { red_v[t >> 6] = best; red_i[t >> 6] = bi; }
      __syncthreads();
      double bv = red_v[0];
      int p = red_i[0];
#pragma unroll
      for (int w = 1; w < NW; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < p)) {
          bv = red_v[w];
          p = red_i[w];
        }
      if (!(bv > 0.0) || !isfinite(bv)) {
        if (t == 0) atomicExch(&status->flag, 1);   // zero or non-finite pivot
        p = c;
      } else if (t == 0) {
        pv_min = fmin(pv_min, bv);
        pv_max = fmax(pv_max, bv);
      }
      if (t == 0) {
        ipiv[c] = p;
        bsw[jc] = p;
      }
      // rows c and p trade places: the pivot row's block values go to prow
      // (every thread reads them), row c's to xch (for row p's owner)
      const int tc = c % NT, ic = c / NT, tp = p % NT, ip = p / NT;
      if (t == tp)
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == ip)
#pragma unroll
            for (int j = 0; j < BW; ++j) prow[j] = x[i][j];
      if (t == tc && p != c)
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == ic)
#pragma unroll
            for (int j = 0; j < BW; ++j) xch[j] = x[i][j];
      __syncthreads();
      if (p != c) {
        if (t == tc)
#pragma unroll
          for (int i = 0; i < RPT; ++i)
            if (i == ic)
#pragma unroll
              for (int j = 0; j < BW; ++j) x[i][j] = prow[j];
        if (t == tp)
#pragma unroll
          for (int i = 0; i < RPT; ++i)
            if (i == ip)
#pragma unroll
              for (int j = 0; j < BW; ++j) x[i][j] = xch[j];
      }
      C piv = prow[jc];
      if (cabs2(piv) == 0.0) piv = cmake<C>(1.0, 0.0);
      const C ipv = cdiv(cmake<C>(1.0, 0.0), piv);
      // scale the column below the pivot, rank-1 update of the block's
      // remaining columns
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = t + i * NT;
        if (r > c && r < R) {
          const C l = cmul(x[i][jc], ipv);
          x[i][jc] = l;
#pragma unroll
          for (int j = 0; j < BW; ++j)
            if (j > jc && j < bw) cfms(x[i][j], l, prow[j]);
        }
      }
    }
    // the block's row swaps, composed into moves dst <- src (at most 2 BW
    // rows), applied at once to the columns outside the block and to the
    // row permutation: every value is loaded before any is stored
    if (t == 0) {
      // dst[q]: a touched row, src[q]: the row whose content ends there
      int m = 0;
      for (int j = 0; j < bw; ++j) {
        const int ra = c0 + j, rb = bsw[j];
        int qa = -1, qb = -1;
        for (int q = 0; q < m; ++q) {
          if (dst[q] == ra) qa = q;
          if (dst[q] == rb) qb = q;
        }
        if (qa < 0) { qa = m; dst[m] = ra; src[m] = ra; ++m; }
        if (qb < 0) { qb = m; dst[m] = rb; src[m] = rb; ++m; }
        const int y = src[qa];
        src[qa] = src[qb];
        src[qb] = y;
      }
      int nm = 0;
      for (int q = 0; q < m; ++q)
        if (src[q] != dst[q]) { dst[nm] = dst[q]; src[nm] = src[q]; ++nm; }
      nmove = nm;
    }
    __syncthreads();
    const int nm = nmove;
    if (nm > 0) {
      // through LDS: every moved value is read before any is written (all
      // of a thread's loads issued before its first LDS store)
      constexpr int MV = (NBMAX * 2 * BW + NT - 1) / NT;
      C mvv[MV];
#pragma unroll
      for (int i = 0; i < MV; ++i) {
        const int e = t + NT * i, cc = e / nm, q = e % nm;
        const bool ok = e < nbf * nm && (cc < c0 || cc >= c1);
        mvv[i] = ld_or_zero(ok, P + (ok ? src[q] + (long long)cc * R : 0));
      }
#pragma unroll
      for (int i = 0; i < MV; ++i) {
        const int e = t + NT * i, cc = e / nm, q = e % nm;
        if (e < nbf * nm && (cc < c0 || cc >= c1)) mv[cc][q] = mvv[i];
      }
      int pv = 0;
      if (t < nm) pv = perm[k + src[t]];
      __syncthreads();
      for (int e = t; e < nbf * nm; e += NT) {
        const int cc = e / nm, q = e % nm;
        if (cc < c0 || cc >= c1) P[dst[q] + (long long)cc * R] = mv[cc][q];
      }
      if (t < nm) perm[k + dst[t]] = pv;
    }
    // the block's columns back to the global copy; the block rows' factors
    // to LDS for the trailing solve
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = t + i * NT;
      if (r < R)
#pragma unroll
        for (int j = 0; j < BW; ++j)
          if (j < bw) P[r + (long long)(c0 + j) * R] = x[i][j];
      if (r >= c0 && r < c1)
#pragma unroll
        for (int j = 0; j < BW; ++j) L11[r - c0][j] = x[i][j];
    }
    __syncthreads();
    if (c1 >= nbf) break;
    const int W = nbf - c1;
    // block rows of the trailing columns: U12 = L11^-1 A12 (unit lower),
    // the column's block rows loaded together first
    for (int cc = t; cc < W; cc += NT) {
      const long long col = (long long)(c1 + cc) * R;
      C u[BW];
#pragma unroll
      for (int i = 0; i < BW; ++i) u[i] = i < bw ? P[c0 + i + col] : czero<C>();
#pragma unroll
      for (int i = 0; i < BW; ++i) {
        if (i >= bw) break;
        C y = u[i];
#pragma unroll
        for (int j = 0; j < BW; ++j)
          if (j < i) cfms(y, L11[i][j], u[j]);
        u[i] = y;
        U12[i][cc] = y;
        P[c0 + i + col] = y;
      }
    }
    __syncthreads();
    // rank-bw update of the trailing columns below the block (own rows):
    // a group of TG columns of all the thread's rows loaded before any of
    // their stores, so that RPT x TG loads are in flight per thread
    constexpr int TG = CG < (NT >= 1024 ? 16 : 32) / RPT ? CG : (NT >= 1024 ? 16 : 32) / RPT;
    for (int cg = 0; cg < W; cg += TG) {
      C y[RPT][TG];
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = t + i * NT;
        const bool ok = r >= c1 && r < R;
#pragma unroll
        for (int q = 0; q < TG; ++q) {
          const bool in = ok && cg + q < W;
          y[i][q] = ld_or_zero(in, P + (in ? r + (long long)(c1 + cg + q) * R : 0));
        }
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = t + i * NT;
        if (r < c1 || r >= R) continue;
#pragma unroll
        for (int q = 0; q < TG; ++q) {
          if (cg + q >= W) break;
#pragma unroll
          for (int j = 0; j < BW; ++j)
            if (j < bw) cfms(y[i][q], x[i][j], U12[j][cg + q]);
          P[r + (long long)(c1 + cg + q) * R] = y[i][q];
        }
      }
    }
    __syncthreads();
  }
  if (t == 0 && pv_max > 0.0) {
    atomicMin(&status->pmin, (unsigned long long)__double_as_longlong(pv_min));
    atomicMax(&status->pmax, (unsigned long long)__double_as_longlong(pv_max));
  }
  panel_inverse<T, NT, false>(P, R, nbf, nb, D);
}

// --------------------------------------------------------------------------
// apply the nbf row swaps to every column, then rows J <- D * rows J for the
// columns outside J.  One workgroup per 64-column tile.
// The swaps are composed first (one wave, in registers): row k + jj of J
// ends up holding old row srcJ[jj], and each row outside J that a swap
// touches (at most nbf of them) holds old row srcO[i].  Every new value is
// then one independent load, so the column tile is read once, in parallel,
// instead of through nbf dependent swaps per column.
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
  __shared__ int srcJ[NBMAX], rowO[NBMAX], srcO[NBMAX];
  __shared__ int nO;
  __shared__ C V[NBMAX][GT + 1];
  __shared__ C DsT[NBMAX][NBMAX + 1];  // DsT[q][r] = D(r, q)
  if (t < 64) {
    // lane i holds srcJ[i] and outside entry i (row ro, source so)
    int vJ = k + t, ro = -1, so = 0, cnt = 0;
    const int piv = ld(ipiv + (t < nbf ? t : 0));
    for (int jj = 0; jj < nbf; ++jj) {
      const int r2 = k + __builtin_amdgcn_readlane(piv, jj);
      const int cur = __builtin_amdgcn_readlane(vJ, jj);
      if (r2 < k + nbf) {
        const int other = __builtin_amdgcn_readlane(vJ, r2 - k);
        if (t == jj) vJ = other;
        if (t == r2 - k) vJ = cur;
      } else {
        const unsigned long long hit = __ballot(ro == r2);
        if (hit) {
          const int i = __ffsll((long long)hit) - 1;
          const int other = __builtin_amdgcn_readlane(so, i);
          if (t == jj) vJ = other;
          if (t == i) so = cur;
        } else {
          if (t == jj) vJ = r2;
          if (t == cnt) { ro = r2; so = cur; }
          ++cnt;
        }
      }
    }
    if (t < nbf) srcJ[t] = vJ;
    if (t < cnt) { rowO[t] = ro; srcO[t] = so; }
    if (t == 0) nO = cnt;
  }
  __syncthreads();
  const int no = nO;
  // every read of the tile before any write
  constexpr int WPT = NBMAX * GT / 256;
  C w[WPT];
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int e = t + 256 * i, r = e / GT, gc = c0 + e % GT;
    const bool ok = r < no && gc < n;
    w[i] = ld_or_zero(ok, F + (ok ? (long long)srcO[r] + (long long)gc * n : 0));
  }
  // the rows J of the tile and D: every load issued before the first store
  C vj[WPT], dw[WPT];
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int e = t + 256 * i, r = e % NBMAX, c = e / NBMAX, gc = c0 + c;
    const bool ok = r < nbf && gc < n;
    vj[i] = ld_or_zero(ok, F + (ok ? (long long)srcJ[r] + (long long)gc * n : 0));
    const bool dok = r < nbf && c < nbf;
    dw[i] = ld_or_zero(dok, D + (dok ? r + c * nb : 0));
  }
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int e = t + 256 * i, r = e % NBMAX, c = e / NBMAX;
    V[r][c] = vj[i];
    DsT[c][r] = dw[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int e = t + 256 * i, r = e / GT, gc = c0 + e % GT;
    if (r < no && gc < n) st(F + (long long)rowO[r] + (long long)gc * n, w[i]);
  }
  // rows J of the tile: thread (rg, cg) owns rows rg + 16 i and columns
  // cg + 16 j (i, j < 4), so each LDS value read feeds four products
  const int rg = t & 15, cg = t >> 4;
  C acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = czero<C>();
  for (int q = 0; q < nbf; ++q) {
    C dv[4], vv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) dv[i] = DsT[q][rg + 16 * i];
#pragma unroll
    for (int j = 0; j < 4; ++j) vv[j] = V[q][cg + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) cfma(acc[i][j], dv[i], vv[j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rg + 16 * i, c = cg + 16 * j, gc = c0 + c;
      if (r >= nbf || gc >= n) continue;
      const bool inJ = gc >= k && gc < k + nbf;
      st(F + (long long)(k + r) + (long long)gc * n, inJ ? V[r][c] : acc[i][j]);
    }
}

// --------------------------------------------------------------------------
// rank-nb update of every entry outside the pivot rows / columns J:
//   F(O, O) -= F(O, J) F(J, O)     (J rows already hold D * F(J, O))
// Computed as C^T = B^T A^T so that the MFMA column index walks the
// contiguous (row) dimension of the column-major front.  Entries of rows
// already eliminated (< k) in boundary columns (>= s) are skipped: they
// would accumulate F11^-1 F12, which neither the factor store (the
// symmetric operator's backward step uses the transpose of -F21 F11^-1) nor
// the parent's extend-add (the Schur block) ever reads.  Tiles that lie
// wholly in J or in that block return at once.
// --------------------------------------------------------------------------
template <typename T, bool M3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (M3 ? 3 : 4) : 1, 8)))
k_sweep_gemm(const FrontDev* __restrict__ fronts, const int* __restrict__ ids,
             int n_active, const int2* __restrict__ tmap, int k, int nb,
             void* ws0, void* ws1) {
  using C = C_t<T>;
  __shared__ GemmSmem<T, 64, 64, false, M3> sm;
  const int2 tm = tmap[blockIdx.x];
  const int a = tm.x;
  const FrontDev f = fronts[ids[a]];
  const int n = f.s + f.b;
  const int nbf = (f.s - k) < nb ? (f.s - k) : nb;
  const int nt = (n + GT - 1) / GT;
  const int tile = tm.y;
  const int i0 = (tile % nt) * GT;   // rows of F
  const int j0 = (tile / nt) * GT;   // columns of F
  const bool rowsJ = i0 >= k && i0 + GT <= k + nbf, colsJ = j0 >= k && j0 + GT <= k + nbf;
  if (rowsJ || colsJ || (i0 + GT <= k && j0 >= f.s)) return;   // uniform per block
  C* F = front_ptr<T>(ws0, ws1, f);
  // P rows = C columns j: B^T(j, q) = F[(k+q) + j n]
  View<T> pv{F + k, (long long)n, 1, n, nbf};
  // Q columns = C rows i: A^T(q, i) = F[i + (k+q) n]
  View<T> qv{F + (long long)k * n, 1, (long long)n, n, nbf};
  WaveAcc<T, 64, 64, M3> acc;
  gemm_tile<T, 64, false, true>(sm, acc, pv, qv, j0, i0, 0, nbf);
  // F(i, j) -= acc: every entry of the lane is loaded before the first store
  // (one latency for the group instead of a load-store chain per entry)
  using O = LaneOut<T, 64, 64>;
  const O o;
  auto outside = [&](int gi, int gj) {
    return gi < n && gj < n && (gi < k || gi >= k + nbf) && (gj < k || gj >= k + nbf) &&
           !(gi < k && gj >= f.s);
  };
  C cv[O::NR][O::NC];
#pragma unroll
  for (int i = 0; i < O::NR; ++i)
#pragma unroll
    for (int j = 0; j < O::NC; ++j) {
      const int gi = i0 + o.c[j], gj = j0 + o.r[i];
      cv[i][j] = ld_or_zero(outside(gi, gj), F + (long long)gi + (long long)gj * n);
    }
#pragma unroll
  for (int i = 0; i < O::NR; ++i)
#pragma unroll
    for (int j = 0; j < O::NC; ++j) {
      const int gi = i0 + o.c[j], gj = j0 + o.r[i];
      if (outside(gi, gj))
        st(F + (long long)gi + (long long)gj * n, csub(cv[i][j], acc_at(acc, i, j)));
    }
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
  // every load of the tile and of D issued before the first LDS store
  constexpr int WPT = NBMAX * GT / 256;
  C w[WPT], dw[WPT];
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int e = t + 256 * i, r = e % GT, c = e / GT;
    const bool ok = r0 + r < n && c < nbf;
    w[i] = ld_or_zero(ok, F + (ok ? (long long)(r0 + r) + (long long)(k + c) * n : 0));
    const int dr = e % NBMAX, dc = e / NBMAX;
    const bool dok = dr < nbf && dc < nbf;
    dw[i] = ld_or_zero(dok, D + (dok ? dr + dc * nb : 0));
  }
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    const int e = t + 256 * i;
    V[e % GT][e / GT] = w[i];
    Ds[e % NBMAX][e / NBMAX] = dw[i];
  }
  __syncthreads();
  // thread (rg, cg) owns rows rg + 16 i and columns cg + 16 j (i, j < 4)
  const int rg = t & 15, cg = t >> 4;
  C acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = czero<C>();
  for (int q = 0; q < nbf; ++q) {
    C vv[4], dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) vv[i] = V[rg + 16 * i][q];
#pragma unroll
    for (int j = 0; j < 4; ++j) dv[j] = Ds[q][cg + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) cfma(acc[i][j], vv[i], dv[j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rg + 16 * i, c = cg + 16 * j, gr = r0 + r;
      if (gr >= n || c >= nbf) continue;
      const bool inJ = gr >= k && gr < k + nbf;
      st(F + (long long)gr + (long long)(k + c) * n, inJ ? Ds[gr - k][c] : cneg(acc[i][j]));
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
                         void* ws0, void* ws1, const GridDev& g, int skip_front,
                         FactorStatus* status, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_orig_entries<T>, dim3(total), dim3(256), 0, st, fronts, ids,
                     n_ids, tmap, layers, ws0, ws1, g, skip_front, status);
}
template <typename T>
void launch_panel(const FrontDev* fronts, const int* ids, int n_active, int max_rows,
                  int k, int nb, void* ws0, void* ws1, void* panel,
                  const long long* panel_off, void* D, int* ipiv, int* perm,
                  const long long* perm_off, FactorStatus* status, hipStream_t st) {
  if (n_active <= 0) return;
  // threads and panel home from the tallest panel of the launch
#define HELM_PANEL(NT, PR)                                                          \
  hipLaunchKernelGGL((k_panel<T, NT, PR>), dim3(n_active), dim3(NT), 0, st,        \
                     fronts, ids, k, nb, ws0, ws1, panel, panel_off, D, ipiv, perm, \
                     perm_off, status)
#define HELM_PANEL_RB(NT, RPT, BW)                                                  \
  hipLaunchKernelGGL((k_panel_rb<T, NT, RPT, BW>), dim3(n_active), dim3(NT), 0, st, \
                     fronts, ids, k, nb, ws0, ws1, panel, panel_off, D, ipiv, perm, \
                     perm_off, status)
  // complex64 up to 512 rows: a row per thread, the panel in registers;
  // taller than the LDS holds: the column block in registers, 4 rows per
  // thread at most (complex128 at 512 threads: at 1024 a lane's register
  // share of 128 would spill), else the global copy alone
  constexpr bool C64 = sizeof(T) == 4;
#define HELM_PANEL_REGS(NW)                                                         \
  hipLaunchKernelGGL((k_panel_regs<T, NW>), dim3(n_active), dim3(64 * NW), 0, st,  \
                     fronts, ids, k, nb, ws0, ws1, D, ipiv, perm, perm_off, panel_off, status)
  if constexpr (C64) {
    if (max_rows <= 512) {
      if (max_rows <= 64) HELM_PANEL_REGS(1);
      else if (max_rows <= 128) HELM_PANEL_REGS(2);
      else if (max_rows <= 192) HELM_PANEL_REGS(3);
      else if (max_rows <= 256) HELM_PANEL_REGS(4);
      else HELM_PANEL_REGS(8);
      return;
    }
  }
  if (max_rows <= 64) HELM_PANEL(64, 64);
  else if (max_rows <= panel_lds_rows<T>()) HELM_PANEL(256, panel_lds_rows<T>());
  else if (max_rows <= 1024) HELM_PANEL_RB(256, 4, PB);
  else if constexpr (C64) {
    if (max_rows <= 2048) HELM_PANEL_RB(1024, 2, PB);
    else if (max_rows <= 4096) HELM_PANEL_RB(1024, 4, PB);
    else if (max_rows <= 6144) HELM_PANEL_RB(1024, 6, PB / 2);
    else HELM_PANEL(1024, 0);
  } else {
    if (max_rows <= 2048) HELM_PANEL_RB(512, 4, PB);
    else HELM_PANEL(1024, 0);
  }
#undef HELM_PANEL_REGS
#undef HELM_PANEL_RB
#undef HELM_PANEL
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
                       void* ws1, bool m3, hipStream_t st) {
  if (total <= 0) return;
  constexpr bool C64 = sizeof(T) == 4;   // the three-product form is for complex64
  if (C64 && m3)
    hipLaunchKernelGGL((k_sweep_gemm<T, C64>), dim3(total), dim3(256), 0, st, fronts, ids,
                       n_active, tmap, k, nb, ws0, ws1);
  else
    hipLaunchKernelGGL((k_sweep_gemm<T, false>), dim3(total), dim3(256), 0, st, fronts, ids,
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
                                       void*, const GridDev&, int, FactorStatus*,   \
                                       hipStream_t);                                \
  template void launch_panel<T>(const FrontDev*, const int*, int, int, int, int, void*, \
                                void*, void*, const long long*, void*, int*, int*, \
                                const long long*, FactorStatus*, hipStream_t);     \
  template void launch_swap_JO<T>(const FrontDev*, const int*, int, const int2*,    \
                                  int, int, int, void*, void*, const void*,        \
                                  const int*, const long long*, const long long*,  \
                                  hipStream_t);                                    \
  template void launch_sweep_gemm<T>(const FrontDev*, const int*, int, const int2*, \
                                     int, int, int, void*, void*, bool, hipStream_t); \
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
