// Volume, interface-trace and Krylov kernels of the online stage.
//
//  * source partition f^l = f chi_l (Algorithm 2) and the volume
//    reconstruction (the last step of Algorithm 2) between the global grid (RHS-major, FP64)
//    and a layer's solve vector (ND order, columns fastest, working precision);
//  * interface sources: the plane deltas of Section "Formulation" scaled to
//    this discretisation (coefficient B = 1/(h^2 beta_x beta_y), the matrix
//    coupling across an interior interface):
//      top of layer l:    -B a on plane s_l,  +B b on plane s_l - 1,
//      bottom of layer l: -B b on plane e_l,  +B a on plane e_l + 1,
//    and the trace read-outs of two planes (Algorithms 3-10);
//  * FP64 column-batched BLAS-1 for GMRES on the interface system;
//  * the FP64 residual f - H u of the global 7-point operator.
// Interface pair vectors use the layout [plane a|b][y][x][column], FP64.
#include "kernels.h"
#include "kernels_common.h"

namespace helm {
namespace kern {

namespace {

// Volume <-> layer copies of the bulk planes [s, e] for a few columns: one
// element per thread, consecutive threads on consecutive nodes.
template <typename T>
__global__ void k_scatter_flat(LayerDev L, const double2* __restrict__ f, int nx, int ny,
                               long long N, int k) {
  using C = C_t<T>;
  const long long plane = (long long)nx * ny;
  const long long nb = plane * (L.e - L.s + 1);
  C* X = reinterpret_cast<C*>(L.X);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nb * k;
       e += (long long)gridDim.x * blockDim.x) {
    const long long sp = e % nb;
    const int c = (int)(e / nb);
    X[(long long)L.nat2nd[sp + plane * (L.s - L.lo)] * k + c] =
        from_d2<C>(f[(long long)c * N + sp + plane * L.s]);
  }
}
template <typename T>
__global__ void k_gather_flat(LayerDev L, double2* __restrict__ u, int nx, int ny,
                              long long N, int k) {
  using C = C_t<T>;
  const long long plane = (long long)nx * ny;
  const long long nb = plane * (L.e - L.s + 1);
  const C* X = reinterpret_cast<const C*>(L.X);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nb * k;
       e += (long long)gridDim.x * blockDim.x) {
    const long long sp = e % nb;
    const int c = (int)(e / nb);
    u[(long long)c * N + sp + plane * L.s] =
        to_d2(X[(long long)L.nat2nd[sp + plane * (L.s - L.lo)] * k + c]);
  }
}

// The same copies for many columns, as tiles of 64 nodes x
// 64 columns staged in LDS: f and u hold each column contiguously over the
// nodes, X holds each node's k values contiguously, so both sides are read
// or written along their contiguous direction.  Grid: (node tiles, column
// tiles); wave w of the block handles tile rows w, w + 4, ...
constexpr int VT = 64;
constexpr int RESID_COLS = 8;   // columns per block row of k_residual

template <typename T>
__global__ void __launch_bounds__(256)
k_scatter_source(LayerDev L, const double2* __restrict__ f, int nx, int ny, long long N, int k) {
  using C = C_t<T>;
  __shared__ C tile[VT][VT + 1];   // [node][column]
  const long long plane = (long long)nx * ny;
  const long long nb = plane * (L.e - L.s + 1);
  const long long n0 = (long long)blockIdx.x * VT;
  const int c0 = blockIdx.y * VT, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  C* X = reinterpret_cast<C*>(L.X);
  {
    const long long sp = n0 + lane;
#pragma unroll
    for (int j = 0; j < VT / 4; ++j) {
      const int c = w + 4 * j;
      const bool ok = sp < nb && c0 + c < k;
      tile[lane][c] = from_d2<C>(ld_or_zero(ok, f + (ok ? (long long)(c0 + c) * N + sp + plane * L.s : 0)));
    }
  }
  __syncthreads();
  long long dst[VT / 4];
#pragma unroll
  for (int j = 0; j < VT / 4; ++j) {
    const long long sp = n0 + w + 4 * j;
    dst[j] = sp < nb ? (long long)ld(L.nat2nd + sp + plane * (L.s - L.lo)) * k : -1;
  }
  if (c0 + lane < k)
#pragma unroll
    for (int j = 0; j < VT / 4; ++j)
      if (dst[j] >= 0) st(X + dst[j] + c0 + lane, tile[w + 4 * j][lane]);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_gather_volume(LayerDev L, double2* __restrict__ u, int nx, int ny, long long N, int k) {
  using C = C_t<T>;
  __shared__ C tile[VT][VT + 1];   // [node][column]
  const long long plane = (long long)nx * ny;
  const long long nb = plane * (L.e - L.s + 1);
  const long long n0 = (long long)blockIdx.x * VT;
  const int c0 = blockIdx.y * VT, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const C* X = reinterpret_cast<const C*>(L.X);
  long long src[VT / 4];
#pragma unroll
  for (int j = 0; j < VT / 4; ++j) {
    const long long sp = n0 + w + 4 * j;
    src[j] = sp < nb ? (long long)ld(L.nat2nd + sp + plane * (L.s - L.lo)) * k : -1;
  }
#pragma unroll
  for (int j = 0; j < VT / 4; ++j) {
    const bool ok = src[j] >= 0 && c0 + lane < k;
    tile[w + 4 * j][lane] = ld_or_zero(ok, X + (ok ? src[j] + c0 + lane : 0));
  }
  __syncthreads();
  const long long sp = n0 + lane;
  if (sp < nb)
#pragma unroll
    for (int j = 0; j < VT / 4; ++j) {
      const int c = w + 4 * j;
      if (c0 + c < k) u[(long long)(c0 + c) * N + sp + plane * L.s] = to_d2(tile[lane][c]);
    }
}

// whole extended layer, natural order <-> ND order (inspection entry point)
template <typename T>
__global__ void k_local_to_X(LayerDev L, const double2* __restrict__ r, int k) {
  using C = C_t<T>;
  C* X = reinterpret_cast<C*>(L.X);
  const long long total = (long long)L.n_loc * k;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long sp = e % L.n_loc;
    const int c = (int)(e / L.n_loc);
    X[(long long)L.nat2nd[sp] * k + c] = from_d2<C>(r[e]);
  }
}
template <typename T>
__global__ void k_X_to_local(LayerDev L, double2* __restrict__ w, int k) {
  using C = C_t<T>;
  const C* X = reinterpret_cast<const C*>(L.X);
  const long long total = (long long)L.n_loc * k;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long sp = e % L.n_loc;
    const int c = (int)(e / L.n_loc);
    w[e] = to_d2(X[(long long)L.nat2nd[sp] * k + c]);
  }
}

// add the interface source of a pair (a, b) = c0 in0 + c1 in1 + c2 in2 (in1
// and in2 may be null)
template <typename T>
__global__ void k_jump(LayerDev L, JumpTerms t, const double2* __restrict__ B, int bottom,
                       int nx, int ny, int k) {
  using C = C_t<T>;
  C* X = reinterpret_cast<C*>(L.X);
  const long long plane = (long long)nx * ny;
  const long long total = plane * k;
  // planes (global): top: a -> s (coef -B), b -> s - 1 (+B)
  //                  bottom: b -> e (-B), a -> e + 1 (+B)
  const int za = bottom ? L.e + 1 : L.s;
  const int zb = bottom ? L.e : L.s - 1;
  const double sa = bottom ? 1.0 : -1.0;
  const double sb = bottom ? -1.0 : 1.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long sp = e / k;
    const int c = (int)(e % k);
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (!t.in[i]) continue;
      const double2 ai = t.in[i][e], bi = t.in[i][e + total];
      a.x += t.c[i] * ai.x; a.y += t.c[i] * ai.y;
      b.x += t.c[i] * bi.x; b.y += t.c[i] * bi.y;
    }
    const double2 cf = B[sp];
    const double2 va = make_double2(sa * (cf.x * a.x - cf.y * a.y), sa * (cf.x * a.y + cf.y * a.x));
    const double2 vb = make_double2(sb * (cf.x * b.x - cf.y * b.y), sb * (cf.x * b.y + cf.y * b.x));
    const long long ia = L.nat2nd[sp + plane * (za - L.lo)];
    const long long ib = L.nat2nd[sp + plane * (zb - L.lo)];
    C& xa = X[ia * k + c];
    xa = cadd(xa, from_d2<C>(va));
    C& xb = X[ib * k + c];
    xb = cadd(xb, from_d2<C>(vb));
  }
}

template <typename T>
__global__ void k_readout(LayerDev L, int bottom, double sx, ReadTerms terms,
                          double2* __restrict__ out, int nx, int ny, int k) {
  using C = C_t<T>;
  const C* X = reinterpret_cast<const C*>(L.X);
  const long long plane = (long long)nx * ny;
  const long long total = plane * k;
  // R_top = (w(s - 1), w(s)),  R_bot = (w(e), w(e + 1))
  const int z0 = bottom ? L.e : L.s - 1;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < 2 * total;
       e += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(e / total);
    if (!((terms.planes >> p) & 1)) continue;
    const long long r = e % total;
    const long long sp = r / k;
    const int c = (int)(r % k);
    double2 v = make_double2(0.0, 0.0);
    if (sx != 0.0) {
      const long long idx = L.nat2nd[sp + plane * (z0 + p - L.lo)];
      double2 x = to_d2(X[idx * k + c]);
      v.x = sx * x.x;
      v.y = sx * x.y;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (!terms.in[i]) continue;
      const double cf = p ? terms.cb[i] : terms.ca[i];
      if (cf == 0.0) continue;
      const double2 y = terms.in[i][e];
      v.x += cf * y.x;
      v.y += cf * y.y;
    }
    out[e] = v;
  }
}

// ----------------------------------------------------------------------------
// FP64 column-batched vector kernels; vectors are V x k with k fastest.
// ----------------------------------------------------------------------------
constexpr int DOT_COLS = 32, DOT_ROWS = 8, DOT_BLOCKS = 256;

// partial[c][blk] = sum_v conj(x[v, c]) y[v, c] over this block's rows
__global__ void __launch_bounds__(256)
k_dot_partial(const double2* __restrict__ x, const double2* __restrict__ y,
              long long V, int k, double2* __restrict__ partial) {
  const int tx = threadIdx.x % DOT_COLS, ty = threadIdx.x / DOT_COLS;
  const int c = blockIdx.y * DOT_COLS + tx;
  double re = 0, im = 0;
  if (c < k) {
    for (long long v = blockIdx.x * DOT_ROWS + ty; v < V; v += (long long)gridDim.x * DOT_ROWS) {
      const double2 a = x[v * k + c], b = y[v * k + c];
      re += a.x * b.x + a.y * b.y;
      im += a.x * b.y - a.y * b.x;
    }
  }
  __shared__ double sre[DOT_ROWS][DOT_COLS], sim[DOT_ROWS][DOT_COLS];
  sre[ty][tx] = re;
  sim[ty][tx] = im;
  __syncthreads();
  if (ty == 0 && c < k) {
    for (int q = 1; q < DOT_ROWS; ++q) { re += sre[q][tx]; im += sim[q][tx]; }
    partial[(long long)c * gridDim.x + blockIdx.x] = make_double2(re, im);
  }
}

// out[c] = sum over blocks (fixed order, reproducible)
__global__ void k_dot_final(const double2* __restrict__ partial, int nblk, int k,
                            double2* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double re = 0, im = 0;
  for (int b = 0; b < nblk; ++b) {
    re += partial[(long long)c * nblk + b].x;
    im += partial[(long long)c * nblk + b].y;
  }
  out[c] = make_double2(re, im);
}

// y[v, c] += sign * alpha[c] * x[v, c]     (alpha per column, complex)
__global__ void k_axpy_cols(double2* __restrict__ y, const double2* __restrict__ x,
                            const double2* __restrict__ alpha, double sign,
                            long long V, int k) {
  const long long total = V * k;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % k);
    const double2 a = alpha[c], b = x[e];
    double2 o = y[e];
    o.x += sign * (a.x * b.x - a.y * b.y);
    o.y += sign * (a.x * b.y + a.y * b.x);
    y[e] = o;
  }
}

// y[v, c] = x[v, c] * s[c]  (s real, per column); y may be x (each element
// is read and written by one thread), so y and x are not restrict
__global__ void k_scale_cols(double2* y, const double2* x, const double* __restrict__ s,
                             long long V, int k) {
  const long long total = V * k;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const double a = s[e % k];
    const double2 b = x[e];
    y[e] = make_double2(a * b.x, a * b.y);
  }
}

// the columns map.col[0..m) of an interleaved batch of k into a batch of w
__global__ void k_gather_cols(double2* __restrict__ out, const double2* __restrict__ in,
                              long long V, int k, int w, int m, ColMap map) {
  const long long total = V * w;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long e = i / w;
    const int j = (int)(i % w);
    out[i] = j < m ? in[e * k + map.col[j]] : make_double2(0.0, 0.0);
  }
}

// back: column c of the batch of k from slot slot.col[c] of the batch of w
__global__ void k_scatter_cols(double2* __restrict__ out, const double2* __restrict__ in,
                               long long V, int k, int w, ColMap slot) {
  const long long total = V * k;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long e = i / k;
    const int s = slot.col[i % k];
    out[i] = s >= 0 ? in[e * w + s] : make_double2(0.0, 0.0);
  }
}

// y = x + z (elementwise); y may be x or z
__global__ void k_add(double2* y, const double2* x, const double2* z, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    y[e] = make_double2(x[e].x + z[e].x, x[e].y + z[e].y);
  }
}

// y[v, c] = x[v, c] + alpha[c] y[v, c]   (alpha per column, complex)
__global__ void k_xpay_cols(double2* __restrict__ y, const double2* __restrict__ x,
                            const double2* __restrict__ alpha, long long V, int k) {
  const long long total = V * k;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const double2 a = alpha[e % k], b = y[e], c = x[e];
    y[e] = make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
  }
}

// y = z - y in place: each element is read and written by one thread, so y
// is the only pointer that aliases nothing else
__global__ void k_rsub(double2* y, const double2* __restrict__ z, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double2 a = y[e], b = z[e];
    y[e] = make_double2(b.x - a.x, b.y - a.y);
  }
}

// FP64 residual r = f - H u on the global grid (volumes RHS-major); f may be
// null (then r = H u).  Same operator as the local assembly.
__global__ void __launch_bounds__(256)
k_residual(GridDev g, const double2* __restrict__ f, const double2* __restrict__ u,
           double2* __restrict__ r, int k) {
  // one node per thread and RESID_COLS columns per block row: the node's
  // stencil coefficients are formed once for all of its columns
  const long long N = (long long)g.nx * g.ny * g.nz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  const double ih2 = 1.0 / (g.h * g.h);
  const int x = (int)(idx % g.nx);
  const int y = (int)((idx / g.nx) % g.ny);
  const int z = (int)(idx / ((long long)g.nx * g.ny));
  const double2 bx = g.bx[x], by = g.by[y], bz = g.bz[z];
  auto mul = [](double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  };
  const double2 bxy = mul(bx, by), bxz = mul(bx, bz), byz = mul(by, bz);
  double2 cp[6];
  cp[0] = cdiv(g.bxh[x], byz);
  cp[1] = cdiv(g.bxh[x + 1], byz);
  cp[2] = cdiv(g.byh[y], bxz);
  cp[3] = cdiv(g.byh[y + 1], bxz);
  cp[4] = cdiv(g.bzh[z], bxy);
  cp[5] = cdiv(g.bzh[z + 1], bxy);
  const double2 dg = cdiv(make_double2(g.omega * g.omega * g.m[idx], 0.0), mul(bxy, bz));
  const long long st[6] = {-1, 1, -(long long)g.nx, (long long)g.nx,
                           -(long long)g.nx * g.ny, (long long)g.nx * g.ny};
  const bool ok[6] = {x > 0, x < g.nx - 1, y > 0, y < g.ny - 1, z > 0, z < g.nz - 1};
  const int cend = min(k, (int)(blockIdx.y + 1) * RESID_COLS);
  for (int c = blockIdx.y * RESID_COLS; c < cend; ++c) {
    const double2* uc = u + (long long)c * N;
    const double2 u0 = uc[idx];
    double2 acc = mul(dg, u0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      double2 nb = ok[q] ? uc[idx + st[q]] : make_double2(0.0, 0.0);
      double2 d = make_double2((nb.x - u0.x) * ih2, (nb.y - u0.y) * ih2);
      double2 t = mul(cp[q], d);
      acc.x += t.x;
      acc.y += t.y;
    }
    const long long e = (long long)c * N + idx;
    double2 out;
    if (f) out = make_double2(f[e].x - acc.x, f[e].y - acc.y);
    else out = acc;
    r[e] = out;
  }
}


// point sources: f[c * N + node[c]] = amp[c] / h^3 (f zeroed before)
__global__ void k_point_sources(double2* __restrict__ f, const long long* __restrict__ node,
                                const double2* __restrict__ amp, double inv_h3,
                                long long N, int k) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  f[(long long)c * N + node[c]] = make_double2(amp[c].x * inv_h3, amp[c].y * inv_h3);
}

// u[c] += d[c]  over volumes (refinement update)
__global__ void k_accumulate(double2* __restrict__ u, const double2* __restrict__ d,
                             long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    u[e] = make_double2(u[e].x + d[e].x, u[e].y + d[e].y);
  }
}

// per-column squared norms of RHS-major volumes: out[c] = sum |x|^2
__global__ void __launch_bounds__(256)
k_volume_norm2(const double2* __restrict__ x, long long N, int k,
               double* __restrict__ partial) {
  const int c = blockIdx.y;
  double s = 0;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < N; e += (long long)gridDim.x * 256) {
    const double2 v = x[(long long)c * N + e];
    s += v.x * v.x + v.y * v.y;
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long long)c * gridDim.x + blockIdx.x] = red[0];
}
__global__ void k_norm_final(const double* __restrict__ partial, int nblk, int k,
                             double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += partial[(long long)c * nblk + b];
  out[c] = s;
}

inline int grid_for(long long n, int block = 256) {
  long long g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------
template <typename T>
void launch_scatter_source(const LayerDev& L, const double2* f, int nx, int ny,
                           long long N, int k, hipStream_t st) {
  const long long nb = (long long)nx * ny * (L.e - L.s + 1);
  if (nb <= 0 || k <= 0) return;
  if (k <= 8) {   // a 64-column tile would leave most lanes idle
    hipLaunchKernelGGL(k_scatter_flat<T>, dim3(grid_for(nb * k)), dim3(256), 0, st, L, f, nx, ny, N, k);
    return;
  }
  const dim3 grid((unsigned)((nb + VT - 1) / VT), (unsigned)((k + VT - 1) / VT));
  hipLaunchKernelGGL(k_scatter_source<T>, grid, dim3(256), 0, st, L, f, nx, ny, N, k);
}
template <typename T>
void launch_gather_volume(const LayerDev& L, double2* u, int nx, int ny,
                          long long N, int k, hipStream_t st) {
  const long long nb = (long long)nx * ny * (L.e - L.s + 1);
  if (nb <= 0 || k <= 0) return;
  if (k <= 8) {   // a 64-column tile would leave most lanes idle
    hipLaunchKernelGGL(k_gather_flat<T>, dim3(grid_for(nb * k)), dim3(256), 0, st, L, u, nx, ny, N, k);
    return;
  }
  const dim3 grid((unsigned)((nb + VT - 1) / VT), (unsigned)((k + VT - 1) / VT));
  hipLaunchKernelGGL(k_gather_volume<T>, grid, dim3(256), 0, st, L, u, nx, ny, N, k);
}
template <typename T>
void launch_local_to_X(const LayerDev& L, const double2* r, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_local_to_X<T>, dim3(grid_for((long long)L.n_loc * k)), dim3(256),
                     0, st, L, r, k);
}
template <typename T>
void launch_X_to_local(const LayerDev& L, double2* w, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_X_to_local<T>, dim3(grid_for((long long)L.n_loc * k)), dim3(256),
                     0, st, L, w, k);
}
template <typename T>
void launch_jump(const LayerDev& L, const JumpTerms& t, const double2* B, int bottom, int nx,
                 int ny, int k, hipStream_t st) {
  long long n = (long long)nx * ny * k;
  hipLaunchKernelGGL(k_jump<T>, dim3(grid_for(n)), dim3(256), 0, st, L, t, B, bottom, nx,
                     ny, k);
}
template <typename T>
void launch_readout(const LayerDev& L, int bottom, double sx, const ReadTerms& terms,
                    double2* out, int nx, int ny, int k, hipStream_t st) {
  long long n = 2LL * nx * ny * k;
  hipLaunchKernelGGL(k_readout<T>, dim3(grid_for(n)), dim3(256), 0, st, L, bottom, sx,
                     terms, out, nx, ny, k);
}

void launch_dot(const double2* x, const double2* y, long long V, int k,
                double2* partial, double2* out, hipStream_t st) {
  dim3 grid(DOT_BLOCKS, (k + DOT_COLS - 1) / DOT_COLS);
  hipLaunchKernelGGL(k_dot_partial, grid, dim3(256), 0, st, x, y, V, k, partial);
  hipLaunchKernelGGL(k_dot_final, dim3((k + 63) / 64), dim3(64), 0, st, partial,
                     DOT_BLOCKS, k, out);
}
void launch_axpy_cols(double2* y, const double2* x, const double2* alpha,
                      double sign, long long V, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_cols, dim3(grid_for(V * k)), dim3(256), 0, st, y, x, alpha,
                     sign, V, k);
}
void launch_gather_cols(double2* out, const double2* in, long long V, int k, int w, int m,
                        const ColMap& map, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(V * w)), dim3(256), 0, st, out, in, V, k, w,
                     m, map);
}
void launch_scatter_cols(double2* out, const double2* in, long long V, int k, int w,
                         const ColMap& slot, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_cols, dim3(grid_for(V * k)), dim3(256), 0, st, out, in, V, k, w,
                     slot);
}
void launch_scale_cols(double2* y, const double2* x, const double* s, long long V,
                       int k, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(V * k)), dim3(256), 0, st, y, x, s, V,
                     k);
}
void launch_add(double2* y, const double2* x, const double2* z, long long n,
                hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(256), 0, st, y, x, z, n);
}
void launch_xpay_cols(double2* y, const double2* x, const double2* alpha, long long V, int k,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_xpay_cols, dim3(grid_for(V * k)), dim3(256), 0, st, y, x, alpha, V, k);
}
void launch_rsub(double2* y, const double2* z, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_rsub, dim3(grid_for(n)), dim3(256), 0, st, y, z, n);
}
void launch_residual(const GridDev& g, const double2* f, const double2* u,
                     double2* r, int k, hipStream_t st) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  if (N <= 0 || k <= 0) return;
  const dim3 grid((unsigned)((N + 255) / 256), (unsigned)((k + RESID_COLS - 1) / RESID_COLS));
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, st, g, f, u, r, k);
}
void launch_point_sources(double2* f, const long long* node, const double2* amp,
                          double inv_h3, long long N, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_point_sources, dim3((k + 63) / 64), dim3(64), 0, st, f, node,
                     amp, inv_h3, N, k);
}
void launch_accumulate(double2* u, const double2* d, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for(n)), dim3(256), 0, st, u, d, n);
}
void launch_volume_norm2(const double2* x, long long N, int k, double* partial,
                         double* out, hipStream_t st) {
  const int nblk = 128;
  hipLaunchKernelGGL(k_volume_norm2, dim3(nblk, k), dim3(256), 0, st, x, N, k, partial);
  hipLaunchKernelGGL(k_norm_final, dim3((k + 63) / 64), dim3(64), 0, st, partial, nblk,
                     k, out);
}

#define HELM_INST_VOL(T)                                                             \
  template void launch_scatter_source<T>(const LayerDev&, const double2*, int, int,  \
                                         long long, int, hipStream_t);               \
  template void launch_gather_volume<T>(const LayerDev&, double2*, int, int,         \
                                        long long, int, hipStream_t);                \
  template void launch_local_to_X<T>(const LayerDev&, const double2*, int,           \
                                     hipStream_t);                                   \
  template void launch_X_to_local<T>(const LayerDev&, double2*, int, hipStream_t);   \
  template void launch_jump<T>(const LayerDev&, const JumpTerms&, const double2*, int, \
                               int, int, int, hipStream_t);                          \
  template void launch_readout<T>(const LayerDev&, int, double, const ReadTerms&,    \
                                  double2*, int, int, int, hipStream_t);
HELM_INST_VOL(float)
HELM_INST_VOL(double)

}  // namespace kern
}  // namespace helm
