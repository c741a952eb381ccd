// Layer decomposition, absorbing-layer tables and nested-dissection plan.
//
// Section "Formulation": the grid (absorbing layer included) is split into L
// layers in z; each internal side of a layer gets alpha extra absorbing
// planes, the outer sides inherit the global absorbing layer.
// Section "Local Solves: Parallel Multi-frontal Methods": every layer is
// reordered by nested dissection and factored by a multifrontal method.
// For a slab of constant thickness the separators of the first levels are
// vertical planes through the whole slab (the quasi-2D problem of the
// complexity section); once a box is thinner laterally than tall it is cut
// in z as well.  Boxes are bisected across their longest side until they
// hold at most `leaf` unknowns.
#include <algorithm>
#include <cmath>
#include <exception>
#include <numeric>
#include <thread>

#include "helm_internal.h"

namespace helm {

namespace {

// sigma(d) = (C/delta) (d/delta)^2 for d > 0 (Eq. appendix:eq:def_alpha)
double sigma_q(double d, double delta, double C) {
  if (d <= 0.0 || delta <= 0.0) return 0.0;
  double r = d / delta;
  return (C / delta) * r * r;
}

cd beta_of(double sigma, double omega) {
  return 1.0 / cd(1.0, sigma / omega);
}

// Global profile of an n-node axis at position x (units of h); the origins
// sit at the half-nodes p - 1/2 and n - 1 - p + 1/2.
double global_sigma(double x, int n, int p, double h, double C) {
  if (p == 0) return 0.0;
  double d = std::max(std::max((p - 0.5) - x, x - (n - 1 - p + 0.5)), 0.0) * h;
  return sigma_q(d, p * h, C);
}

void axis_tables(int n, int p, double h, double omega, double C,
                 std::vector<cd>& node, std::vector<cd>& half) {
  node.resize(n);
  half.resize(n + 1);
  for (int i = 0; i < n; ++i) node[i] = beta_of(global_sigma(i, n, p, h, C), omega);
  for (int i = 0; i <= n; ++i)
    half[i] = beta_of(global_sigma(i - 0.5, n, p, h, C), omega);
}

struct NDBuilder {
  int nx, ny, t;
  long long leaf;
  LayerPlan& P;
  int next_off = 0;

  int dim(int a) const { return a == 0 ? nx : (a == 1 ? ny : t); }

  // returns the front id (post-order), or -1 for an empty box
  int build(const Box& box, int depth) {
    long long vol = box.volume();
    if (vol <= 0) return -1;
    int ext[3] = {box.hi[0] - box.lo[0], box.hi[1] - box.lo[1],
                  box.hi[2] - box.lo[2]};
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (ext[a] > ext[ax]) ax = a;
    FrontHost F;
    F.box = box;
    F.depth = depth;
    if (vol <= leaf || ext[ax] < 3) {
      F.sep = box;
      F.s = (int)vol;
    } else {
      int mid = box.lo[ax] + ext[ax] / 2;
      Box a = box, b = box, sep = box;
      a.hi[ax] = mid;
      b.lo[ax] = mid + 1;
      sep.lo[ax] = mid;
      sep.hi[ax] = mid + 1;
      int ca = build(a, depth + 1);
      int cb = build(b, depth + 1);
      F.child[0] = ca;
      F.child[1] = cb;
      F.sep = sep;
      F.s = (int)sep.volume();
    }
    F.off = next_off;
    // number the pivots: x fastest, then y, then z inside the separator box
    const Box& S = F.sep;
    int o = next_off;
    for (int z = S.lo[2]; z < S.hi[2]; ++z)
      for (int y = S.lo[1]; y < S.hi[1]; ++y)
        for (int x = S.lo[0]; x < S.hi[0]; ++x) {
          int nat = x + nx * (y + ny * z);
          P.nat2nd[nat] = o;
          P.nd2nat[o] = nat;
          ++o;
        }
    next_off = o;
    int id = (int)P.fronts.size();
    P.fronts.push_back(F);
    for (int c = 0; c < 2; ++c)
      if (F.child[c] >= 0) P.fronts[F.child[c]].parent = id;
    return id;
  }
};

}  // namespace

double gj_front_flops(int s, int b, int nb) {
  const int n = s + b, T = 64;
  const int nt = (n + T - 1) / T;
  double fl = 0;
  for (int k = 0; k < s; k += nb) {
    const int nbf = std::min(nb, s - k);
    for (int ti = 0; ti < nt; ++ti) {
      const int i0 = ti * T, ri = std::min(T, n - i0);
      const bool rowsJ = i0 >= k && i0 + T <= k + nbf, rowsDone = i0 + T <= k;
      for (int tj = 0; tj < nt; ++tj) {
        const int j0 = tj * T, cj = std::min(T, n - j0);
        const bool colsJ = j0 >= k && j0 + T <= k + nbf;
        if (rowsJ || colsJ || (rowsDone && j0 >= s)) continue;
        fl += 8.0 * nbf * ri * cj;
      }
    }
    fl += 2.0 * 8.0 * n * (double)nbf * nbf;
  }
  return fl;
}

void build_layer_plan(LayerPlan& P, int nx, int ny, int leaf) {
  const int t = P.t;
  P.n_loc = nx * ny * t;
  P.nat2nd.assign(P.n_loc, -1);
  P.nd2nat.assign(P.n_loc, -1);
  P.fronts.clear();
  NDBuilder B{nx, ny, t, (long long)std::max(leaf, 1), P};
  Box root{{0, 0, 0}, {nx, ny, t}};
  B.build(root, 0);
  HELM_REQUIRE(B.next_off == P.n_loc, HELM_EINVAL, "nested dissection lost unknowns");
  const int nf = (int)P.fronts.size();

  // boundaries: face neighbours of the subtree box, sorted by ND index
  P.bidx.clear();
  P.bidx_off.assign(nf, 0);
  const int dims[3] = {nx, ny, t};
  std::vector<int> tmp;
  for (int f = 0; f < nf; ++f) {
    FrontHost& F = P.fronts[f];
    tmp.clear();
    const Box& bx = F.box;
    for (int a = 0; a < 3; ++a) {
      for (int side = 0; side < 2; ++side) {
        int c = side == 0 ? bx.lo[a] - 1 : bx.hi[a];
        if (c < 0 || c >= dims[a]) continue;
        Box face = bx;
        face.lo[a] = c;
        face.hi[a] = c + 1;
        for (int z = face.lo[2]; z < face.hi[2]; ++z)
          for (int y = face.lo[1]; y < face.hi[1]; ++y)
            for (int x = face.lo[0]; x < face.hi[0]; ++x)
              tmp.push_back(P.nat2nd[x + nx * (y + ny * z)]);
      }
    }
    std::sort(tmp.begin(), tmp.end());
    for (int v : tmp)
      HELM_REQUIRE(v >= F.off + F.s, HELM_EINVAL,
                   "boundary variable eliminated before its front");
    F.b = (int)tmp.size();
    P.bidx_off[f] = (int)P.bidx.size();
    P.bidx.insert(P.bidx.end(), tmp.begin(), tmp.end());
  }

  // front-row -> child-boundary maps (pull form of the extend-add)
  P.inv.clear();
  P.inv_off.assign(2 * nf, -1);
  for (int f = 0; f < nf; ++f) {
    const FrontHost& F = P.fronts[f];
    const int nrow = F.s + F.b;
    for (int slot = 0; slot < 2; ++slot) {
      int c = F.child[slot];
      if (c < 0) continue;
      const FrontHost& Cf = P.fronts[c];
      P.inv_off[2 * f + slot] = (int)P.inv.size();
      size_t base = P.inv.size();
      P.inv.resize(base + nrow, -1);
      const int* cb = P.bidx.data() + P.bidx_off[c];
      int q = 0, found = 0;
      for (int r = 0; r < nrow && q < Cf.b; ++r) {
        int nd = r < F.s ? F.off + r : P.bidx[P.bidx_off[f] + r - F.s];
        while (q < Cf.b && cb[q] < nd) {
          // a child boundary variable missing from the parent front
          HELM_REQUIRE(false, HELM_EINVAL, "child boundary not in parent front");
        }
        if (q < Cf.b && cb[q] == nd) {
          P.inv[base + r] = q++;
          ++found;
        }
      }
      HELM_REQUIRE(found == Cf.b, HELM_EINVAL, "child boundary not in parent front");
    }
  }

  // factor offsets, depth lists, solve-buffer offsets, work counts
  P.fac_off.assign(nf, 0);
  long long acc = 0;
  P.factor_flops = 0;
  P.gj_flops = 0;
  P.solve_elems = 0;
  P.max_front = 0;
  P.max_depth = 0;
  for (int f = 0; f < nf; ++f) {
    const FrontHost& F = P.fronts[f];
    P.fac_off[f] = acc;
    acc += (long long)(F.s + F.b) * F.s;
    const double ss = F.s, bb = F.b;
    P.factor_flops += 4.0 * (2.0 / 3.0 * ss * ss * ss + 2.0 * ss * ss * bb + 2.0 * ss * bb * bb);
    P.gj_flops += gj_front_flops(F.s, F.b, kPivotBlock);
    P.solve_elems += (double)F.s * F.s + 2.0 * F.s * F.b;
    P.max_front = std::max<long long>(P.max_front, F.s + F.b);
    P.max_depth = std::max(P.max_depth, F.depth);
  }
  P.fac_elems = acc;
  P.by_depth.assign(P.max_depth + 1, {});
  for (int f = 0; f < nf; ++f) P.by_depth[P.fronts[f].depth].push_back(f);
  for (auto& v : P.by_depth)
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
      return P.fronts[a].s > P.fronts[b].s;
    });
  P.wt_off.assign(nf, 0);
  P.ub_off.assign(nf, 0);
  P.wt_rows = 0;
  P.ub_rows[0] = P.ub_rows[1] = 0;
  for (int d = 0; d <= P.max_depth; ++d) {
    long long ws = 0, ub = 0;
    for (int f : P.by_depth[d]) {
      P.wt_off[f] = ws;
      P.ub_off[f] = ub;
      ws += P.fronts[f].s;
      ub += P.fronts[f].b;
    }
    P.wt_rows = std::max(P.wt_rows, ws);
    P.ub_rows[d & 1] = std::max(P.ub_rows[d & 1], ub);
  }
}

void build_geometry(Geometry& G, const helm_grid& g, double omega, int pml,
                    int n_layers, int alpha, double C, int leaf) {
  HELM_REQUIRE(g.nx >= 1 && g.ny >= 1 && g.nz >= 1 && g.h > 0, HELM_EINVAL,
               "bad grid");
  HELM_REQUIRE(omega > 0 && std::isfinite(omega), HELM_EINVAL, "bad omega");
  HELM_REQUIRE(pml >= 0 && 2 * pml < g.nx && 2 * pml < g.ny && 2 * pml < g.nz,
               HELM_EINVAL, "PML wider than the grid");
  HELM_REQUIRE(n_layers >= 1, HELM_EINVAL, "need at least one layer");
  HELM_REQUIRE(alpha >= 1 || n_layers == 1, HELM_EINVAL, "pml_local must be >= 1");
  HELM_REQUIRE(C > 0 && std::isfinite(C), HELM_EINVAL, "bad PML strength");
  const int interior = g.nz - 2 * pml;
  HELM_REQUIRE(interior >= n_layers, HELM_EINVAL,
               "layers thinner than one interior plane");
  G.nx = g.nx; G.ny = g.ny; G.nz = g.nz; G.h = g.h; G.omega = omega;
  G.pml = pml; G.L = n_layers; G.alpha = alpha; G.C = C;
  axis_tables(g.nx, pml, g.h, omega, C, G.bx, G.bxh);
  axis_tables(g.ny, pml, g.h, omega, C, G.by, G.byh);
  axis_tables(g.nz, pml, g.h, omega, C, G.bz, G.bzh);

  // interior planes split as evenly as possible, first layers get the extra
  // plane; global absorbing planes attached to the outer layers
  G.layers.assign(n_layers, LayerPlan{});
  G.lbz.assign(n_layers, {});
  G.lbzh.assign(n_layers, {});
  int base = interior / n_layers, extra = interior % n_layers;
  int s = pml;
  for (int l = 0; l < n_layers; ++l) {
    LayerPlan& P = G.layers[l];
    int size = base + (l < extra ? 1 : 0);
    P.index = l;
    P.s = s;
    P.e = s + size - 1;
    s += size;
  }
  G.layers[0].s = 0;
  G.layers[n_layers - 1].e = g.nz - 1;
  for (int l = 0; l < n_layers; ++l) {
    LayerPlan& P = G.layers[l];
    P.lo = l > 0 ? P.s - alpha : P.s;
    P.hi = l < n_layers - 1 ? P.e + alpha : P.e;
    P.t = P.hi - P.lo + 1;
    // z profile: global on [s - 1/2, e + 1/2], local absorbing layer outside
    auto sig = [&](double z) {
      if (l > 0 && z < P.s - 0.5)
        return sigma_q(((P.s - 0.5) - z) * g.h, alpha * g.h, C);
      if (l < n_layers - 1 && z > P.e + 0.5)
        return sigma_q((z - (P.e + 0.5)) * g.h, alpha * g.h, C);
      return global_sigma(z, g.nz, pml, g.h, C);
    };
    G.lbz[l].resize(P.t);
    G.lbzh[l].resize(P.t + 1);
    for (int q = 0; q < P.t; ++q) G.lbz[l][q] = beta_of(sig(P.lo + q), omega);
    for (int q = 0; q <= P.t; ++q) G.lbzh[l][q] = beta_of(sig(P.lo + q - 0.5), omega);
  }

  // The dissection depends only on the layer's extent (nx, ny, t): build one
  // plan per distinct thickness, on threads of their own, and copy it into
  // the other layers of that thickness.
  std::vector<int> first(n_layers, -1), owners;
  for (int l = 0; l < n_layers; ++l) {
    for (int o : owners)
      if (G.layers[o].t == G.layers[l].t) { first[l] = o; break; }
    if (first[l] < 0) { first[l] = l; owners.push_back(l); }
  }
  std::vector<std::exception_ptr> err(owners.size());
  std::vector<std::thread> pool;
  for (size_t i = 0; i < owners.size(); ++i)
    pool.emplace_back([&, i] {
      try {
        build_layer_plan(G.layers[owners[i]], g.nx, g.ny, leaf);
      } catch (...) {
        err[i] = std::current_exception();
      }
    });
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  for (int l = 0; l < n_layers; ++l) {
    if (first[l] == l) continue;
    LayerPlan& P = G.layers[l];
    const LayerPlan keep = P;
    P = G.layers[first[l]];
    P.index = keep.index; P.s = keep.s; P.e = keep.e;
    P.lo = keep.lo; P.hi = keep.hi;
  }
}

}  // namespace helm
