// Offline stage (Algorithm 1): device geometry, memory plan, factorization
// driver, and the level-by-level multi-RHS local solve used by the online
// stage.
#include "handle.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace helm {

DevMem::~DevMem() { release(); }
void DevMem::alloc(size_t b) {
  release();
  if (b == 0) return;
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error{HELM_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
  }
  bytes = b;
}
void DevMem::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

namespace {

// set-up copies (plans, tables): complete before the host vector goes away
template <typename V>
void upload(DevMem& d, const std::vector<V>& h, hipStream_t st) {
  d.alloc(h.size() * sizeof(V));
  if (!h.empty()) {
    HELM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, st));
    HELM_HIP(hipStreamSynchronize(st));
  }
}

// Tile map of a prefix array over items: entry t = (a, t - prefix[a]) for
// prefix[a] <= t < prefix[a + 1].
std::vector<int2> tile_map(const std::vector<int>& prefix) {
  std::vector<int2> m(prefix.empty() ? 0 : (size_t)prefix.back());
  for (size_t a = 0; a + 1 < prefix.size(); ++a)
    for (int t = prefix[a]; t < prefix[a + 1]; ++t) m[t] = make_int2((int)a, t - prefix[a]);
  return m;
}

std::vector<double2> to_d2(const std::vector<cd>& v) {
  std::vector<double2> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = make_double2(v[i].real(), v[i].imag());
  return o;
}

int tiles64(long long n) { return (int)((n + 63) / 64); }
int tiles16(long long n) { return (int)((n + 15) / 16); }

}  // namespace

EventPair::EventPair() {
  HELM_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    a = nullptr;
    throw Error{HELM_EHIP, "hipEventCreate failed"};
  }
}
EventPair::~EventPair() {
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
}
double EventPair::elapsed_ms(hipStream_t) const {
  HELM_HIP(hipEventSynchronize(b));
  float ms = 0;
  HELM_HIP(hipEventElapsedTime(&ms, a, b));
  return ms;
}

void Handle::clear_graphs() {
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
}

Handle::~Handle() {
  if (st) (void)hipStreamSynchronize(st);
  clear_graphs();
  for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : ev_free) (void)hipEventDestroy(e);
  sets.clear();
  if (cap_st) (void)hipStreamDestroy(cap_st);
  if (own_stream && st) (void)hipStreamDestroy(st);
}

void Handle::init_device(const helm_options& o) {
  opt = o;
  device = o.device;
  HELM_HIP(hipSetDevice(device));
  if (o.stream) {
    st = reinterpret_cast<hipStream_t>(o.stream);
    own_stream = false;
  } else {
    HELM_HIP(hipStreamCreate(&st));
    own_stream = true;
  }
  prec = o.precision == HELM_FP64 ? HELM_FP64 : HELM_MIXED;
  elem = prec == HELM_FP64 ? 16 : 8;
  set_profile(o.flags);
}

void Handle::set_profile(int flags) {
  profile_mask = 0;
  if (flags & HELM_FLAG_PROFILE) profile_mask = (1u << K_NCLASS) - 1;
  if (flags & HELM_FLAG_PROFILE_FWD) profile_mask |= 1u << K_FWD_GEMM;
  // the product forms of the complex64 GEMMs; graphs and tile choices made
  // with the other substitution form are dropped
  factor3m = prec == HELM_MIXED && !(flags & HELM_FLAG_FACTOR_4M);
  const bool m3 = prec == HELM_MIXED && !(flags & HELM_FLAG_GEMM_4M);
  if (m3 != gemm3m) {
    if (st) HELM_HIP(hipStreamSynchronize(st));
    clear_graphs();
    tiles.clear();
    tuned.clear();
    gemm3m = m3;
  }
}

// An event recorded on the handle's stream, for the timing of class cls
// (null when that class is not timed).
hipEvent_t Handle::prof_begin(int cls) {
  if (!((profile_mask >> cls) & 1u)) return nullptr;
  return record_event();
}

hipEvent_t Handle::take_event() {
  hipEvent_t e;
  if (!ev_free.empty()) {
    e = ev_free.back();
    ev_free.pop_back();
  } else {
    // timing only: no system-scope fence (cache writeback / invalidate)
    // between the kernels being timed
    HELM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  return e;
}

hipEvent_t Handle::record_event() {
  hipEvent_t e = take_event();
  HELM_HIP(hipEventRecord(e, st));
  return e;
}

void Handle::prof_end(int cls, hipEvent_t a, double flops, double bytes) {
  if (!a) return;
  hipEvent_t b = record_event();
  pending.push_back(PendingEvent{cls, a, b, flops, bytes});
}

void Handle::collect_profile() {
  if (pending.empty()) return;
  HELM_HIP(hipStreamSynchronize(st));
  for (auto& p : pending) {
    float ms = 0;
    HELM_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    KStat& k = kstats[p.cls];
    k.launches += 1;
    k.ms += ms;
    k.flops += p.flops;
    k.bytes += p.bytes;
    ev_free.push_back(p.a);
    ev_free.push_back(p.b);
  }
  pending.clear();
}

void Handle::upload_geometry(const double* m_src, bool m_on_device) {
  const long long N = (long long)G.nx * G.ny * G.nz;
  m.alloc(N * sizeof(double));
  HELM_HIP(hipMemcpyAsync(m.p, m_src, N * sizeof(double),
                          m_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  upload(bx, to_d2(G.bx), st);
  upload(bxh, to_d2(G.bxh), st);
  upload(by, to_d2(G.by), st);
  upload(byh, to_d2(G.byh), st);
  upload(bz, to_d2(G.bz), st);
  upload(bzh, to_d2(G.bzh), st);
  // B(j, i) = 1 / (h^2 beta_x(i) beta_y(j)): matrix coupling across an
  // interior interface, the scale of the interface sources
  std::vector<double2> B((size_t)G.nx * G.ny);
  for (int j = 0; j < G.ny; ++j)
    for (int i = 0; i < G.nx; ++i) {
      cd v = 1.0 / (G.h * G.h * G.bx[i] * G.by[j]);
      B[(size_t)i + (size_t)G.nx * j] = make_double2(v.real(), v.imag());
    }
  upload(Bcoef, B, st);
  const int L = G.L;
  lbz.clear(); lbzh.clear(); nat2nd.clear(); nd2nat.clear(); bidx.clear(); inv.clear();
  for (int l = 0; l < L; ++l) {
    const LayerPlan& P = G.layers[l];
    lbz.emplace_back(new DevMem); upload(*lbz.back(), to_d2(G.lbz[l]), st);
    lbzh.emplace_back(new DevMem); upload(*lbzh.back(), to_d2(G.lbzh[l]), st);
    nat2nd.emplace_back(new DevMem); upload(*nat2nd.back(), P.nat2nd, st);
    nd2nat.emplace_back(new DevMem); upload(*nd2nat.back(), P.nd2nat, st);
    bidx.emplace_back(new DevMem); upload(*bidx.back(), P.bidx, st);
    inv.emplace_back(new DevMem); upload(*inv.back(), P.inv, st);
  }
  grid.nx = G.nx; grid.ny = G.ny; grid.nz = G.nz;
  grid.h = G.h; grid.omega = G.omega;
  grid.m = m.as<double>();
  grid.bx = bx.as<double2>(); grid.bxh = bxh.as<double2>();
  grid.by = by.as<double2>(); grid.byh = byh.as<double2>();
  grid.bz = bz.as<double2>(); grid.bzh = bzh.as<double2>();
}

void Handle::build_fronts() {
  const int L = G.L;
  front_base.assign(L + 1, 0);
  for (int l = 0; l < L; ++l)
    front_base[l + 1] = front_base[l] + (int)G.layers[l].fronts.size();
  n_fronts = front_base[L];
  fronts_h.assign(n_fronts, FrontDev{});
  for (int l = 0; l < L; ++l) {
    const LayerPlan& P = G.layers[l];
    for (size_t q = 0; q < P.fronts.size(); ++q) {
      const FrontHost& F = P.fronts[q];
      FrontDev& d = fronts_h[front_base[l] + q];
      d.s = F.s;
      d.b = F.b;
      d.off = F.off;
      d.layer = l;
      d.fac = P.fac_off[q];
      d.ws = 0;
      d.ws_parity = F.depth & 1;
      d.bidx = P.bidx_off[q];
      for (int c = 0; c < 2; ++c) {
        d.inv[c] = P.inv_off[2 * q + c];
        d.child[c] = F.child[c] >= 0 ? front_base[l] + F.child[c] : -1;
      }
      d.wt = P.wt_off[q];
      d.ub = P.ub_off[q];
      d.ub_parity = F.depth & 1;
    }
  }
  layers_h.assign(L, LayerDev{});
  for (int l = 0; l < L; ++l) {
    const LayerPlan& P = G.layers[l];
    LayerDev& d = layers_h[l];
    d.bidx = bidx[l]->as<int>();
    d.inv = inv[l]->as<int>();
    d.nat2nd = nat2nd[l]->as<int>();
    d.nd2nat = nd2nat[l]->as<int>();
    d.bz = lbz[l]->as<double2>();
    d.bzh = lbzh[l]->as<double2>();
    d.n_loc = P.n_loc;
    d.t = P.t;
    d.lo = P.lo;
    d.s = P.s;
    d.e = P.e;
  }
}

void Handle::upload_layers() {
  if (!layers_d.p || layers_d.bytes < layers_h.size() * sizeof(LayerDev))
    layers_d.alloc(layers_h.size() * sizeof(LayerDev));
  HELM_HIP(hipMemcpyAsync(layers_d.p, layers_h.data(), layers_h.size() * sizeof(LayerDev),
                          hipMemcpyHostToDevice, st));
  HELM_HIP(hipStreamSynchronize(st));
}

size_t plan_factor_elems(const Geometry& G) {
  size_t s = 0;
  for (const auto& P : G.layers) s += (size_t)P.fac_elems;
  return s;
}

// FP64 interface vectors of one column: Krylov basis (up to 16 + 2 vectors)
// and sweep temporaries (about 8), each 2 pair vectors of (L-1) x 2 planes
size_t plan_pair_bytes_per_rhs(const Geometry& G) {
  const size_t pv = (size_t)std::max(G.L - 1, 0) * 2 * G.nx * G.ny * 16;
  return pv * 2 * (18 + 8);
}

size_t lane_bytes_per_slot(const Geometry& G, size_t elem) {
  return plan_bytes_per_rhs(G, elem) + plan_pair_bytes_per_rhs(G);
}

size_t plan_bytes_per_rhs(const Geometry& G, size_t elem) {
  // local solve vectors of every layer (X, Wt, Ub even/odd)
  size_t per = 0;
  for (const auto& P : G.layers)
    per += ((size_t)P.n_loc + P.wt_rows + P.ub_rows[0] + P.ub_rows[1]) * elem;
  per += plan_pair_bytes_per_rhs(G);
  // FP64 volumes: f, u, r, correction
  per += (size_t)G.nx * G.ny * G.nz * 16 * 4;
  return per;
}

// ---------------------------------------------------------------------------
// factorization
// ---------------------------------------------------------------------------
void Handle::factorize() {
  auto t0 = std::chrono::steady_clock::now();
  if (prec == HELM_FP64) factorize_t<double>(); else factorize_t<float>();
  factor_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Frontal workspace of one layer per depth: the sum of (s+b)^2 over its fronts
// and of the panel copies s nb.
std::pair<std::vector<long long>, std::vector<long long>> layer_workspace(const LayerPlan& P,
                                                                          int nb) {
  std::vector<long long> sum(P.max_depth + 1, 0), pan(P.max_depth + 1, 0);
  for (const auto& F : P.fronts) {
    sum[F.depth] += (long long)(F.s + F.b) * (F.s + F.b);
    pan[F.depth] += (long long)F.s * nb;
  }
  return {sum, pan};
}

// Bytes of the two depth-parity frontal buffers and the two panel copies for
// per-depth element counts a (fronts) and p (panels).
size_t workspace_bytes(const std::vector<long long>& a, const std::vector<long long>& p,
                       size_t elem) {
  long long m0 = 0, m1 = 0, mp = 0;
  for (size_t d = 0; d < a.size(); ++d) {
    if (d & 1) m1 = std::max(m1, a[d]); else m0 = std::max(m0, a[d]);
    mp = std::max(mp, p[d]);
  }
  return (size_t)(m0 + m1 + 2 * mp) * elem;
}

template <typename T>
void Handle::factorize_t() {
  const int L = G.L;
  // factor store, one buffer per layer
  fac.clear();
  bytes_factors = 0;
  factor_flops = 0;
  factor_gj_flops = 0;
  HELM_REQUIRE(!opt.hbm_budget_bytes || plan_factor_elems(G) * elem <= opt.hbm_budget_bytes,
               HELM_ENOMEM, "factors exceed the memory budget");
  for (int l = 0; l < L; ++l) {
    fac.emplace_back(new DevMem);
    fac.back()->alloc((size_t)G.layers[l].fac_elems * elem);
    layers_h[l].fac = fac.back()->p;
    bytes_factors += (size_t)G.layers[l].fac_elems * elem;
    factor_flops += G.layers[l].factor_flops;
    factor_gj_flops += G.layers[l].gj_flops;
  }
  // memory left for frontal workspaces: choose groups of consecutive layers
  size_t free_b = 0, total_b = 0;
  HELM_HIP(hipMemGetInfo(&free_b, &total_b));
  size_t budget = opt.hbm_budget_bytes ? opt.hbm_budget_bytes : (size_t)(0.9 * total_b);
  size_t used_now = total_b - free_b;
  size_t avail = budget > used_now ? budget - used_now : 0;
  // leave room for the solve workspace of the default batch
  size_t reserve = plan_bytes_per_rhs(G, elem) * (size_t)std::max(1, opt.max_rhs);
  size_t ws_budget = avail > reserve ? (avail - reserve) : avail / 2;
  auto layer_ws = [&](int l) { return layer_workspace(G.layers[l], nb); };
  std::vector<std::vector<int>> groups;
  {
    std::vector<int> cur;
    std::vector<long long> acc;
    std::vector<long long> accp;
    auto cost = [&](const std::vector<long long>& a, const std::vector<long long>& p) {
      return workspace_bytes(a, p, elem);
    };
    for (int l = 0; l < L; ++l) {
      auto w = layer_ws(l);
      std::vector<long long> na = acc, np = accp;
      if (na.size() < w.first.size()) { na.resize(w.first.size(), 0); np.resize(w.first.size(), 0); }
      for (size_t d = 0; d < w.first.size(); ++d) { na[d] += w.first[d]; np[d] += w.second[d]; }
      if (!cur.empty() && cost(na, np) > ws_budget) {
        groups.push_back(cur);
        cur.clear();
        acc.assign(w.first.begin(), w.first.end());
        accp.assign(w.second.begin(), w.second.end());
        HELM_REQUIRE(cost(acc, accp) <= ws_budget, HELM_ENOMEM,
                     "frontal workspace of one layer exceeds the memory budget");
      } else {
        acc = na;
        accp = np;
      }
      cur.push_back(l);
    }
    if (!cur.empty()) groups.push_back(cur);
  }

  DevMem status;
  status.alloc(sizeof(kern::FactorStatus));
  {
    kern::FactorStatus s0{};
    const double inf = INFINITY;
    std::memcpy(&s0.pmin, &inf, sizeof(double));
    HELM_HIP(hipMemcpyAsync(status.p, &s0, sizeof(s0), hipMemcpyHostToDevice, st));
    HELM_HIP(hipStreamSynchronize(st));
  }
  // test hook: leave the first leaf front of layer 0 unassembled
  int skip_front = -1;
  if (opt.flags & HELM_FLAG_TEST_ZERO_FRONT)
    for (int f = front_base[0]; f < front_base[1] && skip_front < 0; ++f)
      if (fronts_h[f].child[0] < 0 && fronts_h[f].child[1] < 0) skip_front = f;

  for (const auto& grp : groups) {
    int maxd = 0;
    for (int l : grp) maxd = std::max(maxd, G.layers[l].max_depth);
    // per-depth lists, workspace offsets
    std::vector<std::vector<int>> dl(maxd + 1);
    for (int l : grp)
      for (int d = 0; d <= G.layers[l].max_depth; ++d)
        for (int q : G.layers[l].by_depth[d]) dl[d].push_back(front_base[l] + q);
    long long wsz[2] = {0, 0}, pmax = 0, smax_sum = 0;
    for (int d = 0; d <= maxd; ++d) {
      auto& v = dl[d];
      std::stable_sort(v.begin(), v.end(),
                       [&](int a, int b) { return fronts_h[a].s > fronts_h[b].s; });
      long long off = 0, pan = 0, ss = 0;
      for (int f : v) {
        fronts_h[f].ws = off;
        long long n = fronts_h[f].s + fronts_h[f].b;
        off += n * n;
        pan += (long long)fronts_h[f].s * nb;
        ss += fronts_h[f].s;
      }
      wsz[d & 1] = std::max(wsz[d & 1], off);
      pmax = std::max(pmax, pan);
      smax_sum = std::max(smax_sum, ss);
    }
    upload(fronts, fronts_h, st);
    upload_layers();
    DevMem ws0, ws1, panel, Dbuf, ipiv, perm;
    ws0.alloc(std::max<long long>(wsz[0], 1) * elem);
    ws1.alloc(std::max<long long>(wsz[1], 1) * elem);
    panel.alloc(std::max<long long>(pmax, 1) * elem);
    Dbuf.alloc(std::max<long long>(pmax, 1) * elem);
    ipiv.alloc(std::max<long long>(smax_sum, 1) * sizeof(int));
    perm.alloc(std::max<long long>(smax_sum, 1) * sizeof(int));

    for (int d = maxd; d >= 0; --d) {
      const auto& v = dl[d];
      if (v.empty()) continue;
      FactorDepth fd;
      fd.n = (int)v.size();
      std::vector<int> pRow(fd.n + 1, 0), pStore(fd.n + 1, 0);
      std::vector<long long> poff(fd.n + 1, 0), roff(fd.n + 1, 0);
      fd.pFull_h.assign(fd.n + 1, 0);
      fd.pCol_h.assign(fd.n + 1, 0);
      for (int a = 0; a < fd.n; ++a) {
        const FrontDev& F = fronts_h[v[a]];
        int n = F.s + F.b;
        fd.s_sorted.push_back(F.s);
        fd.pFull_h[a + 1] = fd.pFull_h[a] + tiles64(n) * tiles64(n);
        fd.pCol_h[a + 1] = fd.pCol_h[a] + tiles64(n);
        pRow[a + 1] = pRow[a] + (F.s + 255) / 256;
        pStore[a + 1] = pStore[a] + tiles64(n) * tiles64(F.s);
        poff[a + 1] = poff[a] + (long long)F.s * nb;
        roff[a + 1] = roff[a] + F.s;
      }
      upload(fd.ids, v, st);
      upload(fd.pFull, tile_map(fd.pFull_h), st);
      upload(fd.pCol, tile_map(fd.pCol_h), st);
      upload(fd.pRow, tile_map(pRow), st);
      upload(fd.pStore, tile_map(pStore), st);
      upload(fd.panel_off, poff, st);
      upload(fd.perm_off, roff, st);
      const FrontDev* fr = fronts.as<FrontDev>();
      const LayerDev* ld = layers_d.as<LayerDev>();
      const int* ids = fd.ids.as<int>();
      double front_elems = 0;
      for (int a = 0; a < fd.n; ++a) {
        double n = fronts_h[v[a]].s + fronts_h[v[a]].b;
        front_elems += n * n;
      }
      hipEvent_t e0 = prof_begin(K_EXTEND_ADD);
      kern::launch_extend_add<T>(fr, ids, fd.n, fd.pFull.as<int2>(), fd.pFull_h[fd.n], ld,
                                 ws0.p, ws1.p, st);
      prof_end(K_EXTEND_ADD, e0, 0, 2 * front_elems * elem);
      e0 = prof_begin(K_ORIG);
      kern::launch_orig_entries<T>(fr, ids, fd.n, fd.pRow.as<int2>(), pRow[fd.n], ld,
                                   ws0.p, ws1.p, grid, skip_front,
                                   status.as<kern::FactorStatus>(), st);
      prof_end(K_ORIG, e0, 0, 0);
      const int smax = fd.s_sorted[0];
      for (int k = 0; k < smax; k += nb) {
        int n_act = 0;
        while (n_act < fd.n && fd.s_sorted[n_act] > k) ++n_act;
        double sw_flops = 0, sw_bytes = 0;
        if (profile())
          for (int a = 0; a < n_act; ++a) {
            double n = fronts_h[v[a]].s + fronts_h[v[a]].b;
            double nbf = std::min(nb, fronts_h[v[a]].s - k);
            // the LU's trailing update of this step (its share of the
            // algorithmic count 4 (2/3 s^3 + 2 s^2 b + 2 s b^2))
            sw_flops += 8.0 * (n - k - nbf) * (n - k - nbf) * nbf;
            sw_bytes += (2.0 * n * n + 2.0 * n * nbf) * elem;
          }
        hipEvent_t e1 = prof_begin(K_PANEL);
        kern::launch_panel<T>(fr, ids, n_act, smax - k, k, nb, ws0.p, ws1.p, panel.p,
                              fd.panel_off.as<long long>(), Dbuf.p, ipiv.as<int>(),
                              perm.as<int>(), fd.perm_off.as<long long>(),
                              status.as<kern::FactorStatus>(), st);
        prof_end(K_PANEL, e1, 0, 0);
        e1 = prof_begin(K_SWAP_JO);
        kern::launch_swap_JO<T>(fr, ids, n_act, fd.pCol.as<int2>(), fd.pCol_h[n_act], k,
                                nb, ws0.p, ws1.p, Dbuf.p, ipiv.as<int>(),
                                fd.panel_off.as<long long>(), fd.perm_off.as<long long>(),
                                st);
        prof_end(K_SWAP_JO, e1, 0, 0);
        e1 = prof_begin(K_SWEEP_GEMM);
        kern::launch_sweep_gemm<T>(fr, ids, n_act, fd.pFull.as<int2>(), fd.pFull_h[n_act],
                                   k, nb, ws0.p, ws1.p, factor3m, st);
        prof_end(K_SWEEP_GEMM, e1, sw_flops, sw_bytes);
        e1 = prof_begin(K_UPDATE_OJ);
        kern::launch_update_OJ<T>(fr, ids, n_act, fd.pCol.as<int2>(), fd.pCol_h[n_act], k,
                                  nb, ws0.p, ws1.p, Dbuf.p, fd.panel_off.as<long long>(),
                                  st);
        prof_end(K_UPDATE_OJ, e1, 0, 0);
      }
      hipEvent_t e2 = prof_begin(K_STORE);
      kern::launch_store_factor<T>(fr, ids, fd.n, fd.pStore.as<int2>(), pStore[fd.n], ld,
                                   ws0.p, ws1.p, perm.as<int>(),
                                   fd.perm_off.as<long long>(), st);
      prof_end(K_STORE, e2, 0, 0);
      HELM_HIP(hipGetLastError());
      collect_profile();
      // the lists of this depth must outlive the kernels that read them
      HELM_HIP(hipStreamSynchronize(st));
    }
  }
  kern::FactorStatus st_h{};
  HELM_HIP(hipMemcpyAsync(&st_h, status.p, sizeof(st_h), hipMemcpyDeviceToHost, st));
  HELM_HIP(hipStreamSynchronize(st));
  auto as_d = [](unsigned long long b) {
    double v;
    std::memcpy(&v, &b, sizeof(v));
    return v;
  };
  pivot_min = std::sqrt(as_d(st_h.pmin));
  pivot_max = std::sqrt(as_d(st_h.pmax));
  diag_max = std::sqrt(as_d(st_h.dmax));
  zero_pivots = st_h.flag;
  HELM_REQUIRE(st_h.flag == 0, HELM_EZEROPIVOT, "zero or non-finite pivot in a frontal matrix");
  upload(fronts, fronts_h, st);
  upload_layers();
}

template void Handle::factorize_t<float>();
template void Handle::factorize_t<double>();

// ---------------------------------------------------------------------------
// solve workspace and launch lists
// ---------------------------------------------------------------------------
void Handle::ensure_workspace(int k) {
  if (k <= kcap) return;
  HELM_HIP(hipStreamSynchronize(st));
  clear_graphs();
  const int L = G.L;
  X.clear(); Wt.clear(); Ub0.clear(); Ub1.clear();
  for (int l = 0; l < L; ++l) {
    const LayerPlan& P = G.layers[l];
    X.emplace_back(new DevMem); X.back()->alloc((size_t)P.n_loc * k * elem);
    Wt.emplace_back(new DevMem); Wt.back()->alloc((size_t)P.n_loc * k * elem);
    Ub0.emplace_back(new DevMem); Ub0.back()->alloc(std::max<size_t>(P.ub_rows[0], 1) * k * elem);
    Ub1.emplace_back(new DevMem); Ub1.back()->alloc(std::max<size_t>(P.ub_rows[1], 1) * k * elem);
    layers_h[l].X = X[l]->p;
    layers_h[l].Wt = Wt[l]->p;
    layers_h[l].Ub[0] = Ub0[l]->p;
    layers_h[l].Ub[1] = Ub1[l]->p;
  }
  kcap = k;
  upload_layers();
}

const LayerSet& Handle::layer_set(const std::vector<int>& layers) {
  auto it = sets.find(layers);
  if (it != sets.end()) return *it->second;
  auto S = make_set(layers, nullptr);
  auto& ref = *S;
  sets[layers] = std::move(S);
  return ref;
}

// Interface planes of layer l (local z of the extended layer): the top pair
// (s - 1, s) and the bottom pair (e, e + 1), where they exist.
static bool touches(const FrontHost& F, const LayerPlan& P, int mask, int l, int L) {
  if (mask & kPruneAll) return true;
  int pl[4], n = 0;
  if ((mask & kPruneTop) && l >= 1) { pl[n++] = P.s - 1 - P.lo; pl[n++] = P.s - P.lo; }
  if ((mask & kPruneBottom) && l <= L - 2) { pl[n++] = P.e - P.lo; pl[n++] = P.e + 1 - P.lo; }
  for (int i = 0; i < n; ++i)
    if (F.box.lo[2] <= pl[i] && pl[i] < F.box.hi[2]) return true;
  return false;
}

// Launch lists of one local solve of layer l whose sources lie on the
// interface planes of `src` and whose result is read only on those of
// `read` (kPruneTop / kPruneBottom bits).  The right-hand side is zero
// outside the source planes, so a front whose subtree holds none of them has
// a zero forward result and a zero update for its parent: the forward pass
// skips it (and its parent drops it as a child).  Only the values of the
// read-out planes are wanted, and every node is computed by the backward step
// of the front that owns it from the fronts above it, so the backward pass
// keeps the fronts whose subtree holds a read-out plane (with a zero forward
// result where the forward pass skipped them).  The skipped work is exact
// zeros: the result on the read-out planes is the full solve's.
const LayerSet& Handle::pruned_set(int l, int src, int read) {
  const std::vector<int> key{l, src, read};
  auto it = psets.find(key);
  if (it != psets.end()) return *it->second;
  const LayerPlan& P = G.layers[l];
  Prune pr;
  pr.fwd.assign(n_fronts, 1);
  pr.bwd.assign(n_fronts, 1);
  for (size_t q = 0; q < P.fronts.size(); ++q) {
    pr.fwd[front_base[l] + q] = touches(P.fronts[q], P, src, l, G.L);
    pr.bwd[front_base[l] + q] = touches(P.fronts[q], P, read, l, G.L);
  }
  auto S = make_set({l}, &pr);
  auto& ref = *S;
  psets[key] = std::move(S);
  return ref;
}

std::unique_ptr<LayerSet> Handle::make_set(const std::vector<int>& layers, const Prune* pr) {
  auto S = std::make_unique<LayerSet>();
  S->layers = layers;
  int maxd = 0;
  for (int l : layers) maxd = std::max(maxd, G.layers[l].max_depth);
  S->max_depth = maxd;
  // Split a front's K dimension when the depth has too few output tiles to
  // fill the device: aim at ~2048 workgroups, chunks of >= 256.
  const int target = 2048;
  auto split = [&](long long tiles, int K, int& nch, int& kc) {
    nch = 1;
    if (K > 0 && tiles < target / 2) {
      long long want = (target + tiles - 1) / tiles;
      nch = (int)std::max<long long>(1, std::min<long long>(want, K / 256));
    }
    if (K <= 0) { nch = 1; kc = 16; return; }
    kc = (K + nch - 1) / nch;
    kc = (kc + 15) / 16 * 16;
    nch = (K + kc - 1) / kc;
  };
  auto fwd_on = [&](int f) { return !pr || pr->fwd[f]; };
  auto bwd_on = [&](int f) { return !pr || pr->bwd[f]; };
  for (int d = 0; d <= maxd; ++d) {
    auto D = std::make_unique<DepthList>();
    std::vector<int> ids, all;   // backward list (flagged ids: ids_raw)
    for (int l : layers)
      if (d <= G.layers[l].max_depth)
        for (int q : G.layers[l].by_depth[d]) all.push_back(front_base[l] + q);
    std::vector<int> ids_raw;
    for (int f : all)
      if (bwd_on(f)) {
        ids.push_back(f);
        ids_raw.push_back(f | (fwd_on(f) ? 0 : kZeroZ));
      }
    const size_t n = ids.size();
    // backward: every front; a 32-row tile when the pivot blocks are small,
    // K (boundary) split when the depth has few tiles
    double mean_s = 0;
    for (int f : ids) mean_s += fronts_h[f].s;
    mean_s /= std::max<size_t>(n, 1);
    const int bm = mean_s <= 40 ? 32 : 64;
    D->bwd_bm = bm;
    auto tilesB = [&](int s_) { return (s_ + bm - 1) / bm; };
    long long tb = 0;
    for (int f : ids) tb += tilesB(fronts_h[f].s);
    std::vector<SolveTask> tasks(n);
    std::vector<int> pBw(n + 1, 0), rB(n + 1, 0);
    long long scr_b = 0;
    for (size_t a = 0; a < n; ++a) {
      const FrontDev& F = fronts_h[ids[a]];
      SolveTask& t = tasks[a];
      t.nch_f = 1;
      t.kc_f = 16;
      t.scr_f = 0;
      split(tb, F.b, t.nch_b, t.kc_b);
      t.scr_b = scr_b;
      if (t.nch_b > 1) scr_b += (long long)t.nch_b * F.s;
      D->sum_s += F.s;
      D->sum_b += F.b;
      D->sum_sbs += (double)(F.s + F.b) * F.s;
      D->sum_bs += (double)F.b * F.s;
      pBw[a + 1] = pBw[a] + tilesB(F.s) * t.nch_b;
      rB[a + 1] = rB[a] + (t.nch_b > 1 ? tiles16(F.s) : 0);
    }
    // forward: every front takes the GEMM; only fronts with children need
    // the extend-add gather (leaves read their pivots straight from X)
    std::vector<int> idsS, idsL;   // S: fronts with children (gather), L: all
    std::vector<int> idsS_raw, idsL_raw;
    for (int f : all) {
      if (!fwd_on(f)) continue;
      const FrontDev& F = fronts_h[f];
      const double sbs = (double)(F.s + F.b) * F.s;
      int flags = 0;
      for (int c = 0; c < 2; ++c)
        if (F.child[c] >= 0 && !fwd_on(F.child[c])) flags |= kSkipChild0 << c;
      const bool kids = (F.child[0] >= 0 && !(flags & kSkipChild0)) ||
                        (F.child[1] >= 0 && !(flags & kSkipChild1));
      idsL.push_back(f);
      idsL_raw.push_back(f | flags);
      D->fl_s += F.s; D->fl_b += F.b; D->fl_sbs += sbs;
      if (kids) {
        idsS.push_back(f);
        idsS_raw.push_back(f | flags);
        D->fs_s += F.s; D->fs_b += F.b;
      }
    }
    const size_t nl = idsL.size(), ng = idsS.size();
    long long tf = 0;
    for (int f : idsL) tf += tiles64(fronts_h[f].s + fronts_h[f].b);
    std::vector<SolveTask> tasksL(nl);
    std::vector<int> pSB(ng + 1, 0), pF(nl + 1, 0), rF(nl + 1, 0);
    for (size_t a = 0; a < ng; ++a) pSB[a + 1] = pSB[a] + tiles16(fronts_h[idsS[a]].s);
    long long scr_f = 0;
    for (size_t a = 0; a < nl; ++a) {
      const FrontDev& F = fronts_h[idsL[a]];
      SolveTask& t = tasksL[a];
      split(tf, F.s, t.nch_f, t.kc_f);
      t.nch_b = 1;
      t.kc_b = 16;
      t.scr_b = 0;
      t.scr_f = scr_f;
      if (t.nch_f > 1) scr_f += (long long)t.nch_f * (F.s + F.b);
      pF[a + 1] = pF[a] + tiles64(F.s + F.b) * t.nch_f;
      rF[a + 1] = rF[a] + (t.nch_f > 1 ? tiles16(F.s + F.b) : 0);
    }
    D->n = (int)n;
    D->nS = (int)idsS.size();
    D->nL = (int)nl;
    for (int f : ids) S->elems += (double)fronts_h[f].b * fronts_h[f].s;
    for (int f : idsL) S->elems += (double)(fronts_h[f].s + fronts_h[f].b) * fronts_h[f].s;
    upload(D->ids, ids_raw, st);
    upload(D->tasks, tasks, st);
    upload(D->pBw, tile_map(pBw), st);
    upload(D->rB, tile_map(rB), st);
    upload(D->idsS, idsS_raw, st);
    upload(D->idsL, idsL_raw, st);
    upload(D->tasksL, tasksL, st);
    upload(D->pSB, tile_map(pSB), st);
    upload(D->pF, tile_map(pF), st);
    upload(D->rF, tile_map(rF), st);
    D->tSB = pSB.back();
    D->tF = pF.back();
    D->tBw = pBw.back();
    D->tRF = rF.back();
    D->tRB = rB.back();
    D->scratch_rows = std::max(scr_f, scr_b);
    S->scratch_rows = std::max(S->scratch_rows, D->scratch_rows);
    S->depth.push_back(std::move(D));
  }
  HELM_HIP(hipStreamSynchronize(st));
  return S;
}

double Handle::solve_elems(const LayerSet& set) const { return set.elems; }

void Handle::solve_layers(const LayerSet& set, int k) {
  size_t need = (size_t)std::max<long long>(set.scratch_rows, 1) * std::max(k, kcap) * elem;
  if (scratch.bytes < need) {
    HELM_HIP(hipStreamSynchronize(st));
    clear_graphs();
    scratch.alloc(need);
  }
  // The ~35 dependent launches of one multi-RHS solve are captured once per
  // (layer set, width) into a HIP graph and replayed; the sequence holds no
  // memset or host work.  Event timing needs the launches one by one.
  (void)tile_plan(set, k);   // measured choices, if asked for, are taken here
  const bool use_graph = capture && !profile() && !(opt.flags & HELM_FLAG_NO_GRAPHS);
  if (use_graph) {
    GraphKey key{&set, k};
    auto it = graphs.find(key);
    if (it == graphs.end()) {
      // Captured on a stream of its own that does not synchronize with the
      // legacy default stream: while a stream that does is capturing, work
      // that another thread puts on the legacy stream (an allocation by the
      // caller, say) is an error.  A capture records and runs nothing, so
      // the stream it is recorded on needs no ordering with st.
      if (!cap_st) HELM_HIP(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
      struct Restore {
        hipStream_t& s;
        hipStream_t keep;
        ~Restore() { s = keep; }
      } restore{st, st};
      st = cap_st;
      hipGraph_t g = nullptr;
      HELM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        if (prec == HELM_FP64) solve_layers_t<double>(set, k); else solve_layers_t<float>(set, k);
      } catch (...) {
        if (hipStreamEndCapture(st, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
        throw;
      }
      HELM_HIP(hipStreamEndCapture(st, &g));
      hipGraphExec_t ex;
      const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HELM_HIP(ie);
      it = graphs.emplace(key, ex).first;
    }
    HELM_HIP(hipGraphLaunch(it->second, st));
  } else {
    if (prec == HELM_FP64) solve_layers_t<double>(set, k); else solve_layers_t<float>(set, k);
  }
  layer_solves += (long long)set.layers.size();
  solve_bytes += solve_elems(set) * (double)elem;
}

// Tile width from the batch width alone: the vector path for k <= 2 (up to
// 4 columns it is one of the measured candidates), else the narrowest MFMA
// tile of 16 / 32 / 64 columns that covers k (wider batches take several
// 64-column tiles).
static int mfma_bn(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : 64); }
static int width_bn(int k) { return k <= 2 ? 1 : mfma_bn(k); }

// One depth's forward / backward GEMM launch with column width bn (1: the
// vector path).
template <typename T>
void Handle::launch_fwd(const DepthList& D, const FrontDev* fr, const LayerDev* ld, int k,
                        void* scr, int bn, hipEvent_t t0, hipEvent_t t1) {
  if (bn == 1)
    kern::launch_fwd_gemv<T>(fr, D.idsL.as<int>(), D.tasksL.as<SolveTask>(), D.nL,
                             D.pF.as<int2>(), D.tF, ld, k, scr, st, t0, t1);
  else
    kern::launch_fwd_gemm<T>(fr, D.idsL.as<int>(), D.tasksL.as<SolveTask>(), D.nL,
                             D.pF.as<int2>(), D.tF, ld, k, scr, bn, gemm3m, st, t0, t1);
}
template <typename T>
void Handle::launch_bwd(const DepthList& D, const FrontDev* fr, const LayerDev* ld, int k,
                        void* scr, int bn, hipEvent_t t0, hipEvent_t t1) {
  if (bn == 1)
    kern::launch_bwd_gemv<T>(fr, D.ids.as<int>(), D.tasks.as<SolveTask>(), D.n,
                             D.pBw.as<int2>(), D.tBw, ld, k, scr, D.bwd_bm, st, t0, t1);
  else
    kern::launch_bwd_gemm<T>(fr, D.ids.as<int>(), D.tasks.as<SolveTask>(), D.n,
                             D.pBw.as<int2>(), D.tBw, ld, k, scr, D.bwd_bm, bn, gemm3m, st,
                             t0, t1);
}

const std::vector<Handle::TileChoice>& Handle::tile_plan(const LayerSet& set, int k) {
  GraphKey key{&set, k};
  auto it = tiles.find(key);
  if (it != tiles.end()) return it->second;
  std::vector<TileChoice> plan(set.max_depth + 1);
  for (auto& c : plan) c.fwd_bn = c.bwd_bn = width_bn(k);
  if (opt.flags & HELM_FLAG_AUTOTUNE) {
    if (prec == HELM_FP64) autotune_t<double>(set, k, plan);
    else autotune_t<float>(set, k, plan);
  }
  return tiles.emplace(key, std::move(plan)).first->second;
}

// Measured tile choice: every depth's forward and backward GEMM launched
// alone with each admissible width (a width is tried when it is the default
// or narrower than it), best of three launches each, on the solve workspace.
// The right-hand sides already in X are saved and restored around it; the
// other buffers the launches write are rewritten by every solve before they
// are read.
template <typename T>
void Handle::autotune_t(const LayerSet& set, int k, std::vector<TileChoice>& plan) {
  const FrontDev* fr = fronts.as<FrontDev>();
  const LayerDev* ld = layers_d.as<LayerDev>();
  void* scr = scratch.p;
  size_t save_bytes = 0;
  for (int l : set.layers) save_bytes += (size_t)G.layers[l].n_loc * k * elem;
  DevMem save;
  save.alloc(save_bytes);
  {
    size_t off = 0;
    for (int l : set.layers) {
      const size_t b = (size_t)G.layers[l].n_loc * k * elem;
      HELM_HIP(hipMemcpyAsync((char*)save.p + off, X[l]->p, b, hipMemcpyDeviceToDevice, st));
      off += b;
    }
  }
  EventPair ev;
  const int widths[4] = {1, 16, 32, 64};
  auto time_us = [&](auto&& launch) {
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      HELM_HIP(hipEventRecord(ev.a, st));
      launch();
      HELM_HIP(hipEventRecord(ev.b, st));
      best = std::min(best, 1e3 * ev.elapsed_ms(st));
    }
    return best;
  };
  const int widest = mfma_bn(k);
  for (int d = 0; d <= set.max_depth; ++d) {
    const DepthList& D = *set.depth[d];
    TileChoice& c = plan[d];
    c.tuned = true;
    if (D.n == 0) continue;
    auto q = [](double v) { return (long long)std::lround(4.0 * std::log2(1.0 + v)); };
    const std::vector<long long> bucket{k, D.n, q(D.sum_s / D.n), q(D.sum_b / D.n), D.bwd_bm};
    auto hit = tuned.find(bucket);
    if (hit != tuned.end()) {
      c = hit->second;
      continue;
    }
    double bf = 1e30, bb = 1e30;
    for (int w = 0; w < 4; ++w) {
      const int bn = widths[w];
      if (bn > widest || (bn == 1 && k > 4)) continue;
      if (D.nL > 0) {
        double t = time_us([&] {
          launch_fwd<T>(D, fr, ld, k, scr, bn);
        });
        c.t_fwd[w] = t;
        if (t < bf) { bf = t; c.fwd_bn = bn; }
      }
      if (D.bwd_bm == 32 && bn == 16) continue;   // not a distinct tile
      double t = time_us([&] {
        launch_bwd<T>(D, fr, ld, k, scr, bn);
      });
      c.t_bwd[w] = t;
      if (t < bb) { bb = t; c.bwd_bn = bn; }
    }
    tuned[bucket] = c;
  }
  HELM_HIP(hipGetLastError());
  {
    size_t off = 0;
    for (int l : set.layers) {
      const size_t b = (size_t)G.layers[l].n_loc * k * elem;
      HELM_HIP(hipMemcpyAsync(X[l]->p, (char*)save.p + off, b, hipMemcpyDeviceToDevice, st));
      off += b;
    }
  }
  HELM_HIP(hipStreamSynchronize(st));
}

template <typename T>
void Handle::solve_layers_t(const LayerSet& set, int k) {
  run_layers_t<T>(set, k, layers_d.as<LayerDev>(), scratch.p, tile_plan(set, k).data(), true);
}

// The launches of one multi-RHS solve of the layers in `set`: X, Z, the
// update buffers and the layer pointers through the table `ld`, split-K
// partials in `scr`; column-tile widths per depth from `tp`, or from the
// batch width alone when tp is null.  Timing events only when `timing` is
// set and the profiling flags ask for them.
template <typename T>
void Handle::run_layers_t(const LayerSet& set, int k, const LayerDev* ld, void* scr,
                          const TileChoice* tp, bool timing) {
  const FrontDev* fr = fronts.as<FrontDev>();
  auto prof_begin = [&](int cls) { return timing ? this->prof_begin(cls) : nullptr; };
  const double e = (double)elem, kk = (double)k;
  const int wdef = width_bn(k);
  auto fwd_bn = [&](int d) { return tp ? tp[d].fwd_bn : wdef; };
  auto bwd_bn = [&](int d) { return tp ? tp[d].bwd_bn : wdef; };
  for (int d = set.max_depth; d >= 0; --d) {
    const DepthList& D = *set.depth[d];
    if (D.nL == 0) continue;   // (a pruned set may run a front forward only)
    hipEvent_t a = nullptr;
    if (D.nS > 0) {
      a = prof_begin(K_FWD_GATHER);
      kern::launch_fwd_gather<T>(fr, D.idsS.as<int>(), D.nS, D.pSB.as<int2>(), D.tSB, ld, k,
                                 st);
      prof_end(K_FWD_GATHER, a, 0, 3.0 * D.fs_s * kk * e);
    }
    if (D.nL > 0) {
      const int* ids = D.idsL.as<int>();
      const SolveTask* tk = D.tasksL.as<SolveTask>();
      // timed by the launch itself: its start and stop, no event commands
      // between it and its neighbours
      hipEvent_t t0 = nullptr, t1 = nullptr;
      if (timing && timed(K_FWD_GEMM)) {
        t0 = take_event();
        t1 = take_event();
      }
      launch_fwd<T>(D, fr, ld, k, scr, fwd_bn(d), t0, t1);
      // factor block read once; pivots read, Z written, boundary updates
      // written and the children's updates of the boundary rows read
      if (t0)
        pending.push_back(PendingEvent{K_FWD_GEMM, t0, t1, 8.0 * D.fl_sbs * kk,
                                       D.fl_sbs * e + (2.0 * D.fl_s + D.fl_b + D.fs_b) * kk * e});
      if (D.tRF > 0) {
        a = prof_begin(K_FWD_REDUCE);
        kern::launch_fwd_reduce<T>(fr, ids, tk, D.nL, D.rF.as<int2>(), D.tRF, ld, k, scr, st);
        prof_end(K_FWD_REDUCE, a, 0, 0);
      }
    }
  }
  for (int d = 0; d <= set.max_depth; ++d) {
    const DepthList& D = *set.depth[d];
    if (D.n == 0) continue;
    const int* ids = D.ids.as<int>();
    const SolveTask* tk = D.tasks.as<SolveTask>();
    // timed by the launch itself, as the forward GEMM
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timing && timed(K_BWD_GEMM)) {
      t0 = take_event();
      t1 = take_event();
    }
    launch_bwd<T>(D, fr, ld, k, scr, bwd_bn(d), t0, t1);
    // factor block read once; X(B) rows read, Z(S) read, X(S) written
    if (t0)
      pending.push_back(PendingEvent{K_BWD_GEMM, t0, t1, 8.0 * D.sum_bs * kk,
                                     D.sum_bs * e + (D.sum_b + 2.0 * D.sum_s) * kk * e});
    if (D.tRB > 0) {
      hipEvent_t a = prof_begin(K_BWD_REDUCE);
      kern::launch_bwd_reduce<T>(fr, ids, tk, D.n, D.rB.as<int2>(), D.tRB, ld, k, scr, st);
      prof_end(K_BWD_REDUCE, a, 0, 0);
    }
  }
}

template void Handle::solve_layers_t<float>(const LayerSet&, int);
template void Handle::solve_layers_t<double>(const LayerSet&, int);
template void Handle::run_layers_t<float>(const LayerSet&, int, const LayerDev*, void*,
                                          const TileChoice*, bool);
template void Handle::run_layers_t<double>(const LayerSet&, int, const LayerDev*, void*,
                                           const TileChoice*, bool);

const LayerSet* Handle::find_layer_set(const std::vector<int>& layers) const {
  auto it = sets.find(layers);
  return it == sets.end() ? nullptr : it->second.get();
}

}  // namespace helm
