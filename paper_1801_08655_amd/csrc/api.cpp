// C ABI of the library (declarations and contracts in include/helm.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "api_common.h"

namespace helm {

namespace {
thread_local std::string g_last_error;

helm_options resolve(const helm_options* o) {
  helm_options d;
  helm_default_options(&d);
  if (!o) return d;
  helm_options r = *o;
  if (r.pml_local <= 0) r.pml_local = d.pml_local;
  if (r.gmres_tol <= 0) r.gmres_tol = d.gmres_tol;
  if (r.gmres_max_iter <= 0) r.gmres_max_iter = d.gmres_max_iter;
  if (r.ir_tol <= 0) r.ir_tol = d.ir_tol;
  if (r.ir_max_steps <= 0) r.ir_max_steps = d.ir_max_steps;
  if (r.inner_tol <= 0) r.inner_tol = d.inner_tol;
  if (r.inner_tol_refine <= 0) r.inner_tol_refine = r.inner_tol;
  if (r.max_rhs <= 0) r.max_rhs = d.max_rhs;
  if (r.leaf_size <= 0) r.leaf_size = d.leaf_size;
  if (r.gmres_restart < 0) r.gmres_restart = 0;
  return r;
}

double max_velocity(const std::vector<double>& m) {
  double mmin = INFINITY;
  for (double v : m) mmin = std::min(mmin, v);
  return 1.0 / std::sqrt(mmin);
}

void check_model(const std::vector<double>& m) {
  for (double v : m)
    HELM_REQUIRE(std::isfinite(v) && v > 0, HELM_EINVAL,
                 "squared slowness must be finite and positive");
}

Method& method_for(helm_handle* h, int k) {
  if (!h->method || h->method->k != k) {
    h->method.reset();
    h->method.reset(new Method(h->impl, k));
  }
  return *h->method;
}

int factorize_common(const helm_grid* g, const double* m, bool on_device, double omega,
                     int pml_width, int n_layers, const helm_options* opt,
                     helm_handle** out) {
  HELM_REQUIRE(g && m && out, HELM_EINVAL, "null argument");
  *out = nullptr;
  helm_options o = resolve(opt);
  const long long N = (long long)g->nx * g->ny * g->nz;
  HELM_REQUIRE(N > 0, HELM_EINVAL, "empty grid");
  std::vector<double> mh((size_t)N);
  if (on_device) {
    HELM_HIP(hipSetDevice(o.device));
    HELM_HIP(hipMemcpy(mh.data(), m, N * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(mh.data(), m, N * sizeof(double));
  }
  check_model(mh);
  double C = o.pml_C > 0 ? o.pml_C : 20.0 * max_velocity(mh);
  std::unique_ptr<helm_handle> h(new helm_handle);
  Handle& H = h->impl;
  using clk = std::chrono::steady_clock;
  auto since = [](clk::time_point t) { return std::chrono::duration<double>(clk::now() - t).count(); };
  auto t0 = clk::now();
  build_geometry(H.G, *g, omega, pml_width, n_layers, o.pml_local, C, o.leaf_size);
  H.symbolic_seconds = since(t0);
  t0 = clk::now();
  H.init_device(o);
  (void)noalloc_scratch(H.device);   // set-up of the allocation-free entry point
  H.upload_geometry(mh.data(), false);
  H.build_fronts();
  HELM_HIP(hipStreamSynchronize(H.st));
  H.setup_seconds = since(t0);
  H.factorize();
  // the launch lists of every single-layer solve (the sweeps' unit of work)
  t0 = clk::now();
  for (int l = 0; l < H.G.L; ++l) H.single_sets.push_back(&H.layer_set({l}));
  H.lists_seconds = since(t0);
  *out = h.release();
  return HELM_OK;
}

}  // namespace

void set_last_error(const std::string& s) { g_last_error = s; }
const char* last_error_cstr() { return g_last_error.c_str(); }

}  // namespace helm

using namespace helm;

extern "C" {

void helm_default_options(helm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->pml_local = 4;
  o->pml_C = 0.0;
  o->precision = HELM_MIXED;
  o->gmres_tol = 1e-10;
  o->gmres_max_iter = 40;
  o->ir_tol = 1e-9;
  o->ir_max_steps = 6;
  o->inner_tol = 5e-4;
  o->inner_tol_refine = 2e-4;
  o->err_target = 0.0;
  o->hbm_budget_bytes = 0;
  o->device = 0;
  o->stream = nullptr;
  o->max_rhs = 64;
  o->leaf_size = 64;
  o->flags = 0;
  o->gmres_restart = 0;
  o->inner_tol_final = 1e-1;
}

int helm_plan(const helm_grid* g, int pml_width, int n_layers, const helm_options* opt,
              size_t* factor_bytes, size_t* bytes_per_rhs, size_t* max_front) {
  return guard([&] {
    HELM_REQUIRE(g, HELM_EINVAL, "null grid");
    helm_options o = resolve(opt);
    Geometry G;
    // omega and C do not change the symbolic plan
    build_geometry(G, *g, 1.0, pml_width, n_layers, o.pml_local, 1.0, o.leaf_size);
    size_t elem = o.precision == HELM_FP64 ? 16 : 8;
    if (factor_bytes) *factor_bytes = plan_factor_elems(G) * elem;
    if (bytes_per_rhs) *bytes_per_rhs = plan_bytes_per_rhs(G, elem);
    if (max_front) {
      long long mf = 0;
      for (const auto& P : G.layers) mf = std::max(mf, P.max_front);
      *max_front = (size_t)mf;
    }
    return HELM_OK;
  });
}

int helm_plan_lane(const helm_grid* g, int pml_width, int n_layers, const helm_options* opt,
                   size_t* lane_bytes_per_rhs) {
  return guard([&] {
    HELM_REQUIRE(g, HELM_EINVAL, "null grid");
    helm_options o = resolve(opt);
    Geometry G;
    build_geometry(G, *g, 1.0, pml_width, n_layers, o.pml_local, 1.0, o.leaf_size);
    const size_t elem = o.precision == HELM_FP64 ? 16 : 8;
    if (lane_bytes_per_rhs) *lane_bytes_per_rhs = lane_bytes_per_slot(G, elem);
    return HELM_OK;
  });
}

int helm_factorize(const helm_grid* g, const double* m, double omega, int pml_width,
                   int n_layers, const helm_options* opt, helm_handle** out) {
  return guard([&] {
    return factorize_common(g, m, false, omega, pml_width, n_layers, opt, out);
  });
}

int helm_factorize_dev(const helm_grid* g, const double* m_dev, double omega,
                       int pml_width, int n_layers, const helm_options* opt,
                       helm_handle** out) {
  return guard([&] {
    return factorize_common(g, m_dev, true, omega, pml_width, n_layers, opt, out);
  });
}

int helm_solve_dev(helm_handle* h, int n_rhs, const double* f_dev, double* u_dev,
                   helm_solve_info* info) {
  return guard([&] {
    HELM_REQUIRE(h && f_dev && u_dev && n_rhs >= 0, HELM_EINVAL, "bad argument");
    Handle& H = h->impl;
    HELM_HIP(hipSetDevice(H.device));
    if (info) {
      // the caller's per-right-hand-side arrays survive the reset
      double* rr = info->rhs_rel_residual;
      double* re = info->rhs_est_error;
      int* rs = info->rhs_ir_steps;
      int* rg = info->rhs_gmres_iters;
      std::memset(info, 0, sizeof(*info));
      info->n_rhs = n_rhs;
      info->rhs_rel_residual = rr;
      info->rhs_est_error = re;
      info->rhs_ir_steps = rs;
      info->rhs_gmres_iters = rg;
    }
    const long long N = (long long)H.G.nx * H.G.ny * H.G.nz;
    const long long ls0 = H.layer_solves;
    const double sb0 = H.solve_bytes;
    int status = HELM_OK;
    const int kc = std::max(1, H.opt.max_rhs);
    for (int c0 = 0; c0 < n_rhs; c0 += kc) {
      int k = std::min(kc, n_rhs - c0);
      Method& M = method_for(h, k);
      const double2* f = reinterpret_cast<const double2*>(f_dev) + (long long)c0 * N;
      double2* u = reinterpret_cast<double2*>(u_dev) + (long long)c0 * N;
      int s = M.solve(f, u, info, c0);
      if (s != HELM_OK) status = s;
    }
    HELM_HIP(hipStreamSynchronize(H.st));
    // timings are read back when asked for (helm_kernel_stats), or here once
    // many are pending, so that a solve does not spend host time on them
    if (H.pending.size() > (1u << 16)) H.collect_profile();
    if (info) {
      info->layer_solves = H.layer_solves - ls0;
      info->factor_bytes_read = H.solve_bytes - sb0;
    }
    if (status == HELM_ENOCONV) set_last_error("tolerance not reached");
    return status;
  });
}

int helm_solve(helm_handle* h, int n_rhs, const double* f, double* u,
               helm_solve_info* info) {
  return guard([&] {
    HELM_REQUIRE(h && f && u && n_rhs >= 0, HELM_EINVAL, "bad argument");
    Handle& H = h->impl;
    HELM_HIP(hipSetDevice(H.device));
    const long long N = (long long)H.G.nx * H.G.ny * H.G.nz;
    for (long long i = 0; i < 2 * N * n_rhs; ++i)
      HELM_REQUIRE(std::isfinite(f[i]), HELM_EINVAL, "non-finite right-hand side");
    DevMem fd, ud;
    fd.alloc((size_t)N * n_rhs * sizeof(double2));
    ud.alloc((size_t)N * n_rhs * sizeof(double2));
    HELM_HIP(hipMemcpyAsync(fd.p, f, (size_t)N * n_rhs * sizeof(double2),
                            hipMemcpyHostToDevice, H.st));
    int s = helm_solve_dev(h, n_rhs, fd.as<double>(), ud.as<double>(), info);
    if (s != HELM_OK && s != HELM_ENOCONV) return s;
    HELM_HIP(hipMemcpyAsync(u, ud.p, (size_t)N * n_rhs * sizeof(double2),
                            hipMemcpyDeviceToHost, H.st));
    HELM_HIP(hipStreamSynchronize(H.st));
    return s;
  });
}

int helm_solve_points(helm_handle* h, int n_rhs, const int64_t* node_index,
                      const double* amplitude, double* u_dev, helm_solve_info* info) {
  return guard([&] {
    HELM_REQUIRE(h && node_index && amplitude && u_dev && n_rhs >= 0, HELM_EINVAL,
                 "bad argument");
    Handle& H = h->impl;
    HELM_HIP(hipSetDevice(H.device));
    const long long N = (long long)H.G.nx * H.G.ny * H.G.nz;
    for (int r = 0; r < n_rhs; ++r) {
      HELM_REQUIRE(node_index[r] >= 0 && node_index[r] < N, HELM_EINVAL,
                   "point source outside the grid");
      HELM_REQUIRE(std::isfinite(amplitude[2 * r]) && std::isfinite(amplitude[2 * r + 1]),
                   HELM_EINVAL, "non-finite amplitude");
    }
    DevMem fd, nd, ad;
    fd.alloc((size_t)N * n_rhs * sizeof(double2));
    nd.alloc((size_t)std::max(n_rhs, 1) * sizeof(long long));
    ad.alloc((size_t)std::max(n_rhs, 1) * sizeof(double2));
    HELM_HIP(hipMemsetAsync(fd.p, 0, (size_t)N * n_rhs * sizeof(double2), H.st));
    std::vector<long long> nodes(node_index, node_index + n_rhs);
    HELM_HIP(hipMemcpyAsync(nd.p, nodes.data(), n_rhs * sizeof(long long),
                            hipMemcpyHostToDevice, H.st));
    HELM_HIP(hipMemcpyAsync(ad.p, amplitude, n_rhs * sizeof(double2), hipMemcpyHostToDevice,
                            H.st));
    if (n_rhs > 0)
      kern::launch_point_sources(fd.as<double2>(), nd.as<long long>(), ad.as<double2>(),
                                 1.0 / (H.G.h * H.G.h * H.G.h), N, n_rhs, H.st);
    HELM_HIP(hipStreamSynchronize(H.st));
    return helm_solve_dev(h, n_rhs, fd.as<double>(), u_dev, info);
  });
}

int helm_kernel_stats(helm_handle* h, helm_kernel_stat* out, int max, int* count,
                      int reset) {
  return guard([&] {
    HELM_REQUIRE(h, HELM_EINVAL, "null handle");
    Handle& H = h->impl;
    H.collect_profile();
    static const char* names[K_NCLASS] = {
        "solve_fwd_gather", "solve_fwd_gemm", "solve_fwd_reduce", "solve_bwd_gemm",
        "solve_bwd_reduce",
        "factor_sweep_gemm", "factor_panel", "factor_swap_rows", "factor_update_cols",
        "factor_extend_add", "factor_orig_entries", "factor_store"};
    int n = 0;
    for (int c = 0; c < K_NCLASS; ++c) {
      if (out && n < max) {
        helm_kernel_stat& o = out[n];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, names[c], sizeof(o.name) - 1);
        o.launches = H.kstats[c].launches;
        o.total_ms = H.kstats[c].ms;
        o.flops = H.kstats[c].flops;
        o.bytes = H.kstats[c].bytes;
      }
      ++n;
    }
    if (count) *count = n;
    if (reset)
      for (auto& k : H.kstats) k = KStat{};
    return HELM_OK;
  });
}

int helm_tile_choices(helm_handle* h, helm_tile_choice* out, int max, int* count) {
  return guard([&] {
    HELM_REQUIRE(h, HELM_EINVAL, "null handle");
    Handle& H = h->impl;
    int n = 0;
    for (const auto& kv : H.tiles) {
      const LayerSet& S = *kv.first.set;
      for (int d = 0; d <= S.max_depth && d < (int)kv.second.size(); ++d) {
        const DepthList& D = *S.depth[d];
        const Handle::TileChoice& c = kv.second[d];
        if (out && n < max) {
          helm_tile_choice& o = out[n];
          std::memset(&o, 0, sizeof(o));
          o.set_layers = (int)S.layers.size();
          o.k = kv.first.k;
          o.depth = d;
          o.fronts = D.n;
          o.mean_s = D.n ? D.sum_s / D.n : 0.0;
          o.mean_b = D.n ? D.sum_b / D.n : 0.0;
          o.fwd_bn = c.fwd_bn;
          o.bwd_bn = (D.bwd_bm == 32 && c.bwd_bn == 16) ? 32 : c.bwd_bn;
          o.bwd_bm = D.bwd_bm;
          o.tuned = c.tuned ? 1 : 0;
          for (int w = 0; w < 4; ++w) {
            o.t_fwd_us[w] = c.t_fwd[w];
            o.t_bwd_us[w] = c.t_bwd[w];
          }
          o.fwd_elems = D.fl_sbs;
          o.bwd_elems = D.sum_bs;
        }
        ++n;
      }
    }
    if (count) *count = n;
    return HELM_OK;
  });
}

int helm_set_solve_options(helm_handle* h, const helm_options* opt) {
  return guard([&] {
    HELM_REQUIRE(h && opt, HELM_EINVAL, "null argument");
    helm_options o = resolve(opt);
    Handle& H = h->impl;
    H.opt.gmres_tol = o.gmres_tol;
    H.opt.gmres_max_iter = o.gmres_max_iter;
    H.opt.gmres_restart = o.gmres_restart;
    H.opt.ir_tol = o.ir_tol;
    H.opt.ir_max_steps = o.ir_max_steps;
    H.opt.inner_tol = o.inner_tol;
    H.opt.inner_tol_refine = o.inner_tol_refine;
    H.opt.inner_tol_final = o.inner_tol_final;
    H.opt.err_target = o.err_target;
    H.opt.max_rhs = o.max_rhs;
    H.opt.flags = o.flags;
    H.set_profile(o.flags);
    return HELM_OK;
  });
}

int helm_get_factor_info(const helm_handle* h, helm_factor_info* out) {
  return guard([&] {
    HELM_REQUIRE(h && out, HELM_EINVAL, "null argument");
    const Handle& H = h->impl;
    std::memset(out, 0, sizeof(*out));
    out->seconds = H.factor_seconds;
    out->lu_flops = H.factor_flops;
    out->gj_flops = H.factor_gj_flops;
    out->pivot_min = H.pivot_min;
    out->pivot_max = H.pivot_max;
    out->diag_max = H.diag_max;
    out->factor_bytes = H.bytes_factors;
    out->n_fronts = H.n_fronts;
    long long mf = 0;
    for (const auto& P : H.G.layers) mf = std::max(mf, P.max_front);
    out->max_front = mf;
    out->symbolic_seconds = H.symbolic_seconds;
    out->setup_seconds = H.setup_seconds;
    out->lists_seconds = H.lists_seconds;
    return HELM_OK;
  });
}

int helm_free(helm_handle* h) {
  return guard([&] {
    if (!h) return HELM_OK;
    (void)hipSetDevice(h->impl.device);
    h->method.reset();
    delete h;
    return HELM_OK;
  });
}

const char* helm_strerror(int status) {
  switch (status) {
    case HELM_OK: return "success";
    case HELM_EINVAL: return "invalid argument";
    case HELM_ENOMEM: return "out of memory (plan exceeds the budget or allocation failed)";
    case HELM_EZEROPIVOT: return "zero or non-finite pivot";
    case HELM_ENOCONV: return "iteration limit reached before the tolerance";
    case HELM_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* helm_last_error(void) { return helm::last_error_cstr(); }

int helm_layer_info(const helm_handle* h, int l, int* s, int* e, int* lo, int* hi) {
  return guard([&] {
    HELM_REQUIRE(h, HELM_EINVAL, "null handle");
    const Geometry& G = h->impl.G;
    HELM_REQUIRE(l >= 0 && l < G.L, HELM_EINVAL, "layer index out of range");
    const LayerPlan& P = G.layers[l];
    if (s) *s = P.s;
    if (e) *e = P.e;
    if (lo) *lo = P.lo;
    if (hi) *hi = P.hi;
    return HELM_OK;
  });
}

int helm_layer_solve_dev(helm_handle* h, int l, int k, const double* r_dev, double* w_dev) {
  return guard([&] {
    HELM_REQUIRE(h && r_dev && w_dev && k >= 1, HELM_EINVAL, "bad argument");
    Handle& H = h->impl;
    HELM_REQUIRE(l >= 0 && l < H.G.L, HELM_EINVAL, "layer index out of range");
    HELM_HIP(hipSetDevice(H.device));
    H.ensure_workspace(k);
    const LayerSet& S = H.layer_set({l});
    const double2* r = reinterpret_cast<const double2*>(r_dev);
    double2* w = reinterpret_cast<double2*>(w_dev);
    if (H.prec == HELM_FP64) kern::launch_local_to_X<double>(H.layers_h[l], r, k, H.st);
    else kern::launch_local_to_X<float>(H.layers_h[l], r, k, H.st);
    H.solve_layers(S, k);
    if (H.prec == HELM_FP64) kern::launch_X_to_local<double>(H.layers_h[l], w, k, H.st);
    else kern::launch_X_to_local<float>(H.layers_h[l], w, k, H.st);
    HELM_HIP(hipGetLastError());
    HELM_HIP(hipStreamSynchronize(H.st));
    return HELM_OK;
  });
}

int helm_apply_operator_dev(helm_handle* h, int k, const double* f_dev, const double* u_dev,
                            double* r_dev) {
  return guard([&] {
    HELM_REQUIRE(h && u_dev && r_dev && k >= 1, HELM_EINVAL, "bad argument");
    Handle& H = h->impl;
    HELM_HIP(hipSetDevice(H.device));
    kern::launch_residual(H.grid, reinterpret_cast<const double2*>(f_dev),
                          reinterpret_cast<const double2*>(u_dev),
                          reinterpret_cast<double2*>(r_dev), k, H.st);
    HELM_HIP(hipGetLastError());
    HELM_HIP(hipStreamSynchronize(H.st));
    return HELM_OK;
  });
}

int helm_polarized_op_dev(helm_handle* h, int op, int k, const double* in_dev,
                          double* out_dev) {
  return guard([&] {
    HELM_REQUIRE(h && in_dev && out_dev && k >= 1, HELM_EINVAL, "bad argument");
    Handle& H = h->impl;
    HELM_REQUIRE(H.G.L >= 2, HELM_EINVAL, "interface operators need at least two layers");
    HELM_REQUIRE(op >= 0 && op <= 4, HELM_EINVAL, "unknown operator");
    HELM_HIP(hipSetDevice(H.device));
    Method& M = method_for(h, k);
    const double2* in = reinterpret_cast<const double2*>(in_dev);
    double2* out = reinterpret_cast<double2*>(out_dev);
    switch (op) {
      case 0: M.apply_P(in, in + M.Vp, out, out + M.Vp); break;
      case 1: M.apply_A(in, out); break;
      case 2: M.apply_U(in, out); break;
      case 3: M.polarized_rhs(in, out, out + M.Vp); break;
      case 4: M.precondition_source(in, out, out + M.Vp); break;
    }
    HELM_HIP(hipGetLastError());
    HELM_HIP(hipStreamSynchronize(H.st));
    return HELM_OK;
  });
}

}  // extern "C"
