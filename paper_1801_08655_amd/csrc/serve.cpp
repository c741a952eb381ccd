// Request server: continuous batching of point-source requests over resident
// factorizations (contracts in include/helm_serve.h).
//
// One lane per model: K column slots in FP64 volumes F (source), U (iterate),
// R (residual) and D (correction), Methods of widths 1, 2, 4, ..., K on the
// handle's stream, and a host thread.  A lane step is one refinement step
// over the occupied slots, which are kept at the front (Method::refine_step
// at the narrowest width covering them); between steps finished columns are
// copied out, the last live slots move into their places, and queued
// columns take the free slots.  Empty slots inside the width hold zero
// volumes, which every stage of the solve maps to zero (GMRES treats a zero
// right-hand side as converged), so they never change the other columns.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "serve_internal.h"

namespace helm {

double wall_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Account a finished column (lock held).
void Server::finish_column(Request* r, int status, int nsteps, double rel, double est) {
  helm_request_info& I = r->info;
  if (status != HELM_OK && I.status == HELM_OK) I.status = status;
  I.ir_steps_max = std::max(I.ir_steps_max, nsteps);
  I.rel_residual_max = std::max(I.rel_residual_max, rel);
  I.est_error_max = std::max(I.est_error_max, est);
  ++cols_done;
  if (++r->done_cols == r->n) {
    r->finished = true;
    I.t_done_ms = wall_ms() - t0;
    I.latency_ms = I.t_done_ms - I.t_submit_ms;
    lat.push_back(I.latency_ms);
    ++req_done;
    t_last_done = std::max(t_last_done, I.t_done_ms);
    cv_done.notify_all();
  }
}

// The Method of the narrowest width (1, 2, 4, ... up to K) that covers the
// occupied slots; one is created per width on first use.
Method& Lane::method_for(int occ) {
  int w = 1;
  while (w < occ) w *= 2;
  w = std::min(w, K);
  auto it = methods.find(w);
  if (it == methods.end()) {
    it = methods.emplace(w, std::make_unique<Method>(h->impl, w)).first;
    it->second->narrow_allowed = false;   // the lane's memory is planned per slot
  }
  return *it->second;
}

void Server::run_lane(Lane& ln) {
  Handle& H = ln.h->impl;
  (void)hipSetDevice(H.device);
  const long long N = (long long)H.G.nx * H.G.ny * H.G.nz;
  const size_t col_bytes = (size_t)N * sizeof(double2);
  const bool fp64 = H.prec == HELM_FP64;
  const double inv_h3 = 1.0 / (H.G.h * H.G.h * H.G.h);
  Method::StepNorms nm;
  std::vector<int> fresh;
  struct Done { int slot, status, steps; double rel, est; };
  std::vector<Done> done;
  std::vector<std::pair<int, int>> moves;   // (from, to) slot moves after a step
  while (true) {
    fresh.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return stop || ln.retire || ln.occupied() > 0 || !ln.queue.empty();
      });
      if (stop) return;
      if (ln.retire && ln.occupied() == 0 && ln.queue.empty()) return;
      // admission: queued columns take the free slots (after the occupied
      // ones, which are kept at the front), oldest request first
      for (int s = ln.occupied(); s < ln.K && !ln.queue.empty(); ++s) {
        Request* r = ln.queue.front();
        const int c = r->next_col++;
        ln.slots[s] = Slot{r, c, 0, RefineTrack{}};
        if (r->info.t_first_ms < 0) r->info.t_first_ms = wall_ms() - t0;
        ln.node_h[s] = r->nodes[c];
        ln.amp_h[s] = r->amps[c];
        fresh.push_back(s);
        if (r->next_col == r->n) ln.queue.pop_front();
      }
    }
    const int occ = ln.occupied();
    done.clear();
    moves.clear();
    int step_status = HELM_OK;
    std::string step_error;
    try {
      double2* F = ln.F.as<double2>();
      double2* U = ln.U.as<double2>();
      double2* R = ln.R.as<double2>();
      if (!fresh.empty()) {
        HELM_HIP(hipMemcpyAsync(ln.nodes_d.p, ln.node_h.data(), ln.K * sizeof(long long),
                                hipMemcpyHostToDevice, H.st));
        HELM_HIP(hipMemcpyAsync(ln.amps_d.p, ln.amp_h.data(), ln.K * sizeof(double2),
                                hipMemcpyHostToDevice, H.st));
      }
      for (int s : fresh) {
        // new column: f = point source, u = 0, r = f
        HELM_HIP(hipMemsetAsync(F + s * N, 0, col_bytes, H.st));
        HELM_HIP(hipMemsetAsync(U + s * N, 0, col_bytes, H.st));
        kern::launch_point_sources(F + s * N, ln.nodes_d.as<long long>() + s,
                                   ln.amps_d.as<double2>() + s, inv_h3, N, 1, H.st);
        HELM_HIP(hipMemcpyAsync(R + s * N, F + s * N, col_bytes, hipMemcpyDeviceToDevice,
                                H.st));
      }
      // one refinement step over the occupied slots 0..occ-1 at the
      // narrowest width covering them (the extra columns are empty)
      Method& M = ln.method_for(occ);
      const int w = M.k;
      std::vector<double> tol(w, 0.0);
      for (int s = 0; s < w; ++s)
        tol[s] = fp64 ? H.opt.gmres_tol
                      : refinement_tol(ln.slots[s].steps, ln.slots[s].track, H.opt);
      M.refine_step(F, U, R, ln.D.as<double2>(), tol, nm, nullptr);
      std::vector<char> fin(ln.K, 0);
      for (int s = 0; s < occ; ++s) {
        Slot& sl = ln.slots[s];
        const int st = sl.steps++;
        const double rel = nm.rel[s];
        const double teff = M.last_resid.size() > (size_t)s ? M.last_resid[s] : tol[s];
        const double est =
            fp64 ? 0.0 : refinement_error(st, sl.track, nm.dn[s], nm.un[s], teff);
        bool f;
        int status = HELM_OK;
        if (fp64) {
          // one step: GMRES to gmres_tol (a single layer is a direct solve)
          f = true;
          if (H.G.L > 1 && !(M.last_resid.size() > (size_t)s && M.last_resid[s] <= H.opt.gmres_tol))
            status = HELM_ENOCONV;
        } else {
          const bool ok = refinement_met(st, rel, est, H.opt);
          f = ok || sl.steps >= std::max(1, H.opt.ir_max_steps);
          if (!ok) status = HELM_ENOCONV;
        }
        if (!std::isfinite(rel)) { f = true; status = HELM_ENOCONV; }
        if (!f) continue;
        fin[s] = 1;
        HELM_HIP(hipMemcpyAsync(sl.req->out + (long long)sl.col * N, U + s * N, col_bytes,
                                hipMemcpyDefault, H.st));
        HELM_HIP(hipMemsetAsync(F + s * N, 0, col_bytes, H.st));
        HELM_HIP(hipMemsetAsync(U + s * N, 0, col_bytes, H.st));
        HELM_HIP(hipMemsetAsync(R + s * N, 0, col_bytes, H.st));
        done.push_back(Done{s, status, sl.steps, rel, est});
      }
      // keep the occupied slots at the front: the last live slots move down
      // into the holes (their three volumes are copied, the source cleared)
      int lo = 0, hi = occ - 1;
      while (true) {
        while (lo < hi && !fin[lo]) ++lo;
        while (hi > lo && fin[hi]) --hi;
        if (lo >= hi || !fin[lo] || fin[hi]) break;
        for (double2* V : {F, U, R}) {
          HELM_HIP(hipMemcpyAsync(V + lo * N, V + hi * N, col_bytes, hipMemcpyDeviceToDevice,
                                  H.st));
          HELM_HIP(hipMemsetAsync(V + hi * N, 0, col_bytes, H.st));
        }
        moves.push_back({hi, lo});
        fin[lo] = 0;
        fin[hi] = 1;
        ++lo;
        --hi;
      }
      HELM_HIP(hipStreamSynchronize(H.st));
    } catch (const Error& e) {
      step_status = e.code;
      step_error = e.msg;
    } catch (const std::exception& e) {
      step_status = HELM_EINVAL;
      step_error = e.what();
    }
    std::lock_guard<std::mutex> lk(mu);
    ++steps;
    slot_steps += occ;
    if (step_status != HELM_OK) {
      // a failed step ends every column of the lane; the volumes are reset
      // before the lane takes new columns
      set_last_error(step_error);
      for (int s = 0; s < ln.K; ++s) {
        Slot& sl = ln.slots[s];
        if (!sl.req) continue;
        finish_column(sl.req, step_status, sl.steps, INFINITY, INFINITY);
        sl = Slot{};
      }
      (void)hipGetLastError();
      (void)hipMemsetAsync(ln.F.p, 0, ln.F.bytes, H.st);
      (void)hipMemsetAsync(ln.U.p, 0, ln.U.bytes, H.st);
      (void)hipMemsetAsync(ln.R.p, 0, ln.R.bytes, H.st);
      (void)hipStreamSynchronize(H.st);
      continue;
    }
    for (const Done& d : done) {
      Slot& sl = ln.slots[d.slot];
      finish_column(sl.req, d.status, d.steps, d.rel, d.est);
      sl = Slot{};
    }
    for (const auto& mv : moves) {
      ln.slots[mv.second] = ln.slots[mv.first];
      ln.slots[mv.first] = Slot{};
    }
  }
}


int Server::add_model(helm_handle* h, int max_slots, int* slots_out) {
  Handle& H = h->impl;
  HELM_REQUIRE(H.device == opt.device, HELM_EINVAL, "handle lives on another device");
  HELM_HIP(hipSetDevice(H.device));
  std::lock_guard<std::mutex> lk(mu);
  for (auto& l : lanes) HELM_REQUIRE(l->gone || l->h != h, HELM_EINVAL, "handle already served");
  const size_t per = lane_bytes_per_slot(H.G, H.elem);
  size_t free_b = 0, total_b = 0;
  HELM_HIP(hipMemGetInfo(&free_b, &total_b));
  // memory admission: the largest slot count whose workspace fits
  int K = std::max(1, max_slots);
  auto fits = [&](int k) {
    // the lane's full-width workspace plus the Krylov and sweep vectors of
    // its narrower widths (together at most those of one more full width)
    const size_t ws = per * (size_t)k;
    if (opt.hbm_budget_bytes) return reserved + H.bytes_factors + ws <= opt.hbm_budget_bytes;
    return ws <= (size_t)(0.9 * (double)free_b);
  };
  while (K > 1 && !fits(K)) K /= 2;
  HELM_REQUIRE(fits(K), HELM_ENOMEM, "model does not fit the server's memory budget");
  std::unique_ptr<Lane> ln(new Lane);
  ln->model = (int)lanes.size();
  ln->h = h;
  ln->K = K;
  ln->bytes = H.bytes_factors + per * (size_t)K;
  const long long N = (long long)H.G.nx * H.G.ny * H.G.nz;
  const size_t vol = (size_t)N * K * sizeof(double2);
  ln->F.alloc(vol);
  ln->U.alloc(vol);
  ln->R.alloc(vol);
  ln->D.alloc(vol);
  ln->nodes_d.alloc(K * sizeof(long long));
  ln->amps_d.alloc(K * sizeof(double2));
  for (DevMem* d : {&ln->F, &ln->U, &ln->R}) HELM_HIP(hipMemsetAsync(d->p, 0, vol, H.st));
  HELM_HIP(hipStreamSynchronize(H.st));
  h->method.reset();   // the lane's Methods own the solve workspace from here
  H.capture = false;   // launched one by one while the lane's thread drives it
  H.ensure_workspace(K);
  ln->methods.emplace(K, std::make_unique<Method>(H, K))
      .first->second->narrow_allowed = false;
  ln->slots.assign(K, Slot{});
  ln->node_h.assign(K, 0);
  ln->amp_h.assign(K, make_double2(0, 0));
  Lane* lp = ln.get();
  reserved += ln->bytes;
  lanes.push_back(std::move(ln));
  lp->th = std::thread([this, lp] { run_lane(*lp); });
  if (slots_out) *slots_out = K;
  return lp->model;
}

Request* Server::submit(int model, int n, const int64_t* nodes, const double* amps,
                        double* u) {
  Lane* ln = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    HELM_REQUIRE(!stop, HELM_EINVAL, "server is stopping");
    HELM_REQUIRE(model >= 0 && model < (int)lanes.size() && !lanes[model]->retire,
                 HELM_EINVAL, "unknown model");
    ln = lanes[model].get();
  }
  const Geometry& G = ln->h->impl.G;
  const long long N = (long long)G.nx * G.ny * G.nz;
  std::unique_ptr<Request> r(new Request);
  r->n = n;
  r->model = model;
  r->out = reinterpret_cast<double2*>(u);
  r->nodes.resize(n);
  r->amps.resize(n);
  for (int c = 0; c < n; ++c) {
    HELM_REQUIRE(nodes[c] >= 0 && nodes[c] < N, HELM_EINVAL, "point source outside the grid");
    HELM_REQUIRE(std::isfinite(amps[2 * c]) && std::isfinite(amps[2 * c + 1]), HELM_EINVAL,
                 "non-finite amplitude");
    r->nodes[c] = nodes[c];
    r->amps[c] = make_double2(amps[2 * c], amps[2 * c + 1]);
  }
  std::lock_guard<std::mutex> lk(mu);
  // the model may have been removed since the check above
  HELM_REQUIRE(!stop && !ln->retire, HELM_EINVAL, "model removed or server stopping");
  r->id = next_id++;
  r->info.status = HELM_OK;
  r->info.n_rhs = n;
  r->info.model = model;
  r->info.t_submit_ms = wall_ms() - t0;
  r->info.t_first_ms = -1;
  if (t_first_submit < 0) t_first_submit = r->info.t_submit_ms;
  Request* rp = r.get();
  reqs.emplace(r->id, std::move(r));
  if (n == 0) {
    rp->finished = true;
    rp->info.t_first_ms = rp->info.t_done_ms = rp->info.t_submit_ms;
    cv_done.notify_all();
  } else {
    ln->queue.push_back(rp);
    cv_work.notify_all();
  }
  return rp;
}

void Server::remove_model(int model) {
  Lane* ln = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    HELM_REQUIRE(model >= 0 && model < (int)lanes.size() && !lanes[model]->retire,
                 HELM_EINVAL, "unknown model");
    ln = lanes[model].get();
    ln->retire = true;
  }
  cv_work.notify_all();
  if (ln->th.joinable()) ln->th.join();
  Handle& H = ln->h->impl;
  (void)hipSetDevice(H.device);
  HELM_HIP(hipStreamSynchronize(H.st));
  ln->methods.clear();
  H.capture = true;
  for (DevMem* d : {&ln->F, &ln->U, &ln->R, &ln->D, &ln->nodes_d, &ln->amps_d}) d->release();
  std::lock_guard<std::mutex> lk(mu);
  reserved -= ln->bytes;
  ln->gone = true;
}

void Server::shutdown() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_work.notify_all();
  for (auto& l : lanes)
    if (l->th.joinable()) l->th.join();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : reqs) {
      Request* r = kv.second.get();
      if (!r->finished) {
        r->finished = true;
        r->info.status = HELM_EINVAL;
      }
    }
    cv_done.notify_all();
  }
  for (auto& l : lanes) {
    if (l->gone) continue;
    (void)hipSetDevice(l->h->impl.device);
    (void)hipStreamSynchronize(l->h->impl.st);
    l->methods.clear();
  }
}

}  // namespace helm

struct helm_server {
  helm::Server impl;
};

using namespace helm;

extern "C" {

void helm_server_default_options(helm_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget_bytes = 0;
  o->slots = 32;
  o->device = 0;
}

int helm_server_create(const helm_server_options* opt, helm_server** out) {
  return guard([&] {
    HELM_REQUIRE(out, HELM_EINVAL, "null argument");
    *out = nullptr;
    std::unique_ptr<helm_server> s(new helm_server);
    helm_server_default_options(&s->impl.opt);
    if (opt) s->impl.opt = *opt;
    if (s->impl.opt.slots <= 0) s->impl.opt.slots = 32;
    HELM_HIP(hipSetDevice(s->impl.opt.device));
    s->impl.t0 = wall_ms();
    *out = s.release();
    return HELM_OK;
  });
}

int helm_server_add_model(helm_server* sv, helm_handle* h, int* model_id, int* slots_out) {
  return guard([&] {
    HELM_REQUIRE(sv && h && model_id, HELM_EINVAL, "null argument");
    *model_id = sv->impl.add_model(h, sv->impl.opt.slots, slots_out);
    return HELM_OK;
  });
}

int helm_server_remove_model(helm_server* sv, int model_id) {
  return guard([&] {
    HELM_REQUIRE(sv, HELM_EINVAL, "null server");
    sv->impl.remove_model(model_id);
    return HELM_OK;
  });
}

int helm_server_submit(helm_server* sv, int model_id, int n_rhs, const int64_t* node_index,
                       const double* amplitude, double* u, int64_t* request_id) {
  return guard([&] {
    HELM_REQUIRE(sv && request_id && n_rhs >= 0, HELM_EINVAL, "bad argument");
    HELM_REQUIRE(n_rhs == 0 || (node_index && amplitude && u), HELM_EINVAL, "null argument");
    *request_id = sv->impl.submit(model_id, n_rhs, node_index, amplitude, u)->id;
    return HELM_OK;
  });
}

int helm_server_wait(helm_server* sv, int64_t request_id, helm_request_info* info) {
  return guard([&] {
    HELM_REQUIRE(sv, HELM_EINVAL, "null server");
    Server& S = sv->impl;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.reqs.find(request_id);
    HELM_REQUIRE(it != S.reqs.end(), HELM_EINVAL, "unknown request (or already waited for)");
    Request* r = it->second.get();
    S.cv_done.wait(lk, [&] { return r->finished; });
    if (info) *info = r->info;
    int st = r->info.status;
    S.reqs.erase(it);
    if (st != HELM_OK) set_last_error(st == HELM_ENOCONV ? "tolerance not reached" : "request failed");
    return st;
  });
}

int helm_server_poll(helm_server* sv, int64_t request_id, int* done) {
  return guard([&] {
    HELM_REQUIRE(sv && done, HELM_EINVAL, "null argument");
    Server& S = sv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(request_id);
    HELM_REQUIRE(it != S.reqs.end(), HELM_EINVAL, "unknown request (or already waited for)");
    *done = it->second->finished ? 1 : 0;
    return HELM_OK;
  });
}

int helm_server_get_stats(helm_server* sv, helm_server_summary* out) {
  return guard([&] {
    HELM_REQUIRE(sv && out, HELM_EINVAL, "null argument");
    Server& S = sv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    std::memset(out, 0, sizeof(*out));
    out->requests_done = S.req_done;
    out->columns_done = S.cols_done;
    out->steps = S.steps;
    out->bytes_reserved = S.reserved;
    out->mean_active_slots = S.steps ? S.slot_steps / S.steps : 0.0;
    if (!S.lat.empty()) {
      std::vector<double> v = S.lat;
      std::sort(v.begin(), v.end());
      auto pct = [&](double q) {
        size_t i = (size_t)std::ceil(q / 100.0 * v.size());
        return v[std::min(v.size() - 1, i > 0 ? i - 1 : 0)];
      };
      out->p50_ms = pct(50);
      out->p99_ms = pct(99);
      double sum = 0;
      for (double x : v) sum += x;
      out->mean_ms = sum / v.size();
    }
    if (S.t_first_submit >= 0 && S.t_last_done > S.t_first_submit) {
      out->elapsed_s = (S.t_last_done - S.t_first_submit) * 1e-3;
      out->columns_per_s = S.cols_done / out->elapsed_s;
    }
    return HELM_OK;
  });
}

int helm_server_free(helm_server* sv) {
  return guard([&] {
    if (!sv) return HELM_OK;
    sv->impl.shutdown();
    delete sv;
    return HELM_OK;
  });
}

}  // extern "C"
