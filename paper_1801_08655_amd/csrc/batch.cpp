// Batched solves of independent problems (contracts in include/helm_batch.h):
// admission by planned memory, factorization of the next problem overlapped
// with the solves of the resident ones, one request-server lane per problem.
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/helm_batch.h"
#include "serve_internal.h"

using namespace helm;

namespace {

struct Resident {
  int idx;
  int model;
  helm_handle* h;
  Request* req;
  size_t bytes;
};

}  // namespace

extern "C" {

void helm_batch_default_options(helm_batch_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  helm_default_options(&o->opt);
  o->hbm_budget_bytes = 0;
  o->slots = 64;
  o->max_resident = 0;
}

int helm_solve_batch(int n, const helm_problem* P, const helm_batch_options* bo,
                     helm_problem_info* info, helm_batch_summary* summary) {
  return guard([&] {
    HELM_REQUIRE(n >= 0 && (n == 0 || P), HELM_EINVAL, "null problem array");
    helm_batch_options o;
    if (bo) o = *bo; else helm_batch_default_options(&o);
    if (o.slots <= 0) o.slots = 64;
    for (int i = 0; i < n; ++i) {
      const helm_problem& p = P[i];
      HELM_REQUIRE(p.m && p.n_rhs >= 0 && p.grid.nx > 0 && p.grid.ny > 0 && p.grid.nz > 0,
                   HELM_EINVAL, "problem " + std::to_string(i) + ": bad grid or model");
      HELM_REQUIRE(p.n_rhs == 0 || (p.node_index && p.amplitude && p.u), HELM_EINVAL,
                   "problem " + std::to_string(i) + ": null source or output array");
    }
    const double t0 = wall_ms();
    HELM_HIP(hipSetDevice(o.opt.device));
    size_t budget = o.hbm_budget_bytes;
    if (!budget) {
      size_t free_b = 0, total_b = 0;
      HELM_HIP(hipMemGetInfo(&free_b, &total_b));
      budget = (size_t)(0.9 * (double)free_b);
    }
    std::vector<helm_problem_info> inf((size_t)n);
    for (auto& I : inf) std::memset(&I, 0, sizeof(I));
    Server S;
    S.opt.device = o.opt.device;
    S.opt.slots = o.slots;
    S.opt.hbm_budget_bytes = budget;
    S.t0 = t0;
    std::vector<Resident> res;
    size_t planned = 0, peak = 0;
    int max_res = 0;
    double fsum = 0;
    long long cols = 0;
    int next = 0;
    try {
      while (next < n || !res.empty()) {
        // admission in order while the plan fits
        while (next < n && (o.max_resident <= 0 || (int)res.size() < o.max_resident)) {
          const helm_problem& p = P[next];
          helm_problem_info& I = inf[next];
          if (p.n_rhs == 0) {
            I.status = HELM_OK;
            I.t_admit_ms = I.t_done_ms = wall_ms() - t0;
            ++next;
            continue;
          }
          const int K = std::max(1, std::min(p.n_rhs, o.slots));
          size_t fb = 0, br = 0;
          int st = helm_plan(&p.grid, p.pml_width, p.n_layers, &o.opt, &fb, nullptr, nullptr);
          if (st == HELM_OK)
            st = helm_plan_lane(&p.grid, p.pml_width, p.n_layers, &o.opt, &br);
          if (st != HELM_OK) { I.status = st; ++next; continue; }
          // what the server's lane will reserve for K slots
          const size_t need = fb + br * (size_t)K;
          if (planned + need > budget) {
            if (res.empty()) { I.status = HELM_ENOMEM; ++next; continue; }
            break;   // wait for a resident problem to finish
          }
          I.t_admit_ms = wall_ms() - t0;
          I.slots = K;
          I.planned_bytes = need;
          helm_handle* h = nullptr;
          const double tf = wall_ms();
          // the factorization keeps room for the solve workspace of max_rhs
          // columns: the lane's K
          helm_options po = o.opt;
          po.max_rhs = K;
          st = helm_factorize(&p.grid, p.m, p.omega, p.pml_width, p.n_layers, &po, &h);
          I.factor_ms += wall_ms() - tf;
          I.t_factored_ms = wall_ms() - t0;
          fsum += (wall_ms() - tf) * 1e-3;
          // the factorization's transient frontal workspace did not fit beside
          // the resident problems: retry once one of them has finished
          if (st == HELM_ENOMEM && !res.empty()) break;
          if (st != HELM_OK) { I.status = st; ++next; continue; }
          int model = -1;
          try {
            model = S.add_model(h, K, nullptr);
          } catch (const Error& e) {
            helm_free(h);
            I.status = e.code;
            ++next;
            continue;
          }
          Request* r = S.submit(model, p.n_rhs, p.node_index, p.amplitude, p.u);
          planned += need;
          peak = std::max(peak, planned);
          res.push_back(Resident{next, model, h, r, need});
          max_res = std::max(max_res, (int)res.size());
          ++next;
        }
        if (res.empty()) continue;
        // retire the problems that have finished
        std::vector<size_t> fin;
        {
          std::unique_lock<std::mutex> lk(S.mu);
          S.cv_done.wait(lk, [&] {
            for (const Resident& x : res)
              if (x.req->finished) return true;
            return false;
          });
          for (size_t a = 0; a < res.size(); ++a)
            if (res[a].req->finished) fin.push_back(a);
        }
        for (size_t q = fin.size(); q-- > 0;) {
          const Resident x = res[fin[q]];
          helm_problem_info& I = inf[x.idx];
          const helm_request_info& R = x.req->info;
          I.status = R.status;
          I.t_done_ms = R.t_done_ms;
          I.ir_steps_max = R.ir_steps_max;
          I.rel_residual_max = R.rel_residual_max;
          I.est_error_max = R.est_error_max;
          cols += P[x.idx].n_rhs;
          S.remove_model(x.model);
          helm_free(x.h);
          planned -= x.bytes;
          res.erase(res.begin() + (long)fin[q]);
        }
      }
    } catch (...) {
      S.shutdown();
      for (const Resident& x : res) helm_free(x.h);
      throw;
    }
    S.shutdown();
    const double wall = (wall_ms() - t0) * 1e-3;
    int status = HELM_OK;
    for (int i = 0; i < n; ++i) {
      if (info) info[i] = inf[i];
      if (status == HELM_OK && inf[i].status != HELM_OK) status = inf[i].status;
    }
    if (summary) {
      std::memset(summary, 0, sizeof(*summary));
      summary->wall_s = wall;
      summary->factor_s = fsum;
      summary->columns = cols;
      summary->rhs_per_s = wall > 0 ? cols / wall : 0.0;
      summary->max_resident = max_res;
      summary->peak_planned_bytes = peak;
    }
    if (status != HELM_OK) set_last_error("a problem of the batch failed (see its info record)");
    return status;
  });
}

}  // extern "C"
