// Online stage of the method on one batch of k right-hand-side columns.
#pragma once

#include <functional>
#include <map>
#include <memory>
#include <vector>

#include "handle.h"

namespace helm {

struct Method {
  Handle& H;
  int k;
  long long plane = 0, pair_elems = 0, Vp = 0, N = 0;
  DevMem y, zd, zu, keep, dot_partial, hcol, norm_partial, norm_out, scale;
  DevMem fpol, bpol, xpol;   // polarized right-hand side, P b and the iterate
  DevMem vr, vd;             // FP64 volumes: residual and correction
  DevMem vf, vu;             // gathered source and solution (narrowed steps)
  // a narrower batch for the refinement steps that only some columns need
  std::unique_ptr<Method> child;
  bool narrow_ok = true;     // cleared when device memory refused one
  // narrower batches may be created (off for the request server's lanes,
  // whose device memory is planned per slot)
  bool narrow_allowed = true;
  Method* narrower(int w);
  // narrower batches for the operator products of the GMRES iterations
  // whose running columns fit in half the width, by width, with their
  // gathered operand and product
  std::map<int, std::unique_ptr<Method>> krylov_narrow;
  DevMem kv_in, kv_out;
  bool krylov_narrow_ok = true;
  Method* krylov_narrower(int w, long long V);
  const LayerSet* set_all = nullptr;
  const LayerSet* set_lower = nullptr;
  std::vector<const LayerSet*> single;
  std::vector<double> last_resid;
  std::vector<int> col_iters;   // GMRES iterations per column (last call)
  // Krylov basis and temporaries, grown on demand and kept between calls
  std::vector<std::unique_ptr<DevMem>> basis;
  DevMem gw, gr;
  double2* basis_vec(int i);

  Method(Handle& h, int k);

  double2* pair(double2* v, int j) const;
  const double2* pair(const double2* v, int j) const;
  void zero_X(int l);
  template <typename T> void jump_t(int l, const kern::JumpTerms& t, int bottom);
  // X^l += J_top or J_bot (bottom) of ca a + cb b + cc c (b, c may be null)
  void jump(int l, const double2* a, const double2* b, int bottom, double ca = 1.0,
            double cb = 1.0, const double2* c = nullptr, double cc = 1.0);
  void readout(int l, int bottom, double sx, const kern::ReadTerms& t, double2* out);
  // the same terms with only the read-out planes of `mask` written (1: a, 2: b)
  static kern::ReadTerms planes(kern::ReadTerms t, int mask);
  static kern::ReadTerms terms(const double2* a = nullptr, double ca = 0, double cb = 0,
                               const double2* b = nullptr, double cb_a = 0,
                               double cb_b = 0, const double2* c = nullptr,
                               double cc_a = 0, double cc_b = 0);
  void solve_single(int l);
  void solve_planes(int l, int src, int read);
  void apply_P(const double2* vd, const double2* vu, double2* od, double2* ou);
  void apply_U(const double2* xu, double2* out);
  void apply_A(const double2* x, double2* out);
  void scatter_sources(const double2* f);
  void polarized_rhs(const double2* f, double2* fd, double2* fu);
  void precondition_source(const double2* f, double2* od, double2* ou);
  void reconstruct(const double2* f, const double2* tr, double2* u);
  void dot(const double2* a, const double2* b, long long V, double2* out);
  // A linear system for the Krylov solvers: per column, vectors of V
  // elements (column fastest); the Krylov space lives on the elements
  // [off, off + Vs k) of a vector; with `block`, A applied to a vector that
  // is zero below off also returns a part below off that belongs to the
  // solution's down half (the block-triangular polarized system).
  struct KrylovSystem {
    long long V = 0, off = 0, Vs = 0;
    bool block = false;
    bool polarized = false;   // P M (a narrower batch can apply it)
    std::function<void(const double2*, double2*)> apply;
  };
  // S.apply to the columns with run[c] set; the others' products are zero
  // (their operands are zero).  Gathered into a narrower batch when they fit
  // in half the width.
  void apply_running(const KrylovSystem& S, const double2* v, double2* out,
                     const std::vector<char>& run, helm_solve_info* info);
  KrylovSystem polarized_system();
  KrylovSystem sie_system();
  int gmres(const KrylovSystem& S, const double2* b, double2* x,
            const std::vector<double>& tol, int max_iter, int restart, int* iters,
            helm_solve_info* info = nullptr);
  int bicgstab(const KrylovSystem& S, const double2* b, double2* x,
               const std::vector<double>& tol, int max_iter, int* iters);
  void apply_sie(const double2* x, double2* out);
  void sie_rhs(const double2* f, double2* v);
  double krylov_bytes() const;
  int polarized_solve(const double2* f, double2* u, double tol, int max_iter,
                      int restart, helm_solve_info* info);
  int polarized_solve(const double2* f, double2* u, const std::vector<double>& tol,
                      int max_iter, int restart, helm_solve_info* info);
  struct StepNorms {
    std::vector<double> rel, dn, un;
  };
  int refine_step(const double2* F, double2* U, double2* R, double2* D,
                  const std::vector<double>& tol, StepNorms& out, helm_solve_info* info);
  void ensure_volumes();
  void residual(const double2* f, const double2* u, double2* r, std::vector<double>& rel);
  void norms(const double2* x, std::vector<double>& out);
  int solve(const double2* f, double2* u, helm_solve_info* info, int col0 = 0);
  int gmres_restart(int max_iter) const;
};

// Per-column record of the refinement's corrections for the error estimate.
struct RefineTrack {
  double dprev = 0;   // |d| of the previous step
  double qprev = 0;   // contraction ratio measured at the previous step
  double est = 1;     // estimated error after the last step (1: unknown)
};
// Estimated relative error |u - H^-1 f| / |u| after a step whose correction
// has norm dcur and whose GMRES ran to tolerance tol (see method.cpp);
// updates the record.
double refinement_error(int step, RefineTrack& tr, double dcur, double unorm, double tol);
// GMRES tolerance of a column's next step (0-based step index).
double refinement_tol(int step, const RefineTrack& tr, const helm_options& o);
// Whether a column may stop after step `step` (0-based): FP64 residual at
// ir_tol, or estimated error at most a quarter of err_target after the
// second solve (the estimate rests on one measured contraction) and at most
// half of it from the third on.
bool refinement_met(int step, double rel, double est, const helm_options& o);

}  // namespace helm
