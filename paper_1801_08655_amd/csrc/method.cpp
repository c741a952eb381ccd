// Online stage (Algorithm 2): polarized interface system, preconditioned
// GMRES, reconstruction, and FP64 iterative refinement for complex64 factors.
//
// Pair vectors (interface traces) hold, for every interface j = 0..L-2
// between layers j and j+1, the planes (u(e_j), u(e_j + 1)); polarized
// vectors are [x_down | x_up].  With G^l = (H^l)^-1, the interface sources
// J_top/J_bot and the read-outs R_top(w) = (w(s-1), w(s)), R_bot(w) =
// (w(e), w(e+1)), the blocks of Eq. polarized_SIE are
//   (D_down x)_0 = -x_0,      (D_down x)_j = R_bot^j G^j J_top^j(x_{j-1}) - x_j
//   (D_up x)_{L-2} = -x_{L-2}, (D_up x)_j = R_top^{j+1} G^{j+1} J_bot^{j+1}(x_{j+1}) - x_j
//   (L x)_j = R_top^{j+1} G^{j+1}[J_top^{j+1}(x_j) + J_bot^{j+1}(x_{j+1})] - (0, x_{j,b})
//   (U x)_j = R_bot^j G^j [J_top^j(x_{j-1}) + J_bot^j(x_j)] - (x_{j,a}, 0)
// (terms with an index outside 0..L-2 dropped), and the right-hand side is
//   f_down_j = -R_bot^j G^j f^j,  f_up_j = -R_top^{j+1} G^{j+1} f^{j+1}.
// P of Eq. preconditioner_GS is the block Gauss-Seidel inverse, applied by the
// downward sweep (Algorithm 4), the reflections L (Algorithm 6) and the
// upward sweep (Algorithm 5).  As the paper notes, D_down and L can be
// applied together: the solve of the downward sweep at layer l also yields
// the first term of (L x)_{l-1}, and the two solves of the upward step at
// layer j+1 (sweep and the second L term) share one right-hand side by
// linearity.  One application of P costs 2L - 3 sequential layer solves.
// Since P inverts the block lower-triangular part exactly,
//   P M x = x + P (U x_up, 0);
// the local solves of U are folded into those of the sweeps by linearity
// (apply_A), so a GMRES iteration costs 2L - 2 sequential layer solves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "handle.h"
#include "method.h"

namespace helm {

namespace {
double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

Method::Method(Handle& h, int k_) : H(h), k(k_) {
  const int L = H.G.L;
  plane = (long long)H.G.nx * H.G.ny;
  pair_elems = 2 * plane * k;
  Vp = (long long)std::max(L - 1, 0) * pair_elems;   // one pair vector
  N = (long long)H.G.nx * H.G.ny * H.G.nz;
  H.ensure_workspace(k);
  auto a = [&](DevMem& d, long long n) { d.alloc((size_t)std::max<long long>(n, 1) * sizeof(double2)); };
  a(y, Vp); a(zd, Vp); a(zu, Vp); a(keep, Vp);
  a(dot_partial, (long long)k * kern::DOT_PARTIAL_BLOCKS);
  a(hcol, (long long)k * 64);
  norm_partial.alloc((size_t)k * kern::NORM_PARTIAL_BLOCKS * sizeof(double));
  norm_out.alloc((size_t)k * sizeof(double));
  scale.alloc((size_t)k * sizeof(double));
  std::vector<int> all, lower;
  for (int l = 0; l < L; ++l) all.push_back(l);
  for (int l = 0; l + 1 < L; ++l) lower.push_back(l);
  set_all = &H.layer_set(all);
  set_lower = L > 1 ? &H.layer_set(lower) : nullptr;
  for (int l = 0; l < L; ++l) single.push_back(&H.layer_set({l}));
}

double2* Method::pair(double2* v, int j) const { return v + (long long)j * pair_elems; }
const double2* Method::pair(const double2* v, int j) const {
  return v + (long long)j * pair_elems;
}

void Method::zero_X(int l) {
  HELM_HIP(hipMemsetAsync(H.layers_h[l].X, 0,
                          (size_t)H.layers_h[l].n_loc * k * H.elem, H.st));
}

template <typename T>
void Method::jump_t(int l, const kern::JumpTerms& t, int bottom) {
  kern::launch_jump<T>(H.layers_h[l], t, H.Bcoef.as<double2>(), bottom, H.G.nx, H.G.ny, k,
                       H.st);
}
void Method::jump(int l, const double2* a, const double2* b, int bottom, double ca, double cb,
                  const double2* c, double cc) {
  const kern::JumpTerms t{{a, b, c}, {ca, cb, cc}};
  if (H.prec == HELM_FP64) jump_t<double>(l, t, bottom); else jump_t<float>(l, t, bottom);
}

void Method::readout(int l, int bottom, double sx, const kern::ReadTerms& t, double2* out) {
  if (H.prec == HELM_FP64)
    kern::launch_readout<double>(H.layers_h[l], bottom, sx, t, out, H.G.nx, H.G.ny, k, H.st);
  else
    kern::launch_readout<float>(H.layers_h[l], bottom, sx, t, out, H.G.nx, H.G.ny, k, H.st);
}

kern::ReadTerms Method::planes(kern::ReadTerms t, int mask) {
  t.planes = mask;
  return t;
}

kern::ReadTerms Method::terms(const double2* a, double ca, double cb, const double2* b,
                              double cb_a, double cb_b, const double2* c, double cc_a,
                              double cc_b) {
  kern::ReadTerms t{};
  t.planes = 3;
  t.in[0] = a; t.ca[0] = ca; t.cb[0] = cb;
  t.in[1] = b; t.ca[1] = cb_a; t.cb[1] = cb_b;
  t.in[2] = c; t.ca[2] = cc_a; t.cb[2] = cc_b;
  return t;
}

void Method::solve_single(int l) { H.solve_layers(*single[l], k); }

// A single-layer solve whose sources lie on the interface planes of `src`
// and whose result is read on those of `read` (kPruneTop / kPruneBottom):
// the launch lists keep only the fronts those planes reach (the result on
// the read-out planes is unchanged); HELM_FLAG_NO_PRUNE runs every front.
void Method::solve_planes(int l, int src, int read) {
  if (H.opt.flags & HELM_FLAG_NO_PRUNE) solve_single(l);
  else H.solve_layers(H.pruned_set(l, src, read), k);
}

// (zd, zu) = P (vd, vu); vu may be null (zero)
void Method::apply_P(const double2* vd, const double2* vu, double2* od, double2* ou) {
  const int L = H.G.L;
  double2* kp = keep.as<double2>();
  // z_down_0 = -v_down_0
  readout(0, 1, 0.0, terms(pair(vd, 0), -1, -1), pair(od, 0));
  constexpr int T = kPruneTop, B = kPruneBottom;
  for (int l = 1; l <= L - 2; ++l) {
    zero_X(l);
    jump(l, pair(od, l - 1), nullptr, 0);
    solve_planes(l, T, T | B);
    readout(l, 1, 1.0, terms(pair(vd, l), -1, -1), pair(od, l));
    readout(l, 0, 1.0, terms(), pair(kp, l - 1));
  }
  // last layer: only the reflection term is needed
  zero_X(L - 1);
  jump(L - 1, pair(od, L - 2), nullptr, 0);
  solve_planes(L - 1, T, T);
  readout(L - 1, 0, 1.0, terms(), pair(kp, L - 2));
  // upward: z_up_{L-2} = keep_{L-1} - (0, z_down_{L-2,b}) - v_up_{L-2}
  readout(L - 1, 0, 0.0,
          terms(pair(kp, L - 2), 1, 1, pair(od, L - 2), 0, -1,
                vu ? pair(vu, L - 2) : nullptr, -1, -1),
          pair(ou, L - 2));
  for (int j = L - 3; j >= 0; --j) {
    zero_X(j + 1);
    jump(j + 1, pair(ou, j + 1), pair(od, j + 1), 1);
    solve_planes(j + 1, B, T);
    readout(j + 1, 0, 1.0,
            terms(pair(kp, j), 1, 1, pair(od, j), 0, -1, vu ? pair(vu, j) : nullptr, -1, -1),
            pair(ou, j));
  }
}

// y = U x_up
void Method::apply_U(const double2* xu, double2* out) {
  const int L = H.G.L;
  for (int l = 0; l <= L - 2; ++l) {
    zero_X(l);
    if (l >= 1) jump(l, pair(xu, l - 1), nullptr, 0);
    jump(l, pair(xu, l), nullptr, 1);
  }
  H.solve_layers(*set_lower, k);
  for (int l = 0; l <= L - 2; ++l)
    readout(l, 1, 1.0, terms(pair(xu, l), -1, 0), pair(out, l));
}

// out = P M x = x + P (U x_up, 0), with the solves of U folded into the
// sweeps.  With w = U x_up, the downward sweep's step at layer l
// (1 <= l <= L-2) is
//   z_l = R_bot^l G^l J_top^l(z_{l-1}) - w_l
//       = R_bot^l G^l [J_top^l(z_{l-1} - x_{l-1}) - J_bot^l(x_l)] + (x_{l,a}, 0)
// (x = x_up), one local solve instead of two, and z_0 = -w_0 takes one solve of
// layer 0.  The same solve read at the top gives keep_{l-1} - V_{l-1} with
// V_j = R_top^{j+1} G^{j+1} [J_top^{j+1}(x_j) + J_bot^{j+1}(x_{j+1})]; the upward
// step at layer j+1 adds J_top(x_j) + J_bot(x_{j+1}) to its sources, which
// adds V_j back.  The last layer's solve (only keep_{L-2}) keeps its plain
// source.  Cost: 2L - 2 sequential layer solves and no batched U solve.
void Method::apply_A(const double2* x, double2* out) {
  const int L = H.G.L;
  const double2* xd = x;
  const double2* xu = x + Vp;
  double2* od = zd.as<double2>();
  double2* ou = zu.as<double2>();
  double2* kp = keep.as<double2>();
  if (L >= 2) {
    // z_down_0 = -(U x_up)_0
    constexpr int T = kPruneTop, B = kPruneBottom;
    zero_X(0);
    jump(0, pair(xu, 0), nullptr, 1, -1.0);
    solve_planes(0, B, B);
    readout(0, 1, 1.0, terms(pair(xu, 0), 1, 0), pair(od, 0));
    for (int l = 1; l <= L - 2; ++l) {
      zero_X(l);
      jump(l, pair(od, l - 1), pair(xu, l - 1), 0, 1.0, -1.0);
      jump(l, pair(xu, l), nullptr, 1, -1.0);
      solve_planes(l, T | B, T | B);
      readout(l, 1, 1.0, terms(pair(xu, l), 1, 0), pair(od, l));
      readout(l, 0, 1.0, terms(), pair(kp, l - 1));      // keep_{l-1} - V_{l-1}
    }
    zero_X(L - 1);
    jump(L - 1, pair(od, L - 2), nullptr, 0);
    solve_planes(L - 1, T, T);
    readout(L - 1, 0, 1.0, terms(), pair(kp, L - 2));    // keep_{L-2}
    // upward: z_up_{L-2} = keep_{L-2} - (0, z_down_{L-2,b})
    readout(L - 1, 0, 0.0, terms(pair(kp, L - 2), 1, 1, pair(od, L - 2), 0, -1),
            pair(ou, L - 2));
    for (int j = L - 3; j >= 0; --j) {
      zero_X(j + 1);
      jump(j + 1, pair(ou, j + 1), pair(od, j + 1), 1, 1.0, 1.0, pair(xu, j + 1), 1.0);
      jump(j + 1, pair(xu, j), nullptr, 0);
      solve_planes(j + 1, T | B, T);
      readout(j + 1, 0, 1.0, terms(pair(kp, j), 1, 1, pair(od, j), 0, -1), pair(ou, j));
    }
  }
  kern::launch_add(out, xd, od, Vp, H.st);
  kern::launch_add(out + Vp, xu, ou, Vp, H.st);
}

void Method::scatter_sources(const double2* f) {
  for (int l = 0; l < H.G.L; ++l) {
    zero_X(l);
    if (H.prec == HELM_FP64)
      kern::launch_scatter_source<double>(H.layers_h[l], f, H.G.nx, H.G.ny, N, k, H.st);
    else
      kern::launch_scatter_source<float>(H.layers_h[l], f, H.G.nx, H.G.ny, N, k, H.st);
  }
}

// (f_down, f_up) from the volume source f (the first steps of Algorithm 2:
// local solves of the partitioned source and their interface read-outs)
void Method::polarized_rhs(const double2* f, double2* fd, double2* fu) {
  const int L = H.G.L;
  scatter_sources(f);
  H.solve_layers(*set_all, k);
  for (int l = 0; l < L; ++l) {
    if (l <= L - 2) readout(l, 1, -1.0, terms(), pair(fd, l));
    if (l >= 1) readout(l, 0, -1.0, terms(), pair(fu, l - 1));
  }
}

// (od, ou) = P (f_down, f_up) for the volume source f, with the local solves
// of the polarized right-hand side folded into the sweeps by linearity:
//   z_0 = R_bot^0 G^0 f^0,  z_l = R_bot^l G^l [J_top^l(z_{l-1}) + f^l],
// and the top read-out of the same solve is keep_{l-1} - f_up_{l-1}, which is
// the term the upward step subtracts.  2L - 2 sequential layer solves and no
// batched solve over all layers.
void Method::precondition_source(const double2* f, double2* od, double2* ou) {
  const int L = H.G.L;
  constexpr int T = kPruneTop, B = kPruneBottom;
  double2* kp = keep.as<double2>();
  for (int l = 0; l <= L - 1; ++l) {
    zero_X(l);
    if (H.prec == HELM_FP64)
      kern::launch_scatter_source<double>(H.layers_h[l], f, H.G.nx, H.G.ny, N, k, H.st);
    else
      kern::launch_scatter_source<float>(H.layers_h[l], f, H.G.nx, H.G.ny, N, k, H.st);
    if (l >= 1) jump(l, pair(od, l - 1), nullptr, 0);
    solve_planes(l, kPruneAll, T | B);   // volume source: every front forward
    if (l <= L - 2) readout(l, 1, 1.0, terms(), pair(od, l));
    if (l >= 1) readout(l, 0, 1.0, terms(), pair(kp, l - 1));   // keep_{l-1} - f_up_{l-1}
  }
  readout(L - 1, 0, 0.0, terms(pair(kp, L - 2), 1, 1, pair(od, L - 2), 0, -1), pair(ou, L - 2));
  for (int j = L - 3; j >= 0; --j) {
    zero_X(j + 1);
    jump(j + 1, pair(ou, j + 1), pair(od, j + 1), 1);
    solve_planes(j + 1, B, T);
    readout(j + 1, 0, 1.0, terms(pair(kp, j), 1, 1, pair(od, j), 0, -1), pair(ou, j));
  }
}

// u = volume from traces (the reconstruction that ends Algorithm 2)
void Method::reconstruct(const double2* f, const double2* tr, double2* u) {
  const int L = H.G.L;
  scatter_sources(f);
  for (int l = 0; l < L; ++l) {
    if (l >= 1) jump(l, pair(tr, l - 1), nullptr, 0);
    if (l <= L - 2) jump(l, pair(tr, l), nullptr, 1);
  }
  H.solve_layers(*set_all, k);
  for (int l = 0; l < L; ++l) {
    if (H.prec == HELM_FP64)
      kern::launch_gather_volume<double>(H.layers_h[l], u, H.G.nx, H.G.ny, N, k, H.st);
    else
      kern::launch_gather_volume<float>(H.layers_h[l], u, H.G.nx, H.G.ny, N, k, H.st);
  }
}

void Method::dot(const double2* a, const double2* b, long long V, double2* out) {
  kern::launch_dot(a, b, V, k, dot_partial.as<double2>(), out, H.st);
}

// Batched GMRES (one independent Krylov space per column) on P M x = b.
// Arnoldi (modified Gram-Schmidt), norms and basis updates in FP64 on the
// device; the (j+2) x k Hessenberg column is copied to the host where the
// Givens rotations and the stopping test are applied per column.
//
// P M = I + K with K x depending on x_up alone (P M x = x + P(U x_up, 0)), so
// the system is block triangular: (I + K_up) x_up = b_up, then x_down =
// b_down - K_down x_up.  By default the Krylov space is built on the
// up-going block only: a basis vector holds v in its up half and zeros in
// its down half when P M is applied to it; the down half of the result,
// K_down v, is then kept in the basis vector's own down half, so the update
// x += sum y_i v_i accumulates K_down x_up there, and x_down = b_down - that
// at the end.  The stopping test is the same as for the whole system: the
// residual (0, r_up) against |b|.  HELM_FLAG_FULL_KRYLOV runs GMRES on the
// whole polarized system instead.
//
// The same driver solves any KrylovSystem: the unpolarized SIE uses it with
// one pair vector per column and no block structure.
int Method::gmres(const KrylovSystem& S, const double2* b, double2* x,
                  const std::vector<double>& tol, int max_iter, int restart, int* iters_out,
                  helm_solve_info* info) {
  const long long V = S.V;                    // vector length per column
  const int m = std::max(1, std::min(restart, max_iter));
  const bool up = S.block;
  const long long off = S.off;                // first element of the Krylov part
  const long long Vs = S.Vs;                  // its length per column
  if (!gw.p) {
    gw.alloc((size_t)2 * Vp * sizeof(double2));
    gr.alloc((size_t)2 * Vp * sizeof(double2));
  }
  DevMem& w = gw;
  DevMem& r = gr;
  HELM_HIP(hipMemsetAsync(x, 0, (size_t)V * k * sizeof(double2), H.st));
  std::vector<double2> hh((size_t)(m + 2) * k);
  std::vector<double> bnorm(k), scl(k);
  // |b| per column
  dot(b, b, V, hcol.as<double2>());
  HELM_HIP(hipMemcpyAsync(hh.data(), hcol.p, k * sizeof(double2), hipMemcpyDeviceToHost, H.st));
  HELM_HIP(hipStreamSynchronize(H.st));
  for (int c = 0; c < k; ++c) bnorm[c] = std::sqrt(std::max(hh[c].x, 0.0));
  std::vector<char> active(k, 1);
  col_iters.assign(k, 0);
  int total = 0;
  bool first = true;
  int status = HELM_OK;
  std::vector<double> resid(k, 1.0);
  while (true) {
    // r = b - A x  (first cycle: x = 0, r = b), on the Krylov part
    const double2* r0 = b + off;
    if (!first) {
      S.apply(x, w.as<double2>());
      HELM_HIP(hipMemcpyAsync(r.as<double2>() + off, b + off, (size_t)Vs * k * sizeof(double2),
                              hipMemcpyDeviceToDevice, H.st));
      HELM_HIP(hipMemsetAsync(hcol.p, 0, k * sizeof(double2), H.st));
      // r -= w  (alpha = 1 per column)
      std::vector<double2> ones(k, make_double2(1.0, 0.0));
      HELM_HIP(hipMemcpyAsync(hcol.p, ones.data(), k * sizeof(double2),
                              hipMemcpyHostToDevice, H.st));
      kern::launch_axpy_cols(r.as<double2>() + off, w.as<double2>() + off, hcol.as<double2>(),
                             -1.0, Vs, k, H.st);
      r0 = r.as<double2>() + off;
    }
    first = false;
    dot(r0, r0, Vs, hcol.as<double2>());
    HELM_HIP(hipMemcpyAsync(hh.data(), hcol.p, k * sizeof(double2), hipMemcpyDeviceToHost, H.st));
    HELM_HIP(hipStreamSynchronize(H.st));
    std::vector<double> beta(k);
    for (int c = 0; c < k; ++c) {
      beta[c] = std::sqrt(std::max(hh[c].x, 0.0));
      double rel = bnorm[c] > 0 ? beta[c] / bnorm[c] : 0.0;
      resid[c] = rel;
      active[c] = (bnorm[c] > 0 && rel > tol[c]) ? 1 : 0;
      scl[c] = active[c] ? 1.0 / beta[c] : 0.0;
    }
    bool any = false;
    for (int c = 0; c < k; ++c) any |= active[c];
    if (!any) break;
    if (total >= max_iter) { status = HELM_ENOCONV; break; }
    HELM_HIP(hipMemcpyAsync(scale.p, scl.data(), k * sizeof(double), hipMemcpyHostToDevice, H.st));
    kern::launch_scale_cols(basis_vec(0) + off, r0, scale.as<double>(), Vs, k, H.st);
    if (up) HELM_HIP(hipMemsetAsync(basis_vec(0), 0, (size_t)off * sizeof(double2), H.st));
    // per-column Hessenberg, rotations and rhs
    std::vector<std::vector<cd>> Hm(k, std::vector<cd>((size_t)(m + 1) * m, 0.0));
    std::vector<std::vector<cd>> cs(k, std::vector<cd>(m)), sn(k, std::vector<cd>(m));
    std::vector<std::vector<cd>> g(k, std::vector<cd>(m + 1, 0.0));
    std::vector<int> kd(k, 0);
    std::vector<char> run = active;
    for (int c = 0; c < k; ++c) g[c][0] = beta[c];
    int j = 0;
    for (; j < m && total < max_iter; ++j) {
      double2* vj = basis_vec(j);
      // (a column that stopped has a zero basis vector from here on)
      apply_running(S, vj, w.as<double2>(), run, info);
      // K_down v_j into the down half of v_j (no longer an operand of P M)
      if (up)
        HELM_HIP(hipMemcpyAsync(vj, w.p, (size_t)off * sizeof(double2),
                                hipMemcpyDeviceToDevice, H.st));
      double2* wk = w.as<double2>() + off;
      for (int i = 0; i <= j; ++i) {
        dot(basis_vec(i) + off, wk, Vs, hcol.as<double2>() + (long long)i * k);
        kern::launch_axpy_cols(wk, basis_vec(i) + off, hcol.as<double2>() + (long long)i * k,
                               -1.0, Vs, k, H.st);
      }
      dot(wk, wk, Vs, hcol.as<double2>() + (long long)(j + 1) * k);
      HELM_HIP(hipMemcpyAsync(hh.data(), hcol.p, (size_t)(j + 2) * k * sizeof(double2),
                              hipMemcpyDeviceToHost, H.st));
      HELM_HIP(hipStreamSynchronize(H.st));
      ++total;
      bool any_run = false;
      for (int c = 0; c < k; ++c) {
        if (!run[c]) { scl[c] = 0.0; continue; }
        ++col_iters[c];
        std::vector<cd>& Hc = Hm[c];
        auto Hat = [&](int r_, int c_) -> cd& { return Hc[(size_t)r_ * m + c_]; };
        for (int i = 0; i <= j; ++i) {
          double2 v = hh[(size_t)i * k + c];
          Hat(i, j) = cd(v.x, v.y);
        }
        double hn = std::sqrt(std::max(hh[(size_t)(j + 1) * k + c].x, 0.0));
        Hat(j + 1, j) = hn;
        for (int i = 0; i < j; ++i) {
          cd t = cs[c][i] * Hat(i, j) + sn[c][i] * Hat(i + 1, j);
          Hat(i + 1, j) = -std::conj(sn[c][i]) * Hat(i, j) + std::conj(cs[c][i]) * Hat(i + 1, j);
          Hat(i, j) = t;
        }
        cd av = Hat(j, j), bv = Hat(j + 1, j);
        double den = std::sqrt(std::norm(av) + std::norm(bv));
        if (den == 0.0) { cs[c][j] = 1.0; sn[c][j] = 0.0; }
        else { cs[c][j] = std::conj(av) / den; sn[c][j] = std::conj(bv) / den; }
        Hat(j, j) = cs[c][j] * av + sn[c][j] * bv;
        Hat(j + 1, j) = 0.0;
        g[c][j + 1] = -std::conj(sn[c][j]) * g[c][j];
        g[c][j] = cs[c][j] * g[c][j];
        kd[c] = j + 1;
        double rel = bnorm[c] > 0 ? std::abs(g[c][j + 1]) / bnorm[c] : 0.0;
        resid[c] = rel;
        // stop this column on convergence or (lucky) breakdown
        if (rel <= tol[c] || hn <= 1e-300 || !(std::isfinite(rel))) {
          run[c] = 0;
          scl[c] = 0.0;
        } else {
          scl[c] = 1.0 / hn;
          any_run = true;
        }
      }
      if (j + 1 <= m) {
        HELM_HIP(hipMemcpyAsync(scale.p, scl.data(), k * sizeof(double), hipMemcpyHostToDevice,
                                H.st));
        kern::launch_scale_cols(basis_vec(j + 1) + off, wk, scale.as<double>(), Vs, k, H.st);
        if (up)
          HELM_HIP(hipMemsetAsync(basis_vec(j + 1), 0, (size_t)off * sizeof(double2), H.st));
      }
      if (!any_run) { ++j; break; }
    }
    // x += V y, y from the triangular systems of each column
    const int jmax = *std::max_element(kd.begin(), kd.end());
    std::vector<double2> ycoef((size_t)std::max(jmax, 1) * k, make_double2(0, 0));
    for (int c = 0; c < k; ++c) {
      int kc = kd[c];
      std::vector<cd> yv(kc, 0.0);
      for (int i = kc - 1; i >= 0; --i) {
        cd s = g[c][i];
        for (int q = i + 1; q < kc; ++q) s -= Hm[c][(size_t)i * m + q] * yv[q];
        cd d = Hm[c][(size_t)i * m + i];
        yv[i] = d != 0.0 ? s / d : 0.0;
      }
      for (int i = 0; i < kc; ++i)
        ycoef[(size_t)i * k + c] = make_double2(yv[i].real(), yv[i].imag());
    }
    if (jmax > 0) {
      HELM_HIP(hipMemcpyAsync(hcol.p, ycoef.data(), (size_t)jmax * k * sizeof(double2),
                              hipMemcpyHostToDevice, H.st));
      for (int i = 0; i < jmax; ++i)
        kern::launch_axpy_cols(x, basis_vec(i), hcol.as<double2>() + (long long)i * k,
                               1.0, V, k, H.st);
      HELM_HIP(hipStreamSynchronize(H.st));
    }
    bool conv = true;
    for (int c = 0; c < k; ++c) conv &= !(active[c] && resid[c] > tol[c]);
    if (conv) break;
    if (total >= max_iter) { status = HELM_ENOCONV; break; }
  }
  if (up) {
    // x_down = b_down - K_down x_up (the down half holds K_down x_up)
    kern::launch_rsub(x, b, off, H.st);
    HELM_HIP(hipStreamSynchronize(H.st));
  }
  last_resid = resid;
  if (iters_out) *iters_out = total;
  return status;
}

// The preconditioned polarized system P M x = P f (on its up-going block
// unless HELM_FLAG_FULL_KRYLOV).
Method::KrylovSystem Method::polarized_system() {
  KrylovSystem S;
  S.V = 2 * Vp / k;
  S.block = !(H.opt.flags & HELM_FLAG_FULL_KRYLOV);
  S.off = S.block ? Vp : 0;
  S.Vs = S.block ? S.V / 2 : S.V;
  S.polarized = true;
  S.apply = [this](const double2* v, double2* w) { apply_A(v, w); };
  return S;
}

// The cached batch of width w for the operator products of narrowed GMRES
// iterations, with its gathered operand and product (V elements per
// column); none (and no further attempts) when device memory refuses it.
Method* Method::krylov_narrower(int w, long long V) {
  if (!krylov_narrow_ok || !narrow_allowed) return nullptr;
  auto it = krylov_narrow.find(w);
  if (it != krylov_narrow.end()) return it->second.get();
  try {
    std::unique_ptr<Method> c(new Method(H, w));
    c->kv_in.alloc((size_t)V * w * sizeof(double2));
    c->kv_out.alloc((size_t)V * w * sizeof(double2));
    return krylov_narrow.emplace(w, std::move(c)).first->second.get();
  } catch (const Error& e) {
    if (e.code != HELM_ENOMEM) throw;
    krylov_narrow_ok = false;
    return nullptr;
  }
}

void Method::apply_running(const KrylovSystem& S, const double2* v, double2* out,
                           const std::vector<char>& run, helm_solve_info* info) {
  int m = 0;
  for (char r : run) m += r ? 1 : 0;
  int w = 1;
  while (w < m) w *= 2;
  Method* C = nullptr;
  if (S.polarized && m > 0 && 2 * w <= k && k <= kern::kMaxGatherCols &&
      !(H.opt.flags & HELM_FLAG_NO_NARROW))
    C = krylov_narrower(w, S.V);
  if (!C) {
    S.apply(v, out);
    return;
  }
  kern::ColMap g{}, slot{};
  for (int c = 0; c < kern::kMaxGatherCols; ++c) slot.col[c] = -1;
  for (int c = 0, j = 0; c < k; ++c)
    if (run[c]) {
      g.col[j] = c;
      slot.col[c] = j++;
    }
  kern::launch_gather_cols(C->kv_in.as<double2>(), v, S.V, k, w, m, g, H.st);
  C->apply_A(C->kv_in.as<double2>(), C->kv_out.as<double2>());
  kern::launch_scatter_cols(out, C->kv_out.as<double2>(), S.V, k, w, slot, H.st);
  if (info) ++info->narrow_products;
}

// The unpolarized SIE (I - GJ) x = v on one pair vector per column.
Method::KrylovSystem Method::sie_system() {
  KrylovSystem S;
  S.V = Vp / k;
  S.off = 0;
  S.Vs = S.V;
  S.block = false;
  S.apply = [this](const double2* v, double2* w) { apply_sie(v, w); };
  return S;
}

// Batched Bi-CGSTAB (one independent iteration per column, van der Vorst's
// recurrences with the shadow residual r_hat = r_0 and x_0 = 0) on the
// system S, as the memory-lean alternative to GMRES: six work vectors per
// column whatever the iteration count.  On the up-going block of the
// polarized system the down half of every A-product (K_down p, K_down s) is
// accumulated with the same coefficients as the up half, so that the down
// half of x ends as K_down x_up and x_down = b_down - K_down x_up as in
// GMRES.  Stopping test: |r| <= tol |b| per column (r the recurrence's
// residual of the Krylov part, |b| of the whole right-hand side); a column
// that converges or breaks down (rho or (r_hat, v) exactly zero) keeps its
// iterate.  The per-column scalars are formed on the host from device dot
// products.
int Method::bicgstab(const KrylovSystem& S, const double2* b, double2* x,
                     const std::vector<double>& tol, int max_iter, int* iters_out) {
  const long long off = S.off, Vs = S.Vs, V = S.V;
  const bool up = S.block;
  double2* r = basis_vec(0) + off;
  double2* rh = basis_vec(1) + off;
  double2* pf = basis_vec(2);          // p, zero outside the Krylov part
  double2* vf = basis_vec(3);          // A p
  double2* sf = basis_vec(4);          // s, zero outside the Krylov part
  double2* tf = basis_vec(5);          // A s
  double2* p = pf + off;
  double2* s = sf + off;
  double2* hc = hcol.as<double2>();
  HELM_HIP(hipMemsetAsync(x, 0, (size_t)V * k * sizeof(double2), H.st));
  if (up) {
    HELM_HIP(hipMemsetAsync(pf, 0, (size_t)off * sizeof(double2), H.st));
    HELM_HIP(hipMemsetAsync(sf, 0, (size_t)off * sizeof(double2), H.st));
  }
  const size_t kb = (size_t)Vs * k * sizeof(double2);
  HELM_HIP(hipMemcpyAsync(r, b + off, kb, hipMemcpyDeviceToDevice, H.st));
  HELM_HIP(hipMemcpyAsync(rh, b + off, kb, hipMemcpyDeviceToDevice, H.st));
  HELM_HIP(hipMemcpyAsync(p, b + off, kb, hipMemcpyDeviceToDevice, H.st));
  // norms: |b| (whole vector) and |r_0|
  std::vector<double2> hh((size_t)4 * k);
  auto fetch = [&](int n) {
    HELM_HIP(hipMemcpyAsync(hh.data(), hc, (size_t)n * k * sizeof(double2),
                            hipMemcpyDeviceToHost, H.st));
    HELM_HIP(hipStreamSynchronize(H.st));
  };
  auto upload = [&](const std::vector<cd>& a, int slot) {
    std::vector<double2> d(k);
    for (int c = 0; c < k; ++c) d[c] = make_double2(a[c].real(), a[c].imag());
    HELM_HIP(hipMemcpyAsync(hc + (long long)slot * k, d.data(), k * sizeof(double2),
                            hipMemcpyHostToDevice, H.st));
  };
  dot(b, b, V, hc);
  dot(r, r, Vs, hc + k);
  fetch(2);
  std::vector<double> bnorm(k), resid(k);
  std::vector<char> active(k);
  for (int c = 0; c < k; ++c) {
    bnorm[c] = std::sqrt(std::max(hh[c].x, 0.0));
    resid[c] = bnorm[c] > 0 ? std::sqrt(std::max(hh[k + c].x, 0.0)) / bnorm[c] : 0.0;
    active[c] = bnorm[c] > 0 && resid[c] > tol[c];
  }
  col_iters.assign(k, 0);
  std::vector<cd> rho_old(k, 1.0), alpha(k, 0.0), omega(k, 1.0), rho(k), beta(k);
  int it = 0, status = HELM_OK;
  auto any_active = [&] {
    for (char a : active) if (a) return true;
    return false;
  };
  while (any_active()) {
    if (it >= max_iter) { status = HELM_ENOCONV; break; }
    dot(rh, r, Vs, hc);
    fetch(1);
    for (int c = 0; c < k; ++c) {
      rho[c] = cd(hh[c].x, hh[c].y);
      if (active[c] && rho[c] == 0.0) active[c] = 0;   // breakdown: keep the iterate
    }
    if (it > 0) {
      // p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega)
      std::vector<cd> mw(k), bt(k);
      for (int c = 0; c < k; ++c) {
        const bool ok = active[c] && omega[c] != 0.0;
        bt[c] = ok ? (rho[c] / rho_old[c]) * (alpha[c] / omega[c]) : 0.0;
        mw[c] = ok ? omega[c] : 0.0;
      }
      upload(mw, 0);
      upload(bt, 1);
      kern::launch_axpy_cols(p, vf + off, hc, -1.0, Vs, k, H.st);
      kern::launch_xpay_cols(p, r, hc + k, Vs, k, H.st);
    }
    S.apply(pf, vf);
    dot(rh, vf + off, Vs, hc);
    fetch(1);
    for (int c = 0; c < k; ++c) {
      const cd den(hh[c].x, hh[c].y);
      alpha[c] = (active[c] && den != 0.0) ? rho[c] / den : 0.0;
      if (active[c] && den == 0.0) active[c] = 0;
    }
    upload(alpha, 0);
    // s = r - alpha v; x += alpha p (and the down half accumulates alpha K_down p)
    HELM_HIP(hipMemcpyAsync(s, r, kb, hipMemcpyDeviceToDevice, H.st));
    kern::launch_axpy_cols(s, vf + off, hc, -1.0, Vs, k, H.st);
    kern::launch_axpy_cols(x + off, p, hc, 1.0, Vs, k, H.st);
    if (up) kern::launch_axpy_cols(x, vf, hc, 1.0, off / k, k, H.st);
    ++it;
    dot(s, s, Vs, hc + k);
    fetch(2);
    std::vector<char> run = active;
    for (int c = 0; c < k; ++c) {
      if (!active[c]) continue;
      ++col_iters[c];
      resid[c] = std::sqrt(std::max(hh[k + c].x, 0.0)) / bnorm[c];
      if (resid[c] <= tol[c]) run[c] = 0;          // converged on the half step
    }
    S.apply(sf, tf);
    dot(tf + off, s, Vs, hc);
    dot(tf + off, tf + off, Vs, hc + k);
    fetch(2);
    for (int c = 0; c < k; ++c) {
      const cd ts(hh[c].x, hh[c].y);
      const double tt = hh[k + c].x;
      omega[c] = (run[c] && tt > 0) ? ts / tt : 0.0;
    }
    upload(omega, 0);
    // x += omega s (down half: omega K_down s); r = s - omega t
    kern::launch_axpy_cols(x + off, s, hc, 1.0, Vs, k, H.st);
    if (up) kern::launch_axpy_cols(x, tf, hc, 1.0, off / k, k, H.st);
    HELM_HIP(hipMemcpyAsync(r, s, kb, hipMemcpyDeviceToDevice, H.st));
    kern::launch_axpy_cols(r, tf + off, hc, -1.0, Vs, k, H.st);
    dot(r, r, Vs, hc);
    fetch(1);
    for (int c = 0; c < k; ++c) {
      if (!run[c]) { active[c] = 0; continue; }
      resid[c] = std::sqrt(std::max(hh[c].x, 0.0)) / bnorm[c];
      if (resid[c] <= tol[c] || omega[c] == 0.0) active[c] = 0;
      rho_old[c] = rho[c];
    }
  }
  if (up) {
    kern::launch_rsub(x, b, off, H.st);
    HELM_HIP(hipStreamSynchronize(H.st));
  }
  last_resid = resid;
  if (iters_out) *iters_out = it;
  return status;
}

// out = (I - GJ) x for the unpolarized SIE: every layer solves the sources
// of its two interfaces (all layers in one batched solve) and is read on its
// own interface planes: out_j = x_j - (w^j(e_j), w^{j+1}(s_{j+1})).
void Method::apply_sie(const double2* x, double2* out) {
  const int L = H.G.L;
  for (int l = 0; l < L; ++l) {
    zero_X(l);
    if (l >= 1) jump(l, pair(x, l - 1), nullptr, 0);
    if (l <= L - 2) jump(l, pair(x, l), nullptr, 1);
  }
  H.solve_layers(*set_all, k);
  for (int l = 0; l < L; ++l) {
    if (l <= L - 2) readout(l, 1, -1.0, planes(terms(pair(x, l), 1, 0), 1), pair(out, l));
    if (l >= 1) readout(l, 0, -1.0, planes(terms(pair(x, l - 1), 0, 1), 2), pair(out, l - 1));
  }
}

// v of the unpolarized SIE: the local solves of the partitioned source read
// on each layer's own interface planes.
void Method::sie_rhs(const double2* f, double2* v) {
  const int L = H.G.L;
  scatter_sources(f);
  H.solve_layers(*set_all, k);
  for (int l = 0; l < L; ++l) {
    if (l <= L - 2) readout(l, 1, 1.0, planes(terms(), 1), pair(v, l));
    if (l >= 1) readout(l, 0, 1.0, planes(terms(), 2), pair(v, l - 1));
  }
}

// Device bytes of the Krylov vectors held (basis or Bi-CGSTAB work vectors,
// plus GMRES's two temporaries).
double Method::krylov_bytes() const {
  return (double)(basis.size() * 2 * Vp + (gw.p ? 4 * Vp : 0)) * sizeof(double2);
}

double2* Method::basis_vec(int i) {
  while ((int)basis.size() <= i) {
    basis.emplace_back(new DevMem);
    basis.back()->alloc((size_t)2 * Vp * sizeof(double2));
  }
  return basis[i]->as<double2>();
}

// u = H^-1 f through the polarized interface system (one inner solve)
int Method::polarized_solve(const double2* f, double2* u, double tol, int max_iter,
                            int restart, helm_solve_info* info) {
  return polarized_solve(f, u, std::vector<double>(k, tol), max_iter, restart, info);
}

int Method::polarized_solve(const double2* f, double2* u, const std::vector<double>& tol,
                            int max_iter, int restart, helm_solve_info* info) {
  const int L = H.G.L;
  double t0 = now_ms();
  col_iters.assign(k, 0);
  if (L == 1) {
    last_resid.assign(k, 0.0);   // a direct solve: no Krylov residual
    scatter_sources(f);
    H.solve_layers(*set_all, k);
    if (H.prec == HELM_FP64)
      kern::launch_gather_volume<double>(H.layers_h[0], u, H.G.nx, H.G.ny, N, k, H.st);
    else
      kern::launch_gather_volume<float>(H.layers_h[0], u, H.G.nx, H.G.ny, N, k, H.st);
    HELM_HIP(hipStreamSynchronize(H.st));
    if (info) info->t_reconstruct_ms += now_ms() - t0;
    return HELM_OK;
  }
  if (!fpol.p) {
    fpol.alloc((size_t)2 * Vp * sizeof(double2));
    bpol.alloc((size_t)2 * Vp * sizeof(double2));
    xpol.alloc((size_t)2 * Vp * sizeof(double2));
  }
  const bool unpol = H.opt.flags & HELM_FLAG_UNPOLARIZED;
  if (unpol) sie_rhs(f, bpol.as<double2>());
  else precondition_source(f, bpol.as<double2>(), bpol.as<double2>() + Vp);
  HELM_HIP(hipStreamSynchronize(H.st));
  double t1 = now_ms();
  int iters = 0;
  int st;
  if (unpol)
    st = gmres(sie_system(), bpol.as<double2>(), xpol.as<double2>(), tol, max_iter, restart,
               &iters);
  else if (H.opt.flags & HELM_FLAG_BICGSTAB)
    st = bicgstab(polarized_system(), bpol.as<double2>(), xpol.as<double2>(), tol, max_iter,
                  &iters);
  else
    st = gmres(polarized_system(), bpol.as<double2>(), xpol.as<double2>(), tol, max_iter,
               restart, &iters, info);
  HELM_HIP(hipStreamSynchronize(H.st));
  double t2 = now_ms();
  // traces u_j = u_down_j + u_up_j (the unpolarized SIE solves for them)
  double2* tr = unpol ? xpol.as<double2>() : fpol.as<double2>();
  if (!unpol) kern::launch_add(tr, xpol.as<double2>(), xpol.as<double2>() + Vp, Vp, H.st);
  reconstruct(f, tr, u);
  HELM_HIP(hipStreamSynchronize(H.st));
  double t3 = now_ms();
  if (info) {
    info->t_setup_ms += t1 - t0;
    info->t_gmres_ms += t2 - t1;
    info->t_reconstruct_ms += t3 - t2;
    info->gmres_iters += iters;
    info->krylov_bytes = std::max(info->krylov_bytes, krylov_bytes());
  }
  return st;
}

// per-column l2 norms of k volumes
void Method::norms(const double2* x, std::vector<double>& out) {
  out.resize(k);
  kern::launch_volume_norm2(x, N, k, norm_partial.as<double>(), norm_out.as<double>(), H.st);
  HELM_HIP(hipMemcpyAsync(out.data(), norm_out.p, k * sizeof(double), hipMemcpyDeviceToHost,
                          H.st));
  HELM_HIP(hipStreamSynchronize(H.st));
  for (double& v : out) v = std::sqrt(v);
}

// per-column |f - H u| / |f| in FP64; r receives the residual
void Method::residual(const double2* f, const double2* u, double2* r,
                      std::vector<double>& rel) {
  kern::launch_residual(H.grid, f, u, r, k, H.st);
  std::vector<double> nr(k), nf(k);
  kern::launch_volume_norm2(r, N, k, norm_partial.as<double>(), norm_out.as<double>(), H.st);
  HELM_HIP(hipMemcpyAsync(nr.data(), norm_out.p, k * sizeof(double), hipMemcpyDeviceToHost, H.st));
  HELM_HIP(hipStreamSynchronize(H.st));
  kern::launch_volume_norm2(f, N, k, norm_partial.as<double>(), norm_out.as<double>(), H.st);
  HELM_HIP(hipMemcpyAsync(nf.data(), norm_out.p, k * sizeof(double), hipMemcpyDeviceToHost, H.st));
  HELM_HIP(hipStreamSynchronize(H.st));
  rel.resize(k);
  for (int c = 0; c < k; ++c) rel[c] = nf[c] > 0 ? std::sqrt(nr[c] / nf[c]) : std::sqrt(nr[c]);
}

// One refinement step on the k columns: D = (polarized solve of R) with a
// tolerance per column, U += D, R = F - H U in FP64, and the per-column
// relative residual |R|/|F| and norms |D|, |U|.  With U = 0 and R = F on
// entry this is the first solve of the column; later steps correct U.
int Method::refine_step(const double2* F, double2* U, double2* R, double2* D,
                        const std::vector<double>& tol, StepNorms& out, helm_solve_info* info) {
  const int restart = gmres_restart(H.opt.gmres_max_iter);
  int s = polarized_solve(R, D, tol, H.opt.gmres_max_iter, restart, info);
  kern::launch_accumulate(U, D, N * k, H.st);
  double tr = now_ms();
  residual(F, U, R, out.rel);
  norms(D, out.dn);
  norms(U, out.un);
  if (info) info->t_residual_ms += now_ms() - tr;
  return s;
}

// The cached batch of width w for narrowed refinement steps, with its
// gathered volumes; none (and no further attempts) when device memory
// refuses it.
Method* Method::narrower(int w) {
  if (!narrow_ok || !narrow_allowed) return nullptr;
  if (!child || child->k != w) {
    child.reset();
    try {
      std::unique_ptr<Method> c(new Method(H, w));
      c->ensure_volumes();
      c->vf.alloc((size_t)N * w * sizeof(double2));
      c->vu.alloc((size_t)N * w * sizeof(double2));
      child = std::move(c);
    } catch (const Error& e) {
      if (e.code != HELM_ENOMEM) throw;
      narrow_ok = false;
      return nullptr;
    }
  }
  return child.get();
}

void Method::ensure_volumes() {
  if (!vr.p) {
    vr.alloc((size_t)N * k * sizeof(double2));
    vd.alloc((size_t)N * k * sizeof(double2));
  }
}

// Full online solve of k columns (device arrays).  col0 is the index of the
// first column in the caller's per-right-hand-side arrays of info.
int Method::solve(const double2* f, double2* u, helm_solve_info* info, int col0) {
  const helm_options& o = H.opt;
  const int restart = gmres_restart(o.gmres_max_iter);
  ensure_volumes();
  double2* r = vr.as<double2>();
  std::vector<double> rel, est_c(k, 0.0);
  std::vector<int> steps_c(k, 0), iters_c(k, 0);
  int status = HELM_OK;
  double t0 = now_ms();
  if (H.prec == HELM_FP64) {
    int it0 = info ? info->gmres_iters : 0;
    status = polarized_solve(f, u, o.gmres_tol, o.gmres_max_iter, restart, info);
    if (col_iters.size() == (size_t)k) iters_c = col_iters;
    std::fill(steps_c.begin(), steps_c.end(), 1);
    double tr = now_ms();
    residual(f, u, r, rel);
    if (info) {
      info->ir_steps = std::max(info->ir_steps, 1);
      info->ir_width[0] = std::max(info->ir_width[0], k);
      info->t_residual_ms += now_ms() - tr;
      double mx = 0;
      for (double v : rel) mx = std::max(mx, v);
      info->ir_residual[0] = std::max(info->ir_residual[0], mx);
      info->ir_gmres_iters[0] = std::max(info->ir_gmres_iters[0], info->gmres_iters - it0);
    }
  } else {
    // iterative refinement: u <- u + solve_c64(f - H u), FP64 residuals.  A
    // column that meets the target is final and takes no further part.  When
    // the columns a later step still has to refine fit in half the batch or
    // less, they are gathered into the first slots of a batch of the
    // narrowest power-of-two width that holds them (its layer solves stream
    // the same factors with fewer columns), and the results scattered back.
    HELM_HIP(hipMemsetAsync(u, 0, (size_t)N * k * sizeof(double2), H.st));
    HELM_HIP(hipMemcpyAsync(r, f, (size_t)N * k * sizeof(double2), hipMemcpyDeviceToDevice,
                            H.st));
    int steps = 0;
    status = HELM_ENOCONV;
    std::vector<RefineTrack> track(k);
    std::vector<char> met(k, 0);
    rel.assign(k, 0.0);
    const size_t col = (size_t)N * sizeof(double2);
    double emx_last = 0;
    for (int it = 0; it < std::max(1, o.ir_max_steps); ++it) {
      int it0 = info ? info->gmres_iters : 0;
      std::vector<int> todo;
      for (int c = 0; c < k; ++c)
        if (!met[c]) todo.push_back(c);
      const int m = (int)todo.size();
      std::vector<double> tol(k, 0.0), teff(k, 0.0);
      std::vector<int> citer(k, 0);
      for (int c : todo) tol[c] = refinement_tol(it, track[c], o);
      int w = 1;
      while (w < m) w *= 2;
      Method* S = (it > 0 && 2 * w <= k && !(o.flags & HELM_FLAG_NO_NARROW)) ? narrower(w)
                                                                               : nullptr;
      StepNorms nm;
      if (S) {
        // slot j < m holds column todo[j]; the slots past m hold zero
        // columns (a zero source: converged at once, zero correction)
        double2* fc = S->vf.as<double2>();
        double2* uc = S->vu.as<double2>();
        double2* rc = S->vr.as<double2>();
        for (int j = 0; j < w; ++j) {
          if (j < m) {
            const size_t src = (size_t)todo[j] * N;
            HELM_HIP(hipMemcpyAsync(fc + (size_t)j * N, f + src, col, hipMemcpyDeviceToDevice, H.st));
            HELM_HIP(hipMemcpyAsync(uc + (size_t)j * N, u + src, col, hipMemcpyDeviceToDevice, H.st));
            HELM_HIP(hipMemcpyAsync(rc + (size_t)j * N, r + src, col, hipMemcpyDeviceToDevice, H.st));
          } else {
            HELM_HIP(hipMemsetAsync(fc + (size_t)j * N, 0, col, H.st));
            HELM_HIP(hipMemsetAsync(uc + (size_t)j * N, 0, col, H.st));
            HELM_HIP(hipMemsetAsync(rc + (size_t)j * N, 0, col, H.st));
          }
        }
        std::vector<double> tol_w(w, 0.0);
        for (int j = 0; j < m; ++j) tol_w[j] = tol[todo[j]];
        StepNorms nw;
        S->refine_step(fc, uc, rc, S->vd.as<double2>(), tol_w, nw, info);
        nm.rel.assign(k, 0.0);
        nm.dn.assign(k, 0.0);
        nm.un.assign(k, 0.0);
        for (int j = 0; j < m; ++j) {
          const int c = todo[j];
          const size_t dst = (size_t)c * N;
          HELM_HIP(hipMemcpyAsync(u + dst, uc + (size_t)j * N, col, hipMemcpyDeviceToDevice, H.st));
          HELM_HIP(hipMemcpyAsync(r + dst, rc + (size_t)j * N, col, hipMemcpyDeviceToDevice, H.st));
          nm.rel[c] = nw.rel[j];
          nm.dn[c] = nw.dn[j];
          nm.un[c] = nw.un[j];
          teff[c] = S->last_resid.size() == (size_t)w ? S->last_resid[j] : tol[c];
          citer[c] = S->col_iters.size() == (size_t)w ? S->col_iters[j] : 0;
        }
      } else {
        // the final columns get a zero residual: converged at once for the
        // Krylov solver, and a zero correction
        for (int c = 0; c < k; ++c)
          if (met[c]) HELM_HIP(hipMemsetAsync(r + (size_t)c * N, 0, col, H.st));
        refine_step(f, u, r, vd.as<double2>(), tol, nm, info);
        for (int c : todo) {
          teff[c] = last_resid.size() == (size_t)k ? last_resid[c] : tol[c];
          citer[c] = col_iters.size() == (size_t)k ? col_iters[c] : 0;
        }
      }
      ++steps;
      for (int c : todo) {
        rel[c] = nm.rel[c];
        // the relative residual GMRES reached stands for the step's tolerance
        est_c[c] = refinement_error(it, track[c], nm.dn[c], nm.un[c], teff[c]);
        iters_c[c] += citer[c];
        if (refinement_met(it, rel[c], est_c[c], o)) {
          met[c] = 1;
          steps_c[c] = steps;
        }
      }
      double mx = 0, emx = 0;
      bool all = true;
      for (int c = 0; c < k; ++c) {
        mx = std::max(mx, std::isfinite(rel[c]) ? rel[c] : 1e300);
        emx = std::max(emx, est_c[c]);
        all = all && met[c];
      }
      if (info && it < 8) {
        info->ir_residual[it] = std::max(info->ir_residual[it], mx);
        info->ir_gmres_iters[it] = std::max(info->ir_gmres_iters[it], info->gmres_iters - it0);
        info->ir_width[it] = std::max(info->ir_width[it], S ? w : k);
      }
      emx_last = emx;
      if (all) {
        status = HELM_OK;
        break;
      }
    }
    if (info) {
      info->ir_steps = std::max(info->ir_steps, steps);
      // the columns' final estimates (max over the internal batches)
      info->est_error_max = std::max(info->est_error_max, emx_last);
    }
    for (int c = 0; c < k; ++c)
      if (steps_c[c] == 0) steps_c[c] = steps;
  }
  if (info) {
    double mx = 0;
    for (double v : rel) mx = std::max(mx, v);
    info->rel_residual_max = std::max(info->rel_residual_max, mx);
    info->t_total_ms += now_ms() - t0;
    for (int c = 0; c < k && c < (int)rel.size(); ++c) {
      if (info->rhs_rel_residual) info->rhs_rel_residual[col0 + c] = rel[c];
      if (info->rhs_est_error) info->rhs_est_error[col0 + c] = est_c[c];
      if (info->rhs_ir_steps) info->rhs_ir_steps[col0 + c] = steps_c[c];
      if (info->rhs_gmres_iters) info->rhs_gmres_iters[col0 + c] = iters_c[c];
    }
  }
  return status;
}

// Error of the refined column after step `step` (0-based), estimated from
// the contraction of the corrections.  The correction of step k
// approximates the error before it, so q_k = |d_k| / |d_{k-1}| measures the
// contraction of the previous step; if the current step contracts by no
// more than q, the remaining error is at most |d_k| q / (1 - q) relative to
// |u|.  Guards:
//  - q is the larger of the last two measured ratios (from the third step
//    on);
//  - a step contracts by no less than kResidualGain times the relative
//    residual its GMRES reached (tol): the correction's error is the inverse
//    of the preconditioned operator applied to that residual, and the
//    polarized preconditioner leaves an operator close to the identity;
//    a step limited by the complex64 rounding shows in the measured ratios;
//  - an estimate with q > 1/2 (slow or erratic contraction) is not trusted
//    (reported as 1, unknown).
// Unknown (1) after the first step.
double refinement_error(int step, RefineTrack& tr, double dcur, double unorm, double tol) {
  constexpr double kResidualGain = 4.0;
  const double dprev = tr.dprev, qprev = tr.qprev;
  tr.dprev = dcur;
  double est = 1.0;
  if (unorm == 0) {
    est = 0.0;
  } else if (step > 0 && dprev > 0) {
    const double qk = dcur / dprev;
    tr.qprev = qk;
    double q = step >= 2 ? std::max(qk, qprev) : qk;
    q = std::max(q, kResidualGain * tol);
    if (q <= 0.5) est = dcur / unorm * q / (1.0 - q);
  }
  tr.est = est;
  return est;
}

// Tolerance of a column's next step: inner_tol for the first solve; once the
// estimated error is within err_target (but not yet within the part of it
// that stops the column), the step only has to shrink the error by a modest
// factor, and runs to the looser inner_tol_final; otherwise inner_tol_refine.
double refinement_tol(int step, const RefineTrack& tr, const helm_options& o) {
  if (step == 0) return o.inner_tol;
  if (o.err_target > 0 && tr.est <= o.err_target && o.inner_tol_final > 0)
    return std::max(o.inner_tol_final, o.inner_tol_refine);
  return o.inner_tol_refine;
}

bool refinement_met(int step, double rel, double est, const helm_options& o) {
  // after the second solve (one measured contraction) a factor 4 against
  // the estimate, from the third on a factor 2
  const double margin = step <= 1 ? 0.25 : 0.5;
  return rel <= o.ir_tol || (o.err_target > 0 && est <= margin * o.err_target);
}

// Restart length: the caller's gmres_restart when set, capped by what device
// memory holds (basis vectors of 2 pair vectors x k columns each) and by 60.
int Method::gmres_restart(int max_iter) const {
  const int asked = H.opt.gmres_restart > 0 ? std::min(H.opt.gmres_restart, 60) : 60;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
    return std::max(1, std::min({max_iter, asked, 16}));
  // vectors already allocated need no new memory
  const size_t per = (size_t)2 * Vp * sizeof(double2);
  const size_t fit = (per ? (size_t)(0.6 * free_b) / per : 64) + basis.size();
  const int m = (int)std::min<size_t>(fit > 3 ? fit - 3 : 1, (size_t)asked);
  return std::max(1, std::min(max_iter, m));
}

}  // namespace helm
