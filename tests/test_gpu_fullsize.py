"""The full-size workloads, checked with properties that hold at any size,
the oracle supplying the operator:

* the headline (200^3, L = 20, 64 sources, the launch configuration of
  bench.py) in mixed precision and on the complex128 path;
* the smooth random medium at 100^3 (L = 10) on the complex128 path, and
  in mixed precision against it;

* the oracle's own assembly of H gives |f - H u| / |f| for sampled columns
  of the GPU solution; the mixed refinement stops at an estimated error of
  1e-6 and its residual must be below that, the complex128 path runs GMRES to
  1e-10 and its residual must be below 1e-9;
* reciprocity of the symmetric operator: for neighbouring sources s, r the
  field of s at r equals the field of r at s."""

import numpy as np
import pytest

from helm_inputs import workload
from oracle.discretization import Problem, point_source_rhs

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::DeprecationWarning")]

torch = pytest.importorskip("torch")


def _check(wl, m, srcs, cols, sample, pairs, res_tol, rec_tol):
    pb = Problem(m, wl.h, wl.omega, wl.pml, wl.pml_C)
    H = pb.operator()
    F = point_source_rhs(pb.shape, [srcs[c] for c in sample], wl.h)
    for j, c in enumerate(sample):
        r = F[:, j] - H @ cols[c]
        rel = np.linalg.norm(r) / np.linalg.norm(F[:, j])
        print(f"column {c} oracle residual {rel:.2e}")
        assert rel <= res_tol
    nx, ny, _ = wl.n
    idx = lambda p: p[0] + nx * (p[1] + ny * p[2])
    for a, b in pairs:
        uab = cols[a][idx(srcs[b])]
        uba = cols[b][idx(srcs[a])]
        print(f"reciprocity {a}-{b}: {abs(uab - uba) / abs(uab):.2e}")
        assert abs(uab - uba) <= rec_tol * abs(uab)


def test_layered_200_fp64_residual_and_reciprocity():
    """The complex128 path at the headline size (GMRES tolerance 1e-10)."""
    import paper_1801_08655_amd as pt
    wl = workload("layered-200")
    m = wl.m()
    srcs = wl.point_sources(64)
    s = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision="fp64",
                  pml_local=wl.pml_local, pml_C=wl.pml_C, gmres_tol=1e-10)
    u, info = s.solve_points(srcs, info=True)
    print(info)
    assert info["rel_residual_max"] <= 1e-9
    sample = [0, 27, 63]
    cols = {c: u[c].cpu().numpy().ravel() for c in sample + [1, 8, 9]}
    s.close()
    del u
    torch.cuda.empty_cache()
    _check(wl, m, srcs, cols, sample, ((0, 1), (0, 8), (1, 9), (8, 9)), 1e-9, 1e-8)


def test_smooth_100_fp64_residual_and_reciprocity():
    """The smooth random medium at 100^3 with L = 10 on the complex128 path:
    its source at depth 15 and two more at other depths."""
    import paper_1801_08655_amd as pt
    wl = workload("smooth-100")
    m = wl.m()
    srcs = list(wl.sources) + [(40, 57, 15), (61, 44, 52)]
    s = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision="fp64",
                  pml_local=wl.pml_local, pml_C=wl.pml_C, gmres_tol=1e-10)
    u, info = s.solve_points(srcs, info=True)
    print(info)
    assert info["rel_residual_max"] <= 1e-9
    cols = {c: u[c].cpu().numpy().ravel() for c in range(3)}
    s.close()
    _check(wl, m, srcs, cols, [0, 1, 2], ((0, 1), (0, 2), (1, 2)), 1e-9, 1e-8)


def test_smooth_100_mixed_matches_the_complex128_path():
    """The same medium and sources in mixed precision with the library's
    default refinement settings and a 1e-6 error target: every column within
    1e-6 of the complex128 path's solution (GMRES to 1e-10, itself pinned
    by the residual test above), and every column's estimate within the
    target."""
    import paper_1801_08655_amd as pt
    wl = workload("smooth-100")
    m = wl.m()
    srcs = list(wl.sources) + [(40, 57, 15), (61, 44, 52)]
    out = {}
    for prec, kw in (("mixed", dict(err_target=1e-6)), ("fp64", dict(gmres_tol=1e-10))):
        s = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision=prec,
                      pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)
        u, info = s.solve_points(srcs, info=True)
        out[prec] = (u.cpu().numpy().reshape(len(srcs), -1), info)
        s.close()
    um, info = out["mixed"]
    ur, _ = out["fp64"]
    err = np.linalg.norm(um - ur, axis=1) / np.linalg.norm(ur, axis=1)
    print("error vs complex128", err, "estimates", info["rhs_est_error"],
          "steps", info["rhs_ir_steps"], "gmres per step", info["ir_gmres_iters"])
    assert info["ir_steps"] < 6   # stopped on the estimate, before the step limit
    assert max(info["rhs_est_error"]) <= 1e-6
    assert err.max() <= 1e-6


def test_layered_200_residual_and_reciprocity():
    import paper_1801_08655_amd as pt
    wl = workload("layered-200")
    m = wl.m()
    srcs = wl.point_sources(64)
    s = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision="mixed",
                  pml_local=wl.pml_local, pml_C=wl.pml_C, ir_tol=1e-10, inner_tol=5e-4,
                  inner_tol_refine=2e-4, err_target=1e-6, ir_max_steps=4,
                  flags=pt._lib.HELM_FLAG_AUTOTUNE)
    u, info = s.solve_points(srcs, info=True)
    print(info)
    assert info["ir_steps"] >= 2 and info["est_error_max"] <= 1e-6
    sample = [0, 9, 36, 63]
    cols = {c: u[c].cpu().numpy().ravel() for c in sample + [1, 8]}
    s.close()
    del u
    torch.cuda.empty_cache()
    _check(wl, m, srcs, cols, sample, ((0, 1), (0, 8), (1, 9), (8, 9)), 1e-6, 1e-5)
