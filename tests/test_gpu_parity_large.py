"""Parity of the whole method with the oracle's direct solve on the largest
grids the oracle handles (40^3, L = 4 and L = 8), GMRES restarts, the
zero-pivot status, the factorization record, and the mixed-precision stop
rule (run on an MI355X).

Every expected value comes from ``oracle/`` alone: SuperLU on the oracle's
own assembly of the global operator (u = H^-1 f, the plain definition of what
the method computes).  Tolerances: complex128 path <= 1e-9 at GMRES
tolerance 1e-10, mixed precision <= 1e-6, per column (relative l2 over the
whole grid, PML included).
"""

import numpy as np
import pytest

from helm_inputs import workload
from oracle.direct import SparseLU, relative_error
from oracle.discretization import Problem, point_source_rhs

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::DeprecationWarning")]

torch = pytest.importorskip("torch")

# sources of the 40^3 cases: the workload's own plus off-axis extras, so that
# a batch spans several surface positions and depths
EXTRA = {"layered-40": [(19, 21, 17), (30, 9, 25)],
         "smooth-40": [(12, 25, 14), (27, 16, 22), (20, 20, 30)]}


def _solver(wl, precision, **kw):
    import paper_1801_08655_amd as pt
    return pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=precision,
                     pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)


_REFS = {}


def _reference(name, srcs=None):
    """(workload, sources, oracle solution columns), computed once per case."""
    key = (name, tuple(srcs) if srcs else None)
    if key not in _REFS:
        wl = workload(name)
        srcs = list(srcs) if srcs else list(wl.sources) + EXTRA.get(name, [])
        pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
        print(f"oracle: direct solve of {name} ({len(srcs)} sources)", flush=True)
        ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, srcs, wl.h))
        _REFS[key] = (wl, srcs, ref)
    return _REFS[key]


@pytest.mark.parametrize("name", ["layered-40", "smooth-40"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_whole_method_at_40_cubed_matches_direct(name, precision, tol):
    """40^3 grids: L = 8 layers of 3-4 interior planes (layered recipe) and L = 4
    (smooth recipe); every column against the oracle's direct solve."""
    wl, srcs, ref = _reference(name)
    kw = {"gmres_tol": 1e-10} if precision == "fp64" else {"err_target": 1e-6}
    s = _solver(wl, precision, **kw)
    u, info = s.solve_points(srcs, info=True)
    err = relative_error(u.cpu().numpy().reshape(len(srcs), -1).T, ref)
    print(name, precision, "L", wl.n_layers, "err", err, "iters", info["gmres_iters"],
          "ir steps", info["ir_steps"])
    assert err.max() <= tol
    s.close()


@pytest.mark.parametrize("krylov", ["block", "whole"])
@pytest.mark.parametrize("precision,tol,restart", [("fp64", 1e-9, 2), ("fp64", 1e-9, 3),
                                                   ("mixed", 1e-6, 1), ("mixed", 1e-6, 2)])
def test_gmres_restart_matches_direct(restart, krylov, precision, tol):
    """Restarted GMRES (1 to 3 basis vectors per cycle, several cycles in a
    solve) on the up-going block and on the whole polarized system: the block
    form carries K_down x_up in the down half of the iterate across restarts."""
    import paper_1801_08655_amd as pt
    wl, srcs, ref = _reference("layered-28", [(8, 9, 6), (14, 14, 9), (20, 8, 12)])
    flags = 0 if krylov == "block" else pt._lib.HELM_FLAG_FULL_KRYLOV
    # mixed: inner tolerances tight enough that every inner solve takes more
    # iterations than one restart cycle holds
    kw = {"gmres_tol": 1e-10} if precision == "fp64" else {
        "err_target": 1e-6, "inner_tol": 1e-5, "inner_tol_refine": 1e-5}
    s = _solver(wl, precision, gmres_restart=restart, gmres_max_iter=120, flags=flags, **kw)
    u, info = s.solve_points(srcs, info=True)
    err = relative_error(u.cpu().numpy().reshape(len(srcs), -1).T, ref)
    print(krylov, precision, "restart", restart, "err", err, "iters", info["gmres_iters"])
    assert max(info["ir_gmres_iters"]) > restart   # more than one cycle
    assert err.max() <= tol
    s.close()


def test_zero_pivot_is_reported():
    """A front whose pivots are exactly zero (left unassembled by the test
    hook): the factorization finishes and returns HELM_EZEROPIVOT, and a
    normal factorization of the same problem in the same process succeeds."""
    import paper_1801_08655_amd as pt
    wl = workload("homogeneous-25")
    for prec in ("fp64", "mixed"):
        with pytest.raises(pt.HelmError) as e:
            _solver(wl, prec, flags=pt._lib.HELM_FLAG_TEST_ZERO_FRONT)
        assert e.value.status == pt.HELM_EZEROPIVOT
        assert "pivot" in str(e.value)
    s = _solver(wl, "fp64")
    _, _, ref = _reference("homogeneous-25")
    u = s.solve_points(wl.sources)
    assert relative_error(u.cpu().numpy().reshape(1, -1).T, ref).max() <= 1e-9
    s.close()


def test_factor_info_counts_and_pivots():
    """The factorization record: its LU flop count equals the count over an
    independent nested-dissection plan written in the tests, the executed
    Gauss-Jordan count exceeds it by less than the inverse-forming work
    allows, and the pivot range and growth are finite and positive."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "tlc", os.path.join(os.path.dirname(__file__), "test_library_cpu.py"))
    tlc = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(tlc)
    wl = workload("layered-28")
    nx, ny, nz = wl.n
    lu = 0.0
    for t in tlc._layer_planes(nz, wl.pml, wl.n_layers, wl.pml_local):
        for s_, b in tlc._nd_count(nx, ny, t, 64):
            lu += 4.0 * (2.0 / 3.0 * s_ ** 3 + 2.0 * s_ ** 2 * b + 2.0 * s_ * b * b)
    import time
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        s = _solver(wl, prec)
        wall = time.perf_counter() - t0
        fi = s.factor_info()
        print(prec, fi)
        assert fi["lu_flops"] == pytest.approx(lu, rel=1e-12)
        assert lu < fi["gj_flops"] < 3.0 * lu
        assert 0 < fi["pivot_min"] <= fi["pivot_max"] < np.inf
        assert 0 < fi["pivot_growth"] < 1e3
        assert fi["seconds"] > 0 and fi["factor_bytes"] > 0
        # the phases of the factorization call are timed and fit in its wall time
        phases = [fi["symbolic_seconds"], fi["setup_seconds"], fi["seconds"], fi["lists_seconds"]]
        assert all(p > 0 for p in phases)
        assert sum(phases) <= wall
        s.close()


def test_narrowed_refinement_steps_match_full_width():
    """A column that meets the target leaves the refinement, and a later
    step whose remaining columns fit in half the batch runs them gathered at
    the narrowest power-of-two width.  err_target is placed in the widest gap
    between the columns' estimates after two steps (a stop there needs the
    estimate within a quarter of err_target), so that 4 to 7 of the 8
    columns stop there: the third step runs at the narrower width, every
    column matches the same solve with every step at full width
    (HELM_FLAG_NO_NARROW) to the complex64 rounding of the corrections, and
    both are within err_target of the oracle."""
    import paper_1801_08655_amd as pt
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12), (11, 17, 15), (5, 20, 9), (16, 6, 18),
            (12, 12, 21), (18, 18, 7)]
    wl, srcs, ref = _reference("layered-28", srcs)
    k = len(srcs)
    # the estimates after two steps (nothing stops on them: err_target tiny)
    s = _solver(wl, "mixed", ir_tol=1e-300, err_target=1e-300, ir_max_steps=2)
    _, info = s.solve_points(srcs, info=True)
    s.close()
    e2 = np.sort(np.array(info["rhs_est_error"]))
    j = max(range(k // 2, k), key=lambda i: e2[i] / e2[i - 1])
    t = float(np.sqrt(e2[j] * e2[j - 1]))
    m = k - j
    w = 1 << (m - 1).bit_length()
    print("estimates after two steps", e2, "stop below", t, "remaining", m, "width", w)
    assert e2[j] > 1.05 * e2[j - 1]
    out = {}
    for label, flags in (("narrow", 0), ("full", pt._lib.HELM_FLAG_NO_NARROW)):
        s = _solver(wl, "mixed", ir_tol=1e-300, err_target=4 * t, ir_max_steps=6, flags=flags)
        u, inf = s.solve_points(srcs, info=True)
        out[label] = (u.cpu().numpy().reshape(k, -1).T, inf)
        print(label, "widths", inf["ir_width"], "steps", inf["rhs_ir_steps"],
              "gmres per step", inf["ir_gmres_iters"], "layer solves", inf["layer_solves"],
              "narrowed products", inf["narrow_products"])
        s.close()
    un, infn = out["narrow"]
    uf, inff = out["full"]
    assert infn["ir_width"][:3] == [k, k, w]
    assert all(x == k for x in inff["ir_width"])
    # (whether a GMRES iteration also narrows depends on how far apart the
    # columns' iteration counts are; the complex128 test below covers that)
    assert inff["narrow_products"] == 0
    assert sorted(infn["rhs_ir_steps"]) == sorted(inff["rhs_ir_steps"])
    assert sum(1 for x in infn["rhs_ir_steps"] if x == 2) == j
    # the narrowed operator products round differently in complex64 (at one
    # or two columns the substitutions take the vector kernels): about 1e-7
    # of a refinement correction that is itself 1e-4 to 1e-3 of u
    assert relative_error(un, uf).max() <= 1e-10
    assert relative_error(un, ref).max() <= 4 * t


def test_narrowed_gmres_products_match_full_width_fp64():
    """The complex128 path: a GMRES iteration whose running columns fit in
    half the batch applies the operator to them alone, gathered at a narrower
    width.  Eight sources plus eight zero-amplitude columns (converged from
    the start) make every product a narrowed one; the eight solutions equal
    the full-width ones (HELM_FLAG_NO_NARROW) to 1e-12 and the oracle's to
    1e-9, and the zero columns stay zero."""
    import paper_1801_08655_amd as pt
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12), (11, 17, 15), (5, 20, 9), (16, 6, 18),
            (12, 12, 21), (18, 18, 7)]
    wl, srcs, ref = _reference("layered-28", srcs)
    k = len(srcs)
    amps = np.r_[np.ones(k), np.zeros(k)].astype(np.complex128)
    out = {}
    for label, flags in (("narrow", 0), ("full", pt._lib.HELM_FLAG_NO_NARROW)):
        s = _solver(wl, "fp64", gmres_tol=1e-10, flags=flags)
        u, inf = s.solve_points(srcs + srcs, amplitudes=amps, info=True)
        out[label] = (u.cpu().numpy().reshape(2 * k, -1).T, inf)
        print(label, "iterations", inf["gmres_iters"], "narrowed products",
              inf["narrow_products"])
        s.close()
    un, infn = out["narrow"]
    uf, inff = out["full"]
    assert infn["narrow_products"] == infn["gmres_iters"] > 0
    assert inff["narrow_products"] == 0
    assert infn["gmres_iters"] == inff["gmres_iters"]
    assert not np.any(un[:, k:]) and not np.any(uf[:, k:])
    assert relative_error(un[:, :k], uf[:, :k]).max() <= 1e-12
    assert relative_error(un[:, :k], ref).max() <= 1e-9


@pytest.mark.parametrize("name", ["homogeneous-25", "smooth-24", "layered-28", "layered-40"])
def test_refinement_stops_on_the_estimate_only_when_the_error_is_met(name):
    """The mixed path with the FP64 residual test switched off (ir_tol far
    below reach), so refinement stops on the estimated error alone: whenever
    it stops, every column's true error against the oracle's direct solve is
    within err_target, and the estimate is not below half the true error."""
    wl, srcs, ref = _reference(name)
    target = 1e-6
    s = _solver(wl, "mixed", ir_tol=1e-300, err_target=target, ir_max_steps=6)
    u, info = s.solve_points(srcs, info=True)
    err = relative_error(u.cpu().numpy().reshape(len(srcs), -1).T, ref)
    est = np.array(info["rhs_est_error"])
    print(name, "true", err, "estimated", est, "steps", info["rhs_ir_steps"],
          "gmres per step", info["ir_gmres_iters"])
    assert info["ir_steps"] < 6                      # stopped on the estimate
    assert (est <= 0.5 * target).all()
    assert err.max() <= target
    assert (est >= 0.5 * err).all()
    s.close()
