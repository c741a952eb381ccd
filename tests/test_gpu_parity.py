"""Parity of the HIP path with the CPU oracle (run on an MI355X).

Every comparison uses seeded inputs from ``helm_inputs`` and an expected
value computed by ``oracle/`` alone (SuperLU on the oracle's own assembly,
or the oracle's step-by-step polarized traces).  Tolerances:
complex128 paths relative l2 <= 1e-9 (GMRES tol 1e-10) and <= 1e-11 for a
single local solve; mixed precision <= 1e-6 against the FP64 reference.
"""

import numpy as np
import pytest

from helm_inputs import workload
from oracle.direct import SparseLU, relative_error
from oracle.discretization import Problem, local_operator, point_source_rhs
from oracle.polarized import PolarizedTraces

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::DeprecationWarning")]

torch = pytest.importorskip("torch")


def _solver(wl, precision, **kw):
    import paper_1801_08655_amd as pt
    return pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=precision,
                     pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)


def _problem(wl):
    return Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)


@pytest.fixture(scope="module")
def homog():
    wl = workload("homogeneous-25")
    pb = _problem(wl)
    F = point_source_rhs(pb.shape, wl.sources, wl.h)
    u = SparseLU(pb.operator()).solve(F)[:, 0]
    return wl, pb, u


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("mixed", 2e-4)])
def test_layer_solve_matches_oracle(homog, precision, tol):
    """One multi-RHS local solve (H^l)^-1 r against SuperLU on the oracle's H^l."""
    wl, pb, _ = homog
    s = _solver(wl, precision)
    nx, ny, nz = wl.n
    for l in range(wl.n_layers):
        _, _, lo, hi = s.layer_info(l)
        t = hi - lo + 1
        r = _rand((3, t, ny, nx), 100 + l)
        w = s.layer_solve(l, torch.from_numpy(r).cuda()).cpu().numpy()
        Hl = local_operator(pb, wl.n_layers, wl.pml_local, l)
        ref = SparseLU(Hl).solve(r.reshape(3, -1).T).T
        err = relative_error(w.reshape(3, -1).T, ref.T)
        print(f"layer {l} ({precision}) rel err {err}")
        assert err.max() <= tol


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("mixed", 2e-5)])
def test_layer_solve_vector_path_matches_oracle(homog, precision, tol, k):
    """One or two columns: the local solve takes the vector substitution
    kernels (one lane group per row set walking the boundary, reduce-scatter
    over the group) instead of the MFMA tiles; every layer against SuperLU on
    the oracle's H^l (complex64 solves measured at 5.5e-7 to 7.5e-7)."""
    wl, pb, _ = homog
    s = _solver(wl, precision)
    nx, ny, nz = wl.n
    for l in range(wl.n_layers):
        _, _, lo, hi = s.layer_info(l)
        t = hi - lo + 1
        r = _rand((k, t, ny, nx), 300 + 10 * l + k)
        w = s.layer_solve(l, torch.from_numpy(r).cuda()).cpu().numpy()
        Hl = local_operator(pb, wl.n_layers, wl.pml_local, l)
        ref = SparseLU(Hl).solve(r.reshape(k, -1).T).T
        err = relative_error(w.reshape(k, -1).T, ref.T)
        print(f"layer {l} ({precision}, k = {k}) rel err {err}")
        assert err.max() <= tol


def test_operator_matches_oracle(homog):
    wl, pb, _ = homog
    s = _solver(wl, "fp64")
    u = _rand((2,) + pb.shape, 7)
    hu = s.apply_operator(torch.from_numpy(u).cuda()).cpu().numpy()
    ref = (pb.operator() @ u.reshape(2, -1).T).T
    assert relative_error(hu.reshape(2, -1).T, ref.T).max() <= 1e-13


def _pairs_gpu_layout(x):
    """oracle pairs (L-1, 2, ny, nx) per column -> [j][p][y][x][c] flat"""
    return np.stack(x, axis=-1).ravel()


def test_interface_operators_match_oracle(homog):
    """U (Alg. 10 read as the mirror of Alg. 6), P (Algs. 4-6) and P M."""
    wl, pb, _ = homog
    s = _solver(wl, "fp64")
    pt_cpu = PolarizedTraces(pb, wl.n_layers, wl.pml_local)
    k = 2
    shape = pt_cpu.zero_pairs().shape
    xd = [_rand(shape, 11 + c) for c in range(k)]
    xu = [_rand(shape, 21 + c) for c in range(k)]
    gx = torch.from_numpy(np.concatenate([_pairs_gpu_layout(xd), _pairs_gpu_layout(xu)])).cuda()
    gxu = torch.from_numpy(_pairs_gpu_layout(xu)).cuda()
    # U
    gu = s.polarized_op(2, gxu, k).cpu().numpy()
    ref = _pairs_gpu_layout([pt_cpu.U_op(x) for x in xu])
    assert relative_error(gu, ref)[0] <= 1e-11
    # P
    gp = s.polarized_op(0, gx, k).cpu().numpy()
    refs = [pt_cpu.precondition(a, b) for a, b in zip(xd, xu)]
    ref = np.concatenate([_pairs_gpu_layout([r[0] for r in refs]),
                          _pairs_gpu_layout([r[1] for r in refs])])
    assert relative_error(gp, ref)[0] <= 1e-11
    # P M
    ga = s.polarized_op(1, gx, k).cpu().numpy()
    refs = [pt_cpu.precondition(*pt_cpu.apply_M(a, b)) for a, b in zip(xd, xu)]
    ref = np.concatenate([_pairs_gpu_layout([r[0] for r in refs]),
                          _pairs_gpu_layout([r[1] for r in refs])])
    assert relative_error(ga, ref)[0] <= 1e-10


@pytest.mark.parametrize("name", ["homogeneous-25", "layered-28", "layered-40"])
def test_pruned_sweep_solves_match_full_solves(name):
    """P M applied with the sweep solves pruned to the fronts their interface
    sources and read-outs reach (the default) and with every front
    (HELM_FLAG_NO_PRUNE): the skipped work is exact zeros, so the results
    agree to rounding (the split of the pruned lists' GEMMs may differ), and
    both match the oracle's P (M x)."""
    import paper_1801_08655_amd as pt
    wl = workload(name)
    pb = _problem(wl)
    k = 3
    nx, ny, _ = wl.n
    Lm = wl.n_layers - 1
    x = _rand((2 * Lm * 2 * ny * nx * k,), 91)
    gx = torch.from_numpy(x).cuda()
    full = _solver(wl, "fp64", flags=pt._lib.HELM_FLAG_NO_PRUNE).polarized_op(1, gx, k)
    pruned = _solver(wl, "fp64").polarized_op(1, gx, k)
    a, b = pruned.cpu().numpy(), full.cpu().numpy()
    dev = np.linalg.norm(a - b) / np.linalg.norm(b)
    print(name, "pruned vs full", dev)
    assert dev <= 1e-12
    # the oracle's P (M x) column by column
    pt_cpu = PolarizedTraces(pb, wl.n_layers, wl.pml_local)
    half = Lm * 2 * ny * nx * k
    xd = x[:half].reshape(Lm, 2, ny, nx, k)
    xu = x[half:].reshape(Lm, 2, ny, nx, k)
    refs = [pt_cpu.precondition(*pt_cpu.apply_M(xd[..., c], xu[..., c])) for c in range(k)]
    ref = np.concatenate([_pairs_gpu_layout([r[0] for r in refs]),
                          _pairs_gpu_layout([r[1] for r in refs])])
    assert relative_error(a, ref)[0] <= 1e-10


def test_profile_flags_time_only_what_they_name(homog):
    """HELM_FLAG_PROFILE times every substitution kernel class,
    HELM_FLAG_PROFILE_FWD only the forward GEMM; timing never changes the
    arithmetic (same solution, bit for bit, as an untimed solve)."""
    import paper_1801_08655_amd as pt
    wl, pb, _ = homog
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12)]
    base = _solver(wl, "mixed").solve_points(srcs).cpu().numpy()
    for flag, timed in ((pt._lib.HELM_FLAG_PROFILE, None),
                        (pt._lib.HELM_FLAG_PROFILE_FWD, {"solve_fwd_gemm"})):
        s = _solver(wl, "mixed", flags=flag)
        s.kernel_stats(reset=True)
        u = s.solve_points(srcs).cpu().numpy()
        assert np.array_equal(u, base)
        st = s.kernel_stats()
        launched = {name for name, v in st.items() if v["launches"] > 0}
        if timed is None:
            assert {"solve_fwd_gemm", "solve_bwd_gemm"} <= launched
        else:
            assert launched == timed
        assert st["solve_fwd_gemm"]["total_ms"] > 0 and st["solve_fwd_gemm"]["flops"] > 0


def test_polarized_rhs_and_its_preconditioned_form_match_oracle(homog):
    """op 3: (f_down, f_up) of a volume source; op 4: P (f_down, f_up) from one
    folded sweep pair (the layer sources join the downward solves), against the
    oracle's polarized right-hand side and its P."""
    wl, pb, _ = homog
    s = _solver(wl, "fp64")
    pt_cpu = PolarizedTraces(pb, wl.n_layers, wl.pml_local)
    k = 2
    nx, ny, nz = wl.n
    f = [_rand((nz, ny, nx), 31 + c) for c in range(k)]
    gf = torch.from_numpy(np.stack(f).ravel()).cuda()
    rhs = [pt_cpu.polarized_rhs(x) for x in f]
    g3 = s.polarized_op(3, gf, k).cpu().numpy()
    ref = np.concatenate([_pairs_gpu_layout([r[0] for r in rhs]),
                          _pairs_gpu_layout([r[1] for r in rhs])])
    assert relative_error(g3, ref)[0] <= 1e-11
    g4 = s.polarized_op(4, gf, k).cpu().numpy()
    pre = [pt_cpu.precondition(*r) for r in rhs]
    ref = np.concatenate([_pairs_gpu_layout([r[0] for r in pre]),
                          _pairs_gpu_layout([r[1] for r in pre])])
    assert relative_error(g4, ref)[0] <= 1e-10


@pytest.mark.parametrize("name", ["homogeneous-25", "smooth-24", "layered-28"])
def test_fp64_solve_matches_direct(name):
    wl = workload(name)
    pb = _problem(wl)
    srcs = wl.sources[:2]
    F = point_source_rhs(pb.shape, srcs, wl.h)
    ref = SparseLU(pb.operator()).solve(F)
    s = _solver(wl, "fp64", gmres_tol=1e-10)
    u, info = s.solve_points(srcs, info=True)
    u = u.cpu().numpy().reshape(len(srcs), -1).T
    err = relative_error(u, ref)
    print(name, "fp64 err", err, info)
    assert err.max() <= 1e-9


@pytest.mark.parametrize("name", ["homogeneous-25", "layered-28"])
def test_mixed_solve_matches_direct(name):
    wl = workload(name)
    pb = _problem(wl)
    srcs = wl.sources[:2]
    F = point_source_rhs(pb.shape, srcs, wl.h)
    ref = SparseLU(pb.operator()).solve(F)
    s = _solver(wl, "mixed")
    u, info = s.solve_points(srcs, info=True)
    u = u.cpu().numpy().reshape(len(srcs), -1).T
    err = relative_error(u, ref)
    print(name, "mixed err", err, info)
    assert err.max() <= 1e-6


def test_single_layer_equals_global_solve():
    """L = 1: the method is one local solve of the global system."""
    from helm_inputs import smooth_random_model, omega_for_ppw
    import paper_1801_08655_amd as pt
    n, p = 16, 4
    h = 1.0 / (n - 1)
    m = smooth_random_model((n, n, n), 0.25, 2.0, 0.75, 1.25, 5)
    om = omega_for_ppw(0.75, h, 10.0)
    pb = Problem(m, h, om, p, 25.0)
    F = point_source_rhs(pb.shape, [(5, 7, 9), (8, 8, 8)], h)
    ref = SparseLU(pb.operator()).solve(F)
    s = pt.Solver(m, h, om, p, 1, precision="fp64", pml_C=25.0)
    u = s.solve(torch.from_numpy(F.T.reshape(2, n, n, n).copy()).cuda()).cpu().numpy()
    assert relative_error(u.reshape(2, -1).T, ref).max() <= 1e-11


def test_layer_solve_wide_batch(homog):
    """k = 70 columns: more than one 64-column tile in every substitution."""
    wl, pb, _ = homog
    s = _solver(wl, "fp64")
    nx, ny, nz = wl.n
    l = 1
    _, _, lo, hi = s.layer_info(l)
    t = hi - lo + 1
    r = _rand((70, t, ny, nx), 3)
    w = s.layer_solve(l, torch.from_numpy(r).cuda()).cpu().numpy()
    Hl = local_operator(pb, wl.n_layers, wl.pml_local, l)
    ref = SparseLU(Hl).solve(r.reshape(70, -1).T).T
    assert relative_error(w.reshape(70, -1).T, ref.T).max() <= 1e-11


def test_batches_wider_than_max_rhs_are_chunked():
    """5 sources with max_rhs = 3: two internal batches, same results."""
    wl = workload("smooth-24")
    pb = _problem(wl)
    srcs = [(8, 9, 7), (12, 12, 12), (15, 7, 16), (6, 14, 10), (11, 11, 6)]
    ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, srcs, wl.h))
    s = _solver(wl, "fp64", max_rhs=3)
    u = s.solve_points(srcs).cpu().numpy().reshape(len(srcs), -1).T
    assert relative_error(u, ref).max() <= 1e-9


def test_batch_composition_does_not_change_results():
    """A column solved alone and inside a batch agree to rounding."""
    wl = workload("layered-28")
    s = _solver(wl, "fp64")
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12)]
    alone = s.solve_points(srcs[1:2]).cpu().numpy()
    mixed = s.solve_points(srcs).cpu().numpy()[1:2]
    assert relative_error(mixed.reshape(1, -1).T, alone.reshape(1, -1).T)[0] <= 1e-10


def test_autotuned_tiles_give_the_same_solution():
    """Column-tile widths chosen by timing (16 or 32 columns for a batch of
    21) change the launch shapes, not the arithmetic of any column."""
    import paper_1801_08655_amd as pt
    wl = workload("layered-28")
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12), (11, 17, 15), (5, 20, 9), (16, 6, 18),
            (12, 12, 21)] * 3
    a = _solver(wl, "fp64")
    ua = a.solve_points(srcs).cpu().numpy().reshape(len(srcs), -1).T
    b = _solver(wl, "fp64", flags=pt._lib.HELM_FLAG_AUTOTUNE)
    ub = b.solve_points(srcs).cpu().numpy().reshape(len(srcs), -1).T
    assert relative_error(ub, ua).max() <= 1e-12
    ch = b.tile_choices()
    print(ch[:4])
    assert ch and all(c["tuned"] for c in ch)
    assert {c["fwd_bn"] for c in ch} <= {16, 32} and {c["bwd_bn"] for c in ch} <= {16, 32}
    assert any(c["t_fwd_us"][1] > 0 and c["t_fwd_us"][2] > 0 for c in ch)
    assert all(c["tuned"] == 0 for c in a.tile_choices())


@pytest.mark.parametrize("name,precision,tol", [("homogeneous-25", "fp64", 1e-9),
                                                ("layered-28", "fp64", 1e-9),
                                                ("layered-28", "mixed", 1e-6)])
def test_solution_matches_stored_oracle_samples(name, precision, tol):
    """Sampled nodes of the solution against tests/golden (written from the
    oracle's direct solve by tests/golden/make_golden.py)."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "make_golden.py")
    spec = importlib.util.spec_from_file_location("make_golden", path)
    g = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(g)
    srcs, rows = g.read(name)
    wl = workload(name)
    s = _solver(wl, precision)
    u = s.solve_points(srcs).cpu().numpy()
    nx, ny, nz = wl.n
    u = u.reshape(len(srcs), -1)
    scale = max(abs(v) for *_, v in rows)
    worst = max(abs(u[c, i + nx * (j + ny * k)] - v) for c, i, j, k, v in rows) / scale
    print(name, precision, "max sampled deviation", worst)
    assert worst <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_non_cubic_grid_matches_direct(precision, tol):
    """nx, ny and nz all different (and not multiples of the tile sizes),
    an uneven layer split and sources off the axes."""
    from helm_inputs import smooth_random_model, omega_for_ppw
    import paper_1801_08655_amd as pt
    nx, ny, nz = 23, 18, 29
    h = 1.0 / 22
    p, L = 4, 3
    m = smooth_random_model((nx, ny, nz), 0.2, 3.0, 0.8, 1.2, 77)
    om = omega_for_ppw(0.8, h, 10.0)
    srcs = [(6, 9, 7), (15, 5, 20), (11, 12, 14)]
    pb = Problem(m, h, om, p, 25.0)
    assert pb.shape == (nz, ny, nx)
    ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, srcs, h))
    s = pt.Solver(m, h, om, p, L, precision=precision, pml_C=25.0, pml_local=3)
    u = s.solve_points(srcs).cpu().numpy()
    assert u.shape == (3, nz, ny, nx)
    err = relative_error(u.reshape(3, -1).T, ref)
    print(precision, "non-cubic err", err)
    assert err.max() <= tol


def test_per_rhs_info():
    """The per-column records: residuals match an independent FP64 residual
    of the oracle, the mixed path records its estimated errors and steps."""
    wl = workload("layered-28")
    pb = _problem(wl)
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12)]
    F = point_source_rhs(pb.shape, srcs, wl.h)
    H = pb.operator()
    for precision in ("fp64", "mixed"):
        s = _solver(wl, precision, err_target=1e-6)
        u, info = s.solve_points(srcs, info=True)
        U = u.cpu().numpy().reshape(len(srcs), -1).T
        rel = np.linalg.norm(F - H @ U, axis=0) / np.linalg.norm(F, axis=0)
        print(precision, info["rhs_rel_residual"], rel, info["rhs_ir_steps"],
              info["rhs_gmres_iters"], info["rhs_est_error"])
        assert len(info["rhs_rel_residual"]) == 3
        assert np.allclose(info["rhs_rel_residual"], rel, rtol=1e-3, atol=1e-15)
        assert max(info["rhs_rel_residual"]) == pytest.approx(info["rel_residual_max"])
        assert all(1 <= g <= info["gmres_iters"] for g in info["rhs_gmres_iters"])
        assert all(1 <= st <= info["ir_steps"] for st in info["rhs_ir_steps"])
        if precision == "mixed":
            assert max(info["rhs_est_error"]) <= 1e-6
        else:
            assert info["rhs_est_error"] == [0.0, 0.0, 0.0]
        s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-3)])
def test_tall_panels_single_layer_residual(precision, tol):
    """L = 1 on 40^3: the top separator has 1600 rows, so as the elimination
    advances its panels take every panel kernel shape (more than 1024 rows,
    up to 1024, up to 192 and up to 64, global and LDS homes).  The local
    solve is checked by its residual under the oracle's own assembly."""
    from helm_inputs import smooth_random_model, omega_for_ppw
    import paper_1801_08655_amd as pt
    n, p = 40, 5
    h = 1.0 / (n - 1)
    m = smooth_random_model((n, n, n), 0.25, 2.0, 0.75, 1.25, 8)
    om = omega_for_ppw(0.75, h, 10.0)
    pb = Problem(m, h, om, p, 25.0)
    s = pt.Solver(m, h, om, p, 1, precision=precision, pml_C=25.0)
    r = _rand((2, n, n, n), 41)
    w = s.layer_solve(0, torch.from_numpy(r).cuda()).cpu().numpy()
    R = r.reshape(2, -1).T
    res = R - pb.operator() @ w.reshape(2, -1).T
    assert (np.linalg.norm(res, axis=0) / np.linalg.norm(R, axis=0)).max() <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_twelve_column_solve_matches_direct(precision, tol):
    """12 sources: the volume <-> layer copies run as 64-column LDS tiles with
    52 masked columns (narrower batches take the element loop); every column
    against the oracle's direct solve."""
    wl = workload("homogeneous-25")
    pb = _problem(wl)
    srcs = [(6 + (3 * i) % 13, 6 + (7 * i) % 13, 6 + (5 * i) % 13) for i in range(12)]
    ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, srcs, wl.h))
    s = _solver(wl, precision)
    u = s.solve_points(srcs).cpu().numpy().reshape(len(srcs), -1).T
    assert relative_error(u, ref).max() <= tol


def test_up_going_block_krylov_matches_whole_system():
    """GMRES on the up-going block of the block-triangular preconditioned
    system (the default) and on the whole polarized system give the same
    solution, and the block needs no more iterations."""
    import paper_1801_08655_amd as pt
    wl = workload("layered-28")
    pb = _problem(wl)
    srcs = [(8, 9, 6), (14, 14, 9), (20, 8, 12)]
    ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, srcs, wl.h))
    out = {}
    for name, flags in (("block", 0), ("whole", pt._lib.HELM_FLAG_FULL_KRYLOV)):
        s = _solver(wl, "fp64", flags=flags)
        u, info = s.solve_points(srcs, info=True)
        out[name] = (u.cpu().numpy().reshape(len(srcs), -1).T, info["gmres_iters"])
        s.close()
    print({k: v[1] for k, v in out.items()})
    assert relative_error(out["block"][0], ref).max() <= 1e-9
    assert relative_error(out["whole"][0], ref).max() <= 1e-9
    assert out["block"][1] <= out["whole"][1]
