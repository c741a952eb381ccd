"""The Krylov variants the paper names, on the GPU, against the oracle (run on
an MI355X):

* Bi-CGSTAB on the preconditioned polarized system (HELM_FLAG_BICGSTAB),
  on its up-going block and on the whole system;
* GMRES on the unpolarized SIE of Algorithms 2-3 with the sign made
  consistent (HELM_FLAG_UNPOLARIZED), without preconditioner;
* the product forms of the complex64 GEMMs (three or four real products
  per complex product, in the substitutions and in the factorization).

Each solution is compared column by column with the oracle's global direct
solve (complex128 <= 1e-9 at tolerance 1e-10, mixed precision <= 1e-6), and
the iteration counts with the oracle's own CPU implementation of the same
variant (oracle/bicgstab.py, PolarizedTraces.solve_unpolarized)."""

import numpy as np
import pytest

from helm_inputs import workload
from oracle.direct import SparseLU, relative_error
from oracle.discretization import Problem, point_source_rhs
from oracle.polarized import PolarizedTraces

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::DeprecationWarning")]

torch = pytest.importorskip("torch")

SOURCES = {"homogeneous-25": [(12, 12, 12), (8, 15, 10)],
           "layered-28": [(8, 9, 6), (14, 14, 9), (20, 8, 12)]}
_CACHE = {}


def _case(name):
    if name not in _CACHE:
        wl = workload(name)
        srcs = SOURCES[name]
        pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
        F = point_source_rhs(pb.shape, srcs, wl.h)
        print(f"oracle: direct solve of {name}", flush=True)
        ref = SparseLU(pb.operator()).solve(F)
        _CACHE[name] = (wl, pb, srcs, F, ref)
    return _CACHE[name]


def _solver(wl, precision, **kw):
    import paper_1801_08655_amd as pt
    return pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=precision,
                     pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)


@pytest.mark.parametrize("name", ["homogeneous-25", "layered-28"])
@pytest.mark.parametrize("krylov", ["block", "whole"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_bicgstab_matches_direct(name, krylov, precision, tol):
    import paper_1801_08655_amd as pt
    wl, pb, srcs, F, ref = _case(name)
    flags = pt._lib.HELM_FLAG_BICGSTAB | (0 if krylov == "block" else
                                          pt._lib.HELM_FLAG_FULL_KRYLOV)
    kw = {"gmres_tol": 1e-10} if precision == "fp64" else {"err_target": 1e-6}
    s = _solver(wl, precision, flags=flags, **kw)
    u, info = s.solve_points(srcs, info=True)
    err = relative_error(u.cpu().numpy().reshape(len(srcs), -1).T, ref)
    print(name, krylov, precision, "Bi-CGSTAB err", err, "iterations", info["gmres_iters"],
          "Krylov bytes", info["krylov_bytes"])
    assert err.max() <= tol
    s.close()


@pytest.mark.parametrize("name", ["homogeneous-25", "layered-28"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_unpolarized_sie_matches_direct(name, precision, tol):
    import paper_1801_08655_amd as pt
    wl, pb, srcs, F, ref = _case(name)
    kw = {"gmres_tol": 1e-10} if precision == "fp64" else {"err_target": 1e-6}
    s = _solver(wl, precision, flags=pt._lib.HELM_FLAG_UNPOLARIZED, gmres_max_iter=400, **kw)
    u, info = s.solve_points(srcs, info=True)
    err = relative_error(u.cpu().numpy().reshape(len(srcs), -1).T, ref)
    print(name, precision, "unpolarized SIE err", err, "iterations", info["gmres_iters"],
          "layer solves", info["layer_solves"])
    assert err.max() <= tol
    s.close()


@pytest.mark.parametrize("name", ["homogeneous-25", "layered-28"])
def test_variant_iteration_counts_follow_the_oracle(name):
    """complex128 on the GPU and the oracle's CPU implementation of each
    variant take the same number of iterations up to rounding (one column at
    a time: the GPU's batched Krylov spaces are independent per column);
    Bi-CGSTAB holds fewer Krylov vectors than GMRES."""
    import paper_1801_08655_amd as pt
    wl, pb, srcs, F, ref = _case(name)
    ptc = PolarizedTraces(pb, wl.n_layers, wl.pml_local)
    f = F[:, 0].reshape(pb.shape)
    _, it_g, _ = ptc.solve(f, tol=1e-10)
    _, it_b, _ = ptc.solve(f, tol=1e-10, krylov="bicgstab")
    _, it_u, _ = ptc.solve_unpolarized(f, tol=1e-10)
    got = {}
    for label, flags in (("gmres", pt._lib.HELM_FLAG_FULL_KRYLOV),
                         ("bicgstab", pt._lib.HELM_FLAG_BICGSTAB | pt._lib.HELM_FLAG_FULL_KRYLOV),
                         ("unpolarized", pt._lib.HELM_FLAG_UNPOLARIZED)):
        s = _solver(wl, "fp64", flags=flags, gmres_tol=1e-10, gmres_max_iter=400)
        _, info = s.solve_points(srcs[:1], info=True)
        got[label] = (info["gmres_iters"], info["krylov_bytes"])
        s.close()
    print(name, "oracle", {"gmres": it_g, "bicgstab": it_b, "unpolarized": it_u}, "gpu", got)
    assert abs(got["gmres"][0] - it_g) <= 1
    assert abs(got["bicgstab"][0] - it_b) <= 1
    assert abs(got["unpolarized"][0] - it_u) <= max(2, it_u // 10)
    assert got["bicgstab"][1] < got["gmres"][1] or got["gmres"][0] <= 4
    assert got["unpolarized"][0] > got["gmres"][0]


@pytest.mark.parametrize("k", [3, 21, 70])
def test_product_forms_of_the_local_solve(k):
    """complex64 local solves with three real products per complex product
    (the default) and with four (HELM_FLAG_GEMM_4M), at batch widths that
    reach the 16-, 32- and 64-column tiles and a ragged second 64-column
    tile, each against SuperLU on the oracle's H^l; complex128 ignores the
    flag bit for bit."""
    import paper_1801_08655_amd as pt
    from oracle.discretization import local_operator
    wl = workload("homogeneous-25")
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    nx, ny, nz = wl.n
    l = 1
    rng = np.random.default_rng(40 + k)
    s3 = _solver(wl, "mixed")
    s4 = _solver(wl, "mixed", flags=pt._lib.HELM_FLAG_GEMM_4M)
    _, _, lo, hi = s3.layer_info(l)
    t = hi - lo + 1
    r = rng.standard_normal((k, t, ny, nx)) + 1j * rng.standard_normal((k, t, ny, nx))
    rt = torch.from_numpy(r).cuda()
    Hl = local_operator(pb, wl.n_layers, wl.pml_local, l)
    ref = SparseLU(Hl).solve(r.reshape(k, -1).T)
    e = {}
    for name, s in (("3M", s3), ("4M", s4)):
        w = s.layer_solve(l, rt).cpu().numpy()
        e[name] = relative_error(w.reshape(k, -1).T, ref)
        s.close()
    print("k", k, "max rel err 3M", e["3M"].max(), "4M", e["4M"].max())
    assert e["3M"].max() <= 2e-4 and e["4M"].max() <= 2e-4
    d64 = _solver(wl, "fp64")
    d64b = _solver(wl, "fp64", flags=pt._lib.HELM_FLAG_GEMM_4M | pt._lib.HELM_FLAG_FACTOR_4M)
    a = d64.layer_solve(l, rt)
    b = d64b.layer_solve(l, rt)
    assert torch.equal(a, b)
    assert relative_error(a.cpu().numpy().reshape(k, -1).T, ref).max() <= 1e-11


@pytest.mark.parametrize("flags", ["GEMM_4M", "FACTOR_4M", "GEMM_4M|FACTOR_4M"])
def test_product_forms_of_the_mixed_solve(flags):
    """The whole mixed-precision method with the other product forms of the
    complex64 GEMMs (the default form is covered by every other mixed test)
    against the oracle's direct solve."""
    import paper_1801_08655_amd as pt
    wl, pb, srcs, F, ref = _case("layered-28")
    fl = 0
    for f in flags.split("|"):
        fl |= getattr(pt._lib, "HELM_FLAG_" + f)
    s = _solver(wl, "mixed", flags=fl, err_target=1e-6)
    u, info = s.solve_points(srcs, info=True)
    err = relative_error(u.cpu().numpy().reshape(len(srcs), -1).T, ref)
    print(flags, "err", err, "refinement steps", info["ir_steps"])
    assert err.max() <= 1e-6
    s.close()
