"""The allocation-free local solve (helm_layer_solve_noalloc_dev) against the
allocating one (helm_layer_solve_dev) and against the oracle's direct solve of
the local operator, on two calls in a row (the second with a smaller input),
through the C ABI (run on an MI355X)."""

import ctypes

import numpy as np
import pytest

from helm_inputs import workload
from oracle.direct import SparseLU, relative_error
from oracle.discretization import Problem, local_operator

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::DeprecationWarning")]

torch = pytest.importorskip("torch")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _noalloc(s, l, r, w):
    import paper_1801_08655_amd as pt
    return pt.lib().helm_layer_solve_noalloc_dev(s._h, l, r.shape[0], r.data_ptr(),
                                                 w.data_ptr())


@pytest.mark.parametrize("name,precision,oracle_tol", [("homogeneous-25", "fp64", 1e-11),
                                                       ("layered-28", "mixed", 2e-4)])
def test_noalloc_layer_solve_matches_allocating_entry_point(name, precision, oracle_tol):
    import paper_1801_08655_amd as pt
    wl = workload(name)
    s = pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=precision,
                  pml_local=wl.pml_local, pml_C=wl.pml_C)
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    nx, ny, _ = wl.n
    # two calls in a row, the second on a smaller input (other layer, fewer
    # columns): the array keeps the first call's contents
    for l, k, seed in ((1, 5, 11), (0, 2, 12)):
        _, _, lo, hi = s.layer_info(l)
        t = hi - lo + 1
        r_h = _rand((k, t, ny, nx), seed)
        r = torch.from_numpy(r_h).cuda()
        w_na = torch.empty_like(r)
        print(f"noalloc layer solve: {name} {precision} layer {l} k {k}", flush=True)
        assert _noalloc(s, l, r, w_na) == pt.HELM_OK
        w_ref = s.layer_solve(l, r)
        a = w_na.cpu().numpy().reshape(k, -1).T
        b = w_ref.cpu().numpy().reshape(k, -1).T
        dev = relative_error(a, b).max()
        print(f"  vs helm_layer_solve_dev: {dev:.2e} (bitwise equal: {np.array_equal(a, b)})")
        assert dev <= 1e-12
        ref = SparseLU(local_operator(pb, wl.n_layers, wl.pml_local, l)).solve(
            r_h.reshape(k, -1).T)
        err = relative_error(a, ref).max()
        print(f"  vs the oracle's direct solve of H^l: {err:.2e}")
        assert err <= oracle_tol
    s.close()


def test_noalloc_allocates_nothing_and_refuses_oversized_batches():
    import paper_1801_08655_amd as pt
    wl = workload("homogeneous-25")
    s = pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision="fp64",
                  pml_local=wl.pml_local, pml_C=wl.pml_C)
    nx, ny, _ = wl.n
    l = 1
    _, _, lo, hi = s.layer_info(l)
    t = hi - lo + 1
    r = torch.from_numpy(_rand((3, t, ny, nx), 5)).cuda()
    w = torch.empty_like(r)
    assert _noalloc(s, l, r, w) == pt.HELM_OK
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    assert _noalloc(s, l, r, w) == pt.HELM_OK
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    # a batch whose workspace exceeds the static array is refused before any
    # launch: X and Z alone of k columns need 2 n_loc k 16 bytes
    n_loc = t * ny * nx
    k_big = pt._lib.HELM_NOALLOC_SCRATCH_BYTES // (2 * n_loc * 16) + 1
    big = torch.zeros((k_big, t, ny, nx), dtype=torch.complex128, device="cuda")
    wb = torch.empty_like(big)
    st = _noalloc(s, l, big, wb)
    assert st == pt.HELM_ENOMEM
    assert "static scratch" in pt.lib().helm_last_error().decode()
    # null arguments and a bad layer are refused too
    assert pt.lib().helm_layer_solve_noalloc_dev(s._h, l, 1, None, None) == pt.HELM_EINVAL
    assert pt.lib().helm_layer_solve_noalloc_dev(s._h, 99, 1, r.data_ptr(),
                                                 w.data_ptr()) == pt.HELM_EINVAL
    # the entry point still works after the refusals
    w2 = torch.empty_like(r)
    assert _noalloc(s, l, r, w2) == pt.HELM_OK
    assert torch.equal(w2, w)
    s.close()
