"""Error paths of the C ABI on the GPU: every failure is a status code, the
handle stays usable after a refused call, and the iteration limit returns
the best iterate with HELM_ENOCONV."""

import ctypes

import numpy as np
import pytest

from helm_inputs import workload
from oracle.direct import SparseLU, relative_error
from oracle.discretization import Problem, point_source_rhs

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::DeprecationWarning")]

torch = pytest.importorskip("torch")


def _solver(wl, precision, **kw):
    import paper_1801_08655_amd as pt
    return pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=precision,
                     pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)


def test_memory_budget_below_the_factors_is_refused():
    import paper_1801_08655_amd as pt
    wl = workload("layered-28")
    with pytest.raises(pt.HelmError) as e:
        _solver(wl, "mixed", hbm_budget_bytes=1 << 20)
    assert e.value.status == pt.HELM_ENOMEM


def test_iteration_limit_returns_enoconv_and_the_iterate():
    import paper_1801_08655_amd as pt
    wl = workload("layered-28")
    s = _solver(wl, "fp64", gmres_tol=1e-14, gmres_max_iter=1)
    nx, ny, nz = wl.n
    N = nx * ny * nz
    idx = np.array([8 + nx * (9 + ny * 6)], dtype=np.int64)
    amp = np.ones(1, dtype=np.complex128)
    u = torch.empty((1, nz, ny, nx), dtype=torch.complex128, device="cuda")
    inf = pt._lib.helm_solve_info()
    st = pt.lib().helm_solve_points(s._h, 1, idx.ctypes.data, amp.ctypes.data, u.data_ptr(),
                                    ctypes.byref(inf))
    assert st == pt.HELM_ENOCONV
    assert inf.gmres_iters == 1 and np.isfinite(inf.rel_residual_max)
    # one iteration from x0 = 0 already points the right way
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, [(8, 9, 6)], wl.h))
    err = relative_error(u.cpu().numpy().reshape(1, -1).T, ref)[0]
    assert 0 < err < 1.0
    # the handle is still usable at the normal tolerance
    s.set_options(gmres_tol=1e-10, gmres_max_iter=40)
    u2 = s.solve_points([(8, 9, 6)])
    assert relative_error(u2.cpu().numpy().reshape(1, -1).T, ref)[0] <= 1e-9
    s.close()


def test_bad_right_hand_sides_are_refused():
    import paper_1801_08655_amd as pt
    wl = workload("homogeneous-25")
    s = _solver(wl, "mixed")
    nx, ny, nz = wl.n
    N = nx * ny * nz
    L = pt.lib()
    f = np.zeros((1, N), dtype=np.complex128)
    f[0, 5] = np.nan
    u = np.zeros_like(f)
    assert L.helm_solve(s._h, 1, f.ctypes.data, u.ctypes.data, None) == pt.HELM_EINVAL
    idx = np.array([N], dtype=np.int64)
    amp = np.ones(1, dtype=np.complex128)
    ud = torch.empty((1, N), dtype=torch.complex128, device="cuda")
    assert L.helm_solve_points(s._h, 1, idx.ctypes.data, amp.ctypes.data, ud.data_ptr(),
                               None) == pt.HELM_EINVAL
    idx[0] = 7
    amp[0] = np.inf
    assert L.helm_solve_points(s._h, 1, idx.ctypes.data, amp.ctypes.data, ud.data_ptr(),
                               None) == pt.HELM_EINVAL
    assert L.helm_layer_solve_dev(s._h, wl.n_layers, 1, ud.data_ptr(),
                                  ud.data_ptr()) == pt.HELM_EINVAL
    # still usable
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    ref = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, wl.sources, wl.h))
    good = s.solve_points(wl.sources)
    assert relative_error(good.cpu().numpy().reshape(1, -1).T, ref)[0] <= 1e-6
    s.close()
