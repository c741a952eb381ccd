"""Request server on the GPU: continuous batching over resident
factorizations, checked against the oracle's global direct solve.

Each request's columns are compared with SuperLU on the oracle's assembly
(relative l2 <= 1e-6 for complex64 factors with FP64 refinement, <= 1e-9
for complex128 factors), and a request solved alone is compared with the
same request solved inside a mix of other requests (<= 1e-6)."""

import time

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


def _reference(wl, nodes, amps=None):
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    F = point_source_rhs(pb.shape, nodes, wl.h)
    if amps is not None:
        F = F * np.asarray(amps)[None, :]
    return SparseLU(pb.operator()).solve(F)


def _cols(u):
    return u.cpu().numpy().reshape(u.shape[0], -1).T


REQS = {
    "a": [(8, 9, 6), (14, 14, 9), (20, 8, 12)],
    "b": [(10, 10, 10), (17, 12, 7)],
    "c": [(6, 6, 15), (12, 18, 20), (21, 21, 8), (9, 15, 11), (15, 9, 18)],
    "d": [(13, 13, 13)],
}


@pytest.fixture(scope="module")
def layered():
    wl = workload("layered-28")
    refs = {k: _reference(wl, v) for k, v in REQS.items()}
    return wl, refs


def test_server_alone_equals_in_mix(layered):
    from paper_1801_08655_amd.serving import Server
    wl, refs = layered
    s = _solver(wl, "mixed", err_target=1e-6)
    srv = Server(slots=4)
    m = srv.add_model(s)
    assert srv.slots(m) == 4
    alone, info_a = srv.submit(m, REQS["a"]).wait()
    alone = _cols(alone)
    assert info_a["status"] == 0
    assert relative_error(alone, refs["a"]).max() <= 1e-6
    # the mix: 11 columns through 4 slots, so columns of later requests enter
    # slots while earlier requests are still being refined
    order = ["b", "c", "a", "d"]
    reqs = {k: srv.submit(m, REQS[k]) for k in order}
    out = {k: reqs[k].wait() for k in order}
    for k in order:
        u, inf = out[k]
        err = relative_error(_cols(u), refs[k])
        print(k, "err", err, inf)
        assert inf["status"] == 0
        assert err.max() <= 1e-6
    mixed_a = _cols(out["a"][0])
    assert relative_error(mixed_a, alone).max() <= 1e-6
    infos = [out[k][1] for k in order]
    # some request entered the lane while another one was still in it
    joined = any(x["t_first_ms"] > y["t_first_ms"] and x["t_first_ms"] < y["t_done_ms"]
                 for x in infos for y in infos if x is not y)
    assert joined
    st = srv.stats()
    print(st)
    assert st["requests_done"] == 5 and st["columns_done"] == 14
    assert st["mean_active_slots"] > 1.0
    srv.close()
    s.close()


def test_server_two_models_run_concurrently(layered):
    """Two resident factorizations (two frequencies of one model, as the
    paper's sources at several frequencies), each with its own lane."""
    from paper_1801_08655_amd.serving import Server
    import paper_1801_08655_amd as pt
    wl, refs = layered
    wl2 = workload("layered-28")
    wl2.ppw = 10.0        # second frequency
    s1 = _solver(wl, "mixed", err_target=1e-6)
    s2 = _solver(wl2, "mixed", err_target=1e-6)
    srv = Server(slots=3)
    m1, m2 = srv.add_model(s1), srv.add_model(s2)
    amps = [1.0 + 0.5j, -2.0, 0.25j]
    r1 = srv.submit(m1, REQS["a"])
    r2 = srv.submit(m2, REQS["a"], amplitudes=amps)
    r3 = srv.submit(m1, REQS["c"])
    u1, i1 = r1.wait()
    u2, i2 = r2.wait()
    u3, i3 = r3.wait()
    assert relative_error(_cols(u1), refs["a"]).max() <= 1e-6
    assert relative_error(_cols(u3), refs["c"]).max() <= 1e-6
    ref2 = _reference(wl2, REQS["a"], amps)
    assert relative_error(_cols(u2), ref2).max() <= 1e-6
    # the second model's request did not wait for the first model's lane
    assert i2["t_first_ms"] < i1["t_done_ms"]
    srv.close()
    s1.close()
    s2.close()


def test_server_fp64_model(layered):
    from paper_1801_08655_amd.serving import Server
    wl, refs = layered
    s = _solver(wl, "fp64", gmres_tol=1e-10)
    srv = Server(slots=2)
    m = srv.add_model(s)
    u, inf = srv.submit(m, REQS["c"]).wait()
    assert inf["status"] == 0 and inf["ir_steps_max"] == 1
    assert relative_error(_cols(u), refs["c"]).max() <= 1e-9
    srv.close()
    s.close()


def test_server_admission_and_errors(layered):
    import paper_1801_08655_amd as pt
    from paper_1801_08655_amd.serving import Server
    wl, _ = layered
    s = _solver(wl, "mixed")
    tiny = Server(slots=8, hbm_budget_bytes=1 << 20)
    with pytest.raises(pt.HelmError) as e:
        tiny.add_model(s)
    assert e.value.status == pt.HELM_ENOMEM
    tiny.close()
    srv = Server(slots=8)
    m = srv.add_model(s)
    with pytest.raises(ValueError):
        srv.submit(m, [(wl.n[0], 0, 0)])     # outside the grid
    # the library's own check of the linear index
    import ctypes
    N = wl.n[0] * wl.n[1] * wl.n[2]
    idx = np.array([N], dtype=np.int64)
    amp = np.ones(1, dtype=np.complex128)
    out = torch.empty((1, N), dtype=torch.complex128, device="cuda")
    rid = ctypes.c_int64()
    st = pt.lib().helm_server_submit(srv._s, m, 1, idx.ctypes.data, amp.ctypes.data,
                                     out.data_ptr(), ctypes.byref(rid))
    assert st == pt.HELM_EINVAL
    amp[0] = np.nan
    idx[0] = 5
    st = pt.lib().helm_server_submit(srv._s, m, 1, idx.ctypes.data, amp.ctypes.data,
                                     out.data_ptr(), ctypes.byref(rid))
    assert st == pt.HELM_EINVAL
    with pytest.raises(ValueError):
        srv.submit(m + 5, [(1, 1, 1)])
    st = pt.lib().helm_server_submit(srv._s, m + 5, 1, idx.ctypes.data, amp.ctypes.data,
                                     out.data_ptr(), ctypes.byref(rid))
    assert st == pt.HELM_EINVAL
    r = srv.submit(m, [])
    u, inf = r.wait()
    assert inf["status"] == 0 and u.shape[0] == 0
    srv.close()
    s.close()


def test_caller_allocations_during_lane_graph_captures(layered):
    """The caller keeps allocating and computing with torch on its default
    stream, and synchronizes the whole device, while the server's lane runs
    requests of new widths (every request size below is a new narrowest
    width, 1 to 8 columns): the lane launches its kernels without graph
    captures, so none of this is an error, and every request still matches
    the oracle."""
    from paper_1801_08655_amd.serving import Server
    wl, refs = layered
    s = _solver(wl, "mixed", err_target=1e-6)
    srv = Server(slots=8)
    mid = srv.add_model(s)
    nodes = REQS["c"] + REQS["a"]
    reqs = []
    for n in (1, 2, 3, 5, 8):
        reqs.append((n, srv.submit(mid, nodes[:n])))
        for _ in range(20):   # default-stream work while the lane runs
            x = torch.empty((1 << 18,), dtype=torch.complex128, device="cuda")
            x.fill_(1.0)
            y = (x * 2).sum()
        torch.cuda.synchronize()
    ref_all = np.concatenate([refs["c"], refs["a"]], axis=1)
    for n, r in reqs:
        u, _ = r.wait()
        err = relative_error(_cols(u), ref_all[:, :n])
        print(n, "columns: max err", err.max())
        assert err.max() <= 1e-6
    assert float(y.real) == 2.0 * (1 << 18)
    srv.close()
    s.close()
