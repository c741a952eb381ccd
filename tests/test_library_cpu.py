"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, and its planner (nested dissection of the
layers) agrees with an independent count written here from the same
geometric rules."""

import ctypes
import os
import re

import pytest

import paper_1801_08655_amd as pt
from paper_1801_08655_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            with open(os.path.join(inc, f)) as fh:
                names |= set(re.findall(r"\b(helm_[a-z_]+)\s*\(", fh.read()))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = pt.lib()
    declared = _declared_symbols()
    assert len(declared) >= 24
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(declared) == sorted(_lib.EXPORTED)


def test_default_options_and_strerror():
    o = pt.options()
    assert o.pml_local == 4 and o.precision == pt.HELM_MIXED and o.max_rhs == 64
    assert pt.lib().helm_strerror(pt.HELM_ENOMEM).decode().startswith("out of memory")


def test_plan_rejects_impossible_geometry():
    g = _lib.helm_grid(20, 20, 20, 1 / 19)
    o = pt.options()
    fb = ctypes.c_size_t()
    # 20 layers need at least 20 interior planes
    st = pt.lib().helm_plan(ctypes.byref(g), 6, 20, ctypes.byref(o), ctypes.byref(fb),
                            None, None)
    assert st == pt.HELM_EINVAL
    st = pt.lib().helm_plan(ctypes.byref(g), 10, 2, ctypes.byref(o), ctypes.byref(fb),
                            None, None)
    assert st == pt.HELM_EINVAL


# --------------------------------------------------------------------------
# independent count of the nested-dissection plan
# --------------------------------------------------------------------------

def _layer_planes(nz, p, L, alpha):
    interior = nz - 2 * p
    base, extra = divmod(interior, L)
    out, s = [], p
    for l in range(L):
        size = base + (1 if l < extra else 0)
        out.append([s, s + size - 1])
        s += size
    out[0][0] = 0
    out[-1][1] = nz - 1
    t = []
    for l, (s, e) in enumerate(out):
        lo = s - alpha if l > 0 else s
        hi = e + alpha if l < L - 1 else e
        t.append(hi - lo + 1)
    return t


def _nd_count(nx, ny, t, leaf):
    """Fronts of the geometric bisection: (s, b) per front."""
    fronts = []

    def rec(lo, hi):
        ext = [hi[a] - lo[a] for a in range(3)]
        vol = ext[0] * ext[1] * ext[2]
        if vol <= 0:
            return
        dims = (nx, ny, t)
        b = 0
        for a in range(3):
            o = [ext[q] for q in range(3) if q != a]
            if lo[a] > 0:
                b += o[0] * o[1]
            if hi[a] < dims[a]:
                b += o[0] * o[1]
        ax = max(range(3), key=lambda a: (ext[a], -a))
        if vol <= leaf or ext[ax] < 3:
            fronts.append((vol, b))
            return
        mid = lo[ax] + ext[ax] // 2
        h1 = list(hi); h1[ax] = mid
        l2 = list(lo); l2[ax] = mid + 1
        rec(lo, h1)
        rec(l2, hi)
        fronts.append((vol // ext[ax], b))

    rec([0, 0, 0], [nx, ny, t])
    return fronts


@pytest.mark.parametrize("n,p,L,alpha,leaf", [((25, 25, 25), 6, 3, 6, 64),
                                              ((40, 36, 44), 5, 4, 3, 32),
                                              ((100, 100, 100), 10, 10, 4, 64)])
def test_plan_matches_independent_count(n, p, L, alpha, leaf):
    nx, ny, nz = n
    elems = 0
    mf = 0
    for t in _layer_planes(nz, p, L, alpha):
        fr = _nd_count(nx, ny, t, leaf)
        assert sum(s for s, _ in fr) == nx * ny * t
        elems += sum((s + b) * s for s, b in fr)
        mf = max(mf, max(s + b for s, b in fr))
    for prec, size in (("fp64", 16), ("mixed", 8)):
        r = pt.plan(n, p, L, precision=prec, pml_local=alpha, leaf_size=leaf)
        assert r["factor_bytes"] == elems * size
        assert r["max_front"] == mf
        assert r["bytes_per_rhs"] > 0


def test_headline_plan_fits_one_gpu():
    """200^3 with 20 layers: complex64 and complex128 factors both fit in
    288 GB of HBM with room for the solve workspace of 64 columns."""
    for prec in ("mixed", "fp64"):
        r = pt.plan((200, 200, 200), 15, 20, precision=prec, pml_local=4)
        total = r["factor_bytes"] + 32 * r["bytes_per_rhs"]
        assert total < 288e9, (prec, r)


def test_server_entry_points_reject_null_arguments():
    """Argument checks of the request server that return before any device call."""
    L = pt.lib()
    assert L.helm_server_create(None, None) == pt.HELM_EINVAL
    assert L.helm_server_add_model(None, None, None, None) == pt.HELM_EINVAL
    rid = ctypes.c_int64()
    assert L.helm_server_submit(None, 0, 1, None, None, None, ctypes.byref(rid)) == pt.HELM_EINVAL
    assert L.helm_server_wait(None, 1, None) == pt.HELM_EINVAL
    assert L.helm_server_poll(None, 1, None) == pt.HELM_EINVAL
    assert L.helm_server_get_stats(None, None) == pt.HELM_EINVAL
    assert L.helm_server_free(None) == pt.HELM_OK
    o = _lib.helm_server_options()
    L.helm_server_default_options(ctypes.byref(o))
    assert o.slots == 32 and o.hbm_budget_bytes == 0


def test_batch_entry_point_rejects_bad_problems():
    """Argument checks of helm_solve_batch that return before any device call."""
    L = pt.lib()
    assert L.helm_solve_batch(1, None, None, None, None) == pt.HELM_EINVAL
    arr = (_lib.helm_problem * 1)()
    arr[0] = _lib.helm_problem(_lib.helm_grid(8, 8, 8, 1 / 7.0), None, 1.0, 2, 1, 0,
                               None, None, None)
    assert L.helm_solve_batch(1, arr, None, None, None) == pt.HELM_EINVAL   # null model
    m = (ctypes.c_double * 512)()
    arr[0] = _lib.helm_problem(_lib.helm_grid(8, 8, 8, 1 / 7.0), ctypes.addressof(m), 1.0,
                               2, 1, 3, None, None, None)
    assert L.helm_solve_batch(1, arr, None, None, None) == pt.HELM_EINVAL   # null sources
    bo = _lib.helm_batch_options()
    L.helm_batch_default_options(ctypes.byref(bo))
    assert bo.slots == 64 and bo.opt.precision == pt.HELM_MIXED


def test_factorize_rejects_bad_models_before_any_device_call():
    """Non-finite or non-positive squared slowness, null arguments and an
    impossible layer split are refused with HELM_EINVAL on the host."""
    import numpy as np
    L = pt.lib()
    n = 12
    g = _lib.helm_grid(n, n, n, 1.0 / (n - 1))
    o = pt.options()
    h = ctypes.c_void_p()
    good = np.full((n, n, n), 1.0)
    for bad_val in (np.nan, np.inf, 0.0, -1.0):
        m = good.copy()
        m[3, 4, 5] = bad_val
        st = L.helm_factorize(ctypes.byref(g), m.ctypes.data, 10.0, 2, 2, ctypes.byref(o),
                              ctypes.byref(h))
        assert st == pt.HELM_EINVAL, bad_val
        assert "squared slowness" in L.helm_last_error().decode()
    assert L.helm_factorize(None, good.ctypes.data, 10.0, 2, 2, ctypes.byref(o),
                            ctypes.byref(h)) == pt.HELM_EINVAL
    assert L.helm_factorize(ctypes.byref(g), None, 10.0, 2, 2, ctypes.byref(o),
                            ctypes.byref(h)) == pt.HELM_EINVAL
    # 9 layers cannot split 8 interior planes
    st = L.helm_factorize(ctypes.byref(g), good.ctypes.data, 10.0, 2, 9, ctypes.byref(o),
                          ctypes.byref(h))
    assert st == pt.HELM_EINVAL


def test_entry_points_reject_null_handles():
    L = pt.lib()
    x = ctypes.c_double()
    assert L.helm_solve(None, 1, ctypes.byref(x), ctypes.byref(x), None) == pt.HELM_EINVAL
    assert L.helm_solve_dev(None, 1, ctypes.byref(x), ctypes.byref(x), None) == pt.HELM_EINVAL
    assert L.helm_solve_points(None, 1, ctypes.byref(x), ctypes.byref(x), ctypes.byref(x),
                               None) == pt.HELM_EINVAL
    assert L.helm_layer_solve_dev(None, 0, 1, ctypes.byref(x), ctypes.byref(x)) == pt.HELM_EINVAL
    assert L.helm_kernel_stats(None, None, 0, None, 0) == pt.HELM_EINVAL
    assert L.helm_tile_choices(None, None, 0, None) == pt.HELM_EINVAL
    assert L.helm_set_solve_options(None, None) == pt.HELM_EINVAL
    assert L.helm_free(None) == pt.HELM_OK


def test_binding_constants_match_the_header():
    """Every HELM_* integer macro of the headers (flags, status codes,
    precisions, limits) has the same value in the binding."""
    inc = os.path.join(ROOT, "include")
    found = 0
    for f in sorted(os.listdir(inc)):
        if not f.endswith(".h"):
            continue
        with open(os.path.join(inc, f)) as fh:
            text = fh.read()
        for name, val in re.findall(r"#define\s+(HELM_[A-Z0-9_]+)\s+\(?(-?\d+)", text):
            if hasattr(_lib, name):
                found += 1
                assert getattr(_lib, name) == int(val) or name == "HELM_NOALLOC_SCRATCH_BYTES", name
    assert found >= 15
    assert _lib.HELM_NOALLOC_SCRATCH_BYTES == 128 << 20


def test_default_refinement_options():
    """Defaults of the refinement stop rule (documented in helm.h)."""
    o = pt.options()
    assert o.inner_tol == pytest.approx(5e-4) and o.inner_tol_refine == pytest.approx(2e-4)
    assert o.inner_tol_final == pytest.approx(1e-1) and o.gmres_restart == 0
