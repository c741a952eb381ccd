"""Method of polarized traces for the 3D Helmholtz equation on MI355X.

The solver lives in the HIP library ``libhelm.so`` (C ABI in
``include/helm.h``); this package is a thin binding with the same names.
PyTorch is used only to hold device memory and streams.

    import paper_1801_08655_amd as pt
    s = pt.Solver(m, h=1/199, omega=234.4, pml=15, n_layers=20,
                  precision="mixed")
    u = s.solve_points(nodes)          # torch complex128 tensor on the GPU
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (HELM_EINVAL, HELM_ENOCONV, HELM_ENOMEM, HELM_EZEROPIVOT,
                   HELM_FP64, HELM_MIXED, HELM_OK, HelmError, check, lib)

__all__ = ["Solver", "plan", "options", "HelmError", "lib", "HELM_FP64",
           "HELM_MIXED", "HELM_OK", "HELM_ENOCONV", "HELM_EINVAL", "HELM_ENOMEM",
           "HELM_EZEROPIVOT"]


def options(**kw) -> _lib.helm_options:
    """helm_options with the library defaults, overridden by keywords."""
    o = _lib.helm_options()
    lib().helm_default_options(ctypes.byref(o))
    prec = kw.pop("precision", None)
    if prec is not None:
        o.precision = HELM_FP64 if prec in ("fp64", HELM_FP64) else HELM_MIXED
    for key, val in kw.items():
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        setattr(o, key, val)
    return o


def plan(n, pml: int, n_layers: int, h: float = None, **kw):
    """Exact factor bytes, device bytes per RHS column (helm_solve and a
    server or batch lane slot) and largest front."""
    nx, ny, nz = n
    g = _lib.helm_grid(nx, ny, nz, h if h else 1.0 / (max(n) - 1))
    o = options(**kw)
    fb, br, mf, lb = (ctypes.c_size_t() for _ in range(4))
    check(lib().helm_plan(ctypes.byref(g), pml, n_layers, ctypes.byref(o),
                          ctypes.byref(fb), ctypes.byref(br), ctypes.byref(mf)), "helm_plan")
    check(lib().helm_plan_lane(ctypes.byref(g), pml, n_layers, ctypes.byref(o),
                               ctypes.byref(lb)), "helm_plan_lane")
    return {"factor_bytes": fb.value, "bytes_per_rhs": br.value, "max_front": mf.value,
            "lane_bytes_per_rhs": lb.value}


def node_indices(nodes: Sequence, n) -> np.ndarray:
    """Linear indices (x fastest) of (i, j, k) nodes; ValueError outside the grid."""
    nx, ny, nz = n
    out = []
    for (i, j, kk) in nodes:
        if not (0 <= i < nx and 0 <= j < ny and 0 <= kk < nz):
            raise ValueError(f"node {(i, j, kk)} outside the {nx}x{ny}x{nz} grid")
        out.append(i + nx * (j + ny * kk))
    return np.array(out, dtype=np.int64)


def device_peaks(device: int = 0) -> dict:
    """Attainable matrix-core rates and HBM bandwidth of the device (see
    helm_device_peaks in include/helm.h)."""
    v = [ctypes.c_double() for _ in range(4)]
    check(lib().helm_device_peaks(device, *[ctypes.byref(x) for x in v]), "helm_device_peaks")
    return {"mfma_f32_tflops": v[0].value, "mfma_f64_tflops": v[1].value,
            "hbm_read_gbps": v[2].value, "hbm_copy_gbps": v[3].value}


def _ptr(t) -> int:
    """Device pointer of a contiguous torch tensor (complex128 / float64)."""
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class Solver:
    """Handle of a factorized problem (offline stage) with its online calls."""

    def __init__(self, m: np.ndarray, h: float, omega: float, pml: int,
                 n_layers: int, **opts):
        m = np.ascontiguousarray(m, dtype=np.float64)
        if m.ndim != 3:
            raise ValueError("m must be (nz, ny, nx)")
        nz, ny, nx = m.shape
        self.shape = (nz, ny, nx)
        self.n = (nx, ny, nz)
        self.N = nx * ny * nz
        self.h = h
        self.omega = omega
        self.n_layers = n_layers
        self.opts = options(**opts)
        self._grid = _lib.helm_grid(nx, ny, nz, h)
        self._h = ctypes.c_void_p()
        st = lib().helm_factorize(ctypes.byref(self._grid), m.ctypes.data, omega, pml,
                                  n_layers, ctypes.byref(self.opts), ctypes.byref(self._h))
        check(st, "helm_factorize")
        self.pml = pml

    # -- online stage ---------------------------------------------------------
    def solve(self, f, info: bool = False):
        """u for f: torch complex128 (k, nz, ny, nx) on the GPU, or NumPy."""
        import torch
        if isinstance(f, np.ndarray):
            fh = np.ascontiguousarray(f, dtype=np.complex128)
            k = fh.size // self.N
            uh = np.empty_like(fh)
            inf = _lib.helm_solve_info().attach(k)
            st = lib().helm_solve(self._h, k, fh.ctypes.data, uh.ctypes.data,
                                  ctypes.byref(inf))
            self._check_solve(st)
            return (uh, inf.as_dict()) if info else uh
        f = f.contiguous()
        if f.dtype != torch.complex128:
            raise TypeError("f must be complex128")
        k = f.numel() // self.N
        u = torch.empty_like(f)
        inf = _lib.helm_solve_info().attach(k)
        st = lib().helm_solve_dev(self._h, k, _ptr(f), _ptr(u), ctypes.byref(inf))
        self._check_solve(st)
        return (u, inf.as_dict()) if info else u

    def solve_points(self, nodes: Sequence, amplitudes=None, info: bool = False,
                     out=None):
        """Point sources at (i, j, k) nodes, amplitude/h^3 each (default 1)."""
        import torch
        nx, ny, nz = self.n
        idx = node_indices(nodes, self.n)
        r = len(idx)
        amp = np.ones(r, dtype=np.complex128) if amplitudes is None else \
            np.ascontiguousarray(amplitudes, dtype=np.complex128)
        u = out if out is not None else torch.empty((r, nz, ny, nx), dtype=torch.complex128,
                                                    device="cuda")
        inf = _lib.helm_solve_info().attach(r)
        st = lib().helm_solve_points(self._h, r, idx.ctypes.data, amp.ctypes.data, _ptr(u),
                                     ctypes.byref(inf))
        self._check_solve(st)
        return (u, inf.as_dict()) if info else u

    def _check_solve(self, st):
        if st == HELM_ENOCONV:
            return  # result returned with the info record; callers inspect it
        check(st, "helm_solve")

    # -- inspection entry points ---------------------------------------------
    def layer_info(self, l: int):
        v = [ctypes.c_int() for _ in range(4)]
        check(lib().helm_layer_info(self._h, l, *[ctypes.byref(x) for x in v]),
              "helm_layer_info")
        return tuple(x.value for x in v)

    def layer_solve(self, l: int, r):
        """(H^l)^-1 r for k local volumes r: torch complex128 (k, t, ny, nx)."""
        import torch
        r = r.contiguous()
        w = torch.empty_like(r)
        k = r.shape[0]
        check(lib().helm_layer_solve_dev(self._h, l, k, _ptr(r), _ptr(w)),
              "helm_layer_solve_dev")
        return w

    def layer_solve_noalloc(self, l: int, r, w=None):
        """Same as layer_solve through the allocation-free entry point (the
        output tensor may be passed in, so that nothing is allocated)."""
        import torch
        r = r.contiguous()
        if w is None:
            w = torch.empty_like(r)
        check(lib().helm_layer_solve_noalloc_dev(self._h, l, r.shape[0], _ptr(r), _ptr(w)),
              "helm_layer_solve_noalloc_dev")
        return w

    def apply_operator(self, u, f=None):
        """f - H u (or H u when f is None), FP64 on the GPU."""
        import torch
        u = u.contiguous()
        r = torch.empty_like(u)
        k = u.numel() // self.N
        check(lib().helm_apply_operator_dev(self._h, k, _ptr(f) if f is not None else None,
                                            _ptr(u), _ptr(r)), "helm_apply_operator_dev")
        return r

    def polarized_op(self, op: int, x, k: int):
        """Interface operators (see include/helm.h): 0 = P, 1 = P M, 2 = U,
        3 = polarized right-hand side of a volume source, 4 = P of it."""
        import torch
        nx, ny, _ = self.n
        vp = (self.n_layers - 1) * 2 * nx * ny * k
        size = vp if op == 2 else 2 * vp
        out = torch.empty(size, dtype=torch.complex128, device=x.device)
        check(lib().helm_polarized_op_dev(self._h, op, k, _ptr(x.contiguous()), _ptr(out)),
              "helm_polarized_op_dev")
        return out

    def set_options(self, **kw):
        """Change online-stage options (tolerances, steps, batch width, flags)."""
        for key, val in kw.items():
            if not hasattr(self.opts, key):
                raise TypeError(f"unknown option {key}")
            setattr(self.opts, key, val)
        check(lib().helm_set_solve_options(self._h, ctypes.byref(self.opts)),
              "helm_set_solve_options")

    def factor_info(self):
        """Offline-stage record: LU and executed flops, pivot range and growth."""
        fi = _lib.helm_factor_info()
        check(lib().helm_get_factor_info(self._h, ctypes.byref(fi)), "helm_get_factor_info")
        d = fi.as_dict()
        d["pivot_growth"] = d["pivot_max"] / d["diag_max"] if d["diag_max"] > 0 else None
        return d

    def kernel_stats(self, reset: bool = False):
        """Event-timed per-kernel-class statistics (needs flags=HELM_FLAG_PROFILE)."""
        arr = (_lib.helm_kernel_stat * 32)()
        cnt = ctypes.c_int()
        check(lib().helm_kernel_stats(self._h, arr, 32, ctypes.byref(cnt), int(reset)),
              "helm_kernel_stats")
        return {arr[i].name.decode(): {"launches": arr[i].launches,
                                       "total_ms": arr[i].total_ms,
                                       "flops": arr[i].flops, "bytes": arr[i].bytes}
                for i in range(cnt.value)}

    def tile_choices(self):
        """Column-tile widths of the substitution GEMMs per (layer set, k, depth)."""
        cnt = ctypes.c_int()
        check(lib().helm_tile_choices(self._h, None, 0, ctypes.byref(cnt)), "helm_tile_choices")
        arr = (_lib.helm_tile_choice * max(cnt.value, 1))()
        check(lib().helm_tile_choices(self._h, arr, cnt.value, ctypes.byref(cnt)),
              "helm_tile_choices")
        return [arr[i].as_dict() for i in range(cnt.value)]

    def close(self):
        if self._h:
            lib().helm_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
