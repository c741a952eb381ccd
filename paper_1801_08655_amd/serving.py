"""Binding of the request server (``include/helm_serve.h``).

Resident factorizations (``Solver`` objects) are added as models; requests
of point sources are submitted against a model and solved by the library's
lanes, which admit queued columns into free slots between refinement steps
(continuous batching) and run the lanes of different models concurrently.

    srv = Server(slots=32)
    m0 = srv.add_model(solver_a)
    req = srv.submit(m0, [(26, 26, 17), (47, 26, 17)])
    u, info = req.wait()
"""

from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np

from . import _lib
from ._lib import HELM_ENOCONV, HELM_OK, HelmError, check, lib
from . import node_indices


class Request:
    """A submitted request; ``wait()`` returns (u, info)."""

    def __init__(self, server, rid: int, u, n: int):
        self._server = server
        self.id = rid
        self.u = u            # kept alive until the library has written it
        self.n = n
        self._result = None

    def done(self) -> bool:
        if self._result is not None:
            return True
        d = ctypes.c_int()
        check(lib().helm_server_poll(self._server._s, self.id, ctypes.byref(d)),
              "helm_server_poll")
        return bool(d.value)

    def wait(self):
        if self._result is None:
            inf = _lib.helm_request_info()
            st = lib().helm_server_wait(self._server._s, self.id, ctypes.byref(inf))
            if st not in (HELM_OK, HELM_ENOCONV):
                raise HelmError(st, "helm_server_wait")
            self._result = (self.u, inf.as_dict())
        return self._result


class Server:
    def __init__(self, slots: int = 32, hbm_budget_bytes: int = 0, device: int = 0):
        o = _lib.helm_server_options()
        lib().helm_server_default_options(ctypes.byref(o))
        o.slots = slots
        o.hbm_budget_bytes = hbm_budget_bytes
        o.device = device
        self._s = ctypes.c_void_p()
        check(lib().helm_server_create(ctypes.byref(o), ctypes.byref(self._s)),
              "helm_server_create")
        self._models = []

    def add_model(self, solver) -> int:
        """Serve ``solver``'s factorization; returns the model id.  The solver
        must not be used otherwise until the server is closed."""
        mid, slots = ctypes.c_int(), ctypes.c_int()
        check(lib().helm_server_add_model(self._s, solver._h, ctypes.byref(mid),
                                          ctypes.byref(slots)), "helm_server_add_model")
        self._models.append((solver, slots.value))
        return mid.value

    def slots(self, model: int) -> int:
        return self._models[model][1]

    def submit(self, model: int, nodes: Sequence, amplitudes=None, out=None) -> Request:
        """Queue point sources at (i, j, k) nodes (amplitude/h^3 each, default 1);
        the result is a torch complex128 tensor (n, nz, ny, nx) on the GPU."""
        import torch
        if not 0 <= model < len(self._models):
            raise ValueError(f"unknown model {model}")
        solver = self._models[model][0]
        nx, ny, nz = solver.n
        idx = node_indices(nodes, solver.n)
        r = len(idx)
        amp = np.ones(r, dtype=np.complex128) if amplitudes is None else \
            np.ascontiguousarray(amplitudes, dtype=np.complex128)
        u = out if out is not None else torch.empty((r, nz, ny, nx), dtype=torch.complex128,
                                                    device="cuda")
        rid = ctypes.c_int64()
        check(lib().helm_server_submit(self._s, model, r, idx.ctypes.data, amp.ctypes.data,
                                       u.data_ptr() if r else None, ctypes.byref(rid)),
              "helm_server_submit")
        return Request(self, rid.value, u, r)

    def remove_model(self, model: int):
        """Wait for the model's queued columns, then release its lane."""
        check(lib().helm_server_remove_model(self._s, model), "helm_server_remove_model")

    def stats(self) -> dict:
        s = _lib.helm_server_summary()
        check(lib().helm_server_get_stats(self._s, ctypes.byref(s)), "helm_server_get_stats")
        return s.as_dict()

    def close(self):
        if self._s:
            lib().helm_server_free(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
