"""Binding of the batched solve of independent problems (``include/helm_batch.h``).

    results, summary = solve_batch([
        Problem(m, h, omega, pml, n_layers, sources),    # one grid each
        ...], slots=64)
    u0, info0 = results[0]
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import _lib, node_indices, options
from ._lib import HELM_ENOCONV, HELM_ENOMEM, HELM_OK, HelmError, lib


@dataclasses.dataclass
class Problem:
    m: np.ndarray              # (nz, ny, nx) squared slowness
    h: float
    omega: float
    pml: int
    n_layers: int
    sources: Sequence          # (i, j, k) nodes
    amplitudes: Optional[Sequence] = None


def solve_batch(problems: List[Problem], slots: int = 64, hbm_budget_bytes: int = 0,
                max_resident: int = 0, host_output: bool = False, **kw):
    """Solve every problem; returns ([(u, info)], summary).  u is a torch
    complex128 tensor (R, nz, ny, nx) on the GPU, or a NumPy array in host
    memory with host_output=True (None for a failed problem); solver options
    (precision, tolerances, flags, pml_local, pml_C ...) are shared by all
    problems."""
    import torch
    bo = _lib.helm_batch_options()
    lib().helm_batch_default_options(ctypes.byref(bo))
    bo.opt = options(**kw)
    bo.slots = slots
    bo.hbm_budget_bytes = hbm_budget_bytes
    bo.max_resident = max_resident
    n = len(problems)
    arr = (_lib.helm_problem * max(n, 1))()
    keep = []
    outs = []
    for i, p in enumerate(problems):
        m = np.ascontiguousarray(p.m, dtype=np.float64)
        nz, ny, nx = m.shape
        idx = node_indices(p.sources, (nx, ny, nz))
        r = len(idx)
        amp = np.ones(r, dtype=np.complex128) if p.amplitudes is None else \
            np.ascontiguousarray(p.amplitudes, dtype=np.complex128)
        if host_output:
            u = np.empty((r, nz, ny, nx), dtype=np.complex128)
            uptr = u.ctypes.data
        else:
            u = torch.empty((r, nz, ny, nx), dtype=torch.complex128, device="cuda")
            uptr = u.data_ptr()
        keep += [m, idx, amp]
        outs.append(u)
        arr[i] = _lib.helm_problem(_lib.helm_grid(nx, ny, nz, p.h), m.ctypes.data, p.omega,
                                   p.pml, p.n_layers, r, idx.ctypes.data if r else None,
                                   amp.ctypes.data if r else None, uptr if r else None)
    infos = (_lib.helm_problem_info * max(n, 1))()
    summ = _lib.helm_batch_summary()
    st = lib().helm_solve_batch(n, arr, ctypes.byref(bo), infos, ctypes.byref(summ))
    if st == _lib.HELM_EINVAL and not any(infos[i].t_admit_ms for i in range(n)):
        raise HelmError(st, "helm_solve_batch")
    results = []
    for i in range(n):
        d = infos[i].as_dict()
        ok = d["status"] in (HELM_OK, HELM_ENOCONV)
        results.append((outs[i] if ok else None, d))
    return results, summ.as_dict()
