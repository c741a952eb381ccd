"""Textbook Bi-CGSTAB (van der Vorst, 1992) for the oracle's polarized system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names Bi-CGSTAB as the Krylov method to use when the memory of
GMRES's basis is the constraint (Section "Method of Polarized traces",
opening paragraph, and the memory remark of Section "Pipelining").  It gives
no details; the reading taken here is the unpreconditioned textbook
iteration applied to the already (left-)preconditioned system, x0 = 0, the
shadow residual r_hat = r0, and the stopping test of the GMRES reading:
|b - A x| <= tol |b| with b the preconditioned right-hand side.
"""

from __future__ import annotations

import numpy as np


def bicgstab(apply_A, b: np.ndarray, tol: float = 1e-10, maxiter: int = 200):
    """Solve A x = b.  Returns (x, iterations, residual history (relative)).
    One iteration applies A twice."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, 0, hist
    r = b.copy()
    r_hat = r.copy()
    rho_old = alpha = omega = 1.0 + 0.0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    it = 0
    while it < maxiter:
        rho = np.vdot(r_hat, r)
        if rho == 0:
            break
        beta = (rho / rho_old) * (alpha / omega) if it > 0 else 0.0
        p = r + beta * (p - omega * v) if it > 0 else r.copy()
        v = apply_A(p)
        alpha = rho / np.vdot(r_hat, v)
        s = r - alpha * v
        it += 1
        if np.linalg.norm(s) / bnorm <= tol:
            x = x + alpha * p
            hist.append(np.linalg.norm(s) / bnorm)
            break
        t = apply_A(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol or omega == 0:
            break
    return x, it, hist
