"""Textbook GMRES (Saad & Schultz) for the oracle's polarized system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves the preconditioned polarized SIE (Eq.
``precond_polarized_SIE``) with GMRES and stops when the residual has been
reduced by a given factor (Section "Numerical Experiments").  Reading taken
for the unstated details: left preconditioning as written, x0 = 0, modified
Gram-Schmidt Arnoldi, Givens rotations, stop when the preconditioned residual
norm |P(f - M x)| <= tol |P f|, restart length ``restart``.
"""

from __future__ import annotations

import numpy as np


def gmres(apply_A, b: np.ndarray, tol: float = 1e-10, restart: int = 50,
          maxiter: int = 200):
    """Solve A x = b.  Returns (x, iterations, residual history (relative))."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, 0, hist
    total = 0
    while total < maxiter:
        r = b - apply_A(x) if total > 0 else b.copy()
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        m = min(restart, maxiter - total)
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        Hh = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for j in range(m):
            w = apply_A(V[j])
            for i in range(j + 1):                     # modified Gram-Schmidt
                Hh[i, j] = np.vdot(V[i], w)
                w = w - Hh[i, j] * V[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] != 0:
                V[j + 1] = w / Hh[j + 1, j]
            for i in range(j):                         # previous rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -np.conj(sn[i]) * Hh[i, j] + np.conj(cs[i]) * Hh[i + 1, j]
                Hh[i, j] = t
            a, bb = Hh[j, j], Hh[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = a / den
                sn[j] = bb / den
            # rotation [c s; -conj(s) conj(c)] applied with c = a/den, s = b/den
            cs[j], sn[j] = np.conj(cs[j]), np.conj(sn[j])
            Hh[j, j] = cs[j] * a + sn[j] * bb
            Hh[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k_done = j + 1
            total += 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or total >= maxiter:
                break
        y = np.linalg.solve(np.triu(Hh[:k_done, :k_done]), g[:k_done])
        x = x + V[:k_done].T @ y
        if hist[-1] <= tol:
            break
    return x, total, hist
