"""Plain definition of what the method computes: u = H^{-1} f (complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The polarized-traces solution is, by construction, the solution of the
discrete global problem H u = f (Eq. ``discrete_Helmholtz``): the SIE on the
interfaces is solved exactly by the restriction of that solution (Theorem 1
of the companion paper, cited in the SIE reduction section) and the
reconstruction inside each layer is exact (the same section, and the remark
that the discrete transmission conditions are algebraically exact).  So the
oracle of the whole method is a direct solve of the global sparse system.

Two independent routes are provided so that each pins the other on tiny
grids: a dense LAPACK solve and SuperLU on the sparse matrix.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def solve_dense(H, F: np.ndarray) -> np.ndarray:
    """numpy.linalg.solve on the densified matrix (N up to a few thousand)."""
    A = H.toarray()
    return np.linalg.solve(A, F)


class SparseLU:
    """SuperLU factorization of a sparse matrix, reusable for many RHS."""

    def __init__(self, H):
        self.lu = spla.splu(H.tocsc(), permc_spec="COLAMD")

    def solve(self, F: np.ndarray) -> np.ndarray:
        F = np.asarray(F, dtype=np.complex128)
        return self.lu.solve(F)


def solve(H, F: np.ndarray) -> np.ndarray:
    """u = H^{-1} F, dense below 4096 unknowns, SuperLU above."""
    if H.shape[0] <= 4096:
        return solve_dense(H, F)
    return SparseLU(H).solve(F)


def relative_error(u: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-column relative l2 error |u - ref|_2 / |ref|_2 over the full grid
    (PML included); a zero reference column gives |u|_2.  Pinned against
    hand-computed values (tests/test_oracle_pins.py)."""
    u = np.atleast_2d(u.T).T if u.ndim == 1 else u
    ref = np.atleast_2d(ref.T).T if ref.ndim == 1 else ref
    num = np.linalg.norm(u - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return num / np.where(den > 0, den, 1.0)
