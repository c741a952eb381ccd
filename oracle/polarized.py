"""The method of polarized traces on the CPU, in the paper's order (complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 (offline): build each local H^l and factor it (SuperLU here).
Algorithm 2 (online): partition f, solve the local problems, form the
interface right-hand side, solve the (polarized, preconditioned) SIE with
GMRES, then reconstruct the volume with one more local solve per layer whose
source is f^l plus the interface measures.
Algorithms 4, 5 and 6 apply the preconditioner blocks (D_down)^-1,
(D_up)^-1 and L; Algorithms 7-10 apply the polarized matrix
[[D_down, U], [L, D_up]] (Eq. ``polarized_SIE``); P is the block
Gauss-Seidel inverse of Eq. ``preconditioner_GS``.

Notation (0-based): layers l = 0..L-1 own bulk planes [s_l, e_l];
interface j = 0..L-2 separates layers j and j+1 and carries the pair
u_j = (a_j, b_j) = (u(e_j), u(e_j + 1)), the paper's trace vector of Eq.
``traces_definition`` grouped by interface.  G^l = (H^l)^-1.

Readings of the paper taken here:

R8  Interface sources (the plane deltas of Section "Formulation" scaled to
    this discretisation): with B = 1/(h^2 beta_x beta_y) the z-coupling of H
    across an interior interface,
      J_top^l(a, b) = -B a on plane s_l,  +B b on plane s_l - 1,
      J_bot^l(a, b) = -B b on plane e_l,  +B a on plane e_l + 1.
    Then G^l (f^l + J_top^l(u_{l-1}) + J_bot^l(u_l)) equals the global
    solution on the bulk planes and vanishes on the local PML planes (the
    exact Green's representation that the online stage of Algorithm 2 uses to
    rebuild the volume).
R9  Read-outs R_top^l(w) = (w(s_l - 1), w(s_l)), R_bot^l(w) = (w(e_l), w(e_l + 1)).
R10 Blocks of the polarized matrix (the "algebraic operations and
    permutations" the paper defers to the 2D paper), for pair vectors x:
      (D_down x)_0 = -x_0,  (D_down x)_j = R_bot^j G^j J_top^j(x_{j-1}) - x_j
      (D_up x)_{L-2} = -x_{L-2},  (D_up x)_j = R_top^{j+1} G^{j+1} J_bot^{j+1}(x_{j+1}) - x_j
      (L x)_j = R_top^{j+1} G^{j+1} [J_top^{j+1}(x_j) + J_bot^{j+1}(x_{j+1}) [j+1 <= L-2]] - (0, x_{j,b})
      (U x)_j = R_bot^j G^j [J_top^j(x_{j-1}) [j >= 1] + J_bot^j(x_j)] - (x_{j,a}, 0)
    and right-hand side f_down_j = -R_bot^j G^j f^j, f_up_j = -R_top^{j+1} G^{j+1} f^{j+1}.
    Algorithms 4 and 5 are the block forward substitutions for D_down and
    D_up; Algorithm 6 is L (its step for the last layer reads the down-going
    input);
    Algorithm 10, a garbled copy of Algorithm 6, is read as U, the mirror
    image of L; Algorithms 8 and 9 are the forward operators D_down and D_up
    (their captions are swapped in the paper).
"""

from __future__ import annotations

from typing import List

import numpy as np

from .bicgstab import bicgstab
from .discretization import Problem, layers, local_operator
from .direct import SparseLU
from .gmres import gmres


class PolarizedTraces:
    """Offline stage (Algorithm 1) and the operators of the online stage."""

    def __init__(self, problem: Problem, n_layers: int, alpha: int):
        self.problem = problem
        self.L = n_layers
        self.alpha = alpha
        self.geo = layers(problem, n_layers, alpha)
        nx, ny, nz = problem.n
        self.nx, self.ny, self.nz = nx, ny, nz
        # Algorithm 1: build and factor every local system
        self.lu: List[SparseLU] = [
            SparseLU(local_operator(problem, n_layers, alpha, l))
            for l in range(n_layers)]
        self.B = problem.interface_coupling()            # (ny, nx)
        self.local_solves = 0

    # ------------------------------------------------------------------
    # local solves, sources and read-outs
    # ------------------------------------------------------------------
    def G(self, l: int, rhs: np.ndarray) -> np.ndarray:
        """w = (H^l)^-1 rhs for a local volume rhs of shape (planes, ny, nx)."""
        self.local_solves += 1
        w = self.lu[l].solve(rhs.reshape(-1))
        return w.reshape(rhs.shape)

    def zeros_local(self, l: int) -> np.ndarray:
        return np.zeros((self.geo[l].nplanes, self.ny, self.nx), np.complex128)

    def restrict_source(self, l: int, f: np.ndarray) -> np.ndarray:
        """f^l: f on the bulk planes of layer l, zero on the local PML."""
        g = self.geo[l]
        out = self.zeros_local(l)
        out[g.local(g.s):g.local(g.e) + 1] = f[g.s:g.e + 1]
        return out

    def add_J_top(self, l: int, vol: np.ndarray, pair) -> None:
        g = self.geo[l]
        a, b = pair
        vol[g.local(g.s)] += -self.B * a
        vol[g.local(g.s) - 1] += self.B * b

    def add_J_bot(self, l: int, vol: np.ndarray, pair) -> None:
        g = self.geo[l]
        a, b = pair
        vol[g.local(g.e)] += -self.B * b
        vol[g.local(g.e) + 1] += self.B * a

    def R_top(self, l: int, w: np.ndarray) -> np.ndarray:
        g = self.geo[l]
        return np.stack([w[g.local(g.s) - 1], w[g.local(g.s)]])

    def R_bot(self, l: int, w: np.ndarray) -> np.ndarray:
        g = self.geo[l]
        return np.stack([w[g.local(g.e)], w[g.local(g.e) + 1]])

    def traces_of(self, u: np.ndarray) -> np.ndarray:
        """Interface pairs (a_j, b_j) of a volume u[k, j, i]."""
        return np.stack([np.stack([u[g.e], u[g.e + 1]]) for g in self.geo[:-1]])

    def zero_pairs(self) -> np.ndarray:
        return np.zeros((self.L - 1, 2, self.ny, self.nx), np.complex128)

    # ------------------------------------------------------------------
    # forward blocks (Algorithms 6-10)
    # ------------------------------------------------------------------
    def D_down(self, x: np.ndarray) -> np.ndarray:
        """Forward operator D_down (Algorithm 8)."""
        y = self.zero_pairs()
        y[0] = -x[0]
        for j in range(1, self.L - 1):
            src = self.zeros_local(j)
            self.add_J_top(j, src, x[j - 1])
            y[j] = self.R_bot(j, self.G(j, src)) - x[j]
        return y

    def D_up(self, x: np.ndarray) -> np.ndarray:
        """Forward operator D_up (Algorithm 9)."""
        y = self.zero_pairs()
        y[-1] = -x[-1]
        for j in range(self.L - 3, -1, -1):
            src = self.zeros_local(j + 1)
            self.add_J_bot(j + 1, src, x[j + 1])
            y[j] = self.R_top(j + 1, self.G(j + 1, src)) - x[j]
        return y

    def L_op(self, x: np.ndarray) -> np.ndarray:
        """Up-going reflections L (Algorithm 6)."""
        y = self.zero_pairs()
        for j in range(self.L - 1):
            src = self.zeros_local(j + 1)
            self.add_J_top(j + 1, src, x[j])
            if j + 1 <= self.L - 2:
                self.add_J_bot(j + 1, src, x[j + 1])
            w = self.G(j + 1, src)
            y[j] = self.R_top(j + 1, w)
            y[j][1] -= x[j][1]
        return y

    def U_op(self, x: np.ndarray) -> np.ndarray:
        """Down-going reflections U (Algorithm 10, read as the mirror of L)."""
        y = self.zero_pairs()
        for j in range(self.L - 1):
            src = self.zeros_local(j)
            if j >= 1:
                self.add_J_top(j, src, x[j - 1])
            self.add_J_bot(j, src, x[j])
            w = self.G(j, src)
            y[j] = self.R_bot(j, w)
            y[j][0] -= x[j][0]
        return y

    def apply_M(self, xd: np.ndarray, xu: np.ndarray):
        """Polarized matrix (Algorithm 7): (D_down xd + U xu, L xd + D_up xu)."""
        return (self.D_down(xd) + self.U_op(xu), self.L_op(xd) + self.D_up(xu))

    # ------------------------------------------------------------------
    # preconditioner (Algorithms 4 and 5, Eq. preconditioner_GS)
    # ------------------------------------------------------------------
    def sweep_down(self, v: np.ndarray) -> np.ndarray:
        """(D_down)^-1 v by block forward substitution (Algorithm 4)."""
        u = self.zero_pairs()
        u[0] = -v[0]
        for j in range(1, self.L - 1):
            src = self.zeros_local(j)
            self.add_J_top(j, src, u[j - 1])
            u[j] = self.R_bot(j, self.G(j, src)) - v[j]
        return u

    def sweep_up(self, v: np.ndarray) -> np.ndarray:
        """(D_up)^-1 v by block backward substitution (Algorithm 5)."""
        u = self.zero_pairs()
        u[-1] = -v[-1]
        for j in range(self.L - 3, -1, -1):
            src = self.zeros_local(j + 1)
            self.add_J_bot(j + 1, src, u[j + 1])
            u[j] = self.R_top(j + 1, self.G(j + 1, src)) - v[j]
        return u

    def precondition(self, vd: np.ndarray, vu: np.ndarray):
        """P (vd, vu) = (D_down^-1 vd, D_up^-1 (vu - L D_down^-1 vd))."""
        yd = self.sweep_down(vd)
        yu = self.sweep_up(vu - self.L_op(yd))
        return yd, yu

    # ------------------------------------------------------------------
    # online stage (Algorithm 2)
    # ------------------------------------------------------------------
    def polarized_rhs(self, f: np.ndarray):
        """Local solves of the partitioned source and the polarized RHS."""
        fd = self.zero_pairs()
        fu = self.zero_pairs()
        for l in range(self.L):
            v = self.G(l, self.restrict_source(l, f))
            if l <= self.L - 2:
                fd[l] = -self.R_bot(l, v)
            if l >= 1:
                fu[l - 1] = -self.R_top(l, v)
        return fd, fu

    def reconstruct(self, f: np.ndarray, traces: np.ndarray) -> np.ndarray:
        """Volume from interface traces (the reconstruction step of Algorithm 2)."""
        u = np.zeros_like(f)
        for l, g in enumerate(self.geo):
            src = self.restrict_source(l, f)
            if l >= 1:
                self.add_J_top(l, src, traces[l - 1])
            if l <= self.L - 2:
                self.add_J_bot(l, src, traces[l])
            w = self.G(l, src)
            u[g.s:g.e + 1] = w[g.local(g.s):g.local(g.e) + 1]
        return u

    def solve(self, f: np.ndarray, tol: float = 1e-10, restart: int = 60,
              maxiter: int = 200, krylov: str = "gmres"):
        """u for the volume source f[k, j, i]; returns (u, iterations, history).
        krylov: "gmres" (Eq. precond_polarized_SIE solved by GMRES, as in the
        experiments) or "bicgstab" (the memory-lean alternative the paper
        names); both on the same left-preconditioned polarized system."""
        f = np.asarray(f, dtype=np.complex128)
        if self.L == 1:
            return self.G(0, f.copy()), 0, [0.0]
        fd, fu = self.polarized_rhs(f)
        shape = fd.shape
        n = fd.size

        def split(x):
            return x[:n].reshape(shape), x[n:].reshape(shape)

        def PM(x):
            xd, xu = split(x)
            md, mu = self.apply_M(xd, xu)
            pd, pu = self.precondition(md, mu)
            return np.concatenate([pd.ravel(), pu.ravel()])

        pd, pu = self.precondition(fd, fu)
        b = np.concatenate([pd.ravel(), pu.ravel()])
        if krylov == "bicgstab":
            x, iters, hist = bicgstab(PM, b, tol=tol, maxiter=maxiter)
        else:
            x, iters, hist = gmres(PM, b, tol=tol, restart=restart, maxiter=maxiter)
        ud, uu = split(x)
        traces = ud + uu
        return self.reconstruct(f, traces), iters, hist

    # ------------------------------------------------------------------
    # the unpolarized surface integral equation (Eq. SIE, Algorithms 2-3)
    # ------------------------------------------------------------------
    # Reading (G12, G13): the Green's representation restricted to the
    # layer's own interface planes gives, for the exact traces u,
    #   a_j = [G^j (f^j + J_top^j(u_{j-1}) + J_bot^j(u_j))](e_j),
    #   b_j = [G^{j+1} (f^{j+1} + J_top^{j+1}(u_j) + J_bot^{j+1}(u_{j+1}))](s_{j+1}),
    # i.e. (I - GJ) u = v with v_j = ([G^j f^j](e_j), [G^{j+1} f^{j+1}](s_{j+1})).
    # Algorithm 3 applies GJ - I and Algorithm 2 pairs it with +v, which is
    # inconsistent in sign; the consistent system (I - GJ) u = v is solved.
    # The index typos of Algorithm 3 (layer 1's planes) are read as the
    # layer's own first and last bulk planes.
    def sie_rhs(self, f: np.ndarray) -> np.ndarray:
        """v of the unpolarized SIE: local solves of the partitioned source read
        on each layer's own interface planes (lines 2-8 of Algorithm 2)."""
        v = self.zero_pairs()
        for l, g in enumerate(self.geo):
            w = self.G(l, self.restrict_source(l, f))
            if l <= self.L - 2:
                v[l][0] = w[g.local(g.e)]
            if l >= 1:
                v[l - 1][1] = w[g.local(g.s)]
        return v

    def apply_sie(self, x: np.ndarray) -> np.ndarray:
        """(I - GJ) x: every layer solves its two interface sources (all layers
        independent, Algorithm 3) and is read on its own interface planes."""
        y = x.copy()
        for l, g in enumerate(self.geo):
            src = self.zeros_local(l)
            if l >= 1:
                self.add_J_top(l, src, x[l - 1])
            if l <= self.L - 2:
                self.add_J_bot(l, src, x[l])
            w = self.G(l, src)
            if l <= self.L - 2:
                y[l][0] -= w[g.local(g.e)]
            if l >= 1:
                y[l - 1][1] -= w[g.local(g.s)]
        return y

    def solve_unpolarized(self, f: np.ndarray, tol: float = 1e-10, restart: int = 60,
                          maxiter: int = 400):
        """u by GMRES on the unpolarized SIE (no preconditioner), then the
        reconstruction of Algorithm 2; returns (u, iterations, history)."""
        f = np.asarray(f, dtype=np.complex128)
        if self.L == 1:
            return self.G(0, f.copy()), 0, [0.0]
        v = self.sie_rhs(f)
        shape = v.shape

        def A(x):
            return self.apply_sie(x.reshape(shape)).ravel()

        x, iters, hist = gmres(A, v.ravel(), tol=tol, restart=restart, maxiter=maxiter)
        return self.reconstruct(f, x.reshape(shape)), iters, hist
