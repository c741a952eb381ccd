"""Discrete global and local Helmholtz operators (oracle side, complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is assembled, and where it comes from:

* Eq. ``Helmholtz``: Laplacian(u) + omega^2 m u = f, m = 1/c^2.
* Eq. ``extended_operator_PML`` and the stretching rule d/dx -> beta_x d/dx with
  beta = 1/(1 + i sigma/omega) (Eq. ``appendix:eq:def_alpha``) and the
  quadratic profile sigma = (C/delta)(d/delta)^2 inside the absorbing layer.
* Second-order 7-point finite differences on the grid x_ijk = (ih, jh, kh)
  (Section "Formulation"), giving H u = f (Eq. ``discrete_Helmholtz``).
* The layered decomposition in z with extra absorbing planes padded at every
  internal interface, and the local systems H^l v = f^l
  (Eqs. ``local_Helmholtz`` and ``discrete_local_Helmholtz``).

Readings of points the paper leaves open:

R1  h = 1/(n-1) for an n-node axis, nodes at i h; n counts the PML nodes.
R2  A face with p PML nodes has its profile origin at the half-node between
    the last PML node and the first interior node; delta = p h; sigma is
    sampled at nodes and at half-nodes (d = distance past the origin).
R3  Discrete stretched Laplacian in the complex-symmetric "divided" form:
    the stretched operator divided row-wise by beta_x(i) beta_y(j) beta_z(k),
      (H u)_ijk = h^-2 sum_axes [c_{+}(u_+ - u) - c_{-}(u - u_-)]
                  + omega^2 m_ijk u_ijk / (beta_x(i) beta_y(j) beta_z(k)),
    with c^x_{i+1/2,j,k} = beta_x(i+1/2) / (beta_y(j) beta_z(k)) and cyclically.
    H is exactly symmetric (not Hermitian).
R4  Homogeneous Dirichlet values one node beyond the last node.
R5  Layers split the interior planes as evenly as possible (the first
    (interior mod L) layers get one extra plane); the global top/bottom PML
    planes are attached to the first and last layer.
R6  A local absorbing layer of alpha planes is added on every internal
    side, with its origin at the half-node just outside the bulk planes and
    delta = alpha h, the same C as the global layer; inside the bulk range
    the global profile is kept.  The model is extended into the local layer
    by copying the nearest bulk plane.  With this choice every bulk row of
    H^l has exactly the coefficients of the matching row of H.
R7  The PML strength C is an input (the paper says only that it is tuned);
    the workloads use C = 20 c_max.
"""

from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# absorbing-layer profiles (Eq. appendix:eq:def_alpha and the sigma profile)
# ----------------------------------------------------------------------------

def sigma_quadratic(d: np.ndarray, delta: float, C: float) -> np.ndarray:
    """sigma(d) = (C/delta) (d/delta)^2 for d > 0, else 0 (d in length units)."""
    d = np.asarray(d, dtype=np.float64)
    if delta <= 0.0:
        return np.zeros_like(d)
    return np.where(d > 0.0, (C / delta) * (d / delta) ** 2, 0.0)


def beta_from_sigma(sigma: np.ndarray, omega: float) -> np.ndarray:
    """beta = 1 / (1 + i sigma / omega)."""
    return 1.0 / (1.0 + 1j * np.asarray(sigma) / omega)


def global_sigma(pos: np.ndarray, n: int, p: int, h: float, C: float) -> np.ndarray:
    """Global profile along one axis at positions ``pos`` (in units of h).

    Origins at half-nodes p - 1/2 and n - 1 - p + 1/2 (reading R2).
    """
    pos = np.asarray(pos, dtype=np.float64)
    if p == 0:
        return np.zeros_like(pos)
    left = (p - 0.5) - pos
    right = pos - (n - 1 - p + 0.5)
    d = np.maximum(np.maximum(left, right), 0.0) * h
    return sigma_quadratic(d, p * h, C)


def axis_beta(n: int, p: int, h: float, omega: float, C: float):
    """beta at the n nodes and at the n+1 half-nodes i - 1/2, i = 0..n."""
    nodes = np.arange(n, dtype=np.float64)
    halves = np.arange(n + 1, dtype=np.float64) - 0.5
    return (beta_from_sigma(global_sigma(nodes, n, p, h, C), omega),
            beta_from_sigma(global_sigma(halves, n, p, h, C), omega))


# ----------------------------------------------------------------------------
# layer decomposition in z (Section "Formulation", Fig. DDM_sketch_PML)
# ----------------------------------------------------------------------------

def layer_bounds(nz: int, p: int, n_layers: int) -> List[Tuple[int, int]]:
    """Bulk plane range [s_l, e_l] (inclusive) of each layer (reading R5)."""
    interior = nz - 2 * p
    if n_layers < 1 or interior < n_layers:
        raise ValueError("need at least one interior plane per layer")
    base, extra = divmod(interior, n_layers)
    bounds = []
    s = p
    for l in range(n_layers):
        size = base + (1 if l < extra else 0)
        bounds.append([s, s + size - 1])
        s += size
    bounds[0][0] = 0
    bounds[-1][1] = nz - 1
    return [tuple(b) for b in bounds]


def layer_extent(bounds, l: int, alpha: int) -> Tuple[int, int]:
    """First and last global plane of the extended layer l (bulk + local PML)."""
    s, e = bounds[l]
    lo = s - alpha if l > 0 else s
    hi = e + alpha if l < len(bounds) - 1 else e
    return lo, hi


def layer_sigma_z(pos: np.ndarray, nz: int, p: int, h: float, C: float,
                  bounds, l: int, alpha: int) -> np.ndarray:
    """z-profile of layer l at global positions ``pos`` (reading R6)."""
    pos = np.asarray(pos, dtype=np.float64)
    s, e = bounds[l]
    sig = global_sigma(pos, nz, p, h, C)
    if l > 0:
        d = ((s - 0.5) - pos) * h
        sig = np.where(pos < s - 0.5, sigma_quadratic(d, alpha * h, C), sig)
    if l < len(bounds) - 1:
        d = (pos - (e + 0.5)) * h
        sig = np.where(pos > e + 0.5, sigma_quadratic(d, alpha * h, C), sig)
    return sig


# ----------------------------------------------------------------------------
# assembly of the 7-point operator (reading R3, R4)
# ----------------------------------------------------------------------------

def assemble(m: np.ndarray, h: float, omega: float, bx, bxh, by, byh, bz, bzh):
    """Sparse H for model m[k, j, i]; unknown index i + nx (j + ny k).

    ``bx`` (nx,) holds beta_x at nodes, ``bxh`` (nx+1,) at half-nodes i-1/2;
    the same for y and z.
    """
    nz, ny, nx = m.shape
    bx = np.asarray(bx); by = np.asarray(by); bz = np.asarray(bz)
    bxh = np.asarray(bxh); byh = np.asarray(byh); bzh = np.asarray(bzh)
    # edge coefficients; cx[k, j, i] belongs to the half-node i - 1/2
    cx = bxh[None, None, :] / (by[None, :, None] * bz[:, None, None])
    cy = byh[None, :, None] / (bx[None, None, :] * bz[:, None, None])
    cz = bzh[:, None, None] / (bx[None, None, :] * by[None, :, None])
    inv_h2 = 1.0 / (h * h)
    diag = -(cx[:, :, :-1] + cx[:, :, 1:] + cy[:, :-1, :] + cy[:, 1:, :]
             + cz[:-1] + cz[1:]) * inv_h2
    diag = diag + omega * omega * m / (
        bx[None, None, :] * by[None, :, None] * bz[:, None, None])
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    # x couplings between (i, i+1): coefficient at half-node i + 1/2
    a = idx[:, :, :-1].ravel(); b = idx[:, :, 1:].ravel()
    v = (cx[:, :, 1:-1] * inv_h2).ravel()
    rows += [a, b]; cols += [b, a]; vals += [v, v]
    a = idx[:, :-1, :].ravel(); b = idx[:, 1:, :].ravel()
    v = (cy[:, 1:-1, :] * inv_h2).ravel()
    rows += [a, b]; cols += [b, a]; vals += [v, v]
    a = idx[:-1].ravel(); b = idx[1:].ravel()
    v = (cz[1:-1] * inv_h2).ravel()
    rows += [a, b]; cols += [b, a]; vals += [v, v]
    H = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    return H


@dataclasses.dataclass
class Problem:
    """Discrete global problem on an n_x x n_y x n_z grid including the PML."""

    m: np.ndarray          # (nz, ny, nx) squared slowness
    h: float
    omega: float
    pml: int
    C: float

    @property
    def shape(self):
        return self.m.shape

    @property
    def n(self):
        nz, ny, nx = self.m.shape
        return nx, ny, nz

    def betas(self):
        nx, ny, nz = self.n
        return (axis_beta(nx, self.pml, self.h, self.omega, self.C),
                axis_beta(ny, self.pml, self.h, self.omega, self.C),
                axis_beta(nz, self.pml, self.h, self.omega, self.C))

    def operator(self):
        """The global H of Eq. ``discrete_Helmholtz``."""
        (bx, bxh), (by, byh), (bz, bzh) = self.betas()
        return assemble(self.m, self.h, self.omega, bx, bxh, by, byh, bz, bzh)

    def interface_coupling(self) -> np.ndarray:
        """B(j, i) = 1/(h^2 beta_x(i) beta_y(j)): the z-coupling of two planes
        where beta_z = 1 (any interior interface), shape (ny, nx)."""
        (bx, _), (by, _), _ = self.betas()
        return 1.0 / (self.h * self.h * by[:, None] * bx[None, :])


@dataclasses.dataclass
class LayerGeometry:
    """Bulk and extended plane ranges of one layer of the decomposition."""

    index: int
    s: int       # first bulk plane (global index)
    e: int       # last bulk plane
    lo: int      # first plane of the extended layer
    hi: int      # last plane of the extended layer

    @property
    def nplanes(self):
        return self.hi - self.lo + 1

    def local(self, z: int) -> int:
        return z - self.lo


def layers(problem: Problem, n_layers: int, alpha: int) -> List[LayerGeometry]:
    nz = problem.n[2]
    bounds = layer_bounds(nz, problem.pml, n_layers)
    out = []
    for l in range(n_layers):
        lo, hi = layer_extent(bounds, l, alpha)
        out.append(LayerGeometry(l, bounds[l][0], bounds[l][1], lo, hi))
    return out


def local_operator(problem: Problem, n_layers: int, alpha: int, l: int):
    """H^l of Eq. ``discrete_local_Helmholtz`` on the extended layer l."""
    nx, ny, nz = problem.n
    bounds = layer_bounds(nz, problem.pml, n_layers)
    geo = layers(problem, n_layers, alpha)[l]
    planes = np.arange(geo.lo, geo.hi + 1)
    # model extended by copying the nearest bulk plane (reading R6)
    m_loc = problem.m[np.clip(planes, geo.s, geo.e)]
    halves = np.arange(geo.lo, geo.hi + 2) - 0.5
    bz = beta_from_sigma(layer_sigma_z(planes, nz, problem.pml, problem.h,
                                       problem.C, bounds, l, alpha), problem.omega)
    bzh = beta_from_sigma(layer_sigma_z(halves, nz, problem.pml, problem.h,
                                        problem.C, bounds, l, alpha), problem.omega)
    (bx, bxh), (by, byh), _ = problem.betas()
    return assemble(m_loc, problem.h, problem.omega, bx, bxh, by, byh, bz, bzh)


def point_source_rhs(shape_zyx, sources, h: float, amplitudes=None) -> np.ndarray:
    """Right-hand sides for point sources, one column per source.

    A unit point source is the discrete delta of amplitude 1/h^3 at a node
    (the normalisation of the plane delta in Section "Formulation").
    Returns an array (N, R) with unknowns ordered x fastest.
    """
    nz, ny, nx = shape_zyx
    F = np.zeros((nx * ny * nz, len(sources)), dtype=np.complex128)
    for r, (i, j, k) in enumerate(sources):
        amp = 1.0 if amplitudes is None else amplitudes[r]
        F[i + nx * (j + ny * k), r] = amp / h ** 3
    return F
