"""Velocity models, frequencies and sources for the synthetic workloads.

Conventions (shared by both sides, stated once here):

* grid of n_x * n_y * n_z nodes *including* the absorbing layer, spacing
  h = 1/(n-1) for a cube, node (i, j, k) at (i h, j h, k h);
* arrays are stored with x fastest, then y, then z (plane-major), i.e.
  ``m[k, j, i]`` in C order;
* ``m`` is the squared slowness 1/c^2 in float64.
"""

from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Callable, Dict, List, Tuple

import numpy as np


def omega_for_ppw(c_min: float, h: float, ppw: float) -> float:
    """Angular frequency giving ``ppw`` grid points per wavelength at c_min.

    wavelength = 2 pi c / omega, and ppw = wavelength / h.
    """
    return 2.0 * math.pi * c_min / (ppw * h)


def constant_model(n: Tuple[int, int, int], c: float = 1.0) -> np.ndarray:
    nx, ny, nz = n
    return np.full((nz, ny, nx), 1.0 / (c * c), dtype=np.float64)


def _smooth_noise(shape_zyx, sigma: float, seed: int) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape_zyx)
    sm = gaussian_filter(noise, sigma=sigma, mode="reflect")
    sm -= sm.mean()
    sd = sm.std()
    if sd > 0:
        sm /= sd
    return sm


def smooth_random_model(n, amplitude: float, sigma: float, cmin: float,
                        cmax: float, seed: int) -> np.ndarray:
    """c = clip(1 + amplitude * N, cmin, cmax), N = normalised smoothed noise.

    N is standard normal noise from ``numpy.random.default_rng(seed)`` on the
    full grid, Gaussian-smoothed with standard deviation ``sigma`` grid points
    (reflecting edges), then shifted and scaled to zero mean and unit std.
    Stands in for the paper's smooth random medium.
    """
    nx, ny, nz = n
    noise = _smooth_noise((nz, ny, nx), sigma, seed)
    c = np.clip(1.0 + amplitude * noise, cmin, cmax)
    return 1.0 / (c * c)


def layered_dipping_model(n, h: float, n_interfaces: int, seed: int,
                          pml: int, cmin: float = 1.5,
                          cmax: float = 4.5) -> np.ndarray:
    """Layered model with dipping planar interfaces and linear gradients.

    Stands in for the paper's fault and SEAM media.  ``n_interfaces`` planes
    z = z_i + tan(theta_i) ((x - x_c) cos(phi_i) + (y - y_c) sin(phi_i)), with
    theta_i ~ U(0, 20 deg), phi_i ~ U(0, 2 pi) and z_i sorted uniform over the
    interior depth range.  A point's layer index q is the number of interfaces
    above it.  In layer q >= 1 the velocity is c_q + g_q * (depth below
    interface q), c_q = 1.5 + 3 q / n_interfaces + U(-0.1, 0.1),
    g_q ~ U(0, 3) per unit depth; the top layer is forced to c = cmin.
    The result is clipped to [cmin, cmax].
    """
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    theta = np.deg2rad(rng.uniform(0.0, 20.0, n_interfaces))
    phi = rng.uniform(0.0, 2.0 * math.pi, n_interfaces)
    z_top = pml * h
    z_bot = (nz - 1 - pml) * h
    z0 = np.sort(rng.uniform(z_top, z_bot, n_interfaces))
    cq = 1.5 + 3.0 * np.arange(n_interfaces + 1) / n_interfaces \
        + rng.uniform(-0.1, 0.1, n_interfaces + 1)
    gq = rng.uniform(0.0, 3.0, n_interfaces + 1)
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    z = np.arange(nz) * h
    xc = 0.5 * (nx - 1) * h
    yc = 0.5 * (ny - 1) * h
    X, Y = np.meshgrid(x, y, indexing="xy")        # (ny, nx)
    # interface depth surfaces, shape (n_interfaces, ny, nx)
    surf = z0[:, None, None] + np.tan(theta)[:, None, None] * (
        (X[None] - xc) * np.cos(phi)[:, None, None]
        + (Y[None] - yc) * np.sin(phi)[:, None, None])
    c = np.empty((nz, ny, nx), dtype=np.float64)
    for k in range(nz):
        above = (surf <= z[k])                      # interfaces above point
        q = above.sum(axis=0)                       # (ny, nx)
        # depth below interface q (the deepest one above the point)
        idx = np.clip(q - 1, 0, n_interfaces - 1)
        depth = z[k] - np.take_along_axis(surf, idx[None], axis=0)[0]
        ck = cq[q] + gq[q] * np.maximum(depth, 0.0)
        ck = np.where(q == 0, cmin, ck)
        c[k] = ck
    c = np.clip(c, cmin, cmax)
    return 1.0 / (c * c)


def surface_grid_sources(n_side: int, lo: int, width: int,
                         depth: int) -> List[Tuple[int, int, int]]:
    """n_side x n_side point sources at plane ``depth``.

    x, y in {lo + round(width (k + 1/2) / n_side)}.
    """
    coords = [lo + int(round(width * (k + 0.5) / n_side)) for k in range(n_side)]
    return [(ix, iy, depth) for iy in coords for ix in coords]


@dataclasses.dataclass
class Workload:
    """A synthetic problem: grid, model, frequency, layers and sources."""

    name: str
    n: Tuple[int, int, int]
    h: float
    pml: int                       # global PML nodes per face
    n_layers: int
    pml_local: int                 # local PML planes per internal interface
    ppw: float
    c_min: float
    c_max: float
    model: Callable[[], np.ndarray]
    sources: List[Tuple[int, int, int]]
    gmres_tol: float = 1e-10
    description: str = ""

    @property
    def omega(self) -> float:
        return omega_for_ppw(self.c_min, self.h, self.ppw)

    @property
    def pml_C(self) -> float:
        """PML strength: 20 c_max (normal-incidence round trip ~ exp(-13))."""
        return 20.0 * self.c_max

    def m(self) -> np.ndarray:
        return self.model()

    def point_sources(self, count=None):
        src = self.sources if count is None else self.sources[:count]
        return list(src)


def _cube(n):
    return (n, n, n), 1.0 / (n - 1)


def _wl_homog(n=25, pml=6, L=3, alpha=6, name="homogeneous-25"):
    dims, h = _cube(n)
    c = n // 2
    return Workload(
        name=name, n=dims, h=h, pml=pml, n_layers=L, pml_local=alpha,
        ppw=10.0, c_min=1.0, c_max=1.0,
        model=lambda: constant_model(dims, 1.0),
        sources=[(c, c, c)],
        description=f"{n}^3 incl. {pml}-pt PML, c=1, 10 ppw, L={L}, "
                    "one point source at the centre")


def _wl_smooth(n=100, pml=10, L=10, alpha=4, seed=1802, sigma=8.0,
               src_depth=15, name="smooth-100"):
    dims, h = _cube(n)
    return Workload(
        name=name, n=dims, h=h, pml=pml, n_layers=L, pml_local=alpha,
        ppw=10.0, c_min=0.75, c_max=1.25,
        model=lambda: smooth_random_model(dims, 0.25, sigma, 0.75, 1.25, seed),
        sources=[(n // 2, n // 2, src_depth)],
        description=f"{n}^3 incl. {pml}-pt PML, c = clip(1 + 0.25 N_sigma={sigma}, "
                    f"0.75, 1.25), seed {seed}, 10 ppw at c_min, L={L}")


def _wl_layered(n=200, pml=15, L=20, alpha=4, seed=1803, n_side=8,
                depth=16, ppw=8.0, name="layered-200"):
    dims, h = _cube(n)
    interior = n - 2 * pml
    return Workload(
        name=name, n=dims, h=h, pml=pml, n_layers=L, pml_local=alpha,
        ppw=ppw, c_min=1.5, c_max=4.5,
        model=lambda: layered_dipping_model(dims, h, 12, seed, pml),
        sources=surface_grid_sources(n_side, pml, interior, depth),
        description=f"{n}^3 incl. {pml}-pt PML, 12 dipping interfaces, "
                    f"c in [1.5, 4.5], seed {seed}, {ppw:g} ppw at c_min, L={L}, "
                    f"{n_side * n_side} sources on a surface grid at depth {depth}")


WORKLOADS: Dict[str, Callable[[], Workload]] = {
    # plain method, complex128, 25^3 with 6-point PML, L = 3
    "homogeneous-25": lambda: _wl_homog(),
    # plain method on the GPU, complex128, 100^3, L = 10
    "smooth-100": lambda: _wl_smooth(),
    # mixed precision headline workload, 200^3, L = 20, 64 sources
    "layered-200": lambda: _wl_layered(),
    # reduced versions of the same recipes, small enough for the oracle's
    # global direct solve (parity cases)
    "smooth-24": lambda: _wl_smooth(n=24, pml=5, L=4, alpha=4, sigma=3.0,
                                     src_depth=7, name="smooth-24"),
    "layered-28": lambda: _wl_layered(n=28, pml=5, L=4, alpha=3, n_side=2,
                                       depth=6, ppw=8.0, name="layered-28"),
    # the headline recipe shrunk until the oracle's direct solve takes seconds
    "layered-32": lambda: _wl_layered(n=32, pml=5, L=4, alpha=3, n_side=8,
                                       depth=6, ppw=8.0, name="layered-32"),
    # the largest grids the oracle's direct solve handles in about half a
    # minute, with many thin layers (L = 8: 3 or 4 interior planes each) and
    # with the smooth recipe at L = 4
    "layered-40": lambda: _wl_layered(n=40, pml=5, L=8, alpha=3, n_side=2,
                                       depth=6, ppw=8.0, name="layered-40"),
    "smooth-40": lambda: _wl_smooth(n=40, pml=5, L=4, alpha=4, sigma=3.0,
                                     src_depth=9, name="smooth-40"),
}


def serving_models(n: int = 160, pml: int = 16, L: int = 16, alpha: int = 4,
                   seed: int = 1805, ppws=(6.0, 8.0, 10.0)) -> List[Workload]:
    """Resident models of the serving workload: one layered-dipping medium
    (seed 1805) at three frequencies (6, 8 and 10 points per wavelength at
    c_min).  The candidate sources are a 16 x 16 surface grid at depth
    pml + 1."""
    out = []
    for ppw in ppws:
        w = _wl_layered(n=n, pml=pml, L=L, alpha=alpha, seed=seed, n_side=16,
                        depth=pml + 1, ppw=ppw, name=f"layered-{n}-ppw{ppw:g}")
        out.append(w)
    return out


@dataclasses.dataclass
class ServingRequest:
    t: float                       # arrival time [s] from the start
    model: int
    sources: List[Tuple[int, int, int]]


def poisson_requests(count: int, rate: float, n_models: int, candidates,
                     max_sources: int = 128, seed: int = 1806) -> List[ServingRequest]:
    """``count`` requests with exponential inter-arrival times of mean
    1/rate, a uniformly random model, and R ~ U{1..max_sources} sources drawn
    without replacement from ``candidates``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        model = int(rng.integers(0, n_models))
        r = int(rng.integers(1, min(max_sources, len(candidates)) + 1))
        pick = rng.choice(len(candidates), size=r, replace=False)
        out.append(ServingRequest(t, model, [tuple(candidates[i]) for i in pick]))
    return out


def batched_problems(count: int = 32, seed: int = 1804, n_lo: int = 64, n_hi: int = 160,
                     pml: int = 8, alpha: int = 4, max_sources: int = 256) -> List[Workload]:
    """Independent problems of the batched workload: n ~ U{n_lo..n_hi} per
    cube, c = clip(1 + 0.2 N, 0.8, 1.2) with N smoothed normalised noise
    (sigma 6 points, its own seed per problem), 10 points per wavelength at
    c_min = 0.8, L = round(n / 10) layers, and R ~ U{1..max_sources} point
    sources drawn without replacement from a 16 x 16 surface grid at depth
    pml + 1.  All draws come from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        mseed = int(rng.integers(0, 2**31 - 1))
        dims, h = _cube(n)
        L = max(1, int(round(n / 10)))
        grid = surface_grid_sources(16, pml, n - 2 * pml, pml + 1)
        r = int(rng.integers(1, min(max_sources, len(grid)) + 1))
        pick = rng.choice(len(grid), size=r, replace=False)
        srcs = [grid[j] for j in sorted(pick)]
        out.append(Workload(
            name=f"batch-{i}-n{n}", n=dims, h=h, pml=pml, n_layers=L, pml_local=alpha,
            ppw=10.0, c_min=0.8, c_max=1.2,
            model=(lambda d=dims, s_=mseed: smooth_random_model(d, 0.2, 6.0, 0.8, 1.2, s_)),
            sources=srcs,
            description=f"{n}^3 incl. {pml}-pt PML, smooth random c in [0.8, 1.2], "
                        f"10 ppw, L={L}, R={r}"))
    return out


def workload(name: str) -> Workload:
    return WORKLOADS[name]()


def checksum(a: np.ndarray) -> str:
    """Short content hash recorded next to results (inputs are reproducible)."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]
