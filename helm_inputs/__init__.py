"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds only what both sides take as *input*: grid descriptions,
squared-slowness models m = 1/c^2, angular frequencies chosen from a
points-per-wavelength target, and point-source positions.  It contains none
of the solver's arithmetic (no stencil, no PML, no layer split), so the
oracle and the HIP path stay independent of each other.

The workloads stand in for the paper's media (Section "Numerical
Experiments": homogeneous, smooth random, fault and SEAM models), whose
generators and data are not published; the recipes are stated in each
function's docstring.
"""

from .models import (
    Workload,
    omega_for_ppw,
    constant_model,
    smooth_random_model,
    layered_dipping_model,
    surface_grid_sources,
    workload,
    WORKLOADS,
    serving_models,
    poisson_requests,
    batched_problems,
    ServingRequest,
)

__all__ = [
    "Workload",
    "omega_for_ppw",
    "constant_model",
    "smooth_random_model",
    "layered_dipping_model",
    "surface_grid_sources",
    "workload",
    "WORKLOADS",
    "serving_models",
    "batched_problems",
    "poisson_requests",
    "ServingRequest",
]
