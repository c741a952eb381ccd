"""Writes the stored expected values under tests/golden from the oracle alone.

    python tests/golden/make_golden.py

field_homogeneous-25.txt: the oracle's global direct solve (SuperLU on its
own assembly of H, complex128) of the constant-velocity problem with a
6-point PML, h = 1/24, 10 points per wavelength and one unit point source at
the centre (the plain-method configuration of the paper's homogeneous
experiment, shrunk to 25^3), sampled at fixed nodes.

field_layered-28.txt: the same for the reduced layered-dipping model with
two point sources.

Nothing here reads the HIP library; the tests compare both the oracle (to
catch drift in its arithmetic) and the GPU path with these values.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from helm_inputs import workload  # noqa: E402
from oracle.direct import SparseLU  # noqa: E402
from oracle.discretization import Problem, point_source_rhs  # noqa: E402

CASES = {
    "homogeneous-25": {
        "sources": None,   # the workload's own (the centre node)
        "nodes": [(12, 12, 12), (12, 12, 14), (15, 12, 12), (12, 17, 12), (8, 8, 8),
                  (20, 5, 11), (3, 3, 3), (12, 12, 22), (0, 12, 12), (24, 24, 24)],
    },
    "layered-28": {
        "sources": [(8, 9, 6), (14, 14, 9)],
        "nodes": [(8, 9, 6), (14, 14, 9), (8, 9, 10), (20, 20, 20), (6, 21, 13),
                  (14, 3, 24), (27, 0, 0), (13, 13, 13)],
    },
}


def solve(name):
    wl = workload(name)
    srcs = CASES[name]["sources"] or wl.sources
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    U = SparseLU(pb.operator()).solve(point_source_rhs(pb.shape, srcs, wl.h))
    return wl, srcs, U


def write(name):
    wl, srcs, U = solve(name)
    nx, ny, _ = wl.n
    path = os.path.join(HERE, f"field_{name}.txt")
    with open(path, "w") as fh:
        fh.write(f"# oracle global direct solve of the {name} workload "
                 f"({wl.description}); written by tests/golden/make_golden.py\n")
        fh.write("# sources (i j k): " + "; ".join(" ".join(map(str, s)) for s in srcs) + "\n")
        fh.write("# column i j k re im\n")
        for c in range(len(srcs)):
            for (i, j, k) in CASES[name]["nodes"]:
                v = U[i + nx * (j + ny * k), c]
                fh.write(f"{c} {i} {j} {k} {v.real:.17e} {v.imag:.17e}\n")
    print("wrote", path)


def read(name):
    """(sources, [(column, i, j, k, value)]) of a stored fixture."""
    rows, srcs = [], None
    with open(os.path.join(HERE, f"field_{name}.txt")) as fh:
        for line in fh:
            if line.startswith("# sources"):
                srcs = [tuple(int(x) for x in s.split()) for s in
                        line.split(":", 1)[1].split(";")]
            if line.startswith("#") or not line.strip():
                continue
            c, i, j, k, re, im = line.split()
            rows.append((int(c), int(i), int(j), int(k), complex(float(re), float(im))))
    return srcs, rows


if __name__ == "__main__":
    for name in CASES:
        write(name)
