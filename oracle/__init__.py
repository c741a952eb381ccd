"""CPU oracle for the method of polarized traces (3D Helmholtz).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library (no kernels,
headers, tables or helpers); the only common module is ``helm_inputs``, which
holds seeded input generators and none of the method's arithmetic.

Everything here is plain NumPy/SciPy in complex128:

* ``discretization`` -- the PML-stretched 7-point operator H of the discrete
  global problem (Eq. ``discrete_Helmholtz``) and the local layer operators
  H^l (Eq. ``discrete_local_Helmholtz``), assembled as scipy sparse matrices;
* ``direct`` -- the plain definition of what the method computes, u = H^{-1} f
  (dense LAPACK solve for tiny grids, SuperLU otherwise);
* ``polarized`` -- the method itself on the CPU, step by step in the paper's
  order (Algorithms 1-10), with an unfused preconditioner and a textbook
  GMRES (or Bi-CGSTAB); used to pin intermediate operators (sweeps,
  reflections, traces); also the unpolarized SIE of Algorithms 2-3;
* ``gmres``, ``bicgstab`` -- textbook Krylov iterations.

Readings of silent or garbled passages are listed in the module docstrings
that use them.  Functions whose results are not pinned by an independent
check say "parity unpinned" in their docstring.
"""

from . import discretization, direct, polarized, gmres, bicgstab  # noqa: F401
