"""FP64 CPU oracle for the short-range MD path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library and
its Python binding never import it, call it or link it; the two share no code.

Contents (each function cites the passage it follows):
  core       ctypes front end of the O(N^2) minimum-image C core (md_oracle.c):
             wrap, brute-force neighbour sets, Lennard-Jones, EAM (spline or
             analytic functions), sampled variants for large systems, pair lists.
  spline     uniform cubic B-spline: clamped interpolation fit and evaluation
             from the definition.
  integrate  velocity Verlet (kick-drift-kick) with the piston and top walls.
  thermostat Langevin velocity update per slab region (NVT), with the Philox4x32-10
             counter-based generator and Box-Muller normals it draws from.
  profiles   slab profiles of the Appendix (centre-of-mass velocity, temperature
             per axis, pressure tensor, potential and internal energy per mass).
  adjoint    force-matching loss and its exact gradient with respect to the
             spline coefficients, by the forward-mode chain rule.

Every function here is pinned by the CPU tests against closed forms,
invariants, library routines or brute force; see tests/test_oracle_*.py.
"""
from . import core, spline, integrate, adjoint, thermostat, profiles  # noqa: F401
