"""MI355X (gfx950) implicit M1 radiative-transfer multigrid solver.

The solver is the nonlinear FAS multigrid of Bloch, Tremblin, Gonzalez and Audit
(arXiv 2208.14703) for the implicit Euler M1 system with sources. It is written
as HIP kernels behind the C ABI of include/m1.h (libm1mg.so).

Modules:
  binding: ctypes access to the library (Plan, step, vcycle, residual, ...).
  build:   hipcc build of the library for gfx950.
  inputs:  seeded synthetic problem generators, shared with the tests.
"""
__all__ = ["binding", "build", "inputs"]
