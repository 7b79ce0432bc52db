"""CPU oracle for the linear solve inside a semi-smooth Newton step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64
numpy/scipy statement of what the GPU path computes, written from the
paper (Jodlbauer, Langer, Wick, "Parallel matrix-free higher-order finite
element solvers for phase-field fracture problems").  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it.
It shares no code with the HIP library: it assembles sparse matrices
from element matrices built with full (not sum-factorised) tensor-product
basis tables, and runs the multigrid and Krylov algorithms on them.

Modules
  fe          1D tables, quadrature, mesh numbering, tensor-product basis
  material    degradation function, the volumetric/deviatoric split and the spectral split
  operator    residual, Jacobian assembly, constraints, diagonal, VJPs
  multigrid   levels, injection, transfers, Lanczos, Chebyshev, V-cycle
  krylov      flexible GMRES with classical Gram-Schmidt twice
  newton      active-set rule and one Newton step
  splitmix    the SplitMix64 counter generator used for start vectors
"""
