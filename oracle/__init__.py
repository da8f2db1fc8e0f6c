"""FP64 CPU oracle for multilevel CC2 / CCSD on Cholesky-factored integrals.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library and is deliberately plain and slow: NumPy in float64 (complex128 where
a derivative is taken by complex step), every step written as the equation it
follows, with the contraction order left to ``numpy.einsum``.

Modules
  mlcc        residual, energy, ground state, Jacobian transform (complex step),
              dense eigenvalues and a full-space Davidson
  bruteforce  determinant-space engine (second quantisation written out) and
              the two-electron FCI used to pin ``mlcc``
"""
