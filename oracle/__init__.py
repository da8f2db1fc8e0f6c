"""FP64 CPU oracle for multilevel CC2 / CCSD on Cholesky-factored integrals.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library and is deliberately plain and slow: float64 arrays (complex128 where
a derivative is taken by complex step), every step written as the equation it
follows.  Multi-index contractions are written as einsum expressions; the
helper ``mlcc._einsum`` evaluates each along numpy's optimal pairwise path,
one pairwise product at a time through torch.einsum on the CPU (host BLAS),
which changes only the rounding order.

Modules
  mlcc        residual, energy, ground state, Jacobian transform (complex step),
              dense eigenvalues and a full-space Davidson
  bruteforce  determinant-space engine (second quantisation written out) and
              the two-electron FCI used to pin ``mlcc``
"""
