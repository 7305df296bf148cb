"""CPU FP64 oracle for the block omega-circulant preconditioned all-at-once solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path (the HIP library and its Python binding) never does, and it shares no
code with that path (only the seeded input generators in `datagen`).

Everything here follows the paper (Fung & Hon, "Block omega-circulant
preconditioners for parabolic optimal control problems") by definition:

* discretisation.py -- theta-method all-at-once system (Section 1,
  eqn:main_system_before, eqn:matrix_A_before), the symmetric form A
  (eqn:main_system, eqn:matrix_A) and the nonsymmetric form A_hat
  (eqn:main_system_nonsym, eqn:matrix_A_hat), assembled from sparse
  Kronecker products; finite differences with Dirichlet data (any a) or
  homogeneous Neumann data (Example 3), or linear / bilinear finite elements
  (mass matrix M_m != I).
* circulant.py -- omega-circulant S_n^(1), S_n^(2) built entry by entry from
  their printed definition, S_n = S^(1) (S^(2))^{-1}, the dense O(n^2)
  time transform and its eigenvalue table taken from the similarity itself.
* spatial.py -- the textbook sine basis and eigenvalues of -L_h, the finite
  element eigenvalues in that basis, and the cosine basis of the Neumann
  operator.
* precond.py -- P_S, |P_S|, P_MS as dense matrices from their definitions
  (tiny sizes) and as three-step applies built from a dense DFT matrix plus
  dense sine matrices (a = 1) or per-frequency sparse LU (variable a).
* krylov.py -- textbook preconditioned MINRES and restarted (flexible)
  GMRES with classical Gram-Schmidt applied twice; stop on the explicit
  true relative residual.
* solver.py -- end-to-end solve, recovery of y and p, the error e_h, and a
  sparse direct solve of the whole system.

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: closed forms printed in the paper, its theorems' spectral statements,
dense definitions at tiny sizes, the printed Table 1 / Table 3 / Table 4
values, element integrals by quadrature, and a sparse direct solve.
"""
