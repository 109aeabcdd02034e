"""FP64 CPU oracle for rank-adaptive matrix-free atomic tomography.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the product path (the HIP
library and its Python binding) never does, and this package never imports
the product.  The two share no code: the only common module is ``synth``,
which draws random inputs and holds none of the method's arithmetic.

Everything here is plain, slow and written for checking by eye against the
paper (complex128 / float64 throughout):

* ``pauli``   -- the per-qubit basis rotations and the Kronecker product
  basis rotation of a Pauli string (numerical-test section, Pauli design).
* ``born``    -- Born probabilities, the atomic Born map, the cross-entropy
  and least-squares losses, the likelihood-ratio vector, the density-level
  gradient matrix, the atom Wirtinger gradient and the weight gradient, in
  three tiers: dense POVM matrices (n <= 4), dense per-setting rotations
  (n <= 12) and per-axis contraction (any n a workstation holds).
* ``simplex`` -- Euclidean projection onto the simplex, the pruning map and
  the coefficient step.
* ``refactor`` -- the density proposal, the exact spectral step of
  Theorem 1 (dense eigendecomposition) and the Lanczos-based spectral
  refactorisation with Ritz candidates and proximal-surrogate selection.
* ``loop``    -- a small acceptance-safeguarded iteration (atom steps,
  coefficient steps, spectral steps) used for the exact-recovery pin.

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``
(closed forms, invariants, brute force, finite differences, Theorem 1);
none is "parity unpinned".
"""
