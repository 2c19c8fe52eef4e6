"""FP64 CPU oracle for Gaussian-charge charge equilibration (QEq).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library
(the seeded input generators live in their own module, ``inputs``).

What it computes (see the docstrings of each function for the passage it
follows):

* ``ewald``   -- dense periodic Coulomb matrix of normalised Gaussian charges
                 by explicit real- and reciprocal-space Ewald sums, the
                 bordered Lagrange system solved by Gaussian elimination,
                 energies, analytic forces and the adjoint gradient.
* ``matfree`` -- the same sums applied to a vector without forming the matrix,
                 with an FP64 projected CG solve, for systems too large for the
                 dense route (tens of thousands of atoms).
* ``direct``  -- the non-periodic pairwise Coulomb kernel of the paper, the
                 plain plane-wave energy sum, and a brute-force constrained
                 minimiser; used only to pin the other two.

Parity status of every function is stated in its docstring; functions whose
results have no external pin say "parity unpinned".
"""
