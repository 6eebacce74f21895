"""CPU reference implementation of the SP2 density-matrix path (TEST INFRASTRUCTURE).

Plain, slow, FP64 NumPy code written from the paper's text.  It exists so that the
GPU library can be checked against something obviously correct; it is not part of
the product.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import it.  The GPU library never calls into it and shares no code with it.

Modules
-------
dm   : the exact zero/finite-temperature density matrices by diagonalization
       (Eqs. 1, 3-6).
sp2  : spectral bounds, the Deep-NN SP2 recursion (Alg. 1) with FP64 or emulated
       mixed-precision activation (Alg. 2, Eqs. Split1/Split2/Square), the FP64
       refinement layer (Eq. Refinement), the same recursion on eigenvalues, and
       the accelerated layers (Sec. Accelerated Deep-NN SP2).
net  : the generalized second-order polynomial network (Eq. general SP2) applied
       to matrices and to eigenvalues, its squared-error loss against a
       Fermi-Dirac target and the hand-derived gradient.
fermi: the optimized finite-temperature expansion (Eq. general SP2 with the read-out
       1 - sum c_i eps_i, Eq. fermi) and its Levenberg-Marquardt fit on a grid.

Parity status: every function is pinned by tests in tests/test_oracle_*.py against
closed forms, invariants, brute force or the paper's printed constants, except the
ones whose docstring says "parity unpinned".
"""
from . import dm, fermi, sp2, net  # noqa: F401
