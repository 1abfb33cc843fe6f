"""Plain CPU reference (oracle) for randomized bilinear matrix multiplication.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (``paper_1905_07439_amd``) and never imports it.

Everything here is written from the paper (Malik & Becker, "Randomization of
Approximate Bilinear Computation for Matrix Multiplication"), in float64 unless
a function says otherwise, with no blocking, fusion or reordering beyond what
the paper's definitions state:

  schemes     -- U, V, W tensors: Strassen, Laderman, the perturbed (approximate)
                 Strassen of Section 3.1, the R=1 all-ones example of Section 2.1.
  tensors     -- the 6-way tensors X, Y (eqs. def-x, def-y), tau (Definition 1),
                 kappa (eq. epsilon-def), ||Y||, and the quantity of
                 eq. square-root-of-sum.
  draws       -- Rademacher signs and uniform permutations per level
                 (Section 2.1, before Definition 2), taken from numpy's Philox
                 bit generator, and the fold of eq. randomized-algorithm.
  recursion   -- F-hat^(Q) of eq. recursive-random-formula, with a standard
                 product at the leaves, zero padding, and an optional float32
                 working precision (sequential summation as in Section 2.2).
  precision   -- rounding to bf16 / fp16 / e4m3 used to emulate reduced
                 precision leaves (sets tolerances; never a parity reference).
  bounds      -- the error bounds of Propositions 4, 5, 8-12 and Example 13.
  decimal2    -- the 2-digit decimal arithmetic of Example 7.
  expectation -- exact enumeration of E[F-hat] over every draw.

Parity status of each function is stated in its module; functions with no
pin other than themselves say "parity unpinned".
"""

from . import schemes, tensors, draws, recursion, precision, bounds, decimal2, expectation  # noqa: F401
from .recursion import rbc, rbc_seeded, standard  # noqa: F401
