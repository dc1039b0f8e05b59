"""Oracle for the great-circle-arc x constant-latitude intersection problem.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, constants or pre/post-processing).

Contents
--------
``geometry``  The plain definition of the result (Chen, Ullrich & Panetta,
              "Fast and Accurate Intersections on a Sphere", Sec. 1.2 problem
              definition and Sec. 2): every point x with n.x = 0, x_z = z0,
              |x| = 1 lying on the closed minor arc x1 -> x2.  Hit counts and
              flags come from exact integer sign predicates; point coordinates
              from Eq. (2.2) evaluated on the exact normal in 100-digit decimal
              arithmetic.
``angle``     An independent second derivation of the same points (angle
              parametrisation of the arc, mpmath at 300 bits), used only to
              cross-check ``geometry``.
``eft``       The paper's algorithms in IEEE binary64, step by step in the
              paper's order and notation: TwoSum, TwoProduct, FastTwoSum,
              CompDotC / CompDot (Alg. 1-2), AccuDOP (Alg. 4), SumOfSquares /
              SumNonNeg / SumOfSquaresC (Alg. 5-7), AccSqrt and AccuX (Alg. 8).
``naive``     The direct binary64 translation of Eq. (2.2) (Sec. 4) with plain
              binary64 existence and containment predicates.
``batch``     Array drivers over the above (multiprocessing over host cores).

Pins (what fixes these functions other than themselves) live in
``tests/test_oracle_*.py``: closed forms, invariants, brute-force sampling,
the angle cross-check, exact identities of the error-free transformations and
the error bounds the paper prints.
"""

from . import geometry, eft, naive  # noqa: F401

U = 2.0 ** -53  # unit roundoff of binary64 (Sec. 3)
