"""CPU oracle for the randomized-multiplier GENP hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; it exists so that tests, the smoke check and
the benchmark's CPU baseline can compare the HIP path against a plain,
slow, obviously correct implementation written from the paper:

* ``oracle.genp``    -- FP64 numpy: multiplier product, textbook GENP and block
                        Gaussian elimination, substitutions, recovery,
                        refinement, backward error, adjoint.
* ``oracle.exact``   -- exact rational arithmetic (``fractions.Fraction``) for
                        n <= 8: product, GENP, determinants, Cramer's rule.
* ``oracle.lowprec`` -- FP32 / BF16 rounding (round to nearest even) and the
                        low-precision mirrors used to bound the mixed path.

Parity status: every function is pinned by a ``-m "not gpu"`` test except
those whose header says "parity unpinned".
"""
