"""The benchmark's flop count (the metric's numerator) against operations counted one by one.

GENP of an n x n matrix (section 1.1): at step k the n-k-1 multipliers take one division each
and the (n-k-1)^2 trailing entries one multiplication and one subtraction each; summed over
the steps this is (2/3) n^3 - n^2/2 - n/6.  C = A G takes n^2 dot products of length n (n
multiplications, n-1 additions, counted as the usual 2n^3); the two substitutions and x = G y
take 4 n^2 k, and each refinement step 6 n^2 k (residual 2 n^2 k plus another solve 4 n^2 k).
"""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _genp_ops(n):
    ops = 0
    for k in range(n - 1):
        m = n - k - 1
        ops += m                     # multipliers l_ik = c_ik / c_kk
        ops += 2 * m * m             # c_ij -= l_ik c_kj
    return ops


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 33])
def test_lu_term_counts_genp_operations(n):
    b = _bench()
    lu = b.method_flops(n, 0, 0) - 2.0 * n ** 3
    assert lu == pytest.approx(_genp_ops(n), abs=1e-9)


def test_solve_and_refinement_terms():
    b = _bench()
    n, k = 10, 3
    base = b.method_flops(n, k, 0)
    assert base - b.method_flops(n, 0, 0) == pytest.approx(4.0 * n * n * k)
    assert b.method_flops(n, k, 2) - base == pytest.approx(2 * 6.0 * n * n * k)
