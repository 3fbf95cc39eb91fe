"""Pins of the block Gaussian elimination oracle (Theorem 2.2; CPU only).

Each check compares the oracle with something other than itself: the point
GENP oracle (whose factors have their own pins), exact rational arithmetic,
the closed form of the inverse of a Schur complement, determinants, the
library's dense solve, and Theorem 2.2's bounds.  Planted mistakes at the end
show that the checks catch a wrong sign, a missing interchange or a wrong
block.
"""
import inspect
import textwrap
import warnings
from fractions import Fraction

import numpy as np
import pytest

from oracle import blockge as obg
from oracle import exact, genp as og


def _gauss(n, seed):
    return np.random.default_rng(seed).standard_normal((n, n))


def _swapped_blocks(n, nb, seed):
    """C = L_b U_b with L_b block unit lower and U_b block upper triangular, the
    leading entry of every diagonal block of U_b zero.  By the uniqueness of the
    block factorization the block pivots are U_b's diagonal blocks (up to
    rounding), so point GENP breaks down at once while every leading nb, 2nb, ...
    block stays nonsingular."""
    g = np.random.default_rng(seed)
    Lb, Ub = np.eye(n), np.zeros((n, n))
    for k in range(0, n, nb):
        e = min(k + nb, n)
        Lb[e:, k:e] = g.standard_normal((n - e, e - k)) / np.sqrt(n)
        Ub[k:e, k:] = g.standard_normal((e - k, n - k))
        Ub[k, k] = 0.0
    return Lb @ Ub


def _pc_minus_lu(res, C):
    L, U = og.unpack(res.LU)
    return np.max(np.abs(C[res.perm] - L @ U)) / np.max(np.abs(L) @ np.abs(U))


@pytest.mark.parametrize("n,nb", [(48, 16), (50, 16), (37, 8)])
def test_block_pivots_are_the_diagonal_blocks_of_the_point_factors(n, nb):
    # Fact 2.1: the k-th block pivot is the leading block of the k-th Schur
    # complement, which GENP factors as L_kk U_kk
    C = _gauss(n, 1)
    res = obg.block_ge(C, nb)
    LU, info = og.genp_unblocked(C)
    assert info.breakdown_col == 0 and res.breakdown_col == 0
    L, U = og.unpack(LU)
    assert len(res.pivots) == -(-n // nb)
    for k, B in zip(range(0, n, nb), res.pivots):
        e = min(k + nb, n)
        ref = L[k:e, k:e] @ U[k:e, k:e]
        assert np.max(np.abs(B - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,nb", [(40, 8), (45, 16)])
def test_inverse_of_each_block_pivot_is_a_block_of_a_leading_inverse(n, nb):
    # the Schur complement of C_{11} in the leading (k+1) nb block has as inverse
    # the trailing block of that leading block's inverse
    C = _gauss(n, 2)
    res = obg.block_ge(C, nb)
    for k, B in zip(range(0, n, nb), res.pivots):
        e = min(k + nb, n)
        ref = np.linalg.inv(C[:e, :e])[k:e, k:e]
        assert np.allclose(np.linalg.inv(B), ref, rtol=1e-9, atol=1e-9 * np.max(np.abs(ref)))


def test_determinant_is_the_product_of_the_block_pivot_determinants():
    C = _gauss(64, 3)
    res = obg.block_ge(C, 16)
    s, ld = np.linalg.slogdet(C)
    parts = [np.linalg.slogdet(B) for B in res.pivots]
    assert np.isclose(sum(p[1] for p in parts), ld, rtol=1e-12, atol=1e-10)
    assert np.prod([p[0] for p in parts]) == s


def test_block_pivots_in_exact_arithmetic():
    # S_{k+1} = S22 - S21 B^{-1} S12 over the rationals (B^{-1} S12 by Cramer's rule)
    n, nb = 6, 2
    C = _swapped_blocks(n, nb, 4)
    res = obg.block_ge(C, nb)
    S = exact.to_frac(C)
    for k in range(0, n, nb):
        B = [row[:nb] for row in S[:nb]]
        got = res.pivots[k // nb]
        assert np.max(np.abs(got - exact.to_float(B))) <= 1e-12 * np.max(np.abs(got))
        if k + nb < n:
            S12 = [row[nb:] for row in S[:nb]]
            X = exact.cramer(B, S12)                     # B^{-1} S12
            S = [[S[i][j] - sum((S[i][t] * X[t][j - nb] for t in range(nb)), Fraction(0))
                  for j in range(nb, len(S))] for i in range(nb, len(S))]


def test_interior_singular_blocks_need_no_pivoting_across_blocks():
    n, nb = 32, 4
    C = _swapped_blocks(n, nb, 5)
    _, info = og.genp_unblocked(C)
    assert info.breakdown_col == 1                      # GENP: c_11 = 0
    res = obg.block_ge(C, nb)
    assert res.breakdown_col == 0
    for k in range(0, n, nb):
        assert sorted(res.perm[k:k + nb]) == list(range(k, k + nb))    # interchanges stay in the block
        assert res.perm[k] != k                                        # the zero is never a pivot
    assert _pc_minus_lu(res, C) <= 64 * og.U64
    b = np.random.default_rng(6).standard_normal((n, 2))
    x = obg.lu_solve_perm(res, b)
    ref = np.linalg.solve(C, b)
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.linalg.cond(C) * np.max(np.abs(ref))


def test_exact_solution_of_a_tiny_system_with_a_zero_leading_entry():
    n, nb = 6, 3
    C = _swapped_blocks(n, nb, 7)
    b = np.random.default_rng(8).standard_normal((n, 1))
    xe = exact.to_float(exact.cramer(exact.to_frac(C), exact.to_frac(b)))
    x = obg.lu_solve_perm(obg.block_ge(C, nb), b)
    assert np.max(np.abs(x - xe)) <= 1e-12 * np.linalg.cond(C) * np.max(np.abs(xe))


def test_block_size_one_is_point_genp():
    C = _gauss(20, 9)
    res = obg.block_ge(C, 1)
    LU, _ = og.genp_unblocked(C)
    assert np.array_equal(res.perm, np.arange(20))
    assert np.allclose(res.LU, LU, rtol=1e-12, atol=1e-12 * np.max(np.abs(LU)))
    assert np.allclose([B[0, 0] for B in res.pivots], np.diag(LU), rtol=1e-12)


@pytest.mark.parametrize("n,nb", [(40, 8), (30, 7)])
def test_theorem_2_2_bounds_hold(n, nb):
    C = _gauss(n, 10)
    top, nm = obg.theorem_2_2_bounds(C)
    res = obg.block_ge(C, nb)
    for B in res.pivots:
        assert np.linalg.norm(B, 2) <= top
        assert np.linalg.norm(np.linalg.inv(B), 2) <= nm * (1 + 1e-10)


def test_singular_leading_block_is_a_breakdown():
    n, nb = 24, 8
    C = _gauss(n, 11)
    M = np.random.default_rng(12).standard_normal((nb, nb))
    C[nb:2 * nb, :2 * nb] = M @ C[:nb, :2 * nb]          # leading 2nb block of rank nb
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        res = obg.block_ge(C, nb, pivot_tol=n * og.U64)
    assert nb < res.breakdown_col <= 2 * nb
    assert len(res.pivots) == 1
    assert obg.block_ge(_gauss(n, 11), nb, pivot_tol=n * og.U64).breakdown_col == 0


@pytest.mark.parametrize("seed", [13, 14])
def test_solve_with_a_multiplier_matches_the_dense_solve(seed):
    g = np.random.default_rng(seed)
    n = 40
    A, G, b = g.standard_normal((n, n)), g.standard_normal((n, n)), g.standard_normal((n, 3))
    res = obg.block_ge(og.precondition(A, G), 8)
    x = obg.solve(res, G, b)
    ref = np.linalg.solve(A, b)
    assert np.max(np.abs(x - ref)) <= 1e-9 * np.max(np.abs(ref))


# -------------------------------------------------------------- planted mistakes ----

def _checks():
    out = []
    n, nb = 24, 4
    C = _swapped_blocks(n, nb, 21)
    b = np.random.default_rng(22).standard_normal((n, 1))
    for f in (
        lambda r: _pc_minus_lu(r, C) <= 64 * og.U64,
        lambda r: np.allclose(obg.lu_solve_perm(r, b), np.linalg.solve(C, b), rtol=1e-8, atol=1e-8),
        lambda r: all(np.allclose(np.linalg.inv(B), np.linalg.inv(C[:k + nb, :k + nb])[k:, k:], rtol=1e-8, atol=1e-8)
                      for k, B in zip(range(0, n, nb), r.pivots)),
        lambda r: all(sorted(r.perm[k:k + nb]) == list(range(k, k + nb)) for k in range(0, n, nb)),
    ):
        try:
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                out.append(bool(f(obg.block_ge(C, nb))))
        except Exception:
            out.append(False)
    return out


MUTANTS = {
    "Schur complement with the wrong sign": ("block_ge", "S = S[w:, w:] - S21 @", "S = S[w:, w:] + S21 @"),
    "earlier L entries not moved with their rows": ("block_ge", "LU[k:e, :k] = LU[k:e, :k][p]", "LU[k:e, :k] = LU[k:e, :k]"),
    "U12 from the unpermuted rows": ("block_ge", "S12[p], lower=True", "S12, lower=True"),
    "permutation without the block offset": ("block_ge", "perm[k:e] = k + p", "perm[k:e] = p"),
    "block pivot read from C instead of the Schur complement": ("block_ge", "B = S[:w, :w].copy()", "B = C[k:e, k:e].copy()"),
    "interchange list read as a permutation": ("_ipiv_to_perm", "p[i], p[j] = p[j], p[i]", "p[i] = j"),
    "L21 against U^T instead of U": ("block_ge", "solve_triangular(U_k.T, S21.T, lower=True).T", "solve_triangular(U_k, S21.T, lower=False).T"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(obg, attr)))
    assert old in src, old
    ns = dict(vars(obg))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    monkeypatch.setattr(obg, attr, ns[attr])
    assert not all(_checks()), f"mutant not caught: {name}"


def test_checks_pass_on_the_oracle():
    assert all(_checks())


def test_hadamard_rows_factor_exactly():
    # powers of two throughout: P C = L U holds without rounding, |L| in {0, 1}
    import scipy.linalg as sl
    n, nb = 128, 32
    g = np.random.default_rng(3)
    P = np.concatenate([k + g.permutation(nb) for k in range(0, n, nb)])
    C = sl.hadamard(n).astype(np.float64)[P]
    res = obg.block_ge(C, nb)
    L, U = og.unpack(res.LU)
    assert res.breakdown_col == 0
    assert np.array_equal(C[res.perm], L @ U)
    assert set(np.unique(np.abs(np.tril(L, -1)))) <= {0.0, 1.0}
