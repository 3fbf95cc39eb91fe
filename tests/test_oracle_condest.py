"""Pins of the oracle's 1-norm condition estimates (oracle/condest.py) against closed forms and
brute force: the Hager-Higham estimator is exact on non-negative and on diagonal matrices, is a
lower bound of ||B||_1 always, and distinguishes B from B^T (a matrix whose 1- and infinity
norms differ); kappa_1 is checked on hand-worked 2 x 2 cases."""
import numpy as np
import pytest

from oracle import condest as oc


def test_norm1_definition_by_hand():
    # columns sum to 3 and 5 in absolute value
    assert oc.norm1(np.array([[1.0, -2.0], [-2.0, 3.0]])) == 5.0


def test_cond1_exact_hand_worked():
    # C = [[2, 1], [1, 1]]: ||C||_1 = 3, C^{-1} = [[1, -1], [-1, 2]], ||C^{-1}||_1 = 3
    assert oc.cond1_exact(np.array([[2.0, 1.0], [1.0, 1.0]])) == pytest.approx(9.0, rel=1e-14)
    # diag(1e-3, 1): 1 * 1e3
    assert oc.cond1_exact(np.diag([1e-3, 1.0])) == pytest.approx(1e3, rel=1e-14)
    # upper triangular [[1, 4], [0, 1]]: ||C||_1 = 5, C^{-1} = [[1, -4], [0, 1]]: 5
    assert oc.cond1_exact(np.array([[1.0, 4.0], [0.0, 1.0]])) == pytest.approx(25.0, rel=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_estimate_exact_on_nonnegative(seed):
    B = np.abs(np.random.default_rng(seed).standard_normal((40, 40)))
    assert oc.norm1_estimate_matrix(B) == pytest.approx(oc.norm1(B), rel=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_estimate_exact_on_diagonal(seed):
    d = np.random.default_rng(seed).standard_normal(33)
    assert oc.norm1_estimate_matrix(np.diag(d)) == pytest.approx(np.max(np.abs(d)), rel=1e-15)


def test_estimate_is_for_b_not_its_transpose():
    # ||B||_1 = 1 but ||B^T||_1 = ||B||_inf = 3
    B = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    assert oc.norm1_estimate_matrix(B) == pytest.approx(1.0, rel=1e-15)
    assert oc.norm1_estimate_matrix(B.T) == pytest.approx(3.0, rel=1e-15)


def test_estimate_n1():
    assert oc.norm1_estimate_matrix(np.array([[-2.5]])) == 2.5


def test_estimate_lower_bound_and_close_on_random():
    """Brute force over 60 random matrices (Gaussian and inverses of Gaussian): never above
    ||B||_1, never below a third of it, and exact for a good share of them."""
    rng = np.random.default_rng(7)
    ratios = []
    for t in range(60):
        n = int(rng.integers(2, 60))
        M = rng.standard_normal((n, n))
        B = np.linalg.inv(M) if t % 2 else M
        e, x = oc.norm1_estimate_matrix(B), oc.norm1(B)
        assert e <= x * (1 + 1e-12)
        ratios.append(e / x)
    assert min(ratios) >= 1.0 / 3.0
    assert np.mean(np.isclose(ratios, 1.0, rtol=1e-12)) >= 0.4
