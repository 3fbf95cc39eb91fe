"""1-norm condition estimates for the oracle (test infrastructure only).

Section 4 of the paper bounds how well conditioned A G is, given A and a Gaussian G
(Theorem 4.1, Corollary 4.1); the library reports an estimate of kappa_1 of the
matrix it factors.  Here:

* ``cond1_exact`` -- the definition, kappa_1(C) = ||C||_1 ||C^{-1}||_1, with the
  inverse formed by a library solve (LAPACK, partial pivoting) as a step;
* ``norm1_estimate`` -- the Hager-Higham estimator of ||B||_1 from products with B
  and B^T only (N. J. Higham, "FORTRAN codes for estimating the one-norm of a real or
  complex matrix", ACM TOMS 14 (1988), Algorithm 4.1), written out from that
  published description: a lower bound of ||B||_1, exact for many matrices (for
  instance every matrix with non-negative entries and every diagonal one).
"""
from __future__ import annotations

from typing import Callable

import numpy as np


def norm1(M: np.ndarray) -> float:
    """||M||_1: the largest column sum of |M|."""
    return float(np.max(np.sum(np.abs(np.asarray(M, dtype=np.float64)), axis=0)))


def cond1_exact(C: np.ndarray) -> float:
    """kappa_1(C) = ||C||_1 ||C^{-1}||_1."""
    C = np.asarray(C, dtype=np.float64)
    return norm1(C) * norm1(np.linalg.inv(C))


def _sign(y: np.ndarray) -> np.ndarray:
    return np.where(y >= 0.0, 1.0, -1.0)


def norm1_estimate(apply: Callable[[np.ndarray], np.ndarray], apply_t: Callable[[np.ndarray], np.ndarray],
                   n: int, max_iter: int = 5) -> float:
    """Hager-Higham estimate of ||B||_1 for y = B x (apply) and y = B^T x (apply_t).

    Start from x = e / n, take the sign vector xi of B x and z = B^T xi; then move to the
    unit vector e_j at the first largest |z_j| and repeat until the sign vector repeats,
    the estimate stops growing, z's largest entry is at the previous j, or max_iter
    products with B^T have been taken.  Finally compare with the alternating vector
    x_i = (-1)^i (1 + i / (n - 1)) (0-based i), which catches matrices whose largest
    column the search misses.  On the exit where the estimate did not grow, the larger
    of the last two values is kept (both are ||B e_j||_1 for some j, hence lower bounds).
    """
    x = np.full(n, 1.0 / n)
    y = apply(x)
    est = float(np.sum(np.abs(y)))
    if n == 1:
        return est
    xi = _sign(y)
    z = apply_t(xi)
    j = int(np.argmax(np.abs(z)))
    it = 2
    while True:
        x = np.zeros(n)
        x[j] = 1.0
        y = apply(x)
        est_old = est
        est = float(np.sum(np.abs(y)))
        s = _sign(y)
        if np.array_equal(s, xi) or est <= est_old:
            est = max(est, est_old)
            break
        xi = s
        z = apply_t(xi)
        jlast = j
        j = int(np.argmax(np.abs(z)))
        if z[jlast] == np.max(np.abs(z)) or it >= max_iter:
            break
        it += 1
    alt = np.array([(-1.0) ** i * (1.0 + i / (n - 1)) for i in range(n)])
    temp = 2.0 * float(np.sum(np.abs(apply(alt)))) / (3.0 * n)
    return max(est, temp)


def norm1_estimate_matrix(B: np.ndarray) -> float:
    """The estimator applied to an explicit matrix."""
    B = np.asarray(B, dtype=np.float64)
    return norm1_estimate(lambda v: B @ v, lambda v: B.T @ v, B.shape[0])
