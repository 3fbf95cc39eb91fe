"""FP64 CPU oracle of randomized low-rank approximation (test infrastructure only).

Proto-Algorithm 5.1 (section 5.3) with the orthogonal basis of Remark 5.4:

    T' = A^T G                       (Stage 1: G Gaussian or Toeplitz, m x rho_+)
    T' P = Q R, pivoted QR           (Stage 2: rank-revealing factorization; s = the
                                      least number of columns with ||R[s:, s:]||_F <= tau ||A||_F)
    T = Q[:, :s],  W = A T           (Stage 3: A_hat = A T T^T, Theorem 5.1 with an
                                      orthogonal basis)
    FAILURE when ||A - A_hat||_F > tau2 ||A||_F

Norms: the Frobenius norm throughout (the residual of the exact projection is then
sqrt(sum_{j > rho} sigma_j^2), the Frobenius form of Theorem 5.1); 2-norms are
reported beside it where a test needs them.  Library steps: scipy's pivoted QR
(LAPACK geqp3) and matrix products.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


def toeplitz_rect(p: np.ndarray, m: int, k: int) -> np.ndarray:
    """m x k Toeplitz matrix from m + k - 1 parameters: G[i, j] = p[i - j + k - 1]."""
    p = np.asarray(p, dtype=np.float64)
    if p.shape != (m + k - 1,):
        raise ValueError("need m + k - 1 parameters")
    i = np.arange(m)[:, None]
    j = np.arange(k)[None, :]
    return p[i - j + k - 1]


@dataclasses.dataclass
class LowRankResult:
    rank: int                 # s of Stage 2
    T: np.ndarray             # n x s, orthonormal columns
    W: np.ndarray             # m x s, A T
    perm: np.ndarray          # pivot order of the columns of T'
    a_fro: float              # ||A||_F
    tail_fro: float           # ||R[s:, s:]||_F
    resid_fro: float          # ||A - W T^T||_F
    failed: bool              # Stage 3 check

    def ahat(self) -> np.ndarray:
        return self.W @ self.T.T


def sketch(A: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Stage 1: T' = A^T G (Theorem 5.2: a basis of the leading right singular space
    up to an error of order sigma_{rho+1}(A))."""
    return np.asarray(A, dtype=np.float64).T @ np.asarray(G, dtype=np.float64)


def rank_revealing(Tp: np.ndarray, tol_abs: float):
    """Stage 2 with pivoted QR: T' P = Q R; s = the least s with ||R[s:, s:]||_F <= tol_abs.
    Returns (s, Q[:, :s], perm, ||R[s:, s:]||_F)."""
    from scipy.linalg import qr
    Q, R, perm = qr(np.asarray(Tp, dtype=np.float64), mode="economic", pivoting=True)
    k = R.shape[1]
    for s in range(k + 1):
        tail = float(np.linalg.norm(R[s:, s:])) if s < k else 0.0
        if tail <= tol_abs:
            return s, Q[:, :s], perm, tail
    return k, Q, perm, 0.0


def lowrank(A: np.ndarray, G: np.ndarray, tau: float, tau2: float) -> LowRankResult:
    """Proto-Algorithm 5.1 with the orthogonal basis of Remark 5.4."""
    A = np.asarray(A, dtype=np.float64)
    a_fro = float(np.linalg.norm(A))
    s, T, perm, tail = rank_revealing(sketch(A, G), tau * a_fro)
    W = A @ T
    resid = float(np.linalg.norm(A - W @ T.T))
    return LowRankResult(s, T, W, perm, a_fro, tail, resid, resid > tau2 * a_fro)


def projection_residual(A: np.ndarray, T: np.ndarray, orthogonal: bool = True, ord=2) -> float:
    """||A - A T (T^T T)^{-1} T^T|| (Theorem 5.1); with orthogonal T, ||A - A T T^T||."""
    A = np.asarray(A, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    P = T @ T.T if orthogonal else T @ np.linalg.solve(T.T @ T, T.T)
    return float(np.linalg.norm(A - A @ P, ord))

