"""Block Gaussian elimination with explicit block pivots (test infrastructure only).

Theorem 2.2 (section 2.2) bounds two eliminations: GENP, whose pivots are
entries, and block Gaussian elimination, whose pivots are blocks.  With block
size nb the block elimination takes, at each step, the leading nb x nb block
of the current Schur complement as the block pivot and replaces the rest by
its Schur complement with respect to that block (Fact 2.1):

    S_0 = C
    B_k = S_k[:nb, :nb]                                   (k-th block pivot)
    S_{k+1} = S_k[nb:, nb:] - S_k[nb:, :nb] B_k^{-1} S_k[:nb, nb:]

It needs only the leading nb, 2nb, 3nb, ... blocks of C to be nonsingular,
not every leading block as GENP does.  B_k^{-1} is applied through Gaussian
elimination with row interchanges inside the block pivot (LAPACK getrf via
scipy, a library primitive); the interchanges never leave the block, so the
factors satisfy P C = L U with P block diagonal (one permutation per block
pivot), L unit lower and U upper triangular.  This is the packed form the
GPU library stores.  Explicit block pivots are kept for Theorem 2.2's
bounds: ||B_k|| <= N + N_- N^2 and ||B_k^{-1}|| <= N_- with N = ||C|| and
N_- the largest norm of the inverse of a leading block of C.

Plain numpy float64, no blocking beyond the elimination's own block size.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


@dataclasses.dataclass
class BlockGEResult:
    """Outcome of block Gaussian elimination.

    pivots: the block pivots B_k in the row order of C (the last one ragged
            when nb does not divide n); only those before a breakdown.
    perm:   row r of the factors is row perm[r] of C; perm[r] stays inside
            the block of r.
    LU:     unit lower L below the diagonal, U on and above it: P C = L U.
    breakdown_col: 1-based column of the first elimination pivot inside a
            block pivot that is non-finite or has |u| <= pivot_tol max|C|
            (the block pivot is numerically singular); 0 when none.
    """

    pivots: List[np.ndarray]
    perm: np.ndarray
    LU: np.ndarray
    breakdown_col: int
    max_abs_c: float


def _ipiv_to_perm(ipiv: np.ndarray) -> np.ndarray:
    """LAPACK's interchange list (row i swapped with ipiv[i], in order) as a
    permutation: row r of P B is row p[r] of B."""
    p = np.arange(ipiv.shape[0])
    for i, j in enumerate(ipiv):
        if j != i:
            p[i], p[j] = p[j], p[i]
    return p


def block_ge(C: np.ndarray, nb: int, pivot_tol: float = 0.0) -> BlockGEResult:
    """Block Gaussian elimination of C with nb x nb block pivots (Theorem 2.2,
    Fact 2.1); see the module docstring for the recurrence."""
    from scipy.linalg import lu_factor, solve_triangular

    if nb < 1:
        raise ValueError("nb >= 1")
    C = np.array(C, dtype=np.float64, copy=True)
    n = C.shape[0]
    maxc = float(np.max(np.abs(C))) if n else 0.0
    tol_abs = pivot_tol * maxc
    perm = np.arange(n)
    LU = np.zeros((n, n))
    S = C.copy()                      # the current Schur complement (rows/cols k..n-1 of C)
    pivots: List[np.ndarray] = []
    for k in range(0, n, nb):
        w = min(nb, n - k)
        e = k + w
        B = S[:w, :w].copy()          # block pivot B_k
        lu, ipiv = lu_factor(B, check_finite=False)
        d = np.diag(lu)
        bad = [t for t in range(w) if (not np.isfinite(d[t])) or abs(d[t]) <= tol_abs]
        p = _ipiv_to_perm(ipiv)
        perm[k:e] = k + p
        LU[k:e, :k] = LU[k:e, :k][p]  # the L entries of earlier steps follow their rows
        LU[k:e, k:e] = lu
        if bad:
            return BlockGEResult(pivots, perm, LU, k + bad[0] + 1, maxc)
        pivots.append(B)
        if e < n:
            S12, S21 = S[:w, w:], S[w:, :w]
            L_k = np.tril(lu, -1) + np.eye(w)
            U_k = np.triu(lu)
            LU[k:e, e:] = solve_triangular(L_k, S12[p], lower=True, unit_diagonal=True)   # L_k^{-1} P_k S12
            LU[e:, k:e] = solve_triangular(U_k.T, S21.T, lower=True).T                   # S21 U_k^{-1}
            S = S[w:, w:] - S21 @ np.linalg.solve(B, S12)                               # Fact 2.1
    return BlockGEResult(pivots, perm, LU, 0, maxc)


def permute_rows(perm: np.ndarray, B: np.ndarray) -> np.ndarray:
    """P B: row r of the result is row perm[r] of B."""
    return np.asarray(B, dtype=np.float64)[perm]


def lu_solve_perm(res: BlockGEResult, B: np.ndarray) -> np.ndarray:
    """C^{-1} B = U^{-1} L^{-1} P B by row-by-row substitution."""
    from oracle.genp import lu_solve

    return lu_solve(res.LU, permute_rows(res.perm, B))


def solve(res: BlockGEResult, G: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X = G C^{-1} B: the solution of A X = B from the block factors of C = A G."""
    return G @ lu_solve_perm(res, B)


def theorem_2_2_bounds(C: np.ndarray):
    """(N + N_- N^2, N_-) of Theorem 2.2 in the spectral norm: N = ||C||_2 and
    N_- = max_j ||C_j^{-1}||_2 over the leading j x j blocks C_j (brute force)."""
    C = np.asarray(C, dtype=np.float64)
    N = float(np.linalg.norm(C, 2))
    Nm = max(float(np.linalg.norm(np.linalg.inv(C[:j, :j]), 2)) for j in range(1, C.shape[0] + 1))
    return N + Nm * N * N, Nm
