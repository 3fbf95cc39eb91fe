"""Exact rational arithmetic for tiny systems (test infrastructure only).

Every float64 is a rational number, so ``fractions.Fraction(x)`` is exact and
so is every sum, product and quotient below.  For n <= 8 this gives:

* the exact product C = A G of the stored floating-point inputs;
* the exact GENP factors of C (section 1.1) -- unique for a strongly
  nonsingular matrix, i.e. one whose leading blocks are all nonsingular
  (section 2.2);
* exact determinants (fraction-valued elimination with row exchanges, a
  different algorithm from GENP) and hence Cramer's rule for A x = b, the
  brute-force solution the floating-point path must agree with.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Optional, Tuple

import numpy as np

Mat = List[List[Fraction]]


def to_frac(M) -> Mat:
    M = np.asarray(M, dtype=np.float64)
    if M.ndim == 1:
        M = M[:, None]
    return [[Fraction(float(v)) for v in row] for row in M]


def to_float(M: Mat) -> np.ndarray:
    return np.array([[float(v) for v in row] for row in M], dtype=np.float64)


def matmul(A: Mat, B: Mat) -> Mat:
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), Fraction(0)) for j in range(m)]
            for i in range(n)]


def genp(C: Mat) -> Tuple[Optional[Mat], Optional[Mat], int]:
    """Exact GENP: returns (L, U, 0) or (None, None, k) if the k-th (1-based)
    pivot is exactly zero."""
    n = len(C)
    U = [row[:] for row in C]
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for k in range(n):
        if U[k][k] == 0:
            return None, None, k + 1
        for i in range(k + 1, n):
            l = U[i][k] / U[k][k]
            L[i][k] = l
            for j in range(k, n):
                U[i][j] -= l * U[k][j]
    return L, U, 0


def det(M: Mat) -> Fraction:
    """Exact determinant by elimination with row exchanges."""
    A = [row[:] for row in M]
    n = len(A)
    sign = 1
    d = Fraction(1)
    for k in range(n):
        p = next((i for i in range(k, n) if A[i][k] != 0), None)
        if p is None:
            return Fraction(0)
        if p != k:
            A[k], A[p] = A[p], A[k]
            sign = -sign
        d *= A[k][k]
        for i in range(k + 1, n):
            f = A[i][k] / A[k][k]
            for j in range(k, n):
                A[i][j] -= f * A[k][j]
    return sign * d


def cramer(A: Mat, b: Mat) -> Mat:
    """x_i = det(A with column i replaced by b) / det(A), column by column of b."""
    n = len(A)
    dA = det(A)
    if dA == 0:
        raise ZeroDivisionError("singular matrix")
    X = [[Fraction(0)] * len(b[0]) for _ in range(n)]
    for c in range(len(b[0])):
        for i in range(n):
            Ai = [row[:i] + [b[r][c]] + row[i + 1:] for r, row in enumerate(A)]
            X[i][c] = det(Ai) / dA
    return X


def leading_minors(C: Mat) -> List[Fraction]:
    """det C_k for k = 1..n (C_k the leading k x k block, section 2.2)."""
    return [det([row[:k] for row in C[:k]]) for k in range(1, len(C) + 1)]
