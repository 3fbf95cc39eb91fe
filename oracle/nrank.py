"""FP64 CPU oracle of the numerical rank without pivoting or orthogonalization (test
infrastructure only): Proto-Algorithm B.1 (Appendix B) with Remarks B.2 and B.4.

    G (m x rho_+), B_s = A^T G_s with G_s the first s columns of G
    bisection over s in [rho_-, rho_+] (Remark B.4: s = ceil((rho_- + rho_+) / 2));
    COND(B_s): full rank and well conditioned, kappa_2(B_s) <= cond_max.

Reading of the update rule: B_s is well conditioned (with probability near 1) exactly when
s <= nrank(A) -- the product of A^T with a Gaussian m x s matrix keeps the numerical rank
min(s, nrank(A)) -- so a passing test raises the lower end (rho_- = s) and a failing one
lowers the upper end (rho_+ = s - 1).  The sketch is formed once for rho_+ columns: its
first s columns are A^T G_s.

COND: `svd` takes kappa_2 from the singular values (the definition); `lanczos` follows
Remark B.2: Lanczos on S = B_s^T B_s (no reorthogonalization), then the extreme eigenvalues
of the tridiagonal by Sturm-sequence bisection; kappa_2 = sqrt(lambda_max / lambda_min).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def sturm_count(alpha: np.ndarray, beta: np.ndarray, x: float) -> int:
    """Number of eigenvalues < x of the symmetric tridiagonal (diagonal alpha, off-diagonal
    beta), from the signs of the pivots of T - x I = L D L^T (no pivoting)."""
    cnt = 0
    d = 1.0
    for i in range(len(alpha)):
        b2 = beta[i - 1] ** 2 if i else 0.0
        d = (alpha[i] - x) - (b2 / d if i else 0.0)
        if d == 0.0:
            d = -1e-300   # x is an eigenvalue of the leading block: perturb to the left
        if d < 0:
            cnt += 1
    return cnt


def tridiag_extremes(alpha: np.ndarray, beta: np.ndarray, iters: int = 200):
    """(lambda_min, lambda_max) of a symmetric tridiagonal by bisection on Sturm counts,
    inside the Gershgorin interval."""
    k = len(alpha)
    r = np.zeros(k)
    r[:-1] += np.abs(beta)
    r[1:] += np.abs(beta)
    lo, hi = float(np.min(alpha - r)), float(np.max(alpha + r))
    out = []
    for target in (1, k):            # the 1st and the k-th eigenvalue: count(x) >= target
        a, b = lo, hi
        for _ in range(iters):
            mid = 0.5 * (a + b)
            if mid == a or mid == b:
                break
            if sturm_count(alpha, beta, mid) >= target:
                b = mid
            else:
                a = mid
        out.append(0.5 * (a + b))
    return out[0], out[1]


def lanczos_tridiag(S: np.ndarray, v0: np.ndarray, steps: int):
    """Lanczos on symmetric S from v0 (no reorthogonalization): (alpha, beta) of T_k; stops
    early when beta vanishes (an invariant subspace)."""
    v = np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    alpha, beta = [], []
    b = 0.0
    for _ in range(steps):
        w = S @ v - b * v_prev
        a = float(v @ w)
        w -= a * v
        alpha.append(a)
        b = float(np.linalg.norm(w))
        if b <= 1e-300:
            break
        beta.append(b)
        v_prev, v = v, w / b
    return np.array(alpha), np.array(beta[:len(alpha) - 1])


def cond_svd(B: np.ndarray) -> float:
    s = np.linalg.svd(np.asarray(B, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else math.inf


LANCZOS_STEPS_PER_COLUMN = 6   # without reorthogonalization the extremes need several sweeps


def cond_lanczos(B: np.ndarray, v0: np.ndarray) -> float:
    """Remark B.2: kappa_2(B) from the extreme eigenvalues of S = B^T B (Lanczos with 6s
    steps, then Sturm bisection on the tridiagonal).  The Ritz values lie inside the
    spectrum of S, so the estimate is a lower bound on kappa_2(B) -- except that eigenvalues
    of S below its rounding level (u lambda_max) come out at that level or <= 0 (kappa inf)."""
    B = np.asarray(B, dtype=np.float64)
    S = B.T @ B
    al, be = lanczos_tridiag(S, v0, LANCZOS_STEPS_PER_COLUMN * S.shape[0])
    lmin, lmax = tridiag_extremes(al, be)
    return float(math.sqrt(lmax / lmin)) if lmin > 0 else math.inf


@dataclasses.dataclass
class NRankResult:
    rank: int
    tests: list       # (s, kappa, passed) in the order tested
    B: np.ndarray     # n x rank: A^T G_rank, an approximate basis of the leading right singular space


def numerical_rank(A: np.ndarray, G: np.ndarray, rho_minus: int, rho_plus: int, cond_max: float,
                   cond: str = "svd") -> NRankResult:
    """Proto-Algorithm B.1: bisection on the conditioning of B_s = A^T G_s."""
    A = np.asarray(A, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    if not (0 <= rho_minus <= rho_plus <= G.shape[1]):
        raise ValueError("need 0 <= rho_- <= rho_+ <= columns of G")
    sk = A.T @ G                          # the sketch, all rho_+ columns at once
    lo, hi = rho_minus, rho_plus
    tests = []
    while lo < hi:
        s = (lo + hi + 1) // 2            # ceil((rho_- + rho_+) / 2) >= 1
        B = sk[:, :s]
        k = cond_svd(B) if cond == "svd" else cond_lanczos(B, G[:s, 0])
        ok = k <= cond_max
        tests.append((s, k, ok))
        if ok:
            lo = s
        else:
            hi = s - 1
    return NRankResult(lo, tests, sk[:, :lo])
