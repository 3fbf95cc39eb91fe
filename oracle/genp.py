"""FP64 CPU oracle of the randomized-multiplier GENP solve (test infrastructure only).

Pan & Qian, "More on the Power of Randomized Matrix Multiplication":
section 1.1 proposes to solve A y = b by applying a random multiplier and then
Gaussian elimination with no pivoting (GENP); Corollary 4.1(ii) (section 4)
is the reason a *right* Gaussian multiplier makes every leading block of
C = A G nonsingular and well conditioned when A is nonsingular.  The method
computed here:

    C = A G                      (multiplier product, section 1.1)
    C = L U                      (GENP / block Gaussian elimination, section 1.1,
                                  Theorem 2.2 and the Schur complement of Fact 2.1)
    Y = U^{-1} L^{-1} B          (substitutions)
    X = G Y                      (so that A X = A G (AG)^{-1} B = B)
    X += G (LU)^{-1} (B - A X)   (iterative refinement, section 7.1 / Table 7.1,
                                  at most two steps per section 7.2)

Everything is plain numpy float64 with no blocking beyond what the paper's
block Gaussian elimination states.  Library primitives used as steps: the
matrix product (``@``), ``scipy.linalg.solve_triangular`` inside the block
variant, and ``numpy.linalg.solve`` (LAPACK, partial pivoting) only as the
textbook definition x = A^{-1} b in the adjoint.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

U64 = np.finfo(np.float64).eps / 2  # unit roundoff of IEEE double, 2^-53


# ---------------------------------------------------------------------------
# multiplier (Definition 3.2; Toeplitz matrices, section 2.3)
# ---------------------------------------------------------------------------

def toeplitz_from_params(p: np.ndarray, n: int) -> np.ndarray:
    """Dense n x n Toeplitz matrix G[i, j] = t_{i-j} stored as p[i - j + n - 1].

    Section 2.3 defines T = (t_{i-j}) by its first row (t_{-h}) and first
    column (t_h); p holds t_{-(n-1)} .. t_{n-1} in increasing subscript order.
    """
    p = np.asarray(p, dtype=np.float64)
    if p.shape != (2 * n - 1,):
        raise ValueError(f"need 2n-1 = {2 * n - 1} parameters, got {p.shape}")
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return p[i - j + n - 1]


def circulant_from_params(c: np.ndarray, n: int) -> np.ndarray:
    """Dense n x n circulant matrix with first column c: G[i, j] = c[(i - j) mod n]
    (the circulant class of Definition 3.2; section 2.3).  Every circulant is
    diagonalized by the DFT (Theorem 2.1), which is what makes it cheap to apply."""
    c = np.asarray(c, dtype=np.float64)
    if c.shape != (n,):
        raise ValueError("need n parameters")
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return c[(i - j) % n]


def circulant_cond(c: np.ndarray) -> float:
    """2-norm condition number of the circulant with first column c.

    Theorem 2.1: the DFT diagonalizes every circulant, whose eigenvalues are
    the DFT of its first column.  A circulant is normal, so its singular values
    are the moduli of those eigenvalues and kappa_2 = max |DFT(c)| / min |DFT(c)|
    (infinite when some DFT coefficient vanishes).  The FFT is a library step."""
    lam = np.abs(np.fft.fft(np.asarray(c, dtype=np.float64)))
    lo = lam.min()
    return float(lam.max() / lo) if lo > 0 else float("inf")


def householder_from_params(uv: np.ndarray, n: int) -> np.ndarray:
    """Dense n x n Householder-type multiplier from uv = (u, v), 2n parameters:
    G = I - 2 u v^T / (v^T u).

    The multipliers named with Table 7.1 are written as I - u v^T / u^T v; taken
    literally that matrix sends u to 0 and is singular for every u, v, so the
    factor 2 is restored: G is then the oblique reflection (G^2 = I, det G = -1),
    the classical Householder reflection when u = v."""
    uv = np.asarray(uv, dtype=np.float64)
    if uv.shape != (2 * n,):
        raise ValueError("need 2n parameters (u, v)")
    u, v = uv[:n], uv[n:]
    return np.eye(n) - (2.0 / (v @ u)) * np.outer(u, v)


def householder_cond(uv: np.ndarray) -> float:
    """2-norm condition number of I - 2 u v^T / (v^T u): with a = ||u|| ||v|| / |v^T u|,
    the singular values are 1 (n - 2 times) and a +- sqrt(a^2 - 1), so kappa_2 =
    (a + sqrt(a^2 - 1))^2 (infinite when v^T u = 0)."""
    uv = np.asarray(uv, dtype=np.float64)
    n = uv.shape[0] // 2
    u, v = uv[:n], uv[n:]
    d = abs(v @ u)
    if d == 0:
        return float("inf")
    a = max(1.0, np.linalg.norm(u) * np.linalg.norm(v) / d)
    return float((a + np.sqrt(a * a - 1.0)) ** 2)


def dense_multiplier(G: Optional[np.ndarray], p: Optional[np.ndarray], n: int) -> np.ndarray:
    """The multiplier as a dense matrix: G itself, or built from its parameters
    (2n - 1 Toeplitz parameters, n circulant parameters, or 2n Householder
    parameters (u, v))."""
    if G is not None:
        return np.asarray(G, dtype=np.float64)
    if p is not None:
        p = np.asarray(p)
        if p.shape[0] == 2 * n:
            return householder_from_params(p, n)
        return circulant_from_params(p, n) if p.shape[0] == n and n > 1 else toeplitz_from_params(p, n)
    raise ValueError("need G or p")


def precondition(A: np.ndarray, G: np.ndarray, H: Optional[np.ndarray] = None) -> np.ndarray:
    """C = A G, the right multiplier of section 1.1 / Corollary 4.1(ii); with a left
    multiplier H (the G M case of Corollary 4.1), C = H A G."""
    C = np.asarray(A, dtype=np.float64) @ np.asarray(G, dtype=np.float64)
    return C if H is None else np.asarray(H, dtype=np.float64) @ C


# ---------------------------------------------------------------------------
# GENP (section 1.1) and block Gaussian elimination (Theorem 2.2, Fact 2.1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class FactorInfo:
    """Outcome of an elimination.

    breakdown_col: 1-based index of the first pivot that is non-finite or
    has |u_kk| <= pivot_tol * max|C| (0 when none).  The elimination stops
    there, so the factors are only meaningful in rows/columns before it.
    """

    breakdown_col: int
    pivots: np.ndarray          # u_kk for k before the breakdown (all n if none)
    max_abs_c: float
    max_abs_u: float

    @property
    def growth(self) -> float:
        return self.max_abs_u / self.max_abs_c if self.max_abs_c > 0 else np.inf


def _is_breakdown(piv: float, tol_abs: float) -> bool:
    return (not np.isfinite(piv)) or abs(piv) <= tol_abs


def genp_unblocked(C: np.ndarray, pivot_tol: float = 0.0):
    """Outer-product Gaussian elimination with no pivoting (section 1.1).

    For k = 1..n: l_ik = c_ik / c_kk and c_ij -= l_ik c_kj for i, j > k.
    Returns (LU, info) with the unit lower L stored below the diagonal and
    U on and above it, the usual packed form.
    """
    LU = np.array(C, dtype=np.float64, copy=True)
    n = LU.shape[0]
    maxc = float(np.max(np.abs(LU))) if n else 0.0
    tol_abs = pivot_tol * maxc
    pivots = []
    for k in range(n):
        piv = LU[k, k]
        if _is_breakdown(piv, tol_abs):
            return LU, FactorInfo(k + 1, np.array(pivots), maxc, _max_abs_u(LU, k))
        pivots.append(piv)
        LU[k + 1:, k] /= piv
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, FactorInfo(0, np.array(pivots), maxc, _max_abs_u(LU, n))


def _max_abs_u(LU: np.ndarray, upto: int) -> float:
    if upto == 0:
        return 0.0
    return float(np.max(np.abs(np.triu(LU[:upto, :]))))


def genp_blocked(C: np.ndarray, nb: int, pivot_tol: float = 0.0):
    """Block Gaussian elimination with block size nb (Theorem 2.2).

    For each diagonal block: factor it by GENP, then L21 = C21 U11^{-1},
    U12 = L11^{-1} C12 and replace C22 by its Schur complement
    C22 - L21 U12 = C22 - C21 C11^{-1} C12 (Fact 2.1).  In exact arithmetic this is
    the same factorization as :func:`genp_unblocked`; a ragged last block is fine.
    """
    from scipy.linalg import solve_triangular

    if nb < 1:
        raise ValueError("nb >= 1")
    LU = np.array(C, dtype=np.float64, copy=True)
    n = LU.shape[0]
    maxc = float(np.max(np.abs(LU))) if n else 0.0
    pivots = []
    for k in range(0, n, nb):
        e = min(k + nb, n)
        D, inf = genp_unblocked(LU[k:e, k:e], 0.0)
        LU[k:e, k:e] = D
        # pivot test against the tolerance scaled by max|C| of the whole matrix
        for t, piv in enumerate(np.diag(D)):
            if inf.breakdown_col and t + 1 >= inf.breakdown_col:
                return LU, FactorInfo(k + t + 1, np.array(pivots), maxc, _max_abs_u(LU, k + t))
            if _is_breakdown(piv, pivot_tol * maxc):
                return LU, FactorInfo(k + t + 1, np.array(pivots), maxc, _max_abs_u(LU, k + t))
            pivots.append(piv)
        if e < n:
            L11 = np.tril(D, -1) + np.eye(e - k)
            U11 = np.triu(D)
            LU[e:, k:e] = solve_triangular(U11.T, LU[e:, k:e].T, lower=True).T
            LU[k:e, e:] = solve_triangular(L11, LU[k:e, e:], lower=True, unit_diagonal=True)
            LU[e:, e:] -= LU[e:, k:e] @ LU[k:e, e:]
    return LU, FactorInfo(0, np.array(pivots), maxc, _max_abs_u(LU, n))


def unpack(LU: np.ndarray):
    """(L, U) from the packed form: L unit lower, U upper."""
    n = LU.shape[0]
    return np.tril(LU, -1) + np.eye(n), np.triu(LU)


# ---------------------------------------------------------------------------
# substitutions, recovery, refinement (section 1.1, section 7.1)
# ---------------------------------------------------------------------------

def forward_unit(LU: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Z = L^{-1} B, L unit lower triangular (row-by-row substitution)."""
    B = np.asarray(B, dtype=np.float64)
    Z = np.array(B, copy=True).reshape(B.shape[0], -1)
    for i in range(LU.shape[0]):
        if i:
            Z[i] -= LU[i, :i] @ Z[:i]
    return Z.reshape(B.shape)


def backward_upper(LU: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Y = U^{-1} Z, U upper triangular (row-by-row substitution, bottom up)."""
    Z = np.asarray(Z, dtype=np.float64)
    Y = np.array(Z, copy=True).reshape(Z.shape[0], -1)
    n = LU.shape[0]
    for i in range(n - 1, -1, -1):
        if i < n - 1:
            Y[i] -= LU[i, i + 1:] @ Y[i + 1:]
        Y[i] /= LU[i, i]
    return Y.reshape(Z.shape)


def lu_solve(LU: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Y = U^{-1} L^{-1} B."""
    return backward_upper(LU, forward_unit(LU, B))


def solve(LU: np.ndarray, G: np.ndarray, B: np.ndarray, H: Optional[np.ndarray] = None) -> np.ndarray:
    """X = G U^{-1} L^{-1} B: the solution of A X = B from the factors of C = A G.
    With a left multiplier, C = H A G and A X = B  <=>  C (G^{-1} X) = H B, so
    X = G U^{-1} L^{-1} H B."""
    if H is not None:
        B = np.asarray(H, dtype=np.float64) @ np.asarray(B, dtype=np.float64)
    return G @ lu_solve(LU, B)


def residual(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    return B - A @ X


def backward_error_inf(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Normwise backward error per column (Rigal-Gaches, infinity norm).

    eta_j = ||b_j - A x_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf).
    """
    X2 = np.asarray(X).reshape(X.shape[0], -1)
    B2 = np.asarray(B).reshape(B.shape[0], -1)
    R = residual(A, X2, B2)
    a = np.max(np.sum(np.abs(A), axis=1))
    return np.max(np.abs(R), axis=0) / (a * np.max(np.abs(X2), axis=0) + np.max(np.abs(B2), axis=0))


def relative_residual(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """||A y - b|| / ||b|| per column (2-norm), the quantity of Table 7.1."""
    X2 = np.asarray(X).reshape(X.shape[0], -1)
    B2 = np.asarray(B).reshape(B.shape[0], -1)
    return np.linalg.norm(A @ X2 - B2, axis=0) / np.linalg.norm(B2, axis=0)


def backward_error_2(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Normwise backward error per column in the 2-norm (Rigal-Gaches):
    eta_j = ||b_j - A x_j||_2 / (||A||_2 ||x_j||_2 + ||b_j||_2), ||A||_2 from the SVD."""
    X2 = np.asarray(X).reshape(X.shape[0], -1)
    B2 = np.asarray(B).reshape(B.shape[0], -1)
    R = residual(A, X2, B2)
    a = np.linalg.norm(A, 2)
    return np.linalg.norm(R, axis=0) / (a * np.linalg.norm(X2, axis=0) + np.linalg.norm(B2, axis=0))


@dataclasses.dataclass
class SolveResult:
    X: np.ndarray
    eta_hist: list            # eta_inf (max over columns) before each step and at the end
    steps: int


def refine(A, G, LU, B, X, max_iter: int = 2, tol: float = 0.0, H: Optional[np.ndarray] = None) -> SolveResult:
    """Iterative refinement in FP64: R = B - A X, X += G (LU)^{-1} R (G (LU)^{-1} H R
    with a left multiplier H).

    Section 7.1 reports one refinement step after GENP (Table 7.1); section
    7.2 performs at most two.  Stops early when max_j eta_j <= tol.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    hist = [float(np.max(backward_error_inf(A, X, B)))]
    steps = 0
    while steps < max_iter and hist[-1] > tol:
        R = residual(A, X, B)
        X += solve(LU, G, R, H)
        steps += 1
        hist.append(float(np.max(backward_error_inf(A, X, B))))
    return SolveResult(X, hist, steps)


def genp_solve(A, B, G, nb: Optional[int] = None, refine_steps: int = 2, tol: float = 0.0,
               pivot_tol: float = 0.0, H: Optional[np.ndarray] = None):
    """The whole path: C = AG (or H A G), GENP, substitutions, X = GY, refinement."""
    C = precondition(A, G, H)
    LU, info = genp_unblocked(C, pivot_tol) if nb is None else genp_blocked(C, nb, pivot_tol)
    if info.breakdown_col:
        return None, LU, info
    X = solve(LU, G, B, H)
    res = refine(A, G, LU, B, X, refine_steps, tol, H)
    return res, LU, info


# ---------------------------------------------------------------------------
# GMRES-based refinement (the correction equation A d = r solved by GMRES,
# right-preconditioned with M^{-1} = G (LU)^{-1}, since A G (LU)^{-1} = I when
# the factors are exact).  The paper refines with the factors directly
# (section 7.1); GMRES on the correction equation is what the low-precision
# form needs when kappa(C) u_low is not small.
# ---------------------------------------------------------------------------

def gmres(matvec, precond, r: np.ndarray, restart: int, max_iter: int, rtol: float):
    """Right-preconditioned restarted GMRES for A d = r, from d = 0.

    Arnoldi on A M^{-1} with modified Gram-Schmidt, Givens rotations on the
    Hessenberg matrix, least-squares update at the end of each cycle.  Stops
    when the (rotated) residual norm is <= rtol ||r||_2 or after max_iter inner
    iterations.  Returns (d, inner iterations, residual-norm history)."""
    r = np.asarray(r, dtype=np.float64)
    n = r.shape[0]
    d = np.zeros(n)
    beta0 = np.linalg.norm(r)
    hist = [beta0]
    if beta0 == 0.0:
        return d, 0, hist
    its = 0
    while its < max_iter:
        res = r - matvec(d)
        beta = np.linalg.norm(res)
        if beta <= rtol * beta0:
            break
        m = min(restart, max_iter - its)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = res / beta
        k = 0
        for j in range(m):
            w = matvec(precond(V[:, j]))
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = w @ V[:, i]
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):                          # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])        # new rotation zeroing H[j+1, j]
            cs[j], sn[j] = (1.0, 0.0) if den == 0.0 else (H[j, j] / den, H[j + 1, j] / den)
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            its += 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * beta0 or H[j, j] == 0.0:
                break
        y = np.zeros(k)                                 # back substitution with the k x k triangle
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:]) / H[i, i]
        d = d + precond(V[:, :k] @ y)
        if hist[-1] <= rtol * beta0:
            break
    return d, its, hist


def gmres_ir(A, G, LU, B, X, restart: int = 50, max_outer: int = 10, max_inner: int = 1000,
             tol: float = 0.0, inner_rtol: float = 1e-10) -> SolveResult:
    """Refinement whose correction d solves A d = r by preconditioned GMRES:
    r = b - A x (FP64), d = GMRES(A, r; M^{-1} = G (LU)^{-1}), x += d, per column,
    until eta_inf <= tol or max_outer steps."""
    X = np.array(X, dtype=np.float64, copy=True)
    X2 = X.reshape(X.shape[0], -1)
    B2 = np.asarray(B, dtype=np.float64).reshape(B.shape[0], -1)
    hist = [float(np.max(backward_error_inf(A, X2, B2)))]
    steps = 0
    inner = 0
    while steps < max_outer and hist[-1] > tol:
        for c in range(X2.shape[1]):
            r = B2[:, c] - A @ X2[:, c]
            d, its, _ = gmres(lambda v: A @ v, lambda v: solve(LU, G, v), r, restart, max_inner, inner_rtol)
            inner += its
            X2[:, c] += d
        steps += 1
        hist.append(float(np.max(backward_error_inf(A, X2, B2))))
    res = SolveResult(X2.reshape(X.shape), hist, steps)
    res.inner = inner
    return res


# ---------------------------------------------------------------------------
# adjoint (the differentiation form: gradient of L = sum(W * X), X = A^{-1} B)
# ---------------------------------------------------------------------------

def adjoint(A: np.ndarray, X: np.ndarray, W: np.ndarray):
    """dB = A^{-T} W and dA = -dB X^T.

    From d(A^{-1}B) = -A^{-1} dA A^{-1} B + A^{-1} dB: with L = sum(W * X),
    dL = <A^{-T} W, dB> - <A^{-T} W X^T, dA>.  Uses the textbook solve
    (LAPACK partial pivoting) for A^{-T} W.
    """
    dB = np.linalg.solve(np.asarray(A).T, W)
    return dB, -dB @ np.asarray(X).T


# ---------------------------------------------------------------------------
# quantities the tests report
# ---------------------------------------------------------------------------

def factor_residual(C: np.ndarray, LU: np.ndarray):
    """(||C - LU||_F / ||C||_F, ||C - LU||_F / || |L||U| ||_F)."""
    L, U = unpack(LU)
    E = C - L @ U
    e = np.linalg.norm(E)
    return e / np.linalg.norm(C), e / np.linalg.norm(np.abs(L) @ np.abs(U))


def gamma(n: int, u: float = U64) -> float:
    """gamma_n = n u / (1 - n u), the constant of standard rounding-error bounds."""
    return n * u / (1 - n * u)
