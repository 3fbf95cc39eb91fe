"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant replaces one oracle function with a plausibly wrong version (a
dropped term, a wrong sign, a wrong index, a transposed operand) and the test
asserts that at least one of the independent checks below fails with it and
that all of them pass without it.
"""
import inspect
import json
import os
import textwrap

import numpy as np
import pytest

from oracle import exact, genp as og

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _arr(x):
    return np.array(x, dtype=np.float64)


# ------------------------------------------------------------------ checks ----

def check_golden():
    g = json.load(open(GOLDEN))
    e = g["genp_3x3"]
    LU, _ = og.genp_unblocked(_arr(e["C"]))
    L, U = og.unpack(LU)
    ok = np.array_equal(L, _arr(e["L"])) and np.array_equal(U, _arr(e["U"]))
    ok &= np.allclose(og.lu_solve(LU, _arr(e["b"])), _arr(e["x"]))
    r = g["right_multiplier_repairs_it"]
    C = og.precondition(_arr(r["A"]), _arr(r["G"]))
    ok &= np.array_equal(C, _arr(r["C"]))
    LU, _ = og.genp_unblocked(_arr(r["C"]))
    ok &= np.allclose(og.solve(LU, _arr(r["G"]), _arr(r["b"])), _arr(r["x"]))
    t = g["toeplitz_3x3"]
    ok &= np.array_equal(og.toeplitz_from_params(_arr(t["p"]), 3), _arr(t["T"]))
    return bool(ok)


def check_exact():
    g = np.random.default_rng(5)
    n = 5
    A, G, b = g.standard_normal((n, n)), g.standard_normal((n, n)), g.standard_normal((n, 1))
    C = og.precondition(A, G)
    Ce = exact.to_float(exact.matmul(exact.to_frac(A), exact.to_frac(G)))
    if not np.all(np.abs(C - Ce) <= og.gamma(n) * (np.abs(A) @ np.abs(G))):
        return False
    Le, Ue, _ = exact.genp(exact.to_frac(C))
    LU, _ = og.genp_unblocked(C)
    L, U = og.unpack(LU)
    if np.max(np.abs(L - exact.to_float(Le))) > 1e-9 or np.max(np.abs(U - exact.to_float(Ue))) > 1e-9 * np.max(np.abs(U)):
        return False
    xc = exact.to_float(exact.cramer(exact.to_frac(A), exact.to_frac(b)))
    res, _, _ = og.genp_solve(A, b, G, refine_steps=2)
    return bool(res is not None and np.max(np.abs(res.X - xc)) <= 1e-10 * np.max(np.abs(xc)))


def check_gepp_and_eta():
    g = np.random.default_rng(7)
    n = 64
    A = g.standard_normal((n, n))
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, 2))
    res, _, info = og.genp_solve(A, B, G, nb=16, refine_steps=2)
    if res is None:
        return False
    Xp = np.linalg.solve(A, B)
    ok = np.max(np.abs(res.X - Xp)) <= 1e-10 * np.max(np.abs(Xp))
    # eta against an independent computation with library norms
    R = B - A @ res.X
    eta = np.array([np.linalg.norm(R[:, j], np.inf) / (np.linalg.norm(A, np.inf) * np.linalg.norm(res.X[:, j], np.inf)
                                                       + np.linalg.norm(B[:, j], np.inf)) for j in range(2)])
    ok &= np.allclose(og.backward_error_inf(A, res.X, B), eta, rtol=1e-12, atol=0)
    ok &= res.eta_hist[-1] <= 1e-14
    return bool(ok)


def check_toeplitz_scipy():
    from scipy.linalg import toeplitz
    n = 9
    p = np.random.default_rng(2).standard_normal(2 * n - 1)
    return bool(np.array_equal(og.toeplitz_from_params(p, n), toeplitz(p[n - 1:], p[n - 1::-1])))


def check_blocked():
    g = np.random.default_rng(4)
    n = 37
    C = g.standard_normal((n, n)) + 2 * n * np.eye(n)
    a, _ = og.genp_unblocked(C)
    b, _ = og.genp_blocked(C, 8)
    L, U = og.unpack(b)
    return bool(np.allclose(a, b, rtol=0, atol=1e-12) and np.allclose(L @ U, C, rtol=0, atol=1e-10))


def check_adjoint_fd():
    g = np.random.default_rng(6)
    n, k = 12, 2
    A = g.standard_normal((n, n)) + 3 * np.eye(n)
    B, W = g.standard_normal((n, k)), g.standard_normal((n, k))
    X = np.linalg.solve(A, B)
    dB, dA = og.adjoint(A, X, W)

    def L(Am, Bm):
        return float(np.sum(W * np.linalg.solve(Am, Bm)))
    h = 1e-6
    E = np.zeros((n, n))
    E[3, 7] = h
    fa = (L(A + E, B) - L(A - E, B)) / (2 * h)
    Eb = np.zeros((n, k))
    Eb[5, 1] = h
    fb = (L(A, B + Eb) - L(A, B - Eb)) / (2 * h)
    return bool(abs(fa - dA[3, 7]) <= 1e-6 * max(1, abs(fa)) and abs(fb - dB[5, 1]) <= 1e-6 * max(1, abs(fb)))


def check_eta2():
    c, s_ = np.cos(np.pi / 6), np.sin(np.pi / 6)
    A = np.array([[c, -s_], [s_, c]]) @ np.diag([3.0, 1.0])
    x = np.array([[0.25], [0.0]])
    b = np.array([[1.0], [0.0]])
    r = np.array([1.0 - 0.75 * c, -0.75 * s_])
    return bool(abs(og.backward_error_2(A, x, b)[0] - np.sqrt(r @ r) / 1.75) <= 1e-15)


def check_gmres():
    g = np.random.default_rng(4)
    n = 30
    A = g.standard_normal((n, n)) + 6 * np.eye(n)
    r = g.standard_normal(n)
    for k in (2, 3):
        d, _, _ = og.gmres(lambda v: A @ v, lambda v: v, r, restart=n, max_iter=k, rtol=0.0)
        K = np.stack([np.linalg.matrix_power(A, j) @ r for j in range(k)], axis=1)
        c, *_ = np.linalg.lstsq(A @ K, r, rcond=None)
        if abs(np.linalg.norm(r - A @ d) - np.linalg.norm(r - A @ K @ c)) > 1e-10 * np.linalg.norm(r):
            return False
    # preconditioned refinement with perturbed factors must reach eta <= 1e-14
    g = np.random.default_rng(6)
    n = 32
    A = g.standard_normal((n, n))
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, 1))
    LU, _ = og.genp_unblocked(og.precondition(A, G))
    LUp = LU * (1 + 1e-4 * g.standard_normal(LU.shape))
    res = og.gmres_ir(A, G, LUp, B, og.solve(LUp, G, B), restart=10, max_outer=4, tol=1e-14)
    return bool(res.eta_hist[-1] <= 1e-14)


def check_circulant():
    from scipy.linalg import circulant
    n = 10
    c = np.random.default_rng(3).standard_normal(n)
    G = og.circulant_from_params(c, n)
    v = np.exp(2j * np.pi * np.arange(n) * 2 / n)
    return bool(np.array_equal(G, circulant(c)) and np.allclose(G @ v, np.fft.fft(c)[2] * v, atol=1e-12))


def check_circulant_cond():
    n = 9
    c = np.random.default_rng(5).standard_normal(n)
    return bool(np.isclose(og.circulant_cond(c), np.linalg.cond(og.circulant_from_params(c, n)), rtol=1e-9))


def check_householder():
    n = 7
    g = np.random.default_rng(6)
    uv = g.standard_normal(2 * n)
    G = og.householder_from_params(uv, n)
    return bool(np.allclose(G @ G, np.eye(n), atol=1e-12) and np.allclose(G @ uv[:n], -uv[:n], atol=1e-12)
                and np.isclose(og.householder_cond(uv), np.linalg.cond(G), rtol=1e-8))


def check_left():
    n = 12
    g = np.random.default_rng(7)
    A, H, G, B = (g.standard_normal((n, n)), g.standard_normal((n, n)), g.standard_normal((n, n)),
                  g.standard_normal((n, 2)))
    LU, _ = og.genp_unblocked(og.precondition(A, G, H))
    X = og.solve(LU, G, B, H)
    res = og.refine(A, G, LU, B, X + 1e-6, 1, 0.0, H)
    x0 = np.linalg.solve(A, B)
    return bool(np.allclose(X, x0, atol=1e-8) and np.allclose(res.X, x0, atol=1e-8))


CHECKS = [check_golden, check_exact, check_gepp_and_eta, check_toeplitz_scipy, check_blocked, check_adjoint_fd,
          check_eta2, check_gmres, check_circulant, check_circulant_cond, check_householder, check_left]


def run_checks():
    out = []
    for c in CHECKS:
        try:
            with np.errstate(all="ignore"):
                out.append(c())
        except Exception:
            out.append(False)
    return out


# ----------------------------------------------------------------- mutants ----

def _genp_sign(C, pivot_tol=0.0):
    LU = np.array(C, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for k in range(n):
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] += np.outer(LU[k + 1:, k], LU[k, k + 1:])      # wrong sign
    return LU, og.FactorInfo(0, np.diag(LU), float(np.max(np.abs(C))), 1.0)


def _genp_no_divide(C, pivot_tol=0.0):
    LU = np.array(C, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for k in range(n):
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k] / LU[k, k], LU[k, k + 1:])  # multipliers not stored
    return LU, og.FactorInfo(0, np.diag(LU), float(np.max(np.abs(C))), 1.0)


def _genp_index(C, pivot_tol=0.0):
    LU = np.array(C, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for k in range(n):
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k:-1])         # pivot row shifted by one
    return LU, og.FactorInfo(0, np.diag(LU), float(np.max(np.abs(C))), 1.0)


def _forward_transposed(LU, B):
    B = np.asarray(B, dtype=np.float64)
    Z = np.array(B, copy=True).reshape(B.shape[0], -1)
    for i in range(LU.shape[0]):
        if i:
            Z[i] -= LU[:i, i] @ Z[:i]                                       # column instead of row
    return Z.reshape(B.shape)


def _backward_no_divide(LU, Z):
    Z = np.asarray(Z, dtype=np.float64)
    Y = np.array(Z, copy=True).reshape(Z.shape[0], -1)
    n = LU.shape[0]
    for i in range(n - 1, -1, -1):
        if i < n - 1:
            Y[i] -= LU[i, i + 1:] @ Y[i + 1:]                              # diagonal never divided
    return Y.reshape(Z.shape)


def _precondition_left(A, G):
    return np.asarray(G) @ np.asarray(A)                                   # wrong side


def _toeplitz_transposed(p, n):
    p = np.asarray(p, dtype=np.float64)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return p[j - i + n - 1]                                                # t_{j-i}


def _solve_no_recovery(LU, G, B):
    return og.lu_solve(LU, B)                                              # forgets x = G y


def _residual_sign(A, X, B):
    return A @ X - B                                                       # wrong sign


def _eta_onenorm(A, X, B):
    X2 = np.asarray(X).reshape(X.shape[0], -1)
    B2 = np.asarray(B).reshape(B.shape[0], -1)
    R = B2 - A @ X2
    a = np.max(np.sum(np.abs(A), axis=0))                                  # column sums (1-norm)
    return np.max(np.abs(R), axis=0) / (a * np.max(np.abs(X2), axis=0) + np.max(np.abs(B2), axis=0))


def _adjoint_no_transpose(A, X, W):
    dB = np.linalg.solve(np.asarray(A), W)                                 # A instead of A^T
    return dB, -dB @ np.asarray(X).T


def _adjoint_sign(A, X, W):
    dB = np.linalg.solve(np.asarray(A).T, W)
    return dB, dB @ np.asarray(X).T                                        # lost minus sign


def _blocked_transposed_l21(C, nb, pivot_tol=0.0):
    from scipy.linalg import solve_triangular
    LU = np.array(C, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for k in range(0, n, nb):
        e = min(k + nb, n)
        D, _ = og.genp_unblocked(LU[k:e, k:e])
        LU[k:e, k:e] = D
        if e < n:
            L11 = np.tril(D, -1) + np.eye(e - k)
            U11 = np.triu(D)
            LU[e:, k:e] = solve_triangular(U11, LU[e:, k:e].T, lower=False).T   # U11 instead of U11^T
            LU[k:e, e:] = solve_triangular(L11, LU[k:e, e:], lower=True, unit_diagonal=True)
            LU[e:, e:] -= LU[e:, k:e] @ LU[k:e, e:]
    return LU, og.FactorInfo(0, np.diag(LU), float(np.max(np.abs(C))), 1.0)


def _from_source(fn, old, new):
    """A copy of oracle function fn with one source line changed (the planted mistake)."""
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, old
    ns = dict(vars(og))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    return ns[fn.__name__]


SOURCE_MUTANTS = {
    "gmres: Gram-Schmidt adds the projection": (
        "gmres", "w = w - H[i, j] * V[:, i]", "w = w + H[i, j] * V[:, i]"),
    "gmres: rotated right-hand side loses its sign": (
        "gmres", "g[j + 1] = -sn[j] * g[j]", "g[j + 1] = sn[j] * g[j]"),
    "gmres: back substitution adds instead of subtracting": (
        "gmres", "y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:]) / H[i, i]",
        "y[i] = (g[i] + H[i, i + 1:k] @ y[i + 1:]) / H[i, i]"),
    "gmres: preconditioner not applied to the correction": (
        "gmres", "d = d + precond(V[:, :k] @ y)", "d = d + V[:, :k] @ y"),
    "gmres: earlier rotation applied with the wrong sign": (
        "gmres", "H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]",
        "H[i + 1, j] = sn[i] * H[i, j] + cs[i] * H[i + 1, j]"),
    "eta_2: Frobenius norm of A": (
        "backward_error_2", "a = np.linalg.norm(A, 2)", "a = np.linalg.norm(A)"),
    "circulant_cond: real part of the spectrum instead of its modulus": (
        "circulant_cond", "lam = np.abs(np.fft.fft(", "lam = np.real(np.fft.fft("),
    "circulant_cond: ratio upside down": (
        "circulant_cond", "return float(lam.max() / lo)", "return float(lo / lam.max())"),
    "householder: the literal formula (factor 2 dropped)": (
        "householder_from_params", "(2.0 / (v @ u))", "(1.0 / (v @ u))"),
    "householder: rank-one term added": (
        "householder_from_params", "np.eye(n) - (2.0", "np.eye(n) + (2.0"),
    "householder_cond: reciprocal of the largest singular value": (
        "householder_cond", "return float((a + np.sqrt(a * a - 1.0)) ** 2)", "return float(a + np.sqrt(a * a - 1.0))"),
    "left multiplier: applied after the substitutions": (
        "solve", "        B = np.asarray(H, dtype=np.float64) @ np.asarray(B, dtype=np.float64)\n    return G @ lu_solve(LU, B)",
        "        return G @ (np.asarray(H, dtype=np.float64) @ lu_solve(LU, B))\n    return G @ lu_solve(LU, B)"),
    "left multiplier: dropped from the product": (
        "precondition", "return C if H is None else np.asarray(H, dtype=np.float64) @ C", "return C"),
    "circulant: transposed index": (
        "circulant_from_params", "return c[(i - j) % n]", "return c[(j - i) % n]"),
    "gmres_ir: residual with the wrong sign": (
        "gmres_ir", "r = B2[:, c] - A @ X2[:, c]", "r = A @ X2[:, c] - B2[:, c]"),
}

MUTANTS = {
    "genp: wrong sign in the Schur update": ("genp_unblocked", _genp_sign),
    "genp: multipliers not stored": ("genp_unblocked", _genp_no_divide),
    "genp: pivot row off by one": ("genp_unblocked", _genp_index),
    "forward substitution: transposed operand": ("forward_unit", _forward_transposed),
    "back substitution: no division by u_ii": ("backward_upper", _backward_no_divide),
    "precondition: multiplier on the left": ("precondition", _precondition_left),
    "Toeplitz: transposed index": ("toeplitz_from_params", _toeplitz_transposed),
    "solve: recovery x = G y dropped": ("solve", _solve_no_recovery),
    "refinement: residual sign": ("residual", _residual_sign),
    "backward error: 1-norm of A": ("backward_error_inf", _eta_onenorm),
    "adjoint: A instead of A^T": ("adjoint", _adjoint_no_transpose),
    "adjoint: lost minus sign on dA": ("adjoint", _adjoint_sign),
    "block GE: L21 with U11 not transposed": ("genp_blocked", _blocked_transposed_l21),
}


def test_all_checks_pass_on_the_oracle():
    assert all(run_checks())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(og, attr, fn)
    res = run_checks()
    assert not all(res), f"mutant not caught: {name}"


@pytest.mark.parametrize("name", sorted(SOURCE_MUTANTS))
def test_source_mutant_is_caught(name, monkeypatch):
    attr, old, new = SOURCE_MUTANTS[name]
    monkeypatch.setattr(og, attr, _from_source(getattr(og, attr), old, new))
    res = run_checks()
    assert not all(res), f"mutant not caught: {name}"
