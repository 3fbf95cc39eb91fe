"""Pins of the numerical-rank oracle (Proto-Algorithm B.1, Remarks B.2 / B.4)."""
import inspect
import math
import textwrap

import numpy as np
import pytest

from oracle import nrank as onr
from paper_1212_4560_amd import workloads as wl


def test_sturm_extremes_against_eigvalsh():
    g = np.random.default_rng(1)
    for k in (1, 2, 7, 40):
        al = g.standard_normal(k)
        be = g.standard_normal(k - 1)
        T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
        ev = np.linalg.eigvalsh(T)
        lo, hi = onr.tridiag_extremes(al, be)
        assert np.isclose(lo, ev[0], rtol=0, atol=1e-12 * max(1, abs(ev).max()))
        assert np.isclose(hi, ev[-1], rtol=0, atol=1e-12 * max(1, abs(ev).max()))
        for x in (ev[0] - 1, 0.5 * (ev[0] + ev[-1]) + 1e-7, ev[-1] + 1):
            assert onr.sturm_count(al, be, x) == int(np.sum(ev < x))


def test_lanczos_cond_against_svd():
    """Remark B.2's COND (Lanczos on B^T B without reorthogonalization, Sturm bisection) against
    kappa_2 from the SVD: accurate for spectra graded up to kappa 1e3 (a lower bound, since Ritz
    values lie inside the spectrum), and -- the case the rank search meets at s = nrank + 1 --
    an isolated singular value of 1e-10 is found (its square is at the rounding level of S,
    so the estimate is huge or infinite)."""
    g = np.random.default_rng(2)
    for s, kap, rtol in ((1, 1.0, 1e-12), (5, 10.0, 1e-8), (16, 1e2, 1e-6), (40, 1e3, 1e-6), (64, 1e3, 1e-2)):
        U = np.linalg.qr(g.standard_normal((200, s)))[0]
        V = np.linalg.qr(g.standard_normal((s, s)))[0]
        sig = np.logspace(0, -np.log10(kap), s) if s > 1 else np.ones(1)
        B = (U * sig) @ V.T
        k = onr.cond_lanczos(B, g.standard_normal(s))
        assert np.isclose(k, onr.cond_svd(B), rtol=rtol) and k <= onr.cond_svd(B) * (1 + 1e-9)
    for s in (9, 33, 64):
        U = np.linalg.qr(g.standard_normal((300, s)))[0]
        V = np.linalg.qr(g.standard_normal((s, s)))[0]
        sig = 1.0 / np.arange(1, s + 1)
        sig[-1] = 1e-10
        B = (U * sig) @ V.T
        assert onr.cond_lanczos(B, g.standard_normal(s)) >= 1e7   # lambda_min(S) ~ 1e-20: at the rounding level


@pytest.mark.parametrize("q", [1, 8, 32])
def test_sketch_conditioning_switches_at_the_numerical_rank(q):
    """Property (a) of Appendix B as read here: kappa(A^T G_s) stays small for s <= nrank(A) and
    jumps by orders of magnitude at s = nrank(A) + 1 (Table 7.2's matrices, tail 1e-10)."""
    n = 128
    A, S, sig, T, G = wl.svd_head_matrix(n, q, seed=3, rho_plus=min(n, q + 8))
    sk = A.T @ G
    ks = [onr.cond_svd(sk[:, :s]) for s in range(1, q + 2)]
    assert max(ks[:q]) <= 1e5
    assert ks[q] >= 1e6 * max(ks[:q]) ** 0.5


@pytest.mark.parametrize("q,lo,hi", [(1, 0, 40), (8, 0, 40), (17, 3, 40), (32, 0, 64), (40, 0, 40)])
def test_bisection_finds_the_numerical_rank(q, lo, hi):
    """The bisection returns nrank(A) = q (exact-rank and tail-1e-10 matrices) in at most
    ceil(log2(hi - lo + 1)) tests; with Remark B.2's COND the same rank; the basis is A^T G_q."""
    n = 96
    g = np.random.default_rng(q)
    for A in (g.standard_normal((n + 20, q)) @ g.standard_normal((q, n)),
              wl.svd_head_matrix(n, q, seed=q)[0]):
        G = g.standard_normal((A.shape[0], hi))
        r = onr.numerical_rank(A, G, lo, hi, 1e6)
        assert r.rank == q
        assert len(r.tests) <= math.ceil(math.log2(hi - lo + 1))
        assert np.allclose(r.B, A.T @ G[:, :q])
        r2 = onr.numerical_rank(A, G, lo, hi, 1e6, cond="lanczos")
        assert r2.rank == q


def test_full_rank_and_zero_matrix():
    g = np.random.default_rng(5)
    A = g.standard_normal((50, 30))
    assert onr.numerical_rank(A, g.standard_normal((50, 30)), 0, 30, 1e6).rank == 30
    Z = np.zeros((50, 30))
    assert onr.numerical_rank(Z, g.standard_normal((50, 30)), 0, 30, 1e6).rank == 0


# -------------------------------------------------------------- planted mistakes ----

def _checks():
    out = []
    g = np.random.default_rng(9)
    A = g.standard_normal((60, 7)) @ g.standard_normal((7, 50))
    try:
        out.append(onr.numerical_rank(A, g.standard_normal((60, 30)), 0, 30, 1e6).rank == 7)
    except Exception:
        out.append(False)
    try:
        B = g.standard_normal((80, 6)) @ np.diag([1, 1e-1, 1e-2, 1e-3, 1e-4, 1e-5])
        out.append(np.isclose(onr.cond_lanczos(B, np.ones(6)), onr.cond_svd(B), rtol=1e-6))
    except Exception:
        out.append(False)
    try:
        al, be = np.array([2.0, 3.0, 1.0]), np.array([0.5, -0.7])
        T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
        ev = np.linalg.eigvalsh(T)
        lo, hi = onr.tridiag_extremes(al, be)
        out.append(np.isclose(lo, ev[0]) and np.isclose(hi, ev[-1]))
    except Exception:
        out.append(False)
    return out


MUTANTS = {
    "update rule as printed (pass lowers the upper end)": ("numerical_rank", "            lo = s\n        else:\n            hi = s - 1",
                                                           "            hi = s\n        else:\n            lo = s"),
    "COND test inverted": ("numerical_rank", "ok = k <= cond_max", "ok = k >= cond_max"),
    "Sturm recurrence without the off-diagonal term": ("sturm_count", "d = (alpha[i] - x) - (b2 / d if i else 0.0)",
                                                       "d = (alpha[i] - x)"),
    "Lanczos without the three-term correction": ("lanczos_tridiag", "w = S @ v - b * v_prev", "w = S @ v"),
    "kappa from the eigenvalues without the square root": ("cond_lanczos", "return float(math.sqrt(lmax / lmin))",
                                                            "return float(lmax / lmin)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(onr, attr)))
    assert old in src, old
    ns = dict(vars(onr))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    monkeypatch.setattr(onr, attr, ns[attr])
    assert not all(_checks()), f"mutant not caught: {name}"


def test_checks_pass_on_the_oracle():
    assert all(_checks())
