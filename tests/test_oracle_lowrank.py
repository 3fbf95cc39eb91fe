"""Pins of the low-rank oracle (Proto-Algorithm 5.1, Theorems 5.1 / 5.2, Remarks 5.2 / 5.4)
against closed forms, exact-rank matrices and library routines; and planted mistakes in
copies of it that the pins must catch."""
import inspect
import textwrap

import numpy as np
import pytest

from oracle import lowrank as ol
from paper_1212_4560_amd import workloads as wl


def test_theorem_5_1_projection_residuals():
    """For exact bases of the leading right singular space, ||A - A T T^T||_2 = sigma_{rho+1}
    and, for any nonsingular mixing U of the basis, ||A - A T (T^T T)^{-1} T^T||_2 is the same;
    in the Frobenius norm both equal sqrt(sum_{j > rho} sigma_j^2)."""
    n, rho = 40, 6
    g = np.random.default_rng(1)
    S = np.linalg.qr(g.standard_normal((n, n)))[0]
    T = np.linalg.qr(g.standard_normal((n, n)))[0]
    sig = np.sort(g.uniform(0.1, 2.0, n))[::-1]
    A = (S * sig) @ T.T
    Tr = T[:, :rho]
    U = g.standard_normal((rho, rho))
    for B, orth in ((Tr, True), (Tr @ U, False)):
        assert np.isclose(ol.projection_residual(A, B, orth), sig[rho], rtol=1e-10)
        assert np.isclose(ol.projection_residual(A, B, orth, "fro"), np.sqrt(np.sum(sig[rho:] ** 2)), rtol=1e-10)


def test_exact_rank_matrix_is_recovered():
    """A of exact rank rho (A = X Y^T): Stage 2 finds s = rho (with oversampling) and the
    residual is at the rounding level."""
    m, n, rho = 70, 50, 5
    g = np.random.default_rng(2)
    A = g.standard_normal((m, rho)) @ g.standard_normal((rho, n))
    r = ol.lowrank(A, g.standard_normal((m, rho + 4)), tau=1e-10, tau2=1e-10)
    assert r.rank == rho and not r.failed
    assert r.resid_fro <= 1e-13 * r.a_fro
    assert np.allclose(r.T.T @ r.T, np.eye(rho), atol=1e-13)
    assert np.allclose(r.W, A @ r.T, atol=1e-13)


@pytest.mark.parametrize("q", [1, 8, 32])
def test_rank_and_remark_5_2_bound_on_table_7_2_matrices(q):
    """sigma_j = 1/j (j <= q), 1e-10 beyond: Stage 2 picks s = q, and with oversampling 5 the
    residual obeys the bound of Remark 5.2, ||A - A T T^T||_2 <= (1 + 9 sqrt(rho_+ n)) sigma_{q+1}
    (it holds with probability >= 1 - 3 * 5^-5 per draw); without oversampling the basis from
    A^T G alone still gives a residual of order sigma_{q+1} (Theorem 5.2)."""
    n = 128
    plain = []
    for seed in range(6):
        A, S, sig, T, G = wl.svd_head_matrix(n, q, seed=seed, rho_plus=q + 5)
        r = ol.lowrank(A, G, tau=1e-8, tau2=1e-4)
        assert r.rank == q and not r.failed
        assert ol.projection_residual(A, r.T) <= (1 + 9 * np.sqrt((q + 5) * n)) * sig[q]
        A0, _, sig0, _, G0 = wl.svd_head_matrix(n, q, seed=100 + seed)
        r0 = ol.lowrank(A0, G0, tau=1e-8, tau2=1e-4)
        assert r0.rank == q
        plain.append(ol.projection_residual(A0, r0.T) / sig0[q])
    # without oversampling the factor kappa(V) of Theorem 5.2(iii) varies from draw to draw
    # (Table 7.2 reaches 1.45e-6 at q = 32, n = 128): typically 1e2-1e3, rarely 1e5
    assert np.median(plain) <= 1e4 and max(plain) <= 1e6


def test_toeplitz_rect_convention_against_scipy():
    from scipy.linalg import toeplitz
    m, k = 9, 4
    p = np.random.default_rng(3).standard_normal(m + k - 1)
    G = ol.toeplitz_rect(p, m, k)
    assert np.array_equal(G, toeplitz(p[k - 1:], p[k - 1::-1]))


def test_tail_is_the_truncation_residual():
    """||R[s:, s:]||_F equals the Frobenius distance from T' P to its truncation Q_s R[:s, :]."""
    g = np.random.default_rng(4)
    Tp = g.standard_normal((60, 3)) @ g.standard_normal((3, 10)) + 1e-9 * g.standard_normal((60, 10))
    s, Q, perm, tail = ol.rank_revealing(Tp, 1e-6)
    from scipy.linalg import qr
    Qf, R, pf = qr(Tp, mode="economic", pivoting=True)
    assert s == 3 and np.array_equal(perm, pf)
    assert np.isclose(tail, np.linalg.norm(Tp[:, pf] - Qf[:, :s] @ R[:s, :]), rtol=1e-6)


def test_failure_is_reported():
    A, S, sig, T, G = wl.svd_head_matrix(64, 8, seed=5)
    assert ol.lowrank(A, G, tau=1e-8, tau2=1e-30).failed
    r = ol.lowrank(A, G, tau=10.0, tau2=1e-5)   # tolerance so loose that no column is kept
    assert r.rank == 0 and r.failed


# -------------------------------------------------------------- planted mistakes ----

def _checks():
    out = []
    g = np.random.default_rng(9)
    A = g.standard_normal((30, 5)) @ g.standard_normal((5, 20))
    try:
        r = ol.lowrank(A, g.standard_normal((30, 7)), 1e-10, 1e-10)
        out.append(r.rank == 5 and r.resid_fro <= 1e-12 * r.a_fro and not r.failed)
    except Exception:
        out.append(False)
    try:
        A2, S, sig, T, G = wl.svd_head_matrix(64, 8, seed=3, rho_plus=12)
        r2 = ol.lowrank(A2, G, 1e-8, 1e-5)
        out.append(r2.rank == 8 and ol.projection_residual(A2, r2.T) <= 1e3 * sig[8])
    except Exception:
        out.append(False)
    return out


MUTANTS = {
    "sketch of A instead of A^T": ("sketch", "np.asarray(A, dtype=np.float64).T @", "np.asarray(A, dtype=np.float64) @"),
    "projection without the transpose of the basis": ("lowrank", "resid = float(np.linalg.norm(A - W @ T.T))",
                                                      "resid = float(np.linalg.norm(A - W @ T[:W.shape[1]]))"),
    "tail measured from the wrong corner": ("rank_revealing", "tail = float(np.linalg.norm(R[s:, s:]))",
                                            "tail = float(np.linalg.norm(R[:s, :s]))"),
    "rank one too small": ("rank_revealing", "return s, Q[:, :s], perm, tail", "return max(s - 1, 0), Q[:, :max(s - 1, 0)], perm, tail"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(ol, attr)))
    assert old in src
    ns = dict(vars(ol))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    monkeypatch.setattr(ol, attr, ns[attr])
    assert not all(_checks()), f"mutant not caught: {name}"


def test_checks_pass_on_the_oracle():
    assert all(_checks())
