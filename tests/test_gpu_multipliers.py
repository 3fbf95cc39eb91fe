"""Householder-type multipliers and left / two-sided multipliers (C = H A G), through the C ABI.

Products are compared entrywise with the oracle's dense products.  Bound, for C = H (A G)
computed as two products (GEMM, FFT or rank-1 pass, each within gamma_n of its operands'
absolute values): |C - C_oracle| <= 4 gamma_n (|H| |A| |G|) plus, for a circulant factor, the
FFT term (10 log2 n + 10) u max|DFT c| times the 2-norm of the transformed vector.
"""
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import genp as og  # noqa: E402
from paper_1212_4560_amd import genp, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

U64 = og.U64


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _draw(kind, n, g):
    """(parameters, dense matrix) of a multiplier of the given kind."""
    if kind == "dense":
        G = g.standard_normal((n, n))
        return G, G
    if kind == "toeplitz":
        p = g.standard_normal(2 * n - 1)
        return p, og.toeplitz_from_params(p, n)
    if kind == "circulant":
        c = g.standard_normal(n)
        return c, og.circulant_from_params(c, n)
    if kind == "householder":
        uv = g.standard_normal(2 * n)
        return uv, og.householder_from_params(uv, n)
    return None, np.eye(n)


def _right_kw(kind, par):
    return {"dense": {"G": par}, "toeplitz": {"p": par}, "circulant": {"c": par},
            "householder": {"uv": par}}.get(kind, {})


def _fft_term(c, X, axis):
    n = X.shape[0]
    return (10 * np.log2(n) + 10) * U64 * np.max(np.abs(np.fft.fft(c))) * np.linalg.norm(X, axis=axis)


def _bound(A, Hd, Gd, lk, hpar, rk, gpar):
    n = A.shape[0]
    b = 4 * og.gamma(n) * (np.abs(Hd) @ (np.abs(A) @ np.abs(Gd)))
    if rk == "circulant":
        b += np.abs(Hd) @ np.repeat(_fft_term(gpar, A, 1)[:, None], n, axis=1)
    if lk == "circulant":
        T = A @ Gd
        b += np.repeat(_fft_term(hpar, T, 0)[None, :], n, axis=0)
    return b


@pytest.mark.parametrize("n", [1, 7, 64, 200, 517])
def test_householder_product_entrywise(n):
    g = np.random.default_rng(40 + n)
    A = g.standard_normal((n, n))
    uv, Gd = _draw("householder", n, g)
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(A), uv=dev(uv))
    C = host(s.work())
    err = np.abs(C - og.precondition(A, Gd))
    assert np.all(err <= _bound(A, np.eye(n), Gd, None, None, "householder", uv))
    k = s.info()["cond_g"]
    assert abs(k - og.householder_cond(uv)) <= 1e-9 * og.householder_cond(uv)


def test_householder_product_fp32():
    n = 300
    g = np.random.default_rng(41)
    A = g.standard_normal((n, n))
    uv, Gd = _draw("householder", n, g)
    s = genp.Solver(n, "f32", 64)
    s.precondition(dev(A), uv=dev(uv))
    Co = og.precondition(A, Gd)
    assert np.all(np.abs(host(s.work()) - Co) <= 2.0 ** -24 * np.abs(Co) + _bound(A, np.eye(n), Gd, None, None, "h", None))


def test_householder_singular_rejected():
    """v^T u = 0 (u all ones, v alternating signs): ESINGULAR, context left unpreconditioned."""
    n = 128
    uv = np.concatenate([np.ones(n), (-1.0) ** np.arange(n)])
    assert og.householder_cond(uv) == float("inf")
    s = genp.Solver(n, "f64", 64)
    A = dev(np.random.default_rng(1).standard_normal((n, n)))
    with pytest.raises(genp.GenpError) as e:
        s.precondition(A, uv=dev(uv))
    assert e.value.status == genp.ESINGULAR
    with pytest.raises(genp.GenpError) as e:
        s.factor()
    assert e.value.status == genp.ESTATE


@pytest.mark.parametrize("lk,rk", [("dense", None), ("toeplitz", None), ("circulant", None), ("householder", None),
                                   ("dense", "toeplitz"), ("toeplitz", "dense"), ("circulant", "toeplitz"),
                                   ("householder", "toeplitz"), ("householder", "circulant"),
                                   ("dense", "householder")])
@pytest.mark.parametrize("n", [64, 256])
def test_left_and_two_sided_products_entrywise(lk, rk, n):
    print(f"C = H A G: left {lk}, right {rk}, n={n}", flush=True)
    g = np.random.default_rng(zlib.crc32(f"{lk}/{rk}/{n}".encode()))
    A = g.standard_normal((n, n))
    hpar, Hd = _draw(lk, n, g)
    gpar, Gd = _draw(rk, n, g)
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(A), left=(lk, dev(hpar)), **{k: dev(v) for k, v in _right_kw(rk, gpar).items()})
    C = host(s.work())
    err = np.abs(C - og.precondition(A, Gd, Hd))
    bound = _bound(A, Hd, Gd, lk, hpar, rk, gpar)
    print(f"  max err {err.max():.2e}, min slack {np.min(bound - err):.2e}", flush=True)
    assert np.all(err <= bound)
    inf = s.info()
    assert inf["mult_left"] == {"dense": 0, "toeplitz": 1, "circulant": 3, "householder": 4}[lk]


@pytest.mark.parametrize("lk,rk,nrhs", [("dense", None, 1), ("toeplitz", "toeplitz", 2), ("circulant", None, 4),
                                         ("householder", "dense", 3), ("householder", "householder", 6),
                                         (None, "householder", 1)])
def test_whole_path_with_left_multipliers(lk, rk, nrhs):
    """Solve + FP64 refinement: eta <= 1e-14 from the oracle; x within 10 kappa max(eta, u)
    of LAPACK."""
    n = 512
    print(f"solve: left {lk}, right {rk}, {nrhs} rhs", flush=True)
    g = np.random.default_rng(50 + nrhs)
    w = wl.haar_logspaced(n, 1e3, wl.MULT_DENSE, nrhs=nrhs, seed=60 + nrhs)
    hpar, _ = _draw(lk, n, g)
    gpar, _ = _draw(rk, n, g)
    left = (lk, dev(hpar)) if lk else None
    X, info, s = genp.solve(dev(w.A), dev(w.B), nb=128, refine=2, tol=1e-14, left=left,
                            **{k: dev(v) for k, v in _right_kw(rk, gpar).items()})
    Xh = host(X)
    eta = og.backward_error_inf(w.A, Xh, w.B)
    assert np.all(eta <= 1e-14)
    x0 = np.linalg.solve(w.A, w.B)
    kappa = np.linalg.cond(w.A, np.inf)
    assert np.max(np.abs(Xh - x0)) <= 10 * kappa * max(eta.max(), U64) * np.max(np.abs(x0))


def test_left_gaussian_multiplier_repairs_breakdown():
    """GENP breaks on the rank-deficient leading block at column 5; with a Gaussian left
    multiplier (the G M case of Corollary 4.1: the leading columns of A have full rank) the
    elimination succeeds and the refined solution reaches eta <= 1e-14."""
    w = wl.make("c1_n256_rankdef")
    n = w.n
    H = np.random.default_rng(22).standard_normal((n, n))
    X, info, _ = genp.solve(dev(w.A), dev(w.B), nb=64, refine=2, tol=1e-14, pivot_tol=1e-10, left=("dense", dev(H)))
    assert info["breakdown_col"] == 0
    assert og.backward_error_inf(w.A, host(X), w.B).max() <= 1e-14


@pytest.mark.parametrize("lk,rk", [("householder", None), ("dense", "toeplitz"), ("circulant", "householder")])
def test_adjoint_with_left_multipliers(lk, rk):
    """dB = A^{-T} W (through H^T L^{-T} U^{-T} G^T) and dA = -dB X^T against the oracle."""
    n, k = 256, 2
    g = np.random.default_rng(70)
    w = wl.haar_logspaced(n, 1e3, wl.MULT_DENSE, nrhs=k, seed=71)
    W = wl.gaussian((n, k), 72)
    hpar, _ = _draw(lk, n, g)
    gpar, _ = _draw(rk, n, g)
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(w.A), left=(lk, dev(hpar)), **{kk: dev(v) for kk, v in _right_kw(rk, gpar).items()})
    assert s.factor() == 0
    X = s.solve(dev(w.B))
    s.refine(dev(w.B), X, 2, 1e-15)
    dB, dA = s.solve_backward(dev(W), X, want_dA=True, refine_iters=1)
    dBo, dAo = og.adjoint(w.A, host(X), W)
    tol = 10 * np.linalg.cond(w.A, np.inf) * U64
    assert np.max(np.abs(host(dB) - dBo)) <= tol * np.max(np.abs(dBo))
    assert np.max(np.abs(host(dA) - dAo)) <= tol * np.max(np.abs(dAo))


def test_left_multiplier_needs_fp64():
    n = 64
    s = genp.Solver(n, "f32", 64)
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(genp.GenpError) as e:
        s.precondition(A, left=("dense", A))
    assert e.value.status == genp.ENOTSUP


def test_householder_fullsize_n16384():
    """The benchmark's A (n = 16384, s <= 1e6) with a +-1 Householder multiplier, nb = 256:
    64 sampled entries of C = A G against the oracle's dot products, and the refined solution's
    eta from the full A on the host."""
    print("householder n=16384: building inputs", flush=True)
    w = wl.make("c3_n16384_haar1e6_toeplitz", device="cuda")
    n = w.n
    g = np.random.default_rng(80)
    uv = wl.pm1_signs(g, 2 * n)
    while not np.isfinite(og.householder_cond(uv)):
        uv = wl.pm1_signs(g, 2 * n)
    s = genp.Solver(n, "f64", 256)
    s.precondition(w.A, uv=dev(uv))
    Ah = host(w.A)
    I = g.integers(0, n, 64)
    J = g.integers(0, n, 64)
    C = s.work()
    Cs = host(C[torch.as_tensor(I, device="cuda"), torch.as_tensor(J, device="cuda")])
    del C
    u, v = uv[:n], uv[n:]
    sc = 2.0 / (v @ u)
    for t, (i, j) in enumerate(zip(I, J)):
        col = -sc * v[j] * u
        col[j] += 1.0                              # G[:, j] = e_j - s v_j u
        exact = Ah[i] @ col
        bound = 4 * og.gamma(n) * (np.abs(Ah[i]) @ np.abs(col))
        assert abs(Cs[t] - exact) <= bound
    print(f"  sampled entries ok; product {s.info()['ms_ag']:.2f} ms; factor", flush=True)
    assert s.factor() == 0
    X = s.solve(w.B)
    st, eta = s.refine(w.B, X, 2, 1e-14)
    assert st == genp.OK
    eta_o = og.backward_error_inf(Ah, host(X), host(w.B))
    print(f"  eta library {max(eta):.2e} oracle {eta_o.max():.2e}", flush=True)
    assert np.all(eta_o <= 1e-14)
