"""Block Gaussian elimination with explicit block pivots on the GPU (genp_factor_block,
genp_block_pivots, genp_row_perm) against the CPU oracle (Theorem 2.2, Fact 2.1).

Bars:
* the row permutation is index work: equal to the oracle's, element by element
  (inputs are seeded Gaussian matrices, whose largest candidates in a column are
  separated far beyond rounding);
* factors: ||P C - L U||_F <= 1e-13 || |L||U| ||_F and the oracle's packed factors
  to 1e-9 relative to max|L||U| (the two eliminations round in different orders);
* explicit block pivots: B_k is a block of a Schur complement, a forward quantity:
  a backward error of relative size e u (times GENP's growth where there is no
  pivoting) moves it by up to kappa_1(C_e) times that, C_e the leading block that
  ends with B_k; the bar is 10 e u kappa_1(C_e) growth max|B_k|;
* solutions: eta_inf <= 1e-14 after refinement, and the oracle's error bound
  ||x_gpu - x_orc||_inf <= 10 kappa_inf(A) max(eta, u) ||x_orc||_inf.
"""
import warnings

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import blockge as obg  # noqa: E402
from oracle import genp as og  # noqa: E402
from paper_1212_4560_amd import genp  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)


def _swapped_blocks(n, nb, seed):
    """C = L_b U_b, block unit lower times block upper triangular, with the leading entry of
    every diagonal block of U_b zero: GENP breaks down at the first column, while every
    leading nb, 2nb, ... block is nonsingular."""
    g = np.random.default_rng(seed)
    Lb, Ub = np.eye(n), np.zeros((n, n))
    for k in range(0, n, nb):
        e = min(k + nb, n)
        Lb[e:, k:e] = g.standard_normal((n - e, e - k)) / np.sqrt(n)
        Ub[k:e, k:] = g.standard_normal((e - k, n - k))
        Ub[k, k] = 0.0
    return Lb @ Ub


def _pivot_tol(C, e, Bo, growth=1.0):
    return 10 * e * og.U64 * np.linalg.cond(C[:e, :e], 1) * growth * np.max(np.abs(Bo))


def _check_factors(s, C, res, nb):
    n = C.shape[0]
    perm = host(s.row_perm()).astype(np.int64)
    assert np.array_equal(perm, res.perm)
    LU = host(s.work())
    L, U = og.unpack(LU)
    scale = np.abs(L) @ np.abs(U)
    assert np.linalg.norm(C[perm] - L @ U) <= 1e-13 * np.linalg.norm(scale)
    assert np.max(np.abs(LU - res.LU)) <= 1e-9 * np.max(scale)
    B = host(s.block_pivots())
    for k, Bo in zip(range(0, n, nb), res.pivots):
        w = Bo.shape[0]
        assert np.max(np.abs(B[k:k + w, :w] - Bo)) <= _pivot_tol(C, k + w, Bo)
        assert not np.any(B[k:k + w, w:])


@pytest.mark.parametrize("n,nb", [(512, 256), (700, 256), (300, 64), (1100, 128)])
def test_factors_permutation_and_block_pivots_match_the_oracle(n, nb):
    _say(f"block GE parity n={n} nb={nb}")
    g = np.random.default_rng(100 + n)
    A = g.standard_normal((n, n))
    p = g.standard_normal(2 * n - 1)
    G = og.toeplitz_from_params(p, n)
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(A), p=dev(p))
    C = host(s.work())
    assert s.factor(0.0, block=True) == 0
    info = s.info()
    assert info["block_ge"] == 1 and info["row_swaps"] > 0
    res = obg.block_ge(og.precondition(A, G), nb)
    assert res.breakdown_col == 0
    _check_factors(s, C, res, nb)
    assert info["row_swaps"] == int(np.sum(res.perm != np.arange(n)))


@pytest.mark.parametrize("n,nb,k", [(512, 256, 1), (700, 256, 3), (320, 64, 8)])
def test_solve_and_refinement_match_the_oracle(n, nb, k):
    _say(f"block GE solve n={n} nb={nb} k={k}")
    g = np.random.default_rng(200 + n)
    A = g.standard_normal((n, n))
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, k))
    X, info, s = genp.solve(dev(A), dev(B), G=dev(G), nb=nb, refine=2, block=True)
    x = host(X)
    eta = og.backward_error_inf(A, x, B)
    assert np.max(eta) <= 1e-14
    xo = obg.solve(obg.block_ge(og.precondition(A, G), nb), G, B)
    kap = np.linalg.cond(A, np.inf)
    ref = np.linalg.solve(A, B)
    assert np.max(np.abs(x - ref)) <= 10 * kap * max(np.max(eta), og.U64) * np.max(np.abs(ref))
    assert np.max(np.abs(xo - ref)) <= 10 * kap * 1e-12 * np.max(np.abs(ref))
    assert info["block_ge"] == 1


@pytest.mark.parametrize("n,nb", [(320, 64), (512, 256)])
def test_singular_interior_blocks_need_block_pivots(n, nb):
    """No multiplier: GENP breaks down at column 1, block GE solves the system."""
    _say(f"block GE zero leading entries n={n} nb={nb}")
    C = _swapped_blocks(n, nb, 7 + n)
    b = np.random.default_rng(8).standard_normal((n, 1))
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(C))
    assert s.factor(0.0) == 1
    s.precondition(dev(C))
    assert s.factor(0.0, block=True) == 0
    res = obg.block_ge(C, nb)
    _check_factors(s, C, res, nb)
    for k in range(0, n, nb):
        assert host(s.row_perm())[k] != k
    X = s.solve(dev(b))
    s.refine(dev(b), X, 2)
    x = host(X)
    assert np.max(og.backward_error_inf(C, x, b)) <= 1e-14
    ref = np.linalg.solve(C, b)
    assert np.max(np.abs(x - ref)) <= 1e-12 * np.linalg.cond(C, np.inf) * np.max(np.abs(ref))


@pytest.mark.parametrize("nb", [64, 256])
def test_singular_leading_block_is_reported_at_the_oracles_column(nb):
    n = 3 * nb
    _say(f"block GE breakdown n={n} nb={nb}")
    g = np.random.default_rng(11)
    C = g.standard_normal((n, n))
    M = g.standard_normal((nb, nb))
    C[nb:2 * nb, :2 * nb] = M @ C[:nb, :2 * nb]
    # the singular block pivot is rounding noise (~1e-13 of max|C| here); the tolerance
    # flags it at its first column on both sides and passes every genuine pivot
    tol = 1e-8
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(C))
    bk = s.factor(tol, block=True)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        res = obg.block_ge(C, nb, pivot_tol=tol)
    assert res.breakdown_col == nb + 1
    assert bk == res.breakdown_col
    with pytest.raises(genp.GenpError):
        s.solve(dev(np.ones((n, 1))))


def test_genp_block_pivots_are_the_same_blocks():
    """After plain GENP the block pivots are L_kk U_kk with P = I, the same matrices."""
    n, nb = 384, 128
    g = np.random.default_rng(12)
    A = g.standard_normal((n, n))
    G = g.standard_normal((n, n))
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(A), G=dev(G))
    assert s.factor(0.0) == 0
    assert np.array_equal(host(s.row_perm()), np.arange(n))
    assert s.info()["block_ge"] == 0 and s.info()["row_swaps"] == 0
    B = host(s.block_pivots())
    C = og.precondition(A, G)
    res = obg.block_ge(C, nb)
    rho = max(1.0, s.info()["growth"])
    for k, Bo in zip(range(0, n, nb), res.pivots):
        assert np.max(np.abs(B[k:k + nb] - Bo)) <= _pivot_tol(C, k + nb, Bo, rho)


def test_adjoint_with_block_factors():
    n, nb, k = 320, 64, 2
    _say(f"block GE adjoint n={n}")
    g = np.random.default_rng(13)
    A = g.standard_normal((n, n))
    G = g.standard_normal((n, n))
    B, W = g.standard_normal((n, k)), g.standard_normal((n, k))
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(A), G=dev(G))
    assert s.factor(0.0, block=True) == 0
    X = s.solve(dev(B))
    s.refine(dev(B), X, 2)
    dB, dA = s.solve_backward(dev(W), X, want_dA=True, refine_iters=1)
    dBo, dAo = og.adjoint(A, host(X), W)
    kap = np.linalg.cond(A, np.inf)
    assert np.max(np.abs(host(dB) - dBo)) <= 10 * kap * 1e-15 * np.max(np.abs(dBo))
    assert np.max(np.abs(host(dA) - dAo)) <= 10 * kap * 1e-15 * np.max(np.abs(dAo))


def test_gmres_refinement_with_block_factors():
    n, nb = 256, 64
    g = np.random.default_rng(14)
    A = g.standard_normal((n, n))
    G = g.standard_normal((n, n))
    b = g.standard_normal((n, 1))
    X, info, _ = genp.solve(dev(A), dev(b), G=dev(G), nb=nb, refine=3, solver="gmres", block=True)
    assert np.max(og.backward_error_inf(A, host(X), b)) <= 1e-14


def test_errors():
    n = 128
    s = genp.Solver(n, "f32", 64)
    s.precondition(dev(np.eye(n)))
    with pytest.raises(genp.GenpError):
        s.factor(0.0, block=True)
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(np.eye(n)))
    with pytest.raises(genp.GenpError):
        s.block_pivots()
    with pytest.raises(genp.GenpError):
        s.row_perm()


def test_ties_follow_the_interchange_order():
    """Rows of a Sylvester Hadamard matrix shuffled inside each block: every column of every
    block pivot has many entries of equal magnitude, and every value is a power of two, so
    both sides compute exactly and must take the same row at every tie (the first in the
    current row order): factors and permutation bit for bit."""
    import scipy.linalg as sl
    n, nb = 256, 64
    g = np.random.default_rng(3)
    P = np.concatenate([k + g.permutation(nb) for k in range(0, n, nb)])
    C = sl.hadamard(n).astype(np.float64)[P]
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(C))
    assert s.factor(0.0, block=True) == 0
    res = obg.block_ge(C, nb)
    assert np.array_equal(host(s.row_perm()).astype(np.int64), res.perm)
    assert np.array_equal(host(s.work()), res.LU)


@pytest.mark.parametrize("n,nb", [(1, 64), (5, 64), (65, 64), (130, 128)])
def test_tiny_and_ragged_block_pivots(n, nb):
    """Fewer rows than one block, one row past a block, a ragged last block: the interchanges
    stay inside the valid rows (the padding is never chosen) and the solution is exact to
    rounding."""
    g = np.random.default_rng(300 + n)
    C = g.standard_normal((n, n))
    b = g.standard_normal((n, 1))
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(C))
    assert s.factor(0.0, block=True) == 0
    res = obg.block_ge(C, nb)
    _check_factors(s, C, res, nb)
    X = s.solve(dev(b))
    s.refine(dev(b), X, 2)
    assert np.max(og.backward_error_inf(C, host(X), b)) <= 1e-14
