"""Refinement with every option (genp_refine_ex), the adjoint refined against A^T by LU-IR or
FP64 GMRES (genp_solve_backward_ex), and the 1-norm condition estimate (genp_condest), against
the oracle.

* condest: the library's estimates are those of the oracle's Hager-Higham estimator run on the
  same operators (C = A G from the FP64 inputs, (L U)^{-1} from the library's own factors), and
  lower bounds of the exact norms, never below a third of them for these inputs.
* refinement: the backward error the library reports is the oracle's for the returned X (5 %),
  the GMRES budget is honoured, and a converged status means eta <= tol by the oracle's measure.
* adjoint: dB against the oracle's A^{-T} W (LAPACK) within 10 kappa_inf(A) max(eta, u), and the
  transposed system's eta (with ||A||_1) against the oracle's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import condest as oc, genp as og  # noqa: E402
from paper_1212_4560_amd import genp, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

U64 = 2.0 ** -53


def same_eta(lib, orc):
    """The library's eta against the oracle's for the same iterate: within 5 %, or both at the
    rounding level, where two summation orders of the residual differ by a few u."""
    lib, orc = np.asarray(lib, dtype=np.float64), np.asarray(orc, dtype=np.float64)
    return bool(np.all(np.abs(lib - orc) <= 0.05 * orc + 4 * U64))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def eta_t(A, dB, W):
    """The adjoint system's backward error A^T db = w (infinity norm of A^T = ||A||_1)."""
    return og.backward_error_inf(np.ascontiguousarray(A.T), dB, W)


@pytest.mark.parametrize("n,prec,mult,nb,block", [
    (1, "f64", "dense", 64, False), (7, "f64", "dense", 64, False), (130, "f64", "toeplitz", 64, False),
    (300, "f32", "dense", 128, False), (257, "f64", "dense", 64, True), (512, "bf16x3", "toeplitz", 128, False)])
def test_condest_against_oracle(n, prec, mult, nb, block):
    print(f"condest n={n} {prec} {mult} block={block}", flush=True)
    w = wl.haar_logspaced(n, 1e3, wl.MULT_DENSE if mult == "dense" else wl.MULT_TOEPLITZ, seed=n)
    G = w.G if w.G is not None else og.toeplitz_from_params(w.p, n)
    s = genp.Solver(n, prec, nb)
    s.precondition(dev(w.A), G=dev(w.G) if w.G is not None else None, p=dev(w.p) if w.p is not None else None)
    assert s.factor(block=block) == 0
    LU = host(s.work())
    perm = host(s.row_perm()).astype(np.int64)
    got = s.condest()
    info = s.info()
    assert info["cond1_c"] == got["kappa1"]
    L, U = og.unpack(LU)
    # P C = L U: C^{-1} = (L U)^{-1} P, i.e. the library's inverse operator
    P = np.eye(n)[perm]
    Minv = np.linalg.solve(L @ U, P)
    C = w.A @ G
    nc_exact, ni_exact = oc.norm1(C), oc.norm1(Minv)
    nc_orc = oc.norm1_estimate_matrix(C)
    ni_orc = oc.norm1_estimate_matrix(Minv)
    print(f"  ||C||_1 {got['norm1_c']:.6e} oracle est {nc_orc:.6e} exact {nc_exact:.6e}; ||(LU)^-1||_1 "
          f"{got['norm1_inv']:.6e} oracle est {ni_orc:.6e} exact {ni_exact:.6e}", flush=True)
    for g, o, x in ((got["norm1_c"], nc_orc, nc_exact), (got["norm1_inv"], ni_orc, ni_exact)):
        assert g <= x * (1 + 1e-8)
        assert g >= x / 3.0
        assert abs(g - o) <= 1e-8 * o
    assert got["kappa1"] == pytest.approx(got["norm1_c"] * got["norm1_inv"], rel=1e-15)


def test_refine_ex_gmres_budget_and_reported_eta():
    """FP32 factors of an ill-conditioned system (kappa(A) = 1e6, kappa(C) u32 >> 1): GMRES-IR
    with restart 8 and a budget of 20 inner steps stops with ENOCONV within the budget, having
    lowered eta, and reports the oracle's eta of the X it returns."""
    n = 400
    w = wl.haar_logspaced(n, 1e6, wl.MULT_TOEPLITZ, nrhs=1, seed=21)
    s = genp.Solver(n, "f32", 128)
    s.precondition(dev(w.A), p=dev(w.p))
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=50, tol=1e-30, solver="gmres", restart=8, max_inner=20)
    info = s.info()
    eta_o = float(og.backward_error_inf(w.A, host(X), w.B).max())
    print(f"  status {st} outer {info['iters']} inner {info['inner_iters']} eta {max(eta):.2e} oracle {eta_o:.2e}",
          flush=True)
    assert st == genp.ENOCONV
    assert info["inner_iters"] <= 20
    assert abs(eta_o - max(eta)) <= 0.05 * eta_o
    assert max(eta) <= info["eta_hist"][0]


@pytest.mark.parametrize("restart", [30, 100, 200])
def test_refine_ex_gmres_converges_f32(restart):
    """The same system with an unbounded budget: GMRES-IR reaches the FP64 bar with cycles of
    30 steps or more (with 5-step cycles a correction soon raises eta and the refinement stops
    at its best iterate)."""
    n = 400
    w = wl.haar_logspaced(n, 1e6, wl.MULT_TOEPLITZ, nrhs=1, seed=21)
    s = genp.Solver(n, "f32", 128)
    s.precondition(dev(w.A), p=dev(w.p))
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=60, tol=1e-14, solver="gmres", restart=restart)
    info = s.info()
    eta_o = og.backward_error_inf(w.A, host(X), w.B)
    print(f"  restart {restart}: status {st} outer {info['iters']} inner {info['inner_iters']} eta {max(eta):.2e} "
          f"oracle {eta_o.max():.2e}", flush=True)
    assert st == genp.OK
    assert np.all(eta_o <= 1e-14)


def test_backward_ex_luir_equals_legacy_call():
    """genp_solve_backward(refine_iters) is genp_solve_backward_ex with LU-IR and tol = 0."""
    n, k = 200, 3
    w = wl.make("c5_n8192_scaled_lowrank", n=n, nrhs=k)
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(w.A), G=dev(w.G))
    assert s.factor() == 0
    X = s.solve(dev(w.B))
    s.refine(dev(w.B), X, 2, 1e-15)
    dB1, dA1 = s.solve_backward(dev(w.W), X, want_dA=True, refine_iters=2)
    dB2, dA2, st, eta = s.solve_backward(dev(w.W), X, want_dA=True, refine_iters=2, solver="luir",
                                         return_status=True)
    assert st == genp.OK
    assert torch.equal(dB1, dB2) and torch.equal(dA1, dA2)
    eo = eta_t(w.A, host(dB2), w.W)
    assert same_eta(eta, eo)


@pytest.mark.parametrize("n,smax", [(256, 1e2), (600, 1e5)])
def test_backward_ex_gmres_fp32_factors(n, smax):
    """FP32 factors, adjoint refined against A^T with FP64 GMRES (preconditioner H^T (LU)^{-T}
    G^T): dB reaches the FP64 bar and matches the oracle's A^{-T} W; dA = -dB X^T likewise."""
    k = 2
    w = wl.haar_logspaced(n, smax, wl.MULT_DENSE, nrhs=k, seed=5)
    W = wl.gaussian((n, k), 55)
    s = genp.Solver(n, "f32", 128)
    s.precondition(dev(w.A), G=dev(w.G))
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, _ = s.refine(Bd, X, max_iter=30, tol=1e-14, solver="gmres", restart=50)
    assert st == genp.OK
    dB, dA, stb, eta = s.solve_backward(dev(W), X, want_dA=True, refine_iters=30, solver="gmres", tol=1e-14,
                                        restart=50, return_status=True)
    info = s.info()
    Xh = host(X)
    dBo, dAo = og.adjoint(w.A, Xh, W)
    eo = eta_t(w.A, host(dB), W)
    kappa = np.linalg.cond(w.A, np.inf)
    err_b = np.max(np.abs(host(dB) - dBo)) / np.max(np.abs(dBo))
    err_a = np.max(np.abs(host(dA) - dAo)) / np.max(np.abs(dAo))
    print(f"  backward gmres: status {stb} outer {info['bwd_iters']} inner {info['bwd_inner_iters']} eta "
          f"{max(eta):.2e} oracle {eo.max():.2e}; rel err dB {err_b:.2e} dA {err_a:.2e} (kappa {kappa:.2e})",
          flush=True)
    assert stb == genp.OK and np.all(eo <= 1e-14)
    assert same_eta(eta, eo)
    assert info["anorm_1"] == pytest.approx(np.max(np.sum(np.abs(w.A), axis=0)), rel=1e-13)
    tol = 10 * kappa * max(eo.max(), U64)
    assert err_b <= tol and err_a <= tol


@pytest.mark.parametrize("smax,expect_switch", [(10.0, False), (1e6, True)])
def test_refine_auto_luir_then_gmres(smax, expect_switch):
    """GENP_SOLVER_AUTO: with FP32 factors and kappa(C) u32 < 1 it stays on LU-IR (no inner GMRES
    steps); with kappa(C) u32 >> 1 it turns to GMRES-IR and still reaches the FP64 bar."""
    n = 400
    w = wl.haar_logspaced(n, smax, wl.MULT_TOEPLITZ, nrhs=2, seed=21)
    s = genp.Solver(n, "f32", 128)
    s.precondition(dev(w.A), p=dev(w.p))
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=60, tol=1e-14, solver="auto", restart=60)
    info = s.info()
    eta_o = og.backward_error_inf(w.A, host(X), w.B)
    print(f"  smax {smax:g}: status {st} outer {info['iters']} inner {info['inner_iters']} eta {max(eta):.2e} "
          f"oracle {eta_o.max():.2e} hist {['%.1e' % e for e in info['eta_hist']]}", flush=True)
    assert st == genp.OK and np.all(eta_o <= 1e-14)
    assert (info["inner_iters"] > 0) == expect_switch


def _fp32_system(n, smax, k, seed):
    w = wl.haar_logspaced(n, smax, wl.MULT_TOEPLITZ, nrhs=k, seed=seed)
    s = genp.Solver(n, "f32", 128)
    s.precondition(dev(w.A), p=dev(w.p))
    assert s.factor() == 0
    return w, s


@pytest.mark.parametrize("k", [2, 7, 64])
def test_refine_gmres_many_columns_matches_column_by_column(k, monkeypatch):
    """GMRES-IR over k right-hand sides at once (one preconditioner solve and one product with A
    per Arnoldi step for all columns) reaches the FP64 bar on every column, and its X agrees with
    the one-cycle-per-column path's (GENP_GMRES=columns) to the accuracy both reach,
    kappa_inf(A) eta."""
    n = 400
    w, s = _fp32_system(n, 1e6, k, 31)
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=60, tol=1e-14, solver="gmres", restart=60)
    info = s.info()
    monkeypatch.setenv("GENP_GMRES", "columns")
    w2, s2 = _fp32_system(n, 1e6, k, 31)
    X2 = s2.solve(Bd)
    st2, eta2 = s2.refine(Bd, X2, max_iter=60, tol=1e-14, solver="gmres", restart=60)
    info2 = s2.info()
    Xh, X2h = host(X), host(X2)
    eta_o = og.backward_error_inf(w.A, Xh, w.B)
    kappa = np.linalg.cond(w.A, np.inf)
    diff = np.max(np.abs(Xh - X2h), axis=0) / np.max(np.abs(X2h), axis=0)
    print(f"  k {k}: batched status {st} outer {info['iters']} inner {info['inner_iters']} eta {max(eta):.2e} "
          f"(oracle {eta_o.max():.2e}); per column status {st2} outer {info2['iters']} inner "
          f"{info2['inner_iters']}; max rel diff {diff.max():.2e} (kappa {kappa:.2e})", flush=True)
    assert st == genp.OK and st2 == genp.OK
    assert np.all(eta_o <= 1e-14)
    assert same_eta(eta, eta_o)
    assert np.all(diff <= 10 * kappa * 1e-14)


def test_refine_gmres_many_columns_budget():
    """The many-column cycle honours the inner-step budget summed over columns: 8 columns,
    restart 8, budget 50 -> cycles of at most 50 // 8 = 6 steps per column, and the refinement
    stops once fewer than 8 steps remain (ENOCONV, eta lowered)."""
    n, k = 400, 8
    w, s = _fp32_system(n, 1e6, k, 21)
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=50, tol=1e-30, solver="gmres", restart=8, max_inner=50)
    info = s.info()
    eta_o = og.backward_error_inf(w.A, host(X), w.B)
    print(f"  status {st} outer {info['iters']} inner {info['inner_iters']} eta {max(eta):.2e} "
          f"hist {['%.1e' % e for e in info['eta_hist']]}", flush=True)
    assert st == genp.ENOCONV
    assert 0 < info["inner_iters"] <= 50 and info["inner_iters"] > 50 - k
    assert same_eta(eta, eta_o)
    assert max(eta) < info["eta_hist"][0]
