"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances are derived from the arithmetic:
* C = A G: both sides satisfy |C_hat - C| <= gamma_n |A||G| (standard dot-product
  bound), so they differ by at most 2 gamma_n |A||G| entrywise.
* factors: ||C - L U||_F <= 1e-13 || |L||U| ||_F (growth-normalized backward
  error of the elimination) and, where the leading blocks are well conditioned
  (strongly diagonally dominant C), entrywise agreement with the oracle's
  factors to 1e-12 relative.
* solutions: eta_inf(x_gpu) <= 1e-14 computed by the oracle from the GPU's x,
  and ||x_gpu - x_orc||_inf <= 10 kappa_inf(A) max(eta_gpu, eta_orc, u) ||x_orc||_inf.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import genp as og  # noqa: E402
from paper_1212_4560_amd import genp, workloads as wl  # noqa: E402

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


# ------------------------------------------------------------------ C = A G ----

@pytest.mark.parametrize("n", [1, 7, 64, 200, 256, 517, 640])
@pytest.mark.parametrize("mult", ["dense", "toeplitz"])
def test_precondition_entrywise(n, mult):
    """Sizes on both sides of the full-tile Toeplitz product (n a multiple of 128: 256, 640)."""
    _say(f"precondition n={n} mult={mult}")
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n))
    if mult == "dense":
        G = g.standard_normal((n, n))
        p = None
    else:
        p = g.standard_normal(2 * n - 1)
        G = og.toeplitz_from_params(p, n)
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(A), G=dev(G) if p is None else None, p=dev(p) if p is not None else None)
    C = host(s.work())
    Co = og.precondition(A, G)
    bound = 2 * og.gamma(n) * (np.abs(A) @ np.abs(G))
    assert np.all(np.abs(C - Co) <= bound + 1e-300)
    info = s.info()
    assert info["max_abs_c"] == np.max(np.abs(C))
    assert abs(info["anorm_inf"] - np.max(np.sum(np.abs(A), axis=1))) <= 1e-13 * info["anorm_inf"]


def test_precondition_strided_inputs():
    n = 130
    g = np.random.default_rng(3)
    Abig = g.standard_normal((n, n + 9))
    Gbig = g.standard_normal((n, n + 5))
    s = genp.Solver(n, "f64", 128)
    s.precondition(dev(Abig)[:, :n], G=dev(Gbig)[:, :n])
    C = host(s.work())
    Co = Abig[:, :n] @ Gbig[:, :n]
    assert np.all(np.abs(C - Co) <= 2 * og.gamma(n) * (np.abs(Abig[:, :n]) @ np.abs(Gbig[:, :n])))


# ------------------------------------------------------------------ factors ----

@pytest.mark.parametrize("n,nb", [(1, 64), (33, 64), (64, 64), (255, 64), (256, 256), (257, 128),
                                  (700, 256), (1000, 128), (1031, 64)])
def test_factor_matches_oracle_well_conditioned(n, nb):
    """No multiplier, strongly diagonally dominant C: factors agree entrywise."""
    _say(f"factor n={n} nb={nb}")
    g = np.random.default_rng(n + nb)
    C = g.standard_normal((n, n)) + 2.0 * n * np.eye(n)
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(C))
    assert s.factor() == 0
    LU = host(s.work())
    LUo, info = og.genp_unblocked(C)
    assert np.max(np.abs(LU - LUo)) <= 1e-12 * np.max(np.abs(LUo))
    i = s.info()
    assert i["breakdown_col"] == 0
    assert abs(i["min_abs_piv"] - np.min(np.abs(np.diag(LUo)))) <= 1e-12 * i["min_abs_piv"]
    assert abs(i["max_abs_piv"] - np.max(np.abs(np.diag(LUo)))) <= 1e-12 * i["max_abs_piv"]
    assert abs(i["growth"] - info.growth) <= 1e-12 * info.growth


@pytest.mark.parametrize("n,nb,mult", [(256, 256, "dense"), (256, 64, "dense"), (600, 128, "toeplitz"),
                                       (1100, 256, "dense")])
def test_factor_backward_error_with_multiplier(n, nb, mult):
    _say(f"factor-residual n={n} nb={nb} {mult}")
    w = wl.rank_deficient_lead(n=n, seed=n)
    if mult == "toeplitz":
        p = np.random.default_rng(7).standard_normal(2 * n - 1)
        G = og.toeplitz_from_params(p, n)
    else:
        p, G = None, w.G
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(w.A), G=dev(G) if p is None else None, p=dev(p) if p is not None else None)
    C = host(s.work())
    assert s.factor(n * og.U64) == 0
    LU = host(s.work())
    L, U = og.unpack(LU)
    E = np.linalg.norm(C - L @ U)
    assert E <= 1e-13 * np.linalg.norm(np.abs(L) @ np.abs(U))
    # raw residual reported next to the oracle's for the same C (agree within 10x)
    LUo, _ = og.genp_blocked(C, nb)
    raw_gpu, _ = og.factor_residual(C, LU)
    raw_orc, _ = og.factor_residual(C, LUo)
    _say(f"  raw ||C-LU||/||C||: gpu {raw_gpu:.2e} oracle {raw_orc:.2e}")
    assert raw_gpu <= 10 * max(raw_orc, 1e-16 * n)


def test_breakdown_on_singular_leading_block():
    """GENP on A itself (no multiplier) breaks down at column 5; on A G it does not."""
    w = wl.make("c1_n256_rankdef")
    tol = 1e-10   # far below every legitimate pivot of A G, far above rounding of the singular block
    _, io = og.genp_unblocked(w.A, tol)
    assert io.breakdown_col == 5
    s = genp.Solver(256, "f64", 64)
    s.precondition(dev(w.A))
    assert s.factor(tol) == 5
    i = s.info()
    assert i["breakdown_col"] == 5
    with pytest.raises(genp.GenpError) as e:
        s.solve(dev(w.B))
    assert e.value.status == genp.ESTATE
    s2 = genp.Solver(256, "f64", 64)
    s2.precondition(dev(w.A), G=dev(w.G))
    assert s2.factor(tol) == 0


def test_nonfinite_input_is_a_breakdown():
    n = 70
    A = np.random.default_rng(0).standard_normal((n, n)) + 50 * np.eye(n)
    A[3, 3] = np.nan
    s = genp.Solver(n, "f64", 64)
    s.precondition(dev(A))
    bk = s.factor()
    assert 1 <= bk <= 4


# ------------------------------------------------------------ solve / refine ----

def _check_solution(A, B, X, eta_gpu, kappa):
    eta = og.backward_error_inf(A, X, B)
    assert np.all(eta <= 1e-14), eta
    Xo = np.linalg.solve(A, B)
    eta_o = og.backward_error_inf(A, Xo, B)
    tol = 10 * kappa * max(np.max(eta), np.max(eta_o), og.U64)
    assert np.max(np.abs(X - Xo)) <= tol * np.max(np.abs(Xo))
    assert np.all(np.asarray(eta_gpu) <= 1e-14)


@pytest.mark.parametrize("name,n,nrhs,nb", [
    ("c1_n256_rankdef", 256, 1, 64),
    ("c1_n256_rankdef", 256, 1, 256),
    ("c2_n4096_haar1e4_dense", 700, 16, 256),
    ("c2_n4096_haar1e4_dense", 513, 3, 128),
    ("c3_n16384_haar1e6_toeplitz", 600, 1, 64),
    ("c4a_n16384_haar1e6_toeplitz", 520, 64, 256),
    ("c5_n8192_scaled_lowrank", 384, 70, 128),
])
def test_solve_refine_backward_error(name, n, nrhs, nb):
    _say(f"solve {name} n={n} nrhs={nrhs} nb={nb}")
    w = wl.make(name, n=n, nrhs=nrhs)
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(w.A), G=dev(w.G) if w.G is not None else None,
                   p=dev(w.p) if w.p is not None else None)
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    X0 = host(X).copy()
    st, eta = s.refine(Bd, X, max_iter=2, tol=0.0)
    Xh = host(X)
    # the unrefined solution is the oracle's solve of the same factors up to rounding
    G = og.dense_multiplier(w.G, w.p, n)
    LUg = host(s.work())
    Xs = og.solve(LUg, G, w.B)
    assert np.max(np.abs(X0 - Xs)) <= 1e-8 * np.max(np.abs(Xs))
    _check_solution(w.A, w.B, Xh, eta, np.linalg.cond(w.A, np.inf))
    i = s.info()
    assert i["iters"] <= 2 and i["n_eta"] >= 2 and i["eta_hist"][-1] <= 1e-14


def test_refine_stops_at_tolerance_and_reports_enoconv():
    w = wl.make("c2_n4096_haar1e4_dense", n=300, nrhs=2)
    s = genp.Solver(300, "f64", 64)
    s.precondition(dev(w.A), G=dev(w.G))
    s.factor()
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=5, tol=1e-15)
    assert st == genp.OK and max(eta) <= 1e-15 and s.info()["iters"] <= 3
    X2 = s.solve(Bd)
    st2, _ = s.refine(Bd, X2, max_iter=0, tol=1e-30)
    assert st2 == genp.ENOCONV


def test_solve_is_deterministic():
    w = wl.make("c2_n4096_haar1e4_dense", n=512, nrhs=8)
    out = []
    for _ in range(2):
        s = genp.Solver(512, "f64", 128)
        s.precondition(dev(w.A), G=dev(w.G))
        s.factor()
        X = s.solve(dev(w.B))
        s.refine(dev(w.B), X, 2)
        out.append(host(X))
    assert np.array_equal(out[0], out[1])


def test_state_and_argument_errors():
    n = 64
    s = genp.Solver(n, "f64", 64)
    B = dev(np.ones((n, 1)))
    with pytest.raises(genp.GenpError) as e:
        s.solve(B)
    assert e.value.status == genp.ESTATE
    with pytest.raises(genp.GenpError) as e:
        s.factor()
    assert e.value.status == genp.ESTATE
    with pytest.raises(genp.GenpError) as e:
        genp.Solver(n, "f64", 100)
    assert e.value.status == genp.EINVAL


# ------------------------------------------------------------------ adjoint ----

@pytest.mark.parametrize("n,nrhs,nb", [(64, 4, 64), (300, 16, 128), (257, 1, 256)])
def test_adjoint_matches_oracle(n, nrhs, nb):
    _say(f"adjoint n={n} nrhs={nrhs}")
    w = wl.make("c5_n8192_scaled_lowrank", n=n, nrhs=nrhs)
    s = genp.Solver(n, "f64", nb)
    s.precondition(dev(w.A), G=dev(w.G))
    assert s.factor() == 0
    X = s.solve(dev(w.B))
    s.refine(dev(w.B), X, 2)
    dB, dA = s.solve_backward(dev(w.W), X, want_dA=True, refine_iters=1)
    Xh = host(X)
    dBo, dAo = og.adjoint(w.A, Xh, w.W)
    kappa = np.linalg.cond(w.A, np.inf)
    tol = 10 * kappa * 1e-15
    assert np.max(np.abs(host(dB) - dBo)) <= tol * np.max(np.abs(dBo))
    assert np.max(np.abs(host(dA) - dAo)) <= tol * np.max(np.abs(dAo))


def test_autograd_central_differences_n64():
    n, k = 64, 3
    w = wl.make("c5_n8192_scaled_lowrank", n=n, nrhs=k)
    GenpSolve = genp.GenpSolve
    A = dev(w.A).requires_grad_(True)
    B = dev(w.B).requires_grad_(True)
    G = dev(w.G)
    W = dev(w.W)
    X = GenpSolve.apply(A, B, G)
    loss = (W * X).sum()
    loss.backward()
    gA, gB = host(A.grad), host(B.grad)

    def L(Ah, Bh):
        Xf, _, _ = genp.solve(dev(Ah), dev(Bh), G=G, refine=2)
        return float(np.sum(w.W * host(Xf)))

    g = np.random.default_rng(1)
    h = 1e-6 * np.max(np.abs(w.A))
    for _ in range(6):
        i, j = g.integers(0, n, 2)
        E = np.zeros((n, n))
        E[i, j] = h
        fd = (L(w.A + E, w.B) - L(w.A - E, w.B)) / (2 * h)
        assert abs(fd - gA[i, j]) <= 1e-6 * max(abs(gA[i, j]), 1e-2 * np.max(np.abs(gA)))
    D = g.standard_normal((n, n))
    hd = 1e-6
    fd = (L(w.A + hd * D, w.B) - L(w.A - hd * D, w.B)) / (2 * hd)
    assert abs(fd - np.sum(gA * D)) <= 1e-6 * abs(fd)
    i, c = 5, 1
    E = np.zeros((n, k))
    E[i, c] = 1e-6
    fd = (L(w.A, w.B + E) - L(w.A, w.B - E)) / 2e-6
    assert abs(fd - gB[i, c]) <= 1e-6 * max(abs(gB[i, c]), 1e-2 * np.max(np.abs(gB)))


def test_gradient_does_not_depend_on_multiplier():
    n, k = 128, 2
    w = wl.make("c5_n8192_scaled_lowrank", n=n, nrhs=k)
    grads = []
    for seed in (11, 12):
        G = dev(wl.gaussian((n, n), seed))
        A = dev(w.A).requires_grad_(True)
        X = genp.GenpSolve.apply(A, dev(w.B), G)
        (dev(w.W) * X).sum().backward()
        grads.append(host(A.grad))
    kappa = np.linalg.cond(w.A, np.inf)
    assert np.max(np.abs(grads[0] - grads[1])) <= 10 * kappa * 1e-15 * np.max(np.abs(grads[0]))


# -------------------------------------------------- schedule and solve variants ----

def _factor_with_env(monkeypatch, var, value, A, G, n, nb, prec="f64"):
    monkeypatch.setenv(var, value)
    s = genp.Solver(n, prec, nb)       # the library reads the switch when the context is created
    s.precondition(dev(A), G=dev(G))
    assert s.factor() == 0
    return s, host(s.work())


@pytest.mark.parametrize("n,nb,prec", [(1280, 256, "f64"), (1100, 128, "f64"), (900, 64, "f32")])
def test_lookahead_does_not_change_the_factors(monkeypatch, n, nb, prec):
    """Look-ahead only moves the diagonal-block factorizations to a second stream: the
    products, their grouping and their order are the same, so the factors are bit-identical."""
    g = np.random.default_rng(n)
    A, G = g.standard_normal((n, n)), g.standard_normal((n, n))
    _, on = _factor_with_env(monkeypatch, "GENP_LOOKAHEAD", "1", A, G, n, nb, prec)
    _, off = _factor_with_env(monkeypatch, "GENP_LOOKAHEAD", "0", A, G, n, nb, prec)
    assert np.array_equal(on, off)


@pytest.mark.parametrize("n,nb", [(2560, 256), (1031, 64), (1500, 128)])
def test_round_cuts_do_not_change_the_factors(monkeypatch, n, nb):
    """FP64: the bulk of a step group is cut into column parts of whole rounds of update
    tiles instead of equal parts of whole blocks.  Every entry takes the same products in the
    same order either way (the cuts fall on 128-column tile edges; with nb = 64 the last part
    takes the half tile), so the factors are bit-identical."""
    g = np.random.default_rng(n + 7)
    A, G = g.standard_normal((n, n)), g.standard_normal((n, n))
    # rounds of 8 tiles, so that these small trailing matrices take the cut by rounds
    _, on = _factor_with_env(monkeypatch, "GENP_ROUND_CUT", "8", A, G, n, nb)
    _, off = _factor_with_env(monkeypatch, "GENP_ROUND_CUT", "0", A, G, n, nb)
    assert np.array_equal(on, off)


@pytest.mark.parametrize("n,nb", [(1280, 256), (1100, 128), (900, 64)])
def test_fp32_update_kernel_matches_general_kernel(monkeypatch, n, nb):
    """FP32 form: the Schur updates on the dedicated 256 x 128 FP32 kernel and on the general
    LDS-staged kernel feed every MFMA the same four consecutive k in the same order, so the
    factors are bit-identical."""
    g = np.random.default_rng(n + 11)
    A, G = g.standard_normal((n, n)), g.standard_normal((n, n))
    _, on = _factor_with_env(monkeypatch, "GENP_F32_UPD", "upd", A, G, n, nb, "f32")
    _, off = _factor_with_env(monkeypatch, "GENP_F32_UPD", "lp", A, G, n, nb, "f32")
    assert np.array_equal(on, off)


@pytest.mark.parametrize("n", [512, 1280, 1100])
def test_split_diagonal_blocks_match_single_workgroup_blocks(monkeypatch, n):
    """FP64 nb = 256: the diagonal block as two LDS-resident 128 halves with the panel solves
    and one update between them (block GE on the block, Theorem 2.2) against one workgroup
    eliminating it column by column: the same pivots in exact arithmetic, so on a strongly well
    conditioned C the factors agree to rounding (1e-12 relative), including a ragged last block."""
    g = np.random.default_rng(n + 7)
    A = g.standard_normal((n, n)) + 2 * np.sqrt(n) * np.eye(n)
    G = np.eye(n) + 0.1 * g.standard_normal((n, n)) / np.sqrt(n)
    _, split = _factor_with_env(monkeypatch, "GENP_DIAG", "split", A, G, n, 256)
    _, single = _factor_with_env(monkeypatch, "GENP_DIAG", "single", A, G, n, 256)
    assert np.max(np.abs(split - single)) <= 1e-12 * np.max(np.abs(single))


@pytest.mark.parametrize("mode", ["split", "single"])
def test_breakdown_in_the_second_half_of_a_diagonal_block(monkeypatch, mode):
    """A leading 200 x 200 block of rank 199 (no multiplier): GENP breaks down at column 200,
    which lies in the second 128-column half of the first 256 block.  The failing pivot is
    rounding noise (2e-10 max|C| on the host, measured up to 2e-10 max|C| with one workgroup
    and 2e-8 max|C| with the split block, whose products sum in another order); every
    regular pivot is >= 5e-3 max|C|, so pivot_tol = 1e-7 separates them with margin."""
    monkeypatch.setenv("GENP_DIAG", mode)
    n = 512
    g = np.random.default_rng(5)
    A = g.standard_normal((n, n))
    A[:200, :200] = g.standard_normal((200, 199)) @ g.standard_normal((199, 200))
    s = genp.Solver(n, "f64", 256)
    s.precondition(dev(A))
    assert s.factor(1e-7) == 200
    inf = s.info()
    assert inf["min_abs_piv"] >= 5e-3 * inf["max_abs_c"]


@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 5, 17, 64])
def test_chained_triangular_solves_match_per_block_solves(monkeypatch, nrhs):
    """The single-launch solves (forward/backward for the solution, transposed for the
    adjoint) against the one-launch-per-block solves, for 1..4 right-hand sides (VALU
    chain) and 5..64 (MFMA chain; the block path is the diagonal-block TRSM and GEMM).  Both are
    substitution with the sums accumulated in a different order, so both must be backward
    stable: eta_inf of X for A X = B and of dB for A^T dB = W small (no refinement here) and
    within 10x of each other; the solutions themselves differ by the factors' conditioning
    times u (GENP factors of A G can be much worse conditioned than A).  No error word may
    be left behind."""
    n, nb = 1000, 128
    g = np.random.default_rng(40 + nrhs)
    A = g.standard_normal((n, n)) + 3 * np.sqrt(n) * np.eye(n)
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, nrhs))
    W = g.standard_normal((n, nrhs))
    res = {}
    for mode in ("chain", "step"):
        s, _ = _factor_with_env(monkeypatch, "GENP_TRSV", mode, A, G, n, nb)
        X = s.solve(dev(B))
        dB, _ = s.solve_backward(dev(W), X, want_dA=False, refine_iters=0)
        s.info()                        # raises if a chained solve reported an error
        res[mode] = (host(X), host(dB))
    eta = {m: (og.backward_error_inf(A, res[m][0], B).max(), og.backward_error_inf(A.T, res[m][1], W).max())
           for m in res}
    _say(f"  nrhs={nrhs}: eta chain {eta['chain']} step {eta['step']}")
    for k in range(2):
        a, b = eta["chain"][k], eta["step"][k]
        # unrefined GENP solves: growth puts eta near 1e-10 here (refinement takes it to u)
        assert a <= 1e-8 and b <= 1e-8
        assert a <= 10 * b + 1e-16 and b <= 10 * a + 1e-16
        x, y = res["chain"][k], res["step"][k]
        assert np.max(np.abs(x - y)) <= 1e-6 * np.max(np.abs(y))
