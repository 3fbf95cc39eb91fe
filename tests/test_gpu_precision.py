"""Parity of the precision form (FP32 / BF16-operand factors + FP64 refinement) with the oracle.

Bounds from the arithmetic (u32 = 2^-24, u_bf16 = 2^-9):
* C = A G with operands rounded FP64 -> FP32 (-> BF16) and FP32 accumulation:
  |C_gpu - Ahat Ghat| <= (n + 1) u32 |Ahat||Ghat| entrywise, where Ahat Ghat is the
  product of the rounded operands computed by the oracle in FP64 (BF16 x BF16
  products are exact in FP32).
* 2-word BF16: the product is hi hi + hi lo + lo hi (each operand x = hi + lo), three FP32
  accumulations per k: |C_gpu - P| <= (3n + 1) u32 (|hi_A| + |lo_A|)(|hi_G| + |lo_G|), P the
  oracle's exact three-term product.
* factors: growth-normalized residual ||C - LU||_F / || |L||U| ||_F <= 4 n u32 (FP32),
  <= 8 u_bf16 (BF16 Schur operands) or <= 8 * 2^-16 (2-word BF16), and within 10x of the
  oracle's mirror.
* after FP64 refinement: eta_inf <= 1e-14 computed by the oracle from the GPU's x.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import genp as og, lowprec as lpo  # noqa: E402
from paper_1212_4560_amd import genp, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

U32 = 2.0 ** -24
UBF = 2.0 ** -9
ROUND = {"f32": lpo.round_fp32, "bf16": lpo.round_bf16}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("n,mult", [(1, "dense"), (64, "dense"), (200, "dense"), (517, "toeplitz"),
                                    (300, "toeplitz"), (512, "toeplitz"), (768, "dense")])
def test_lowprec_precondition_entrywise(prec, n, mult):
    """C = A G in each precision form against the product of the rounded operands.  Sizes whose
    padded order is a multiple of 256 (200, 512, 768) take the BF16 forms' LDS-staged BF16 kernel
    from BF16 copies of A and G^T; FP32 with a Toeplitz G takes the register-operand kernel; the
    others the LDS-staged kernel from FP32 copies."""
    print(f"precondition {prec} n={n} {mult}", flush=True)
    g = np.random.default_rng(n + 1)
    A = g.standard_normal((n, n))
    if mult == "dense":
        G, p = g.standard_normal((n, n)), None
    else:
        p = g.standard_normal(2 * n - 1)
        G = og.toeplitz_from_params(p, n)
    s = genp.Solver(n, prec, 64)
    s.precondition(dev(A), G=dev(G) if p is None else None, p=dev(p) if p is not None else None)
    C = host(s.work())
    if prec == "bf16x3":
        Ce = lpo.product_bf16x3(A, G)
        ha, la = lpo.split_bf16x2(A)
        hg, lg = lpo.split_bf16x2(G)
        bound = (3 * n + 1) * U32 * ((np.abs(ha) + np.abs(la)) @ (np.abs(hg) + np.abs(lg)))
    else:
        r = ROUND[prec]
        Ce = lpo.product_of_rounded(A, G, r)
        bound = (n + 1) * U32 * (np.abs(r(A)) @ np.abs(r(G)))
    assert np.all(np.abs(C - Ce) <= bound)


@pytest.mark.parametrize("prec,nb", [("f32", 64), ("f32", 128), ("bf16", 128), ("bf16", 256), ("bf16x3", 128),
                                     ("bf16x3", 256)])
def test_lowprec_factor_residual(prec, nb):
    n = 600
    print(f"factor {prec} nb={nb}", flush=True)
    w = wl.haar_logspaced(n, 10.0, wl.MULT_DENSE, nrhs=1, seed=7)
    s = genp.Solver(n, prec, nb)
    s.precondition(dev(w.A), G=dev(w.G))
    C = host(s.work())
    assert s.factor() == 0
    LU = host(s.work())
    L, U = og.unpack(LU)
    rel = np.linalg.norm(C - L @ U) / np.linalg.norm(np.abs(L) @ np.abs(U))
    LUo = lpo.genp_blocked_lowprec(C, nb, bf16_update=(prec == "bf16"), bf16x3_update=(prec == "bf16x3"))
    Lo, Uo = og.unpack(LUo)
    rel_o = np.linalg.norm(C - Lo @ Uo) / np.linalg.norm(np.abs(Lo) @ np.abs(Uo))
    print(f"  growth-normalized residual gpu {rel:.2e} mirror {rel_o:.2e}", flush=True)
    assert rel <= {"f32": 4 * n * U32, "bf16": 8 * UBF, "bf16x3": 8 * 2.0 ** -16}[prec]
    assert rel <= 10 * max(rel_o, n * U32)


@pytest.mark.parametrize("prec,solver,smax,mult", [
    ("f32", "luir", 10.0, wl.MULT_DENSE),
    ("f32", "luir", 1e2, wl.MULT_TOEPLITZ),
    ("f32", "gmres", 1e4, wl.MULT_DENSE),
    # 2-word BF16 factors: about 16 bits, so LU-IR contracts only slowly once kappa(C) passes
    # ~1e4 (eta 5e-2 -> 3e-3 in 12 steps at n = 512, s <= 10, dense G); GMRES-IR converges
    ("bf16x3", "gmres", 10.0, wl.MULT_DENSE),
    ("bf16x3", "gmres", 1e2, wl.MULT_TOEPLITZ),
])
def test_lowprec_refinement_reaches_fp64_accuracy(prec, solver, smax, mult):
    n, k = 512, 2
    print(f"refine {prec} {solver} smax={smax} {mult}", flush=True)
    w = wl.haar_logspaced(n, smax, mult, nrhs=k, seed=11)
    s = genp.Solver(n, prec, 128)
    s.precondition(dev(w.A), G=dev(w.G) if w.G is not None else None, p=dev(w.p) if w.p is not None else None)
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=12, tol=1e-14, solver=solver)
    Xh = host(X)
    eta_o = og.backward_error_inf(w.A, Xh, w.B)
    info = s.info()
    print(f"  status {st} outer {info['iters']} inner {info['inner_iters']} eta {max(eta):.2e} "
          f"oracle {eta_o.max():.2e} hist {['%.1e' % e for e in info['eta_hist']]}", flush=True)
    assert st == genp.OK
    assert np.all(eta_o <= 1e-14)


def test_fp32_factors_many_rhs_refine_to_fp64_accuracy():
    """FP32 factors and 24 right-hand sides: every substitution of the solve and of LU-IR goes
    through the chained many-column solve reading an FP32 factor.  The unrefined solve equals
    the oracle's FP64 substitution with the same (FP32-stored) factors up to rounding, and
    LU-IR takes all 24 columns to the FP64 backward-error bar (the oracle's measure).  The
    matrix is the one of the two-column FP32 LU-IR case (kappa(C) ~ 3e5)."""
    n, k = 512, 24
    print(f"refine f32 luir n={n} k={k}", flush=True)
    w = wl.haar_logspaced(n, 10.0, wl.MULT_DENSE, nrhs=k, seed=11)
    s = genp.Solver(n, "f32", 128)
    s.precondition(dev(w.A), G=dev(w.G))
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    X0 = host(X).copy()
    LUg = host(s.work()).astype(np.float64)
    Xs = og.solve(LUg, w.G, w.B)
    print(f"  unrefined vs oracle substitution: {np.max(np.abs(X0 - Xs)) / np.max(np.abs(Xs)):.2e}", flush=True)
    assert np.max(np.abs(X0 - Xs)) <= 1e-8 * np.max(np.abs(Xs))
    st, eta = s.refine(Bd, X, max_iter=20, tol=1e-14, solver="luir")
    Xh = host(X)
    eta_o = og.backward_error_inf(w.A, Xh, w.B)
    info = s.info()
    print(f"  status {st} outer {info['iters']} eta {max(eta):.2e} oracle {eta_o.max():.2e} "
          f"hist {['%.1e' % e for e in info['eta_hist']]}", flush=True)
    assert st == genp.OK
    assert eta_o.shape == (k,) and np.all(eta_o <= 1e-14)


def test_lowprec_adjoint_with_refinement():
    """FP32 factors, adjoint refined against A^T: dB, dA match the oracle's FP64 gradient."""
    n, k = 256, 4
    w = wl.make("c5_n8192_scaled_lowrank", n=n, nrhs=k)
    s = genp.Solver(n, "f32", 64)
    s.precondition(dev(w.A), G=dev(w.G))
    assert s.factor() == 0
    X = s.solve(dev(w.B))
    s.refine(dev(w.B), X, 10, 1e-15)
    dB, dA = s.solve_backward(dev(w.W), X, want_dA=True, refine_iters=8)
    dBo, dAo = og.adjoint(w.A, host(X), w.W)
    kappa = np.linalg.cond(w.A, np.inf)
    tol = 10 * kappa * 1e-15
    assert np.max(np.abs(host(dB) - dBo)) <= tol * np.max(np.abs(dBo))
    assert np.max(np.abs(host(dA) - dAo)) <= tol * np.max(np.abs(dAo))


@pytest.mark.parametrize("solver", ["luir", "gmres"])
def test_bf16_factors_refine_honestly(solver):
    """BF16 Schur operands: kappa(A G) u_bf16 > 1 even for kappa(A) = 10 (G Gaussian makes
    kappa(C) ~ 1e3-1e4), so refinement need not converge.  The path must then say so
    (ENOCONV), keep the best iterate, and report the oracle's backward error of it."""
    n, k = 512, 1
    w = wl.haar_logspaced(n, 10.0, wl.MULT_DENSE, nrhs=k, seed=11)
    s = genp.Solver(n, "bf16", 128)
    s.precondition(dev(w.A), G=dev(w.G))
    assert s.factor() == 0
    Bd = dev(w.B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=6, tol=1e-14, solver=solver)
    info = s.info()
    eta_o = float(og.backward_error_inf(w.A, host(X), w.B).max())
    print(f"  bf16 {solver}: status {st} eta {max(eta):.2e} oracle {eta_o:.2e} hist "
          f"{['%.1e' % e for e in info['eta_hist']]}", flush=True)
    assert st in (genp.OK, genp.ENOCONV)
    assert abs(eta_o - max(eta)) <= 0.05 * eta_o + 1e-17
    assert max(eta) <= info["eta_hist"][0] * (1 + 1e-12)
    if st == genp.OK:
        assert eta_o <= 1e-14


def test_bf16_factors_converge_when_well_conditioned():
    """No multiplier and a strongly diagonally dominant A: kappa u_bf16 < 1, LU-IR converges."""
    n, k = 384, 2
    g = np.random.default_rng(3)
    A = g.standard_normal((n, n)) + 4.0 * n * np.eye(n)
    B = g.standard_normal((n, k))
    s = genp.Solver(n, "bf16", 128)
    s.precondition(dev(A))
    assert s.factor() == 0
    Bd = dev(B)
    X = s.solve(Bd)
    st, eta = s.refine(Bd, X, max_iter=20, tol=1e-14)
    assert st == genp.OK
    assert og.backward_error_inf(A, host(X), B).max() <= 1e-14
