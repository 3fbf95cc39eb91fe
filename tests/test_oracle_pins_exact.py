"""Exact pins of three oracle functions that statistics alone would not catch (CPU only).

* ``relative_residual`` (Table 7.1's quantity) against a hand-worked 2 x 2 case whose
  2-, infinity- and 1-norm ratios differ, one column at a time.
* ``theorem_2_2_bounds`` (Theorem 2.2's N + N_- N^2 and N_-) against two hand-worked
  3 x 3 cases: one whose N_- comes from a leading 1 x 1 block and one whose N_- comes
  from the whole matrix.
* ``genp_blocked_lowprec`` (the FP32 / BF16 / 2-word BF16 mirror of the precision
  form) on a matrix built from its factors so that every rounding the mirror is
  supposed to make, and only those, is visible: the Schur update of one block step is
  exact in FP32 when its operands are rounded the stated way, so the whole packed
  factorization is known in closed form.  The expected values use integer arithmetic
  on the significands (round half to even by ``numpy.round``), not the oracle's
  rounding functions.

Each check is also run against planted mistakes that must fail it.
"""
import inspect
import json
import os
import textwrap

import numpy as np
import pytest

from oracle import blockge as obg, genp as og, lowprec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _arr(x):
    return np.array(x, dtype=np.float64)


# ------------------------------------------------------------- relative residual ----

def check_relative_residual():
    e = _golden()["relative_residual_2x2"]
    r = og.relative_residual(_arr(e["A"]), _arr(e["y"]), _arr(e["b"]))
    return bool(r.shape == (2,) and np.allclose(r, e["rel_2"], rtol=1e-15, atol=0))


def test_relative_residual_hand_example():
    assert check_relative_residual()
    e = _golden()["relative_residual_2x2"]
    # the fixture itself separates the norms: a check that passed for all of them would be vacuous
    assert e["rel_2"][0] != e["rel_inf"][0] != e["rel_1"][0]


# ------------------------------------------------------------- Theorem 2.2 bounds ----

def check_theorem_2_2():
    g = _golden()
    ok = True
    for key in ("theorem_2_2_bounds_3x3", "theorem_2_2_bounds_diag"):
        e = g[key]
        top, nm = obg.theorem_2_2_bounds(_arr(e["C"]))
        ok &= np.isclose(top, e["pivot_bound"], rtol=1e-13, atol=0) and np.isclose(nm, e["N_minus"], rtol=1e-13, atol=0)
    return bool(ok)


def test_theorem_2_2_bounds_hand_examples():
    assert check_theorem_2_2()


# ------------------------------------------------ low-precision mirror, exact case ----

def _bf16_of_fraction_bits(m):
    """bf16 of x = 1 + m / 1024 (0 <= m < 1024): keep 7 fraction bits, ties to even."""
    return 1.0 + np.round(m / 8.0) / 128.0


def _exact_case(mode, seed=3):
    """C (4 x 4) and its packed factors for one nb = 2 block step.

    C11 = L11 U11 with L11 = [[1, 0], [1, 1]], U11 = [[2, 1], [0, 4]]; U12, L21 with
    entries +-(1 + m / 1024), m odd (so BF16 rounding changes every one of them);
    C12 = L11 U12, C21 = L21 U11 (exact).  C22 = P + D where P is the Schur product the
    mode computes (FP32: L21 U12; BF16: bf16(L21) bf16(U12); 2-word BF16: hi hi + hi lo +
    lo hi = L21 U12 - lo(L21) lo(U12)), all exact in FP32, and D = [[2, 1], [4, 3]], whose
    own GENP is exact.  The trailing block after the step is therefore exactly D."""
    g = np.random.default_rng(seed)
    mL = 2 * g.integers(0, 512, (2, 2)) + 1
    mU = 2 * g.integers(0, 512, (2, 2)) + 1
    sL = np.where(g.random((2, 2)) < 0.5, -1.0, 1.0)
    sU = np.where(g.random((2, 2)) < 0.5, -1.0, 1.0)
    L21 = sL * (1.0 + mL / 1024.0)
    U12 = sU * (1.0 + mU / 1024.0)
    hiL, hiU = sL * _bf16_of_fraction_bits(mL), sU * _bf16_of_fraction_bits(mU)
    loL, loU = L21 - hiL, U12 - hiU
    if mode == "f32":
        P = L21 @ U12
    elif mode == "bf16":
        P = hiL @ hiU
    else:
        P = L21 @ U12 - loL @ loU
    L11 = _arr([[1, 0], [1, 1]])
    U11 = _arr([[2, 1], [0, 4]])
    D = _arr([[2, 1], [4, 3]])
    C = np.block([[L11 @ U11, L11 @ U12], [L21 @ U11, P + D]])
    LU = np.block([[np.tril(L11, -1) + U11, U12], [L21, _arr([[2, 1], [2, 1]])]])
    assert np.array_equal(C, C.astype(np.float32).astype(np.float64)), "inputs must be exact in FP32"
    assert np.all(loL != 0) and np.all(loU != 0)
    return C, LU


def check_lowprec_exact():
    ok = True
    for mode, kw in (("f32", {}), ("bf16", {"bf16_update": True}), ("bf16x3", {"bf16x3_update": True})):
        C, LU = _exact_case(mode)
        ok &= np.array_equal(lowprec.genp_blocked_lowprec(C, 2, **kw), LU)
    return bool(ok)


def test_lowprec_mirror_exact_one_block_step():
    assert check_lowprec_exact()


def test_exact_cases_separate_the_three_modes():
    # the matrix built for one mode must not factor exactly in another (else the pin is vacuous)
    for mode in ("f32", "bf16", "bf16x3"):
        C, LU = _exact_case(mode)
        for other, kw in (("f32", {}), ("bf16", {"bf16_update": True}), ("bf16x3", {"bf16x3_update": True})):
            if other != mode:
                assert not np.array_equal(lowprec.genp_blocked_lowprec(C, 2, **kw), LU), (mode, other)


# ------------------------------------------------------------------ planted mistakes ----

CHECKS = [check_relative_residual, check_theorem_2_2, check_lowprec_exact]

MUTANTS = {
    "relative residual: infinity norm": (
        og, "relative_residual", "np.linalg.norm(A @ X2 - B2, axis=0) / np.linalg.norm(B2, axis=0)",
        "np.max(np.abs(A @ X2 - B2), axis=0) / np.max(np.abs(B2), axis=0)"),
    "relative residual: 1-norm": (
        og, "relative_residual", "np.linalg.norm(A @ X2 - B2, axis=0) / np.linalg.norm(B2, axis=0)",
        "np.sum(np.abs(A @ X2 - B2), axis=0) / np.sum(np.abs(B2), axis=0)"),
    "relative residual: Frobenius over all columns": (
        og, "relative_residual", "np.linalg.norm(A @ X2 - B2, axis=0) / np.linalg.norm(B2, axis=0)",
        "np.full(X2.shape[1], np.linalg.norm(A @ X2 - B2) / np.linalg.norm(B2))"),
    "relative residual: scaled by ||A|| ||y||": (
        og, "relative_residual", "/ np.linalg.norm(B2, axis=0)",
        "/ (np.linalg.norm(A, 2) * np.linalg.norm(X2, axis=0))"),
    "Theorem 2.2: Frobenius norm for N": (
        obg, "theorem_2_2_bounds", "N = float(np.linalg.norm(C, 2))", "N = float(np.linalg.norm(C))"),
    "Theorem 2.2: only the whole matrix for N_-": (
        obg, "theorem_2_2_bounds", "for j in range(1, C.shape[0] + 1)", "for j in range(C.shape[0], C.shape[0] + 1)"),
    "Theorem 2.2: leading blocks from 2 x 2": (
        obg, "theorem_2_2_bounds", "for j in range(1, C.shape[0] + 1)", "for j in range(2, C.shape[0] + 1)"),
    "Theorem 2.2: leading blocks stop before the whole matrix": (
        obg, "theorem_2_2_bounds", "for j in range(1, C.shape[0] + 1)", "for j in range(1, C.shape[0])"),
    "Theorem 2.2: N_- N instead of N_- N^2": (
        obg, "theorem_2_2_bounds", "return N + Nm * N * N, Nm", "return N + Nm * N, Nm"),
    "mirror: U12 left unrounded in the BF16 update": (
        lowprec, "genp_blocked_lowprec", "U12 = round_bf16(U12).astype(np.float32)", "U12 = U12"),
    "mirror: L21 left unrounded in the BF16 update": (
        lowprec, "genp_blocked_lowprec", "L21 = round_bf16(L21).astype(np.float32)", "L21 = L21"),
    "mirror: rounded L21 written back into the stored factors": (
        lowprec, "genp_blocked_lowprec", "L21 = round_bf16(L21).astype(np.float32)",
        "L21 = LU[e:, k:e] = round_bf16(L21).astype(np.float32)"),
    "mirror: Schur update with the wrong sign": (
        lowprec, "genp_blocked_lowprec", "LU[e:, e:] -= L21 @ U12", "LU[e:, e:] += L21 @ U12"),
    "mirror: 2-word update as a single BF16 product": (
        lowprec, "genp_blocked_lowprec", "product_bf16x3(L21, U12)", "product_of_rounded(L21, U12, round_bf16)"),
    "mirror: L21 solved against U11 instead of its transpose": (
        lowprec, "genp_blocked_lowprec", "solve_triangular(U11.T, LU[e:, k:e].T, lower=True)",
        "solve_triangular(U11, LU[e:, k:e].T, lower=False)"),
}


def run_checks():
    out = []
    for c in CHECKS:
        try:
            with np.errstate(all="ignore"):
                out.append(c())
        except Exception:
            out.append(False)
    return out


def test_checks_pass_on_the_oracle():
    assert all(run_checks())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    mod, attr, old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(mod, attr)))
    assert old in src, old
    ns = dict(vars(mod))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    monkeypatch.setattr(mod, attr, ns[attr])
    assert not all(run_checks()), f"mutant not caught: {name}"
