"""Low-precision rounding and mirrors for the mixed-precision form (test infrastructure only).

The mixed form stores C = A G and its factors in FP32 or in BF16-operand /
FP32-accumulate arithmetic and restores accuracy by FP64 refinement.  The
paper fixes no precision (its tests are double, section 7.2); the readings
used here are:

* conversion FP64 -> FP32 is IEEE round-to-nearest-even (RNE);
* conversion to BF16 goes FP64 -> FP32 (RNE) -> BF16 (RNE on the upper 16
  bits of the FP32 pattern), NaN kept quiet, overflow to +-inf by rounding;
* a product of BF16 operands is exact in FP64 (8-bit significands), so
  ``product_of_rounded`` gives the exact value the MFMA sums approximate.

* the 2-word BF16 form splits an FP32 value x into hi = bf16(x) and
  lo = bf16(x - hi) (x - hi is exact in FP32: hi shares x's leading bits) and
  takes a product of split operands as hi_a hi_b + hi_a lo_b + lo_a hi_b,
  dropping lo_a lo_b; ``product_bf16x3`` gives the exact value of those three
  terms.

``genp_blocked_lowprec`` is an FP32 block elimination with optionally
BF16-rounded (or 2-word BF16) Schur-update operands.  It is pinned exactly on a
matrix built from its factors, where one block step's update is exact in FP32
when (and only when) its operands are rounded as stated.  On general inputs it
mirrors the kind of factorization the mixed form computes, not its bits (the
MFMA accumulation order is not specified anywhere), so tests compare the
library with it through statistics (growth, factor residual) and bounds.
"""
from __future__ import annotations

import numpy as np


def round_fp32(x) -> np.ndarray:
    """FP64 -> FP32, round to nearest even, returned as float64 values."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """FP32 array -> uint16 BF16 patterns (RNE, NaN quieted)."""
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x32)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(nan, ((u >> 16) | 0x0040) & 0xFFFF, r)
    return r.astype(np.uint16)


def bf16_bits_to_fp64(b: np.ndarray) -> np.ndarray:
    u = (np.asarray(b, dtype=np.uint32) << 16).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    """FP64 -> FP32 (RNE) -> BF16 (RNE), returned as float64 values."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    return bf16_bits_to_fp64(round_bf16_bits(x32)).reshape(np.shape(x))


def product_of_rounded(A, B, rounder) -> np.ndarray:
    """rounder(A) @ rounder(B) in FP64 (exact term-by-term for BF16 operands)."""
    return rounder(A) @ rounder(B)


def split_bf16x2(x):
    """(hi, lo) with hi = bf16(fp32(x)) and lo = bf16(fp32(x) - hi), as float64 values."""
    x32 = round_fp32(x)
    hi = round_bf16(x32)
    lo = round_bf16(x32 - hi)
    return hi, lo


def product_bf16x3(A, B) -> np.ndarray:
    """hi_A hi_B + hi_A lo_B + lo_A hi_B in FP64: the three products the 2-word BF16
    form accumulates (each term exact in FP64)."""
    ha, la = split_bf16x2(A)
    hb, lb = split_bf16x2(B)
    return ha @ hb + (ha @ lb + la @ hb)


def genp_blocked_lowprec(C, nb: int, bf16_update: bool = False, bf16x3_update: bool = False):
    """FP32 block GENP; with bf16_update the Schur-update operands L21 and U12
    are rounded to BF16 before the FP32 product (the stored factors keep their FP32
    values), with bf16x3_update the update is the 2-word BF16 product."""
    from scipy.linalg import solve_triangular

    LU = np.array(C, dtype=np.float32, copy=True)
    n = LU.shape[0]
    for k in range(0, n, nb):
        e = min(k + nb, n)
        for t in range(k, e):
            LU[t + 1:e, t] /= LU[t, t]
            LU[t + 1:e, t + 1:e] -= np.outer(LU[t + 1:e, t], LU[t, t + 1:e])
        if e < n:
            D = LU[k:e, k:e]
            L11 = np.tril(D, -1) + np.eye(e - k, dtype=np.float32)
            U11 = np.triu(D)
            LU[e:, k:e] = solve_triangular(U11.T, LU[e:, k:e].T, lower=True).T.astype(np.float32)
            LU[k:e, e:] = solve_triangular(L11, LU[k:e, e:], lower=True,
                                           unit_diagonal=True).astype(np.float32)
            L21, U12 = LU[e:, k:e], LU[k:e, e:]
            if bf16x3_update:
                LU[e:, e:] -= product_bf16x3(L21, U12).astype(np.float32)
                continue
            if bf16_update:
                L21 = round_bf16(L21).astype(np.float32)
                U12 = round_bf16(U12).astype(np.float32)
            LU[e:, e:] -= L21 @ U12
    return LU.astype(np.float64)
