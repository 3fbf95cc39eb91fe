"""Seeded synthetic inputs for the randomized-multiplier GENP workloads.

This module only draws random numbers and builds test matrices; it holds none
of the method's arithmetic (no multiplier product, no elimination, no
substitution).  Both the HIP path's tests/benchmark and the CPU oracle take
their inputs from here, so the same seed gives the same bytes on both sides.

Random numbers: ``numpy.random.default_rng(seed)`` (PCG64), ``standard_normal``
in C order.  The paper's theory uses Gaussian multipliers (Definition 3.2,
section 3.1); its own Fortran tests drew uniform [-1, 1) numbers (section 7),
which the workloads here do not follow.

Workloads (n, structure, multiplier, right-hand sides):

* ``rank_deficient_lead`` -- A ~ N(0,1) whose leading 8x8 block is the rank-4
  product X(8x4) Y(4x8), so GENP on A itself meets a singular leading block
  (section 1.1: GENP needs every leading block nonsingular); dense Gaussian G;
  one right-hand side.  Draw order: A, X, Y, G, B.
* ``haar_logspaced`` -- A = U diag(s) V^T with U = Q(Z_U), V = Q(Z_V) the
  unique orthogonal QR factors with positive diag(R) of Gaussian matrices
  (Fact 2.2), s_i = smax^((i-1)/(n-1)) ascending, so kappa_2(A) = smax; G dense
  Gaussian or Gaussian Toeplitz (Definition 3.2); nrhs Gaussian right-hand
  sides.  Draw order: Z_U, Z_V, G (or its 2n-1 parameters), B.
* ``scaled_gaussian_lowrank_lead`` -- A ~ N(0,1)/sqrt(n) whose leading 16x16
  block is X(16x8) Y(8x16)/sqrt(n) (rank 8); dense Gaussian G; nrhs
  right-hand sides and a weight matrix W ~ N(0,1) of the same shape.
  Draw order: A, X, Y, G, B, W.

Toeplitz parameter order: p[0 .. 2n-2] with G[i, j] = p[i - j + n - 1]
(0-based), i.e. p[n-1] is the diagonal, p[n-1+h] = t_h down the first column
and p[n-1-h] = t_{-h} along the first row (section 2.3 defines T = (t_{i-j})
by its first row and column but fixes no storage order).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

MULT_DENSE = "dense"
MULT_TOEPLITZ = "toeplitz"
MULT_CIRCULANT = "circulant"
MULT_CIRCULANT_PM1 = "circulant_pm1"   # circulant whose n entries are random signs +-1
MULT_HOUSEHOLDER = "householder"       # 2n parameters (u, v), independent random signs +-1


@dataclasses.dataclass
class Workload:
    """One seeded instance.  Arrays are float64, C-contiguous (row-major).

    ``G`` is the dense n x n multiplier (None for Toeplitz and circulant), ``p`` the
    2n-1 Toeplitz parameters or the n circulant parameters (None for dense).  ``W`` is only set for the
    differentiation workload.  On the ``cuda`` device the arrays are torch
    tensors instead of numpy arrays.
    """

    name: str
    n: int
    seed: int
    A: object
    B: object
    mult: str
    G: object = None
    p: object = None
    W: object = None
    smax: Optional[float] = None

    @property
    def nrhs(self) -> int:
        return int(self.B.shape[1])


def logspaced_singular_values(n: int, smax: float) -> np.ndarray:
    """s_i = smax^((i-1)/(n-1)), i = 1..n, ascending from 1 to smax."""
    if n == 1:
        return np.array([1.0])
    e = np.arange(n, dtype=np.float64) / (n - 1)
    return np.power(10.0, math.log10(smax) * e)


def _q_positive_r_numpy(z: np.ndarray) -> np.ndarray:
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return np.ascontiguousarray(q * d[None, :])


def _multiplier_draw(g: np.random.Generator, n: int, mult: str):
    if mult == MULT_DENSE:
        return g.standard_normal((n, n)), None
    if mult == MULT_TOEPLITZ:
        return None, g.standard_normal(2 * n - 1)
    if mult == MULT_CIRCULANT:
        return None, g.standard_normal(n)
    if mult == MULT_CIRCULANT_PM1:
        return None, pm1_signs(g, n)
    if mult == MULT_HOUSEHOLDER:
        return None, pm1_signs(g, 2 * n)
    raise ValueError(f"unknown multiplier kind {mult!r}")


def pm1_signs(g: np.random.Generator, n: int) -> np.ndarray:
    """n independent fair signs +-1 (FP64)."""
    return g.integers(0, 2, n).astype(np.float64) * 2.0 - 1.0


def pm1_redraw(n: int, seed: int, attempt: int) -> np.ndarray:
    """A fresh sign vector for attempt number `attempt` of the draw with this seed
    (independent stream per (seed, attempt); used when a draw is singular)."""
    return pm1_signs(np.random.default_rng([seed, 7919, attempt]), n)


def cs_illcond_lead(n: int, seed: int = 0, nrhs: int = 1, smallest_cos: float = 0.0) -> Workload:
    """A well conditioned (orthogonal) A whose n/2 x n/2 leading block is ill conditioned,
    with a +-1 circulant multiplier and b uniform in [-1, 1).

    The CS decomposition gives A = diag(U1, U2) [[C, -S], [S, C]] diag(V1, V2)^T with
    Haar U1, U2, V1, V2 of order n/2, C = diag(cos t_i), S = diag(sin t_i): A is
    orthogonal (kappa_2 = 1) and its leading block U1 C V1^T has singular values
    cos t_i.  The cosines are uniform in [0.5, 1) except the last, `smallest_cos`
    (0: the leading block has rank n/2 - 1 in exact arithmetic)."""
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    g = np.random.default_rng(seed)
    h = n // 2
    U1, U2, V1, V2 = (_q_positive_r_numpy(g.standard_normal((h, h))) for _ in range(4))
    cosv = g.uniform(0.5, 1.0, h)
    cosv[-1] = smallest_cos
    sinv = np.sqrt(1.0 - cosv * cosv)
    A = np.block([[(U1 * cosv) @ V1.T, -(U1 * sinv) @ V2.T],
                  [(U2 * sinv) @ V1.T, (U2 * cosv) @ V2.T]])
    B = g.uniform(-1.0, 1.0, (n, nrhs))
    c = pm1_signs(g, n)
    return Workload("cs_illcond_lead", n, seed, np.ascontiguousarray(A), B, MULT_CIRCULANT_PM1, p=c)


def svd_head_matrix(n: int, q: int, seed: int = 0, tail: float = 1e-10, mult: str = MULT_DENSE,
                    rho_plus: Optional[int] = None):
    """Table 7.2's matrices: A = S diag(sigma) T^T with Haar orthogonal S, T (positive-R QR of
    Gaussian matrices), sigma_j = 1/j for j <= q and `tail` beyond, so ||A||_2 = 1 and
    kappa(A) = 1 / tail.  Returns (A, S, sigma, T, G) with G the m x rho_+ multiplier
    (Gaussian, or the m + rho_+ - 1 Toeplitz parameters for mult = MULT_TOEPLITZ)."""
    g = np.random.default_rng(seed)
    S = _q_positive_r_numpy(g.standard_normal((n, n)))
    T = _q_positive_r_numpy(g.standard_normal((n, n)))
    sig = np.full(n, tail)
    sig[:q] = 1.0 / np.arange(1, q + 1)
    A = np.ascontiguousarray((S * sig[None, :]) @ T.T)
    k = q if rho_plus is None else rho_plus
    if mult == MULT_TOEPLITZ:
        G = g.standard_normal(n + k - 1)
    else:
        G = g.standard_normal((n, k))
    return A, S, sig, T, G


def lowrank_plus_noise(m: int, n: int, q: int, rho_plus: int, noise: float = 1e-10, seed: int = 12,
                       device: str = "cpu"):
    """A = X Y^T + E: X (m x q), Y (n x q) Gaussian, E Gaussian scaled so that
    ||E||_F = noise ||X Y^T||_F (numerical rank q); G (m x rho_+) Gaussian.  The large-size
    low-rank workload (the tables of section 7 stop at n = 256).  Returns (A, G)."""
    import torch
    g = np.random.default_rng(seed)
    X = torch.from_numpy(g.standard_normal((m, q))).to(device)
    Y = torch.from_numpy(g.standard_normal((n, q))).to(device)
    A = X @ Y.T
    E = torch.from_numpy(g.standard_normal((m, n))).to(device)
    A += E * (noise * float(torch.linalg.norm(A)) / float(torch.linalg.norm(E)))
    del E
    G = torch.from_numpy(g.standard_normal((m, rho_plus))).to(device)
    return A.contiguous(), G


def rank_deficient_lead(n: int = 256, seed: int = 1, nrhs: int = 1,
                        lead: int = 8, rank: int = 4) -> Workload:
    """A ~ N(0,1) with a rank-`rank` leading lead x lead block; dense G."""
    if not (1 <= rank <= lead <= n):
        raise ValueError("need 1 <= rank <= lead <= n")
    g = np.random.default_rng(seed)
    A = g.standard_normal((n, n))
    X = g.standard_normal((lead, rank))
    Y = g.standard_normal((rank, lead))
    A[:lead, :lead] = X @ Y
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, nrhs))
    return Workload("rank_deficient_lead", n, seed, A, B, MULT_DENSE, G=G)


def scaled_gaussian_lowrank_lead(n: int = 8192, seed: int = 5, nrhs: int = 64,
                                 lead: int = 16, rank: int = 8) -> Workload:
    """A ~ N(0,1)/sqrt(n), leading lead x lead block of rank `rank`; dense G; W."""
    g = np.random.default_rng(seed)
    s = 1.0 / math.sqrt(n)
    A = g.standard_normal((n, n)) * s
    X = g.standard_normal((lead, rank))
    Y = g.standard_normal((rank, lead))
    A[:lead, :lead] = (X @ Y) * s
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, nrhs))
    W = g.standard_normal((n, nrhs))
    return Workload("scaled_gaussian_lowrank_lead", n, seed, A, B, MULT_DENSE, G=G, W=W)


def haar_logspaced(n: int, smax: float, mult: str = MULT_DENSE, nrhs: int = 1,
                   seed: int = 2, device: str = "cpu") -> Workload:
    """A = U diag(s) V^T with Haar U, V; G dense or Toeplitz; B ~ N(0,1).

    ``device="cuda"`` draws the same Gaussian numbers on the host, then forms
    the two QR factorizations and the product with torch on the GPU (the
    host LAPACK route takes minutes at n = 16384).  The factors agree with
    the host route to rounding, not bit for bit; every consumer receives the
    arrays actually produced, so both sides of a comparison still see the
    same bytes.
    """
    g = np.random.default_rng(seed)
    s = logspaced_singular_values(n, smax)
    if device == "cpu":
        zu = g.standard_normal((n, n))
        zv = g.standard_normal((n, n))
        U = _q_positive_r_numpy(zu)
        del zu
        V = _q_positive_r_numpy(zv)
        del zv
        A = np.ascontiguousarray((U * s[None, :]) @ V.T)
        del U, V
        G, p = _multiplier_draw(g, n, mult)
        B = g.standard_normal((n, nrhs))
        return Workload("haar_logspaced", n, seed, A, B, mult, G=G, p=p, smax=smax)
    import torch  # GPU route: torch supplies QR and GEMM for input construction only
    dev = torch.device(device)

    def q_of(zh):
        z = torch.from_numpy(zh).to(dev)
        q, r = torch.linalg.qr(z)
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d[None, :]

    U = q_of(g.standard_normal((n, n)))
    V = q_of(g.standard_normal((n, n)))
    st = torch.from_numpy(s).to(dev)
    A = ((U * st[None, :]) @ V.T.contiguous()).contiguous()
    del U, V
    Gh, ph = _multiplier_draw(g, n, mult)
    Bh = g.standard_normal((n, nrhs))
    G = torch.from_numpy(Gh).to(dev) if Gh is not None else None
    p = torch.from_numpy(ph).to(dev) if ph is not None else None
    B = torch.from_numpy(Bh).to(dev)
    return Workload("haar_logspaced", n, seed, A, B, mult, G=G, p=p, smax=smax)


def haar_family(n: int, smaxes, mult: str = MULT_DENSE, nrhs: int = 1, seed: int = 2, device: str = "cuda"):
    """The haar_logspaced recipe for several smax at once: one draw of Z_U, Z_V, G and B (the
    draws of haar_logspaced with this seed), then A = U diag(s) V^T for each smax in turn.
    Yields one Workload per smax; only the current A is held beside U and V."""
    import torch
    dev = torch.device(device)
    g = np.random.default_rng(seed)

    def q_of(zh):
        z = torch.from_numpy(zh).to(dev)
        q, r = torch.linalg.qr(z)
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d[None, :]

    U = q_of(g.standard_normal((n, n)))
    Vt = q_of(g.standard_normal((n, n))).T.contiguous()
    Gh, ph = _multiplier_draw(g, n, mult)
    Bh = g.standard_normal((n, nrhs))
    G = torch.from_numpy(Gh).to(dev) if Gh is not None else None
    p = torch.from_numpy(ph).to(dev) if ph is not None else None
    B = torch.from_numpy(Bh).to(dev)
    for smax in smaxes:
        st = torch.from_numpy(logspaced_singular_values(n, smax)).to(dev)
        A = ((U * st[None, :]) @ Vt).contiguous()
        yield Workload("haar_logspaced", n, seed, A, B, mult, G=G, p=p, smax=float(smax))
        del A


# The five named workloads, with their sizes; `scale_n` lets tests build the
# same recipe at a size the oracle finishes in seconds.
NAMED = {
    "c1_n256_rankdef": dict(kind="rank_deficient_lead", n=256, seed=1, nrhs=1),
    "c2_n4096_haar1e4_dense": dict(kind="haar_logspaced", n=4096, smax=1e4, mult=MULT_DENSE,
                                   nrhs=16, seed=2),
    "c3_n16384_haar1e6_toeplitz": dict(kind="haar_logspaced", n=16384, smax=1e6,
                                       mult=MULT_TOEPLITZ, nrhs=1, seed=3),
    # plain-FP64 comparison at n = 16384: (a) the n = 16384 Toeplitz instance
    # itself, (b) the n = 4096 recipe (dense G, smax 1e4) grown to n = 16384
    "c4a_n16384_haar1e6_toeplitz": dict(kind="haar_logspaced", n=16384, smax=1e6,
                                        mult=MULT_TOEPLITZ, nrhs=64, seed=3),
    "c4b_n16384_haar1e4_dense": dict(kind="haar_logspaced", n=16384, smax=1e4,
                                     mult=MULT_DENSE, nrhs=64, seed=2),
    "c5_n8192_scaled_lowrank": dict(kind="scaled_gaussian_lowrank_lead", n=8192, seed=5,
                                    nrhs=64),
    # the benchmark's A with a Gaussian circulant multiplier (n parameters), applied by FFT
    "c3c_n16384_haar1e6_circulant": dict(kind="haar_logspaced", n=16384, smax=1e6,
                                         mult=MULT_CIRCULANT, nrhs=1, seed=3),
    "c3h_n16384_haar1e6_householder": dict(kind="haar_logspaced", n=16384, smax=1e6,
                                           mult=MULT_HOUSEHOLDER, nrhs=1, seed=3),
}


def make(name: str, n: Optional[int] = None, seed: Optional[int] = None,
         nrhs: Optional[int] = None, device: str = "cpu") -> Workload:
    """Build a named workload, optionally at another n / seed / nrhs."""
    spec = dict(NAMED[name])
    kind = spec.pop("kind")
    if n is not None:
        spec["n"] = n
    if seed is not None:
        spec["seed"] = seed
    if nrhs is not None:
        spec["nrhs"] = nrhs
    if kind == "rank_deficient_lead":
        return rank_deficient_lead(**spec)
    if kind == "scaled_gaussian_lowrank_lead":
        return scaled_gaussian_lowrank_lead(**spec)
    return haar_logspaced(device=device, **spec)


def gaussian(shape, seed: int) -> np.ndarray:
    """A plain seeded N(0,1) array (test directions, weights)."""
    return np.random.default_rng(seed).standard_normal(shape)
