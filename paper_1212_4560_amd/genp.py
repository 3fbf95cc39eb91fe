"""Python binding of ``libgenp.so`` (ctypes): argument marshalling only.

Every step of the method runs in the HIP library; torch supplies device
memory (tensors) and the stream.  The functions mirror the C ABI of
``include/genp.h`` one to one:

    genp_create / genp_precondition / genp_factor / genp_solve /
    genp_refine(_ex) / genp_solve_backward(_ex) / genp_condest / genp_get_info /
    genp_copy_work

plus :func:`solve` (the whole path in one call) and :class:`GenpSolve`, a
``torch.autograd.Function`` whose backward is the library's adjoint.

There is no fallback: if the library is missing or no gfx950 device is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgenp.so")

F64, F32, BF16, BF16X3 = 0, 1, 2, 3
G_DENSE, G_TOEPLITZ, G_NONE, G_CIRCULANT, G_HOUSEHOLDER = 0, 1, 2, 3, 4
SOLVER_LUIR, SOLVER_GMRES, SOLVER_AUTO = 0, 1, 2
OK, BREAKDOWN, ENOCONV = 0, 1, 2
EINVAL, EDEVICE, ENOMEM, ESTATE, ENOTSUP, ESINGULAR, ESCRATCH = -1, -2, -3, -4, -5, -6, -7
ETA_HIST = 64

PRECS = {"f64": F64, "f32": F32, "bf16": BF16, "bf16x3": BF16X3}
SOLVERS = {"luir": SOLVER_LUIR, "gmres": SOLVER_GMRES, "auto": SOLVER_AUTO}

# the entry points declared in include/genp.h
EXPORTS = ("genp_create", "genp_destroy", "genp_precondition", "genp_precondition2", "genp_factor", "genp_solve",
           "genp_factor_block", "genp_block_pivots", "genp_row_perm",
           "genp_lowrank", "genp_numerical_rank", "genp_numerical_rank_noalloc",
           "genp_refine", "genp_refine_ex", "genp_solve_backward", "genp_solve_backward_ex", "genp_condest",
           "genp_get_info", "genp_copy_work", "genp_strerror")
GMRES_MAX_RESTART = 1024


class GenpInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nb", ctypes.c_int64),
        ("prec", ctypes.c_int32), ("mult", ctypes.c_int32),
        ("breakdown_col", ctypes.c_int64),
        ("min_abs_piv", ctypes.c_double), ("max_abs_piv", ctypes.c_double),
        ("max_abs_c", ctypes.c_double), ("max_abs_u", ctypes.c_double),
        ("growth", ctypes.c_double), ("anorm_inf", ctypes.c_double),
        ("iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
        ("eta", ctypes.c_double), ("n_eta", ctypes.c_int32),
        ("eta_hist", ctypes.c_double * ETA_HIST),
        ("ms_precond", ctypes.c_double), ("ms_factor", ctypes.c_double),
        ("ms_solve", ctypes.c_double), ("ms_refine", ctypes.c_double),
        ("ms_backward", ctypes.c_double),
        ("ms_ag", ctypes.c_double), ("ms_schur", ctypes.c_double), ("ms_panel", ctypes.c_double),
        ("n_schur", ctypes.c_int32),
        ("cond_g", ctypes.c_double),
        ("mult_left", ctypes.c_int32), ("cond_h", ctypes.c_double),
        ("block_ge", ctypes.c_int32), ("row_swaps", ctypes.c_int64),
        ("ms_condest", ctypes.c_double), ("cond1_c", ctypes.c_double), ("norm1_c", ctypes.c_double),
        ("norm1_inv", ctypes.c_double),
        ("bwd_iters", ctypes.c_int32), ("bwd_inner_iters", ctypes.c_int32), ("bwd_eta", ctypes.c_double),
        ("anorm_1", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "eta_hist"}
        d["eta_hist"] = [self.eta_hist[i] for i in range(self.n_eta)]
        return d


class GenpRefineOpts(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("restart", ctypes.c_int32),
        ("max_inner", ctypes.c_int32), ("tol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
    ]


def refine_opts(max_iter: int = 2, tol: float = 0.0, solver: str = "luir", restart: int = 50,
                max_inner: int = 0, inner_rtol: float = 1e-10) -> GenpRefineOpts:
    return GenpRefineOpts(SOLVERS[solver], int(max_iter), int(restart), int(max_inner), float(tol),
                          float(inner_rtol))


class GenpLrInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("rho_plus", ctypes.c_int64),
        ("rank", ctypes.c_int64), ("failed", ctypes.c_int32),
        ("a_fro", ctypes.c_double), ("tail_fro", ctypes.c_double), ("resid_fro", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("ms_sketch", ctypes.c_double), ("ms_basis", ctypes.c_double),
        ("ms_project", ctypes.c_double), ("ms_resid", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class GenpNrankInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("rho_minus", ctypes.c_int64), ("rho_plus", ctypes.c_int64),
        ("rank", ctypes.c_int64), ("tests", ctypes.c_int32),
        ("cond_at_rank", ctypes.c_double), ("cond_above", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("ms_sketch", ctypes.c_double), ("ms_gram", ctypes.c_double),
        ("ms_search", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class GenpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1212_4560_amd.build`")
    L = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.genp_create.argtypes = [ctypes.POINTER(vp), i64, i32, i32, vp]
    L.genp_destroy.argtypes = [vp]
    L.genp_precondition.argtypes = [vp, vp, i64, i32, vp, i64]
    L.genp_precondition2.argtypes = [vp, vp, i64, i32, vp, i64, i32, vp, i64]
    L.genp_numerical_rank.argtypes = [vp, i64, i64, i64, vp, i64, i64, i64, dbl, vp, i64,
                                      ctypes.POINTER(GenpNrankInfo), vp]
    L.genp_numerical_rank_noalloc.argtypes = L.genp_numerical_rank.argtypes
    L.genp_lowrank.argtypes = [vp, i64, i64, i64, i32, vp, i64, i64, dbl, dbl, vp, i64, vp, i64, vp, i64,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(GenpLrInfo), vp]
    L.genp_factor.argtypes = [vp, dbl, ctypes.POINTER(i64)]
    L.genp_factor_block.argtypes = [vp, dbl, ctypes.POINTER(i64)]
    L.genp_block_pivots.argtypes = [vp, vp, i64]
    L.genp_row_perm.argtypes = [vp, vp]
    L.genp_solve.argtypes = [vp, vp, i64, i64, vp, i64]
    L.genp_refine.argtypes = [vp, vp, i64, i64, vp, i64, i32, dbl, i32, ctypes.POINTER(dbl)]
    L.genp_refine_ex.argtypes = [vp, vp, i64, i64, vp, i64, ctypes.POINTER(GenpRefineOpts), ctypes.POINTER(dbl)]
    L.genp_solve_backward.argtypes = [vp, vp, i64, vp, i64, i64, vp, i64, vp, i64, i32]
    L.genp_solve_backward_ex.argtypes = [vp, vp, i64, vp, i64, i64, vp, i64, vp, i64,
                                         ctypes.POINTER(GenpRefineOpts), ctypes.POINTER(dbl)]
    L.genp_condest.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.genp_get_info.argtypes = [vp, ctypes.POINTER(GenpInfo)]
    L.genp_copy_work.argtypes = [vp, vp, i64]
    L.genp_strerror.argtypes = [i32]
    L.genp_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "genp_strerror":
            getattr(L, name).restype = i32
    _lib = L
    return L


def strerror(status: int) -> str:
    try:
        return load().genp_strerror(status).decode()
    except RuntimeError:
        return f"status {status}"


def _check(status: int, where: str, allow=(OK,)) -> int:
    if status not in allow:
        raise GenpError(status, where)
    return status


def _mat(t, name: str, rows: int, cols: Optional[int] = None):
    """(pointer, leading dimension) of a float64 CUDA tensor with unit column stride."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name}: need a float64 CUDA tensor")
    if t.dim() == 1:
        if t.stride(0) != 1 or t.shape[0] != rows:
            raise ValueError(f"{name}: bad shape/stride")
        return t.data_ptr(), 1
    if t.dim() != 2 or t.shape[0] != rows or (cols is not None and t.shape[1] != cols):
        raise ValueError(f"{name}: expected shape ({rows}, {cols}), got {tuple(t.shape)}")
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError(f"{name}: columns must be contiguous")
    return t.data_ptr(), max(t.stride(0), t.shape[1])


class Solver:
    """One genp_ctx: n x n systems, a working precision and a panel width."""

    def __init__(self, n: int, prec: str = "f64", nb: int = 256, stream=None):
        import torch
        L = load()
        self.n = int(n)
        self.nb = int(nb)
        self.prec = prec
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.genp_create(ctypes.byref(h), self.n, PRECS[prec], int(nb), ctypes.c_void_p(self.stream.cuda_stream)),
               "genp_create")
        self._h = h
        self._keep = ()   # tensors the context borrows (A, dense G)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.genp_destroy(h)
        self._h = None
        self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _mult(self, kind, t):
        """(kind code, pointer, leading dimension) of a multiplier given as (kind name, tensor)."""
        n = self.n
        if kind is None:
            return G_NONE, 0, n
        if kind == "dense":
            g, ld = _mat(t, "G", n, n)
            return G_DENSE, g, ld
        shapes = {"toeplitz": (G_TOEPLITZ, 2 * n - 1), "circulant": (G_CIRCULANT, n),
                  "householder": (G_HOUSEHOLDER, 2 * n)}
        if kind not in shapes:
            raise ValueError(f"unknown multiplier kind {kind!r}")
        code, length = shapes[kind]
        g, _ = _mat(t, kind, length)
        return code, g, n

    def precondition(self, A, G=None, p=None, c=None, uv=None, left=None):
        """C = H A G.  The right multiplier G: dense G, Toeplitz with parameters p, circulant
        with first column c, Householder with parameters uv = (u, v), or none.  The left
        multiplier H: left = (kind, tensor) with kind "dense", "toeplitz", "circulant" or
        "householder" (FP64 contexts only), or None."""
        n = self.n
        a, lda = _mat(A, "A", n, n)
        if G is not None:
            right = ("dense", G)
        elif p is not None:
            right = ("toeplitz", p)
        elif c is not None:
            right = ("circulant", c)
        elif uv is not None:
            right = ("householder", uv)
        else:
            right = (None, None)
        rk, g, ldg = self._mult(*right)
        lk, h, ldh = self._mult(*(left if left is not None else (None, None)))
        if lk == G_NONE:
            _check(load().genp_precondition(self._h, a, lda, rk, g, ldg), "genp_precondition")
        else:
            _check(load().genp_precondition2(self._h, a, lda, lk, h, ldh, rk, g, ldg), "genp_precondition2")
        self._keep = (A, right[1], left)
        return self

    def factor(self, pivot_tol: float = 0.0, block: bool = False) -> int:
        """Blocked GENP, or with block=True block Gaussian elimination with row
        interchanges inside each diagonal block pivot (genp_factor_block); returns the
        1-based breakdown column (0 = none)."""
        bk = ctypes.c_int64(0)
        name = "genp_factor_block" if block else "genp_factor"
        _check(getattr(load(), name)(self._h, float(pivot_tol), ctypes.byref(bk)), name, allow=(OK, BREAKDOWN))
        return int(bk.value)

    def block_pivots(self):
        """The explicit block pivots B_k stacked by rows: an n x nb FP64 tensor."""
        import torch
        out = torch.empty((self.n, self.nb), dtype=torch.float64, device="cuda")
        o, ldo = _mat(out, "out", self.n, self.nb)
        _check(load().genp_block_pivots(self._h, o, ldo), "genp_block_pivots")
        return out

    def row_perm(self):
        """Row r of the factors is row perm[r] of C (int32 tensor of n)."""
        import torch
        perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(load().genp_row_perm(self._h, ctypes.c_void_p(perm.data_ptr())), "genp_row_perm")
        return perm

    def solve(self, B, X=None):
        import torch
        k = B.shape[1]
        b, ldb = _mat(B, "B", self.n)
        if X is None:
            X = torch.empty((self.n, k), dtype=torch.float64, device=B.device)
        x, ldx = _mat(X, "X", self.n, k)
        _check(load().genp_solve(self._h, b, ldb, k, x, ldx), "genp_solve")
        return X

    def refine(self, B, X, max_iter: int = 2, tol: float = 0.0, solver: str = "luir", restart: int = None,
               max_inner: int = 0, inner_rtol: float = 0.0):
        """In-place refinement of X; returns (status, eta per column).  Without restart,
        max_inner or inner_rtol this is genp_refine; with any of them genp_refine_ex."""
        k = B.shape[1]
        b, ldb = _mat(B, "B", self.n, k)
        x, ldx = _mat(X, "X", self.n, k)
        eta = (ctypes.c_double * k)()
        if restart is None and not max_inner and not inner_rtol:
            st = _check(load().genp_refine(self._h, b, ldb, k, x, ldx, int(max_iter), float(tol),
                                           SOLVERS[solver], eta), "genp_refine", allow=(OK, ENOCONV))
        else:
            o = refine_opts(max_iter, tol, solver, restart or 0, max_inner, inner_rtol)
            st = _check(load().genp_refine_ex(self._h, b, ldb, k, x, ldx, ctypes.byref(o), eta),
                        "genp_refine_ex", allow=(OK, ENOCONV))
        return st, [eta[i] for i in range(k)]

    def solve_backward(self, W, X, want_dA: bool = True, refine_iters: int = 1, solver: str = None,
                       tol: float = 0.0, restart: int = 0, max_inner: int = 0, inner_rtol: float = 0.0,
                       return_status: bool = False):
        """dB = A^{-T} W and dA = -dB X^T from the stored factors.  With solver=None this is
        genp_solve_backward (refine_iters LU-IR steps against A^T); with a solver name,
        genp_solve_backward_ex (refine_iters outer steps, tol, GMRES restart / budget).
        Returns (dB, dA), or (dB, dA, status, eta per column) with return_status."""
        import torch
        k = W.shape[1]
        w, ldw = _mat(W, "W", self.n, k)
        x, ldx = _mat(X, "X", self.n, k)
        dB = torch.empty((self.n, k), dtype=torch.float64, device=W.device)
        db, lddb = _mat(dB, "dB", self.n, k)
        dA = None
        da, ldda = 0, self.n
        if want_dA:
            dA = torch.empty((self.n, self.n), dtype=torch.float64, device=W.device)
            da, ldda = _mat(dA, "dA", self.n, self.n)
        eta = (ctypes.c_double * k)()
        if solver is None:
            st = _check(load().genp_solve_backward(self._h, w, ldw, x, ldx, k, db, lddb, da, ldda,
                                                   int(refine_iters)), "genp_solve_backward", allow=(OK, ENOCONV))
            etal = [float("nan")] * k
        else:
            o = refine_opts(refine_iters, tol, solver, restart, max_inner, inner_rtol)
            st = _check(load().genp_solve_backward_ex(self._h, w, ldw, x, ldx, k, db, lddb, da, ldda,
                                                      ctypes.byref(o), eta), "genp_solve_backward_ex",
                        allow=(OK, ENOCONV))
            etal = [eta[i] for i in range(k)]
        if return_status:
            return dB, dA, st, etal
        return dB, dA

    def condest(self) -> dict:
        """Hager-Higham estimates of ||C||_1, ||(LU)^{-1}||_1 and their product (genp_condest)."""
        kap, nc, ni = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load().genp_condest(self._h, ctypes.byref(kap), ctypes.byref(nc), ctypes.byref(ni)), "genp_condest")
        return {"kappa1": kap.value, "norm1_c": nc.value, "norm1_inv": ni.value}

    def info(self) -> dict:
        inf = GenpInfo()
        _check(load().genp_get_info(self._h, ctypes.byref(inf)), "genp_get_info")
        return inf.as_dict()

    def work(self):
        """FP64 copy of the working matrix (C, or L \\ U after factor)."""
        import torch
        out = torch.empty((self.n, self.n), dtype=torch.float64, device="cuda")
        o, ldo = _mat(out, "out", self.n, self.n)
        _check(load().genp_copy_work(self._h, o, ldo), "genp_copy_work")
        return out


def solve(A, B, G=None, p=None, prec: str = "f64", nb: int = 256, refine: int = 2,
          tol: float = 0.0, pivot_tol: float = 0.0, solver: str = "luir", c=None, uv=None, left=None,
          block: bool = False):
    """The whole path: C = H A G, GENP, substitutions, X = G Y, refinement.
    The right multiplier: dense G, Toeplitz parameters p, circulant first column c or
    Householder parameters uv; the left one: left = (kind, tensor) or None.
    block=True factors by block Gaussian elimination with explicit block pivots.

    Returns (X, info dict, solver object).  Raises GenpError on breakdown.
    """
    s = Solver(A.shape[0], prec, nb)
    s.precondition(A, G=G, p=p, c=c, uv=uv, left=left)
    bk = s.factor(pivot_tol, block=block)
    if bk:
        raise GenpError(BREAKDOWN, f"genp_factor (column {bk})")
    X = s.solve(B)
    if refine > 0:
        s.refine(B, X, refine, tol, solver)
    return X, s.info(), s


def lowrank(A, rho_plus: int, G=None, p=None, tau: float = 1e-8, tau2: float = 1e-6, want_ahat: bool = False,
            stream=None):
    """Randomized rank-s approximation A ~ W_s T_s^T (Proto-Algorithm 5.1, orthogonal basis of
    Remark 5.4) through genp_lowrank.  G: m x rho_+ multiplier, or p: its m + rho_+ - 1 Toeplitz
    parameters.  Returns dict(rank, T (n x s), W (m x s), Ahat or None, perm, info)."""
    import torch
    m, n = A.shape
    k = int(rho_plus)
    a, lda = _mat(A, "A", m, n)
    if G is not None:
        g, ldg = _mat(G, "G", m, k)
        mult = G_DENSE
    elif p is not None:
        g, _ = _mat(p, "p", m + k - 1)
        ldg, mult = k, G_TOEPLITZ
    else:
        raise ValueError("need G or p")
    T = torch.empty((n, k), dtype=torch.float64, device=A.device)
    W = torch.empty((m, k), dtype=torch.float64, device=A.device)
    Ah = torch.empty((m, n), dtype=torch.float64, device=A.device) if want_ahat else None
    t, ldt = _mat(T, "T", n, k)
    w, ldw = _mat(W, "W", m, k)
    ah, ldah = (_mat(Ah, "Ahat", m, n) if Ah is not None else (0, n))
    perm = (ctypes.c_int32 * k)()
    info = GenpLrInfo()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load().genp_lowrank(a, m, n, lda, mult, g, ldg, k, float(tau), float(tau2), t, ldt, w, ldw, ah, ldah,
                               perm, ctypes.byref(info), ctypes.c_void_p(st.cuda_stream)), "genp_lowrank")
    s = int(info.rank)
    return {"rank": s, "T": T[:, :s], "W": W[:, :s], "Ahat": Ah, "perm": [perm[i] for i in range(k)],
            "info": info.as_dict(), "_keep": (A, G, p)}


def numerical_rank(A, G, rho_minus: int, rho_plus: int, cond_max: float = 1e6, stream=None, B=None,
                   noalloc: bool = False):
    """Numerical rank of A in [rho_-, rho_+] without pivoting or orthogonalization
    (Proto-Algorithm B.1) through genp_numerical_rank, or genp_numerical_rank_noalloc (scratch
    from the library's fixed device array) with noalloc=True.  G: the m x rho_+ Gaussian
    multiplier; B: optional n x rho_+ output tensor.  Returns dict(rank, B (n x rank: the first
    columns of A^T G), info)."""
    import torch
    m, n = A.shape
    k = int(rho_plus)
    a, lda = _mat(A, "A", m, n)
    g, ldg = _mat(G, "G", m, k)
    if B is None:
        B = torch.empty((n, k), dtype=torch.float64, device=A.device)
    b, ldb = _mat(B, "B", n, k)
    info = GenpNrankInfo()
    st = stream if stream is not None else torch.cuda.current_stream()
    name = "genp_numerical_rank_noalloc" if noalloc else "genp_numerical_rank"
    _check(getattr(load(), name)(a, m, n, lda, g, ldg, int(rho_minus), k, float(cond_max), b, ldb,
                                 ctypes.byref(info), ctypes.c_void_p(st.cuda_stream)), name)
    r = int(info.rank)
    return {"rank": r, "B": B[:, :r], "info": info.as_dict()}


def _autograd_function():
    import torch

    class GenpSolve(torch.autograd.Function):
        """X = A^{-1} B through the randomized GENP path; backward = library adjoint.

        Gradients: dB = A^{-T} gX (L^{-T} U^{-T} G^T gX plus refinement),
        dA = -dB X^T.  The multiplier receives no gradient.
        """

        @staticmethod
        def forward(ctx, A, B, G=None, p=None, prec="f64", nb=256, refine=2, refine_bwd=1, c=None, uv=None,
                    left=None):
            X, _, s = solve(A.detach(), B.detach(), G=G, p=p, prec=prec, nb=nb, refine=refine, c=c, uv=uv, left=left)
            ctx.solver = s
            ctx.refine_bwd = refine_bwd
            ctx.save_for_backward(X)
            return X

        @staticmethod
        def backward(ctx, gX):
            (X,) = ctx.saved_tensors
            dB, dA = ctx.solver.solve_backward(gX.contiguous(), X, want_dA=ctx.needs_input_grad[0],
                                               refine_iters=ctx.refine_bwd)
            return dA, dB, None, None, None, None, None, None, None, None, None

    return GenpSolve


_genp_solve_cls = None


def __getattr__(name):
    global _genp_solve_cls
    if name == "GenpSolve":
        if _genp_solve_cls is None:
            _genp_solve_cls = _autograd_function()
        return _genp_solve_cls
    raise AttributeError(name)
