/*
 * genp.h -- C ABI of the randomized-multiplier GENP solver for AMD MI355X (gfx950).
 *
 * Method (Pan & Qian, "More on the Power of Randomized Matrix Multiplication"):
 * section 1.1 solves a nonsingular system A x = b by multiplying A by a random
 * matrix and running Gaussian elimination with no pivoting (GENP) on the
 * product.  Here the multiplier G is applied on the right (Corollary 4.1(ii):
 * the leading blocks of A H are nonsingular with probability 1 and well
 * conditioned with high probability whenever A is nonsingular):
 *
 *     C = A G  ->  C = L U (no pivoting)  ->  Y = U^{-1} L^{-1} B  ->  X = G Y,
 *
 * followed by iterative refinement X += G (LU)^{-1} (B - A X) (section 7.1,
 * Table 7.1; at most two steps in section 7.2).  G is either a dense Gaussian
 * matrix or a Gaussian Toeplitz matrix given by its 2n-1 parameters
 * (Definition 3.2; Toeplitz structure of section 2.3).
 *
 * Conventions shared by every call:
 *  - Matrices are row-major (C order, torch-contiguous): element (i, j) of an
 *    n x m matrix M with leading dimension ldm is M[i * ldm + j], ldm >= m.
 *  - Every matrix/vector pointer is a DEVICE pointer on the context's device.
 *  - Work is ordered on the HIP stream given to genp_create.  Calls that
 *    report a numerical status (genp_factor, genp_refine, genp_get_info)
 *    synchronize that stream before returning; the others only enqueue work.
 *  - Ownership: A and a dense G are BORROWED by genp_precondition and must
 *    stay valid and unchanged until the next genp_precondition or
 *    genp_destroy (refinement and the adjoint read them again).  Toeplitz
 *    parameters are copied.  B, X, W, dB, dA belong to the caller.  The
 *    working matrix C (later L \ U) and all scratch belong to the context.
 *  - Status codes: 0 = success; > 0 = numerical outcome with defined outputs;
 *    < 0 = caller or device error, outputs undefined.  No exception or abort
 *    crosses this interface.
 *  - Call order: create -> precondition -> factor -> solve / refine /
 *    solve_backward (any number of times) -> destroy.  Out of order calls
 *    return GENP_ESTATE.  One context serves one host thread at a time.
 */
#ifndef GENP_H
#define GENP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct genp_ctx genp_ctx;

/* Working precision of C = A G and of its LU factors. */
enum {
    GENP_F64 = 0,   /* FP64 MFMA product and factorization                        */
    GENP_F32 = 1,   /* FP32 MFMA product and factorization, FP32 storage           */
    GENP_BF16 = 2,  /* BF16 operands with FP32 accumulation for A G and the Schur  */
                    /* updates; panel and triangular blocks in FP32; FP32 storage  */
    GENP_BF16X3 = 3 /* as GENP_BF16 with 2-word BF16 operands: x = hi + lo,         */
                    /* hi = bf16(x), lo = bf16(x - hi); a b = hi hi + hi lo + lo hi */
                    /* (three BF16 MFMA products, about 16 significand bits)        */
};

/* Kind of multiplier passed to genp_precondition. */
enum {
    GENP_G_DENSE = 0,     /* G: n x n dense, row-major, leading dimension ldg        */
    GENP_G_TOEPLITZ = 1,  /* G: 2n-1 parameters p, G[i][j] = p[i - j + n - 1]        */
    GENP_G_NONE = 2,      /* no multiplier: C = A (plain GENP, for tests)            */
    GENP_G_CIRCULANT = 3, /* G: n parameters c, G[i][j] = c[(i - j) mod n]; applied by
                             FFT; n a power of two, 4 <= n <= 16384                    */
    GENP_G_HOUSEHOLDER = 4 /* G: 2n parameters (u, v), G = I - 2 u v^T / (v^T u): the
                             Householder-type multipliers named with Table 7.1, read as a
                             reflection (the printed I - u v^T / u^T v sends u to 0 and is
                             singular); applied as rank-1 updates in O(n^2)             */
};

/* Refinement solvers for genp_refine. */
enum {
    GENP_SOLVER_LUIR = 0,   /* classical refinement: X += G (LU)^{-1} (B - A X)          */
    GENP_SOLVER_GMRES = 1,  /* FP64 GMRES on A x = r right-preconditioned by G (LU)^{-1} */
    GENP_SOLVER_AUTO = 2    /* LU-IR while each correction divides eta by 4 or more, then
                               GMRES-IR from the best iterate                                */
};

enum {
    GENP_OK = 0,
    GENP_BREAKDOWN = 1,   /* a pivot was non-finite or |u_kk| <= pivot_tol * max|C|    */
    GENP_ENOCONV = 2,     /* refinement stopped above tol; the best X is returned      */
    GENP_EINVAL = -1,     /* bad argument                                              */
    GENP_EDEVICE = -2,    /* no usable gfx950 device, or a HIP call failed             */
    GENP_ENOMEM = -3,     /* device allocation failed                                  */
    GENP_ESTATE = -4,     /* call out of order                                         */
    GENP_ENOTSUP = -5,    /* combination not supported by this build                   */
    GENP_ESINGULAR = -6,  /* the multiplier is singular to working precision           */
    GENP_ESCRATCH = -7    /* the problem needs more than the fixed scratch of the
                             allocation-free entry point holds                          */
};

#define GENP_ETA_HIST 64

/* Diagnostics of the last factorization / refinement. */
typedef struct {
    int64_t n, nb;
    int32_t prec, mult;
    int64_t breakdown_col;      /* 1-based first failing pivot, 0 = none                  */
    double min_abs_piv;         /* min |u_kk| over the n pivots (before a breakdown)      */
    double max_abs_piv;         /* max |u_kk|                                             */
    double max_abs_c;           /* max |c_ij| of C = A G                                  */
    double max_abs_u;           /* max |u_ij| of the computed U                           */
    double growth;              /* max_abs_u / max_abs_c                                  */
    double anorm_inf;           /* ||A||_inf (computed once per precondition)             */
    int32_t iters;              /* refinement (outer) steps taken by the last genp_refine */
    int32_t inner_iters;        /* GMRES inner iterations of the last genp_refine         */
    double eta;                 /* final max_j eta_j of the last genp_refine              */
    int32_t n_eta;              /* entries of eta_hist                                    */
    double eta_hist[GENP_ETA_HIST]; /* eta before each refinement step and at the end     */
    double ms_precond, ms_factor, ms_solve, ms_refine, ms_backward; /* HIP-event times   */
    double ms_ag;               /* the C = A G product kernel alone (last genp_precondition) */
    double ms_schur;            /* last genp_factor: sum over its step groups of the main-stream
                                   interval from the group's first Schur update to its last
                                   block solve (updates, plus the block solves between them) */
    double ms_panel;            /* sum over panels of diagonal-block LU start to block-solve
                                   end (overlaps the updates)                                 */
    int32_t n_schur;            /* number of step groups summed in ms_schur                  */
    double cond_g;              /* 2-norm condition number of G when it is known cheaply:
                                   circulant: max_f |DFT(c)[f]| / min_f |DFT(c)[f]| (exact, the
                                   circulant being normal, Theorem 2.1); Householder:
                                   (a + sqrt(a^2 - 1))^2, a = ||u|| ||v|| / |v^T u| (exact);
                                   none: 1; dense and Toeplitz: NaN (not computed)           */
    int32_t mult_left;          /* kind of the left multiplier H (GENP_G_NONE without one)   */
    double cond_h;              /* the same for H                                            */
    int32_t block_ge;           /* 1 after genp_factor_block, 0 after genp_factor             */
    int64_t row_swaps;          /* genp_factor_block: rows r with perm[r] != r (0 for GENP)   */
    double ms_condest;          /* HIP-event time of the last genp_condest                    */
    double cond1_c;             /* last genp_condest: norm1_c * norm1_inv (NaN before one)     */
    double norm1_c;             /*   its estimate of ||C||_1, C = H A G from the FP64 A        */
    double norm1_inv;           /*   its estimate of ||(L U)^{-1}||_1 from the stored factors  */
    int32_t bwd_iters;          /* last genp_solve_backward(_ex): refinement steps taken       */
    int32_t bwd_inner_iters;    /*   its GMRES inner iterations                                */
    double bwd_eta;             /*   its final max_j eta_j against A^T (norm ||A||_1)          */
    double anorm_1;             /* ||A||_1 (computed by the first adjoint solve after a
                                   genp_precondition; NaN before)                             */
} genp_info;

/*
 * Create a context for n x n systems on the current HIP device.
 *   n        >= 1.
 *   prec     GENP_F64 / GENP_F32 / GENP_BF16 / GENP_BF16X3.
 *   nb       panel width of the blocked elimination: 64, 128 or 256 (0 = default 256).
 *   stream   hipStream_t to order all work on (NULL = the null stream).
 * Allocates the working matrix (padded to a multiple of nb) and scratch (among it
 * 512 n_pad bytes for the values published along the chained substitutions).
 * Errors: GENP_EINVAL, GENP_EDEVICE (no gfx950 device), GENP_ENOMEM.
 */
int genp_create(genp_ctx** ctx, int64_t n, int prec, int nb, void* stream);

/* Release everything the context owns.  NULL is accepted. */
int genp_destroy(genp_ctx* ctx);

/*
 * C = A G (section 1.1; right multiplier per Corollary 4.1(ii)), in the
 * context's working precision.  A: n x n FP64 (lda >= n).  mult selects G:
 * dense (G n x n FP64, ldg >= n), Toeplitz (G = the 2n-1 FP64 parameters,
 * ldg ignored, copied), circulant (G = the n FP64 parameters c, ldg ignored;
 * the multiplier's spectrum is kept, and every product with G or G^T runs as
 * FFTs of length n, Theorem 2.1 -- n must be a power of two with
 * 4 <= n <= 16384, else GENP_ENOTSUP), Householder (G = the 2n FP64 parameters
 * (u, v), ldg ignored, copied; A G = A - (2 / v^T u) (A u) v^T costs two passes over A),
 * or none (G ignored).  Also computes ||A||_inf.  Resets the context to the
 * "preconditioned" state.
 * A circulant multiplier whose spectrum has min |DFT(c)| <= n 2^-53 max |DFT(c)|, a
 * Householder one with |v^T u| <= n 2^-53 ||u|| ||v||, or a non-finite one, is rejected
 * with GENP_ESINGULAR (the context is then left unpreconditioned): C = A G would be
 * singular to working precision.  Circulant draws with entries +-1 hit this with
 * probability about 2 sqrt(2 / (pi n)), whenever the signs balance (DFT(c)[0] = 0) or
 * balance over the even and odd positions (DFT(c)[n/2] = 0), and +-1 Householder draws
 * whenever v^T u = 0; the caller draws new signs.
 */
int genp_precondition(genp_ctx* ctx, const double* A, int64_t lda, int mult,
                      const double* G, int64_t ldg);

/*
 * C = H A G: a left multiplier H, a right multiplier G, or both (Corollary 4.1 covers the
 * products G M and M H with Gaussian multipliers; the solve then takes C (G^{-1} x) = H b, so
 * x = G U^{-1} L^{-1} H b, and refinement and the adjoint apply H and H^T likewise).
 * left / H / ldh and right / G / ldg each take the kinds and layouts of genp_precondition
 * (GENP_G_NONE: no multiplier on that side).  genp_precondition(ctx, A, lda, mult, G, ldg)
 * is genp_precondition2(ctx, A, lda, GENP_G_NONE, NULL, 0, mult, G, ldg).
 * A left multiplier needs the FP64 context (else GENP_ENOTSUP).  A dense H is borrowed like a
 * dense G; with both a right multiplier and a dense or Toeplitz H the library allocates an
 * n x n FP64 buffer (kept until genp_destroy).  Errors as genp_precondition; a singular
 * circulant or Householder multiplier on either side gives GENP_ESINGULAR.
 */
int genp_precondition2(genp_ctx* ctx, const double* A, int64_t lda, int left, const double* H,
                       int64_t ldh, int right, const double* G, int64_t ldg);

/*
 * Blocked right-looking GENP of C in place (section 1.1; block Gaussian
 * elimination of Theorem 2.2; each step replaces the trailing block by its
 * Schur complement, Fact 2.1).  No pivoting, no row exchanges.
 *   pivot_tol    breakdown threshold relative to max|C| (0 = only non-finite
 *                or exactly zero pivots).
 *   breakdown_col (nullable, host) receives the 1-based first failing pivot
 *                column, 0 if none.
 * Returns GENP_OK or GENP_BREAKDOWN (factors are then only meaningful in the
 * columns before breakdown_col).  Synchronizes the stream.
 */
int genp_factor(genp_ctx* ctx, double pivot_tol, int64_t* breakdown_col);

/*
 * Block Gaussian elimination of C in place with the diagonal nb x nb blocks of
 * the successive Schur complements as explicit block pivots (Theorem 2.2 and
 * Fact 2.1: B_k is the leading block of the k-th Schur complement, which is then
 * replaced by its Schur complement with respect to B_k).  B_k^{-1} is applied
 * through Gaussian elimination with row interchanges inside B_k only: at each
 * column the row of the block with the largest |entry| (the first on ties)
 * becomes the pivot row, and the interchange is applied to the whole row of C.
 * The result is P C = L U with P block diagonal (one permutation per block
 * pivot), L unit lower and U upper triangular, stored like genp_factor's.
 * Needs only the leading nb, 2nb, 3nb, ... blocks of C to be nonsingular, where
 * GENP needs every leading block.  FP64 contexts only (else GENP_ENOTSUP).
 *   pivot_tol, breakdown_col  as for genp_factor; a breakdown now means that a
 *                block pivot is numerically singular (its largest candidate in
 *                some column is non-finite or <= pivot_tol * max|C|).
 * Solve, refine and the adjoint then apply P (and P^T) themselves.  A new
 * genp_precondition returns the context to GENP.  Synchronizes the stream.
 */
int genp_factor_block(genp_ctx* ctx, double pivot_tol, int64_t* breakdown_col);

/*
 * The explicit block pivots of the last successful factorization (FP64
 * contexts): out (device, n x ldo, ldo >= nb) receives B_k = P_k^T L_kk U_kk in
 * rows k nb .. k nb + w - 1 (w = min(nb, n - k nb)), columns 0 .. w - 1, in the
 * row order of C; columns w .. nb - 1 of a ragged last block are set to 0.
 * After genp_factor P_k = I (B_k = L_kk U_kk, the same blocks of the Schur
 * complements).  The caller owns out.  Stream-ordered; GENP_ESTATE before a
 * successful factorization, GENP_ENOTSUP for FP32/BF16 contexts.
 */
int genp_block_pivots(const genp_ctx* ctx, double* out, int64_t ldo);

/*
 * The row permutation of the last factorization: perm (device, n int32) receives
 * the row of C that factor row r came from (P C = L U, row r of P C = row
 * perm[r] of C).  The identity after genp_factor.  Stream-ordered; GENP_ESTATE
 * before a factorization.
 */
int genp_row_perm(const genp_ctx* ctx, int32_t* perm);

/*
 * X = G U^{-1} L^{-1} B for nrhs right-hand sides (section 1.1: the system
 * C y = b of the preconditioned matrix C = A G is solved by the two triangular
 * substitutions of GENP, and x = G y solves A x = b).  B: n x nrhs, ldb >= nrhs;
 * X: n x nrhs, ldx >= nrhs; X may equal B.  FP64 arithmetic over the stored
 * factors.  Requires a successful genp_factor.  Stream-ordered, does not
 * synchronize.  With nrhs <= 64 each triangular solve is one launch whose
 * workgroups wait on each other with a bounded spin; the bound is a safety limit
 * that a running solve never reaches, and if it were ever exceeded the next
 * genp_refine or genp_get_info returns GENP_EDEVICE once (the solutions computed
 * since are then invalid; the error word is cleared when it is reported).  More than 64 right-hand sides are solved block by block
 * (diagonal-block solve, then a product per block).  Environment GENP_TRSV=step
 * selects one launch per 128-row block (nrhs <= 4) or the block-by-block solve
 * (5 <= nrhs <= 64) instead.
 */
int genp_solve(genp_ctx* ctx, const double* B, int64_t ldb, int64_t nrhs,
               double* X, int64_t ldx);

/*
 * Iterative refinement of X (in/out) against the original A and B in FP64:
 * solver GENP_SOLVER_LUIR repeats R = B - A X, X += G (LU)^{-1} R (section
 * 7.1); GENP_SOLVER_GMRES runs restarted FP64 GMRES preconditioned by the
 * factors for the correction.  Stops when max_j eta_j <= tol or after
 * max_iter outer steps, where eta_j = ||r_j||_inf / (||A||_inf ||x_j||_inf +
 * ||b_j||_inf).  eta_out (nullable, host, nrhs doubles) receives the final
 * eta_j.  Returns GENP_OK (eta <= tol, or tol = 0) or GENP_ENOCONV (X holds
 * the best iterate).  GMRES runs one cycle of at most 50 steps per column and
 * outer step, to a residual reduction of 1e-10 (genp_refine_ex sets these).
 * Synchronizes the stream.
 */
int genp_refine(genp_ctx* ctx, const double* B, int64_t ldb, int64_t nrhs,
                double* X, int64_t ldx, int max_iter, double tol, int solver,
                double* eta_out);

/* Options of genp_refine_ex and genp_solve_backward_ex. */
#define GENP_GMRES_MAX_RESTART 1024
typedef struct {
    int32_t solver;       /* GENP_SOLVER_LUIR, GENP_SOLVER_GMRES or GENP_SOLVER_AUTO             */
    int32_t max_outer;    /* corrections (outer steps) at most, >= 0                               */
    int32_t restart;      /* GMRES: steps of one cycle (one cycle per column and outer step),
                             1 .. GENP_GMRES_MAX_RESTART; 0 = 50                                   */
    int32_t max_inner;    /* GMRES: inner steps summed over all cycles and columns at most (0 = no
                             cap); the last cycle is shortened to fit                               */
    double tol;           /* stop once max_j eta_j <= tol (0: run the steps, no target)             */
    double inner_rtol;    /* GMRES: a cycle stops once its residual 2-norm has dropped by this
                             factor (0 = 1e-10)                                                      */
} genp_refine_opts;

/*
 * genp_refine with every option: LU-IR (section 7.1) or FP64 GMRES-IR for the correction
 * equation A d = r, right-preconditioned by M^{-1} = G (LU)^{-1} H (the factors' inverse, so
 * that A M^{-1} = I for exact factors).  Each outer step computes R = B - A X in FP64 from the
 * original A, then the correction (LU-IR: D = M^{-1} R; GMRES: one cycle of at most
 * o->restart steps per column, classical Gram-Schmidt applied twice, within the o->max_inner
 * budget), X += D.  With 2 to 64 right-hand sides the columns' cycles run side by side (one
 * preconditioner solve and one product with A per step for all columns; a column stops
 * growing once it meets inner_rtol), each cycle then gets at most
 * (max_inner - steps so far) / nrhs steps, and the budget counts as spent once fewer than
 * nrhs steps remain.  Stops at max_j eta_j <= o->tol, after o->max_outer steps, when the budget
 * is spent, or when a step raised eta (it is undone; X holds the best iterate).  Returns GENP_OK
 * (eta <= tol, or tol = 0) or GENP_ENOCONV; eta_out (nullable, host, nrhs doubles) receives the
 * final eta_j; genp_info records the steps, the inner steps and the eta history.
 * Errors: GENP_EINVAL (bad options or arguments), GENP_ESTATE, GENP_ENOMEM (the Krylov basis,
 * (restart + 1) n_pad doubles per column, is allocated on first use of a larger one),
 * GENP_EDEVICE.
 * Synchronizes the stream.
 */
int genp_refine_ex(genp_ctx* ctx, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                   const genp_refine_opts* opts, double* eta_out);

/*
 * Not in the paper: the differentiation of its solve.  For X = A^{-1} B and a
 * loss with gradient W = dL/dX, dL = <A^{-T} W, dB> - <A^{-T} W X^T, dA>, so the
 * adjoint of the loss sum(W .* X) is dB = A^{-T} W and dA = -dB X^T.  dB is computed
 * from the stored factors as L^{-T} U^{-T} (G^T W), followed by refine_iters
 * FP64 refinement steps against A^T; if dA is not NULL, dA = -dB X^T
 * (n x n, ldda >= n).  W, X: n x nrhs (ldw, ldx >= nrhs); dB: n x nrhs.
 * Requires a successful genp_factor.
 */
int genp_solve_backward(genp_ctx* ctx, const double* W, int64_t ldw,
                        const double* X, int64_t ldx, int64_t nrhs,
                        double* dB, int64_t lddb, double* dA, int64_t ldda,
                        int refine_iters);

/*
 * genp_solve_backward with the refinement of dB against A^T chosen by opts (as for
 * genp_refine_ex, with A^T in place of A, M^{-T} = H^T (LU)^{-T} G^T as the preconditioner and
 * eta_j = ||w_j - A^T db_j||_inf / (||A||_1 ||db_j||_inf + ||w_j||_inf)).  genp_solve_backward is
 * this call with LU-IR, refine_iters steps and tol = 0.  Returns GENP_OK or GENP_ENOCONV (dB
 * holds the best iterate, dA is formed from it); eta_out (nullable, host, nrhs doubles) receives
 * the final eta_j; genp_info records bwd_iters, bwd_inner_iters and bwd_eta.  Synchronizes
 * the stream.
 */
int genp_solve_backward_ex(genp_ctx* ctx, const double* W, int64_t ldw, const double* X, int64_t ldx,
                           int64_t nrhs, double* dB, int64_t lddb, double* dA, int64_t ldda,
                           const genp_refine_opts* opts, double* eta_out);

/*
 * Condition estimate of the factored matrix, kappa_1 ~ ||C||_1 ||(L U)^{-1}||_1, by the
 * Hager-Higham 1-norm estimator (Higham, ACM TOMS 14 (1988), Algorithm 4.1: at most five
 * products with the transposed operator, then the alternating-sign vector): ||C||_1 from
 * products with C = H A G and C^T computed from the FP64 A and the multipliers, and
 * ||(L U)^{-1}||_1 from substitutions with the stored factors (in the working precision, so for
 * FP32 / BF16 contexts it is the inverse of the low-precision factors that refinement uses).
 * Each estimate is a lower bound of the norm it estimates (rarely below a third of it).  This is
 * what section 4 bounds (the conditioning of A G given that of A and G, Theorem 4.1 and
 * Corollary 4.1).  kappa, norm_c, norm_inv: host, nullable.  Requires a successful factorization
 * (else GENP_ESTATE).  Synchronizes the stream.
 */
int genp_condest(genp_ctx* ctx, double* kappa, double* norm_c, double* norm_inv);

/* Copy diagnostics (host struct).  Synchronizes the stream. */
int genp_get_info(const genp_ctx* ctx, genp_info* info);

/*
 * Copy the n x n working matrix (C after genp_precondition, packed L \ U
 * after genp_factor) to out (device, FP64, ldo >= n), widening FP32 storage.
 * For tests and diagnostics.
 */
int genp_copy_work(const genp_ctx* ctx, double* out, int64_t ldo);

/* Static description of a status code. */
const char* genp_strerror(int status);

/* ------------------------------------------------------------------------- */
/* Randomized low-rank approximation (Proto-Algorithm 5.1, section 5.3, with the
 * orthogonal basis of Remark 5.4).  Independent of the GENP context.          */

typedef struct {
    int64_t m, n, rho_plus;
    int64_t rank;               /* s: columns kept at Stage 2                                */
    int32_t failed;             /* 1: ||A - A_hat||_F > tau2 ||A||_F (the FAILURE of Stage 3) */
    double a_fro;               /* ||A||_F                                                   */
    double tail_fro;            /* Frobenius norm of the columns of T' left after Stage 2    */
    double resid_fro;           /* ||A - W_s T_s^T||_F                                        */
    double ms_total, ms_sketch, ms_basis, ms_project, ms_resid;   /* HIP-event times       */
} genp_lr_info;

/*
 * Rank-s approximation A_hat = W_s T_s^T of an m x n FP64 matrix A (row-major, lda >= n),
 * all device pointers, on `stream` (hipStream_t, NULL = null stream) of the current device:
 *   Stage 1  T' = A^T G, n x rho_+; mult = GENP_G_DENSE: G is m x rho_+ (ldg >= rho_+);
 *            GENP_G_TOEPLITZ: G holds the m + rho_+ - 1 parameters of G[i][j] = p[i - j + rho_+ - 1]
 *            (ldg ignored).  The random numbers are the caller's.
 *   Stage 2  Gram-Schmidt with column pivoting on T' (each projection applied twice), a
 *            rank-revealing QR: it stops at the least s for which the remaining columns have
 *            Frobenius norm <= tau ||A||_F; T_s = its first s orthonormal columns.
 *   Stage 3  W = A T; failed = ||A - W_s T_s^T||_F > tau2 ||A||_F.
 * Outputs: T (n x rho_+, ldt >= rho_+) and W (m x rho_+, ldw >= rho_+), of which the first
 * `rank` columns are the result (the others are scratch); A_hat = W_s T_s^T (m x n, ldah >= n)
 * when Ahat is not NULL; perm_out (host, rho_+ entries, may be NULL): the columns of T' in
 * pivot order; info (host).  1 <= rho_+ <= min(64, m, n).  Allocates and frees its own device
 * scratch (O((m + n) rho_+) plus one double per 64 x 64 tile of A).  Waits for the stream
 * once, at the end.  Errors: GENP_EINVAL, GENP_ENOTSUP (other multiplier kinds),
 * GENP_ENOMEM, GENP_EDEVICE.
 */
int genp_lowrank(const double* A, int64_t m, int64_t n, int64_t lda, int mult, const double* G,
                 int64_t ldg, int64_t rho_plus, double tau, double tau2, double* T, int64_t ldt,
                 double* W, int64_t ldw, double* Ahat, int64_t ldah, int32_t* perm_out,
                 genp_lr_info* info, void* stream);

/* ------------------------------------------------------------------------- */
/* Numerical rank without pivoting or orthogonalization (Proto-Algorithm B.1,
 * Appendix B, with the COND of Remark B.2 and the bisection of Remark B.4).    */

typedef struct {
    int64_t m, n, rho_minus, rho_plus;
    int64_t rank;               /* the numerical rank found                               */
    int32_t tests;              /* COND evaluations (at most ceil(log2(rho_+ - rho_- + 1)))  */
    double cond_at_rank;        /* COND's kappa_2 estimate of B_rank (NaN when not tested)  */
    double cond_above;          /* the estimate of B_{rank+1} (NaN when not tested)        */
    double ms_total, ms_sketch, ms_gram, ms_search;   /* HIP-event times                 */
} genp_nrank_info;

/*
 * Numerical rank of an m x n FP64 matrix A (row-major, lda >= n; device pointers; `stream`
 * as for genp_lowrank) in the range [rho_minus, rho_plus], 0 <= rho_- < rho_+ <= min(64, m, n).
 * G: the caller's m x rho_+ Gaussian multiplier (ldg >= rho_+).  The sketch B = A^T G is formed
 * once; the candidates s are tested by bisection (s = ceil((lo + hi) / 2)) on B_s = its first s
 * columns (= A^T G_s): COND passes when the kappa_2 estimate of B_s is <= cond_max, and a pass
 * raises the lower end (B_s keeps full rank with high probability exactly when
 * s <= nrank(A)), a failure lowers the upper end to s - 1.  COND runs Lanczos (6 s steps, no
 * reorthogonalization) on the leading s x s block of B^T B and locates the extreme
 * eigenvalues of the tridiagonal by Sturm-count multisection; the estimate is a lower bound
 * on kappa_2 except below the rounding level of B^T B (about 1e8 for kappa_2), so cond_max
 * should lie well below 1e8.  Output B (n x rho_+, ldb >= rho_+): the sketch; its first `rank`
 * columns approximate a basis of the leading right singular space.  Allocates and frees its
 * own scratch; waits for the stream once.  Errors: GENP_EINVAL, GENP_ENOMEM, GENP_EDEVICE.
 */
int genp_numerical_rank(const double* A, int64_t m, int64_t n, int64_t lda, const double* G,
                        int64_t ldg, int64_t rho_minus, int64_t rho_plus, double cond_max, double* B,
                        int64_t ldb, genp_nrank_info* info, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): genp_numerical_rank with the same arguments and
 * results, whose scratch comes from one fixed 64 MiB device array per GPU (held from the first
 * call on that GPU until the process ends) instead of hipMalloc; it calls no allocating routine.
 * The scratch holds the m x 64 multiplier and n x 64 sketch (rows padded to 16), the 64 x 64
 * Gram matrix and at least one n x 64 slice of split-K partials:
 * 512 (ceil16(m) + ceil16(n) + max(n, 64)) + 33 KiB <= 64 MiB, about m + 2n <= 131000;
 * larger problems return GENP_ESCRATCH.  Every call on a GPU uses that GPU's one array, which
 * keeps the last call's contents (each call clears what it reads before writing it): calls that
 * overlap on one GPU (other host threads, other streams) race and must be serialized by the
 * caller.  The stage times of info are NaN (no events are created).  Waits for the stream once.
 * Errors: GENP_EINVAL, GENP_ESCRATCH, GENP_EDEVICE.
 */
int genp_numerical_rank_noalloc(const double* A, int64_t m, int64_t n, int64_t lda, const double* G,
                                int64_t ldg, int64_t rho_minus, int64_t rho_plus, double cond_max, double* B,
                                int64_t ldb, genp_nrank_info* info, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GENP_H */
