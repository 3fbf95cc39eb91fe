// Host side of the GENP library: the C ABI of include/genp.h, context and
// workspace management, and the orchestration of the kernels into the method's
// steps (section 1.1): C = A G, blocked GENP, substitutions, recovery X = G Y,
// refinement (section 7.1) and the adjoint solve.
#include "../../include/genp.h"
#include "common.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#define HIPCK(x)                                      \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) return GENP_EDEVICE;    \
    } while (0)
#define CK(x)                                         \
    do {                                              \
        int r_ = (x);                                 \
        if (r_ != GENP_OK) return r_;                 \
    } while (0)

namespace {

enum { ST_CREATED = 0, ST_PRECOND = 1, ST_FACTORED = 2, ST_BROKEN = 3 };
enum { EV_PRE = 0, EV_FAC = 1, EV_SOL = 2, EV_REF = 3, EV_BWD = 4, EV_CEST = 5, EV_N = 6 };

// device reduction slots (bit patterns of non-negative doubles)
enum { R_MAXC = 0, R_MAXU = 1, R_ANORM = 2, R_ANORM1 = 3, R_COLS = 8 };   // R_COLS: 3 * 256 per-column maxima

// One multiplier (right G or left H) as the library keeps it.
struct Mult {
    int kind = GENP_G_NONE;
    const double* G = nullptr;   // dense: borrowed
    int64_t ldg = 0;
    double* p = nullptr;         // Toeplitz: the 2n - 1 parameters (owned copy)
    double* p_rev = nullptr;     //           reversed: the parameters of the transpose
    double2* spec = nullptr;     // circulant: spectrum X[0..n/2], then (max, min) modulus
    double* uv = nullptr;        // Householder: u (n), v (n), then (v^T u, u^T u, v^T v)
};

}  // namespace

struct genp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0, n_pad = 0, nb = 256;
    int prec = GENP_F64;
    void* C = nullptr;
    int64_t ldc = 0;
    PanelStats* stats = nullptr;
    unsigned long long* red = nullptr;
    // borrowed / copied inputs
    const double* A = nullptr;
    int64_t lda = 0;
    Mult mr, ml;               // right multiplier G and left multiplier H (C = H A G)
    // FFT twiddles shared by circulant multipliers (n / 4 and n / 2 + 1 entries)
    double2* circ_tw = nullptr;
    double2* circ_wp = nullptr;
    double* hw = nullptr;      // Householder: a length-n_pad work vector
    // precision form: FP32 (or BF16-valued) copies of A and of the multiplier, zero-padded to
    // n_pad (the operands of the register-operand FP32 product)
    float* A32 = nullptr;      // n_pad x n_pad
    float* G32 = nullptr;      // dense G: n_pad x n_pad; Toeplitz: 2 n_pad - 1 parameters
    size_t g32_bytes = 0;
    double* dwork = nullptr;   // FP32 forms, nb = 256: an FP64 copy of the current diagonal block
    // BF16 forms: BF16 copies of A and of G^T (hi words; lo words for the 2-word form), n_pad x n_pad
    unsigned short* Abf[2] = {nullptr, nullptr};
    unsigned short* Gtbf[2] = {nullptr, nullptr};
    // ... and of the update operands L21 (n_pad x K) and U12^T (n_pad x K), K <= 8 nb
    unsigned short* Lbf[2] = {nullptr, nullptr};
    unsigned short* Ubf[2] = {nullptr, nullptr};
    double* w2 = nullptr;      // two-sided products with a dense or Toeplitz H: n x n copy of A G
    // right-hand-side scratch, capacity kcap columns
    int64_t kcap = 0;
    double* Z = nullptr;       // n_pad x kcap
    double* R = nullptr;       // n_pad x kcap
    double* Dx = nullptr;      // n_pad x kcap
    double* Xb = nullptr;      // n_pad x kcap: the best iterate of a GMRES refinement
    double* part = nullptr;    // split-K partials: KSPLIT_MAX x n_pad x kcap
    // GMRES-IR: Krylov basis (gm_cap + 1 vectors of n_pad), the Gram-Schmidt coefficients of
    // one Arnoldi step (2 (gm_cap + 2) doubles), three n_pad work vectors
    int gm_cap = 0;
    double* gm_V = nullptr;
    double* gm_w = nullptr;
    double* gm_z = nullptr;
    double* gm_r = nullptr;
    double* gm_h = nullptr;
    // GMRES-IR over several columns at once: Krylov blocks ((restart + 1) x n_pad x k), two
    // n_pad x 64 work blocks, the coefficients of a step (2 (restart + 2) 64 + 64 doubles)
    size_t gmb_cap = 0;
    double* gmb_V = nullptr;
    double* gmb_w = nullptr;
    double* gmb_z = nullptr;
    double* gmb_h = nullptr;
    double* gmb_part = nullptr;        // row-chunk partial dots: (GENP_GMRES_MAX_RESTART + 2 + 1024) x 64
    // 1-norm estimator: four n_pad vectors, then 8 scalars
    double* cest = nullptr;
    double anorm1 = -1.0;              // ||A||_1 (= ||A^T||_inf), < 0 until the adjoint needs it
    int state = ST_CREATED;
    genp_info info{};
    hipEvent_t ev0[EV_N]{}, ev1[EV_N]{};
    bool ev_used[EV_N]{};
    hipEvent_t ev_ag[2]{};
    // per elimination step: Schur start/end (main stream), panel start/end (panel stream),
    // cross-update done, panel done (ordering only)
    std::vector<hipEvent_t> ev_step;
    hipStream_t side = nullptr;        // look-ahead stream for the next panel (default priority)
    bool lookahead = true;
    // chained triangular solves (<= 64 right-hand sides): ticket and sticky error word; the
    // solved values as published along the chain (n_pad x 64)
    unsigned* tsync = nullptr;
    unsigned long long* tpub = nullptr;
    bool trsv_chain = true;
    bool diag_split = true;            // FP64 nb = 256 diagonal blocks as two LDS-resident halves
    bool lp_regs = true;               // precision forms: product from FP32 copies of A and G
    bool f32_upd = true;               // FP32 form: updates on the 256 x 128 FP32 kernel
    bool gm_batched = true;            // GMRES-IR over 2..64 columns: one cycle for all columns
    // steps per group of the factorization: g_big while the trailing matrix has at least
    // g_switch rows, then g_small
    int g_big = 3, g_small = 2;
    int64_t g_switch = 8192;
    // FP64 update products: 128 x 128 tiles, two workgroups per CU, so a launch runs in
    // rounds of round_tiles tiles; the bulk of a step group is cut into parts of whole
    // rounds (the last part takes the rest) so that only one part pays a partly filled round
    int64_t round_tiles = 512;
    bool round_cut = true;
    // block Gaussian elimination: rows interchanged inside the diagonal blocks, P C = L U;
    // factor row r came from row perm[r] of C (n_pad entries)
    bool block_ge = false;
    int* perm = nullptr;
    double anorm = 0.0;
};

namespace {

constexpr int KSPLIT_MAX = 8;

size_t esize(int prec) { return prec == GENP_F64 ? 8 : 4; }

int ensure_rhs(genp_ctx* c, int64_t k) {
    if (k <= c->kcap) return GENP_OK;
    const int64_t cap = std::max<int64_t>(k, 4);
    hipFree(c->Z);
    hipFree(c->R);
    hipFree(c->Dx);
    hipFree(c->Xb);
    hipFree(c->part);
    c->Z = c->R = c->Dx = c->Xb = c->part = nullptr;
    c->kcap = 0;
    const size_t sz = (size_t)c->n_pad * cap * sizeof(double);
    if (hipMalloc(&c->Z, sz) != hipSuccess || hipMalloc(&c->R, sz) != hipSuccess ||
        hipMalloc(&c->Dx, sz) != hipSuccess || hipMalloc(&c->Xb, sz) != hipSuccess ||
        hipMalloc(&c->part, sz * KSPLIT_MAX) != hipSuccess)
        return GENP_ENOMEM;
    c->kcap = cap;
    return GENP_OK;
}

void ev_begin(genp_ctx* c, int e) {
    hipEventRecord(c->ev0[e], c->stream);
}
void ev_end(genp_ctx* c, int e) {
    hipEventRecord(c->ev1[e], c->stream);
    c->ev_used[e] = true;
}

double bits_to_double(unsigned long long b) {
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

// y (M x k) = beta * yin + alpha * op(A) (M x K) * X (K x k); FP64 arithmetic.
// Few right-hand sides: one wave per row; more: FP64 MFMA with split-K.
int skinny(genp_ctx* c, int M, int K, int k, double alpha, const void* A, int64_t lda, int amode,
           int a_f32, const double* X, int64_t ldx, double beta, const double* Yin, int64_t ldyi,
           double* Y, int64_t ldy) {
    if (M <= 0 || k <= 0) return GENP_OK;
    if (K <= 0) {
        if (beta == 0.0) HIPCK(launch_fill2d(0.0, Y, ldy, M, k, c->stream));
        else if (beta != 1.0 || Yin != Y) return GENP_ENOTSUP;
        return GENP_OK;
    }
    if (k <= 4) {
        if (amode == OP_TOEP && c->kcap > 0) {
            // Toeplitz operand (the multiplier): LDS-staged windows of its parameters, split over K
            HIPCK(launch_toep_gemv(M, K, k, alpha, (const double*)A, lda, X, ldx, beta, Yin, ldyi, Y, ldy, c->part,
                                   (long long)KSPLIT_MAX * c->n_pad * c->kcap, c->stream));
            return GENP_OK;
        }
        if (amode == OP_T && M >= 64 && c->kcap > 0) {
            // transposed operand: partial sums over row slices (coalesced), then their sum
            HIPCK(launch_gemv_t_f64(M, K, k, alpha, A, lda, a_f32, X, ldx, beta, Yin, ldyi, Y, ldy, c->part,
                                    (long long)KSPLIT_MAX * c->n_pad * c->kcap, c->stream));
            return GENP_OK;
        }
        HIPCK(launch_gemv_f64(M, K, k, alpha, A, lda, amode, a_f32, X, ldx, beta, Yin, ldyi, Y, ldy,
                              c->stream));
        return GENP_OK;
    }
    if (a_f32 && amode == OP_TOEP) return GENP_ENOTSUP;
    for (int c0 = 0; c0 < k; c0 += 64) {
        const int kc = std::min(64, k - c0);
        GemmF64Args g{};
        g.M = M;
        g.N = kc;
        g.K = K;
        g.A = (const double*)A;
        g.lda = lda;
        g.amode = amode;
        g.B = X + c0;
        g.ldb = ldx;
        g.bmode = OP_N;
        g.alpha = alpha;
        g.beta = beta;
        g.Cin = Yin ? Yin + c0 : nullptr;
        g.ldci = ldyi;
        g.a_f32 = a_f32;
        const int ntm = (M + 127) / 128;
        int ks = std::max(1, std::min(KSPLIT_MAX, (1024 + ntm - 1) / ntm));
        ks = std::min(ks, std::max(1, K / 64));
        if (ks > 1 && (int64_t)M * kc * ks > c->n_pad * c->kcap * KSPLIT_MAX) ks = 1;
        if (ks == 1) {
            g.D = Y + c0;
            g.ldd = ldy;
            g.ksplit = 1;
            HIPCK(launch_gemm_f64(g, 4, c->stream));
        } else {
            g.D = c->part;
            g.ldd = kc;
            g.ksplit = ks;
            g.split_stride = (long long)M * kc;
            HIPCK(launch_gemm_f64(g, 4, c->stream));
            HIPCK(launch_splitk_reduce_f64(M, kc, ks, c->part, kc, (long long)M * kc, 1.0, beta,
                                           Yin ? Yin + c0 : nullptr, ldyi, Y + c0, ldy, c->stream));
        }
    }
    return GENP_OK;
}

int lu_solve_trans_core(genp_ctx* c, double* Z, int64_t ldz, int k);

// Z (n_pad x k, ldz) := U^{-1} L^{-1} P Z (P = I for GENP), block by block: substitution with the
// diagonal block, then the block column below (above) updates the remaining rows.
int lu_solve_inplace(genp_ctx* c, double* Z, int64_t ldz, int k) {
    const int64_t nb = c->nb, nblk = c->n_pad / nb;
    const int f32 = c->prec != GENP_F64;
    const size_t es = esize(c->prec);
    const char* Cb = (const char*)c->C;
    if (c->block_ge) {
        // P Z through the split-K scratch (at least n_pad x k)
        HIPCK(launch_permute_rows((int)c->n_pad, k, Z, ldz, c->part, k, c->perm, 0, c->stream));
        HIPCK(launch_copy2d(c->part, k, Z, ldz, (int)c->n_pad, k, c->stream));
    }
    if (k <= 4) {
        // few right-hand sides: one chained launch per triangle (or one launch per 128-row block)
        if (c->trsv_chain) {
            HIPCK(launch_trsv_chain(TRSM_L_UNIT, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub, c->stream));
            HIPCK(launch_trsv_chain(TRSM_U, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub, c->stream));
            return GENP_OK;
        }
        const int bs = nb >= 128 ? 128 : 64;
        HIPCK(launch_trsv_full(TRSM_L_UNIT, f32, c->C, c->ldc, (int)c->n_pad, bs, Z, ldz, k, c->stream));
        HIPCK(launch_trsv_full(TRSM_U, f32, c->C, c->ldc, (int)c->n_pad, bs, Z, ldz, k, c->stream));
        return GENP_OK;
    }
    if (k <= 64 && c->trsv_chain) {
        // up to 64 right-hand sides: one chained launch per triangle, MFMA block products
        HIPCK(launch_trsm_chain(TRSM_L_UNIT, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub, c->stream));
        HIPCK(launch_trsm_chain(TRSM_U, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub, c->stream));
        return GENP_OK;
    }
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t r0 = b * nb;
        HIPCK(launch_trsm(TRSM_L_UNIT, f32, 0, Cb + (r0 * c->ldc + r0) * es, c->ldc, (int)nb, Z + r0 * ldz,
                          ldz, k, c->stream));
        const int64_t below = c->n_pad - r0 - nb;
        if (below > 0) {
            const void* Lp = Cb + ((r0 + nb) * c->ldc + r0) * es;
            CK(skinny(c, (int)below, (int)nb, k, -1.0, Lp, c->ldc, OP_N, f32, Z + r0 * ldz, ldz, 1.0,
                      Z + (r0 + nb) * ldz, ldz, Z + (r0 + nb) * ldz, ldz));
        }
    }
    for (int64_t b = nblk - 1; b >= 0; --b) {
        const int64_t r0 = b * nb;
        HIPCK(launch_trsm(TRSM_U, f32, 0, Cb + (r0 * c->ldc + r0) * es, c->ldc, (int)nb, Z + r0 * ldz, ldz,
                          k, c->stream));
        if (r0 > 0) {
            const void* Up = Cb + r0 * es;
            CK(skinny(c, (int)r0, (int)nb, k, -1.0, Up, c->ldc, OP_N, f32, Z + r0 * ldz, ldz, 1.0, Z, ldz,
                      Z, ldz));
        }
    }
    return GENP_OK;
}

// Z (n_pad x k) := P^T L^{-T} U^{-T} Z (the transposed solve of the adjoint; P = I for GENP).
int lu_solve_trans_inplace(genp_ctx* c, double* Z, int64_t ldz, int k) {
    CK(lu_solve_trans_core(c, Z, ldz, k));
    if (c->block_ge) {
        HIPCK(launch_copy2d(Z, ldz, c->part, k, (int)c->n_pad, k, c->stream));
        HIPCK(launch_permute_rows((int)c->n_pad, k, c->part, k, Z, ldz, c->perm, 1, c->stream));
    }
    return GENP_OK;
}

int lu_solve_trans_core(genp_ctx* c, double* Z, int64_t ldz, int k) {
    const int64_t nb = c->nb, nblk = c->n_pad / nb;
    const int f32 = c->prec != GENP_F64;
    const size_t es = esize(c->prec);
    const char* Cb = (const char*)c->C;
    if (k <= 4) {
        if (c->trsv_chain) {
            HIPCK(launch_trsv_chain(TRSM_UT, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub, c->stream));
            HIPCK(launch_trsv_chain(TRSM_LT_UNIT, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync,
                                    c->tpub, c->stream));
            return GENP_OK;
        }
        const int bs = nb >= 128 ? 128 : 64;
        HIPCK(launch_trsv_full(TRSM_UT, f32, c->C, c->ldc, (int)c->n_pad, bs, Z, ldz, k, c->stream));
        HIPCK(launch_trsv_full(TRSM_LT_UNIT, f32, c->C, c->ldc, (int)c->n_pad, bs, Z, ldz, k, c->stream));
        return GENP_OK;
    }
    if (k <= 64 && c->trsv_chain) {
        HIPCK(launch_trsm_chain(TRSM_UT, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub, c->stream));
        HIPCK(launch_trsm_chain(TRSM_LT_UNIT, f32, c->C, c->ldc, (int)c->n_pad, Z, ldz, k, c->tsync, c->tpub,
                                c->stream));
        return GENP_OK;
    }
    // U^T is lower triangular: forward substitution
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t r0 = b * nb;
        HIPCK(launch_trsm(TRSM_UT, f32, 0, Cb + (r0 * c->ldc + r0) * es, c->ldc, (int)nb, Z + r0 * ldz, ldz,
                          k, c->stream));
        const int64_t below = c->n_pad - r0 - nb;
        if (below > 0) {
            // (U^T)(r0+nb+i, r0+t) = U(r0+t, r0+nb+i): transposed access of the U row block
            const void* Up = Cb + (r0 * c->ldc + r0 + nb) * es;
            CK(skinny(c, (int)below, (int)nb, k, -1.0, Up, c->ldc, OP_T, f32, Z + r0 * ldz, ldz, 1.0,
                      Z + (r0 + nb) * ldz, ldz, Z + (r0 + nb) * ldz, ldz));
        }
    }
    // L^T is unit upper triangular: backward substitution
    for (int64_t b = nblk - 1; b >= 0; --b) {
        const int64_t r0 = b * nb;
        HIPCK(launch_trsm(TRSM_LT_UNIT, f32, 0, Cb + (r0 * c->ldc + r0) * es, c->ldc, (int)nb, Z + r0 * ldz,
                          ldz, k, c->stream));
        if (r0 > 0) {
            // (L^T)(i, r0+t) = L(r0+t, i) for i < r0
            const void* Lp = Cb + (r0 * c->ldc) * es;
            CK(skinny(c, (int)r0, (int)nb, k, -1.0, Lp, c->ldc, OP_T, f32, Z + r0 * ldz, ldz, 1.0, Z, ldz,
                      Z, ldz));
        }
    }
    return GENP_OK;
}

// Y (n x k) = alpha * M Z + beta * Yin, or with M^T (trans), for a stored multiplier M.
int apply_mult(genp_ctx* c, const Mult& m, int trans, int k, double alpha, const double* Zin, int64_t ldz,
               double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy) {
    const int n = (int)c->n;
    switch (m.kind) {
        case GENP_G_NONE:
            if (alpha != 1.0) return GENP_ENOTSUP;
            if (beta == 0.0) HIPCK(launch_copy2d(Zin, ldz, Y, ldy, n, k, c->stream));
            else if (beta == 1.0 && Yin == Y) HIPCK(launch_axpy2d(1.0, Zin, ldz, Y, ldy, n, k, c->stream));
            else return GENP_ENOTSUP;
            return GENP_OK;
        case GENP_G_TOEPLITZ:
            return skinny(c, n, n, k, alpha, trans ? m.p_rev : m.p, n, OP_TOEP, 0, Zin, ldz, beta, Yin, ldyi, Y, ldy);
        case GENP_G_CIRCULANT:
            // the k columns as k vectors: element t of column b at Z[t * ldz + b]
            HIPCK(launch_circ_apply(n, k, trans, Zin, ldz, 1, m.spec, c->circ_tw, c->circ_wp, alpha, beta, Yin, ldyi,
                                    1, Y, 0, ldy, 1, c->stream));
            return GENP_OK;
        case GENP_G_HOUSEHOLDER: {
            // M Z = Z - (2 / v^T u) u (v^T Z);  M^T Z = Z - (2 / v^T u) v (u^T Z)
            const double* u = m.uv;
            const double* v = m.uv + n;
            const double* a = trans ? v : u;
            const double* b = trans ? u : v;
            HIPCK(launch_gemv_t_f64(k, n, 1, 1.0, Zin, ldz, 0, b, 1, 0.0, nullptr, 0, c->hw, 1, c->part,
                                    (long long)KSPLIT_MAX * c->n_pad * c->kcap, c->stream));
            HIPCK(launch_rank1(n, k, alpha, Zin, ldz, a, c->hw, m.uv + 2 * n, 2.0, beta, Yin, ldyi, Y, 0, ldy,
                               c->stream));
            return GENP_OK;
        }
        default:
            return skinny(c, n, n, k, alpha, m.G, m.ldg, trans ? OP_T : OP_N, 0, Zin, ldz, beta, Yin, ldyi, Y, ldy);
    }
}

// X (n x k) = G U^{-1} L^{-1} H Bin, using Z as workspace (n_pad x k, ldz = k).
int solve_into(genp_ctx* c, const double* Bin, int64_t ldb, int k, double* X, int64_t ldx) {
    double* Z = c->Z;
    const int64_t ldz = k;
    CK(apply_mult(c, c->ml, 0, k, 1.0, Bin, ldb, 0.0, nullptr, 0, Z, ldz));   // H B (a copy without H)
    if (c->n_pad > c->n)
        HIPCK(launch_fill2d(0.0, Z + c->n * ldz, ldz, (int)(c->n_pad - c->n), k, c->stream));
    CK(lu_solve_inplace(c, Z, ldz, k));
    return apply_mult(c, c->mr, 0, k, 1.0, Z, ldz, 0.0, nullptr, 0, X, ldx);
}

// eta_j = ||r_j||_inf / (anorm ||x_j||_inf + ||b_j||_inf), host result (anorm = ||A||_inf, or
// ||A^T||_inf = ||A||_1 for the transposed system).
int backward_error(genp_ctx* c, const double* R, int64_t ldr, const double* X, int64_t ldx,
                   const double* B, int64_t ldb, int k, std::vector<double>& eta, double anorm) {
    unsigned long long* cols = c->red + R_COLS;
    HIPCK(hipMemsetAsync(cols, 0, sizeof(unsigned long long) * 3 * 256, c->stream));
    HIPCK(launch_col_abs_max(R, ldr, (int)c->n, k, cols, c->stream));
    HIPCK(launch_col_abs_max(X, ldx, (int)c->n, k, cols + 256, c->stream));
    HIPCK(launch_col_abs_max(B, ldb, (int)c->n, k, cols + 512, c->stream));
    std::vector<unsigned long long> h(3 * 256);
    HIPCK(hipMemcpyAsync(h.data(), cols, sizeof(unsigned long long) * 3 * 256, hipMemcpyDeviceToHost,
                         c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    eta.resize(k);
    for (int j = 0; j < k; ++j) {
        const double r = bits_to_double(h[j]), x = bits_to_double(h[256 + j]), b = bits_to_double(h[512 + j]);
        const double den = anorm * x + b;
        eta[j] = (den > 0) ? r / den : (r > 0 ? INFINITY : 0.0);
        if (isnan(r) || isnan(x)) eta[j] = NAN;
    }
    return GENP_OK;
}

double max_of(const std::vector<double>& v) {
    double m = 0.0;
    for (double e : v) {
        if (isnan(e)) return NAN;
        m = std::max(m, e);
    }
    return m;
}


// ------------------------------------------------------------------ GMRES-IR ---
// FP64 restarted GMRES for A d = r with the right preconditioner M^{-1} = G (LU)^{-1}
// built from the stored (possibly low-precision) factors.  Classical Gram-Schmidt
// applied twice on the device; Hessenberg QR by Givens rotations on the host.

int ensure_gmres(genp_ctx* c, int m) {
    const size_t np = (size_t)c->n_pad;
    if (!c->gm_w) {
        if (hipMalloc(&c->gm_w, np * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gm_z, np * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gm_r, np * sizeof(double)) != hipSuccess)
            return GENP_ENOMEM;
    }
    if (m > c->gm_cap) {
        hipFree(c->gm_V);
        hipFree(c->gm_h);
        c->gm_V = c->gm_h = nullptr;
        c->gm_cap = 0;
        if (hipMalloc(&c->gm_V, (size_t)(m + 1) * np * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gm_h, 2 * (size_t)(m + 2) * sizeof(double)) != hipSuccess)
            return GENP_ENOMEM;
        c->gm_cap = m;
    }
    return GENP_OK;
}

constexpr long long GMB_PART = (long long)(GENP_GMRES_MAX_RESTART + 2 + 1024) * 64;

int ensure_gmres_batched(genp_ctx* c, int m, int k) {
    const size_t np = (size_t)c->n_pad;
    if (!c->gmb_w) {
        if (hipMalloc(&c->gmb_w, np * 64 * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gmb_z, np * 64 * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gmb_h, ((size_t)2 * (GENP_GMRES_MAX_RESTART + 2) * 64 + 64) * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gmb_part, (size_t)GMB_PART * sizeof(double)) != hipSuccess)
            return GENP_ENOMEM;
    }
    const size_t need = (size_t)(m + 1) * np * k;
    if (need > c->gmb_cap) {
        hipFree(c->gmb_V);
        c->gmb_V = nullptr;
        c->gmb_cap = 0;
        if (hipMalloc(&c->gmb_V, need * sizeof(double)) != hipSuccess) return GENP_ENOMEM;
        c->gmb_cap = need;
    }
    return GENP_OK;
}

// X (n x k) = H^T U^{-T} L^{-T} G^T Bin (the transposed solve: C^T = G^T A^T H^T), Z as workspace.
int solve_t_into(genp_ctx* c, const double* Bin, int64_t ldb, int k, double* X, int64_t ldx) {
    double* Z = c->Z;
    const int64_t ldz = k;
    if (c->n_pad > c->n)
        HIPCK(launch_fill2d(0.0, Z + c->n * ldz, ldz, (int)(c->n_pad - c->n), k, c->stream));
    CK(apply_mult(c, c->mr, 1, k, 1.0, Bin, ldb, 0.0, nullptr, 0, Z, ldz));
    CK(lu_solve_trans_inplace(c, Z, ldz, k));
    return apply_mult(c, c->ml, 1, k, 1.0, Z, ldz, 0.0, nullptr, 0, X, ldx);
}

// z = M^{-1} v with M^{-1} = G (LU)^{-1} H, or its transpose for the adjoint system (n rows)
int precond(genp_ctx* c, bool trans, const double* v, double* z) {
    return trans ? solve_t_into(c, v, 1, 1, z, 1) : solve_into(c, v, 1, 1, z, 1);
}

// w = A z, or A^T z (n rows, FP64)
int op_a(genp_ctx* c, bool trans, const double* z, double* w) {
    const int n = (int)c->n;
    return skinny(c, n, n, 1, 1.0, c->A, c->lda, trans ? OP_T : OP_N, 0, z, 1, 0.0, nullptr, 1, w, 1);
}

// One cycle of at most m steps of FP64 GMRES for Op d = r (Op = A, or A^T when trans), right-
// preconditioned by M^{-1}, from d = 0: Arnoldi with classical Gram-Schmidt applied twice, the
// products and the new basis vector on the device, the Hessenberg matrix and its Givens
// rotations on the host (one round trip per step).  r (n doubles) is read before anything is
// written; d receives the correction.  Stops early once the rotated residual norm is
// <= tol_rel ||r||_2.  *iters_out = steps taken.
int gmres_cycle(genp_ctx* c, bool trans, int m, const double* r, double* d, double tol_rel, int* iters_out) {
    const int n = (int)c->n;
    const int64_t np = c->n_pad;
    double* V = c->gm_V;
    double* hd = c->gm_h;               // device: h (m + 2), then the second pass h2 (m + 2)
    double* hd2 = hd + (m + 2);
    *iters_out = 0;
    HIPCK(hipMemcpyAsync(V, r, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCK(launch_multidot(n, 1, V, np, V, hd, c->stream));
    double beta = 0.0;
    HIPCK(hipMemcpyAsync(&beta, hd, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    beta = sqrt(beta);
    if (!(beta > 0) || !std::isfinite(beta)) {
        HIPCK(launch_fill2d(0.0, d, 1, n, 1, c->stream));
        return GENP_OK;
    }
    HIPCK(launch_scale2d(1.0 / beta, V, 1, n, 1, c->stream));   // v_0 = r / beta
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0), hh(2 * (m + 2));
    g[0] = beta;
    int k = 0;
    for (; k < m; ++k) {
        double* vk = V + (size_t)k * np;
        double* vk1 = V + (size_t)(k + 1) * np;
        CK(precond(c, trans, vk, c->gm_z));
        CK(op_a(c, trans, c->gm_z, vk1));                       // w, built in place of v_{k+1}
        // w -= V h, h = V^T w; twice (the second pass restores orthogonality lost in the first)
        HIPCK(launch_multidot(n, k + 1, V, np, vk1, hd, c->stream));
        HIPCK(launch_gemv_f64(n, k + 1, 1, -1.0, V, np, OP_T, 0, hd, 1, 1.0, vk1, 1, vk1, 1, c->stream));
        HIPCK(launch_multidot(n, k + 1, V, np, vk1, hd2, c->stream));
        HIPCK(launch_gemv_f64(n, k + 1, 1, -1.0, V, np, OP_T, 0, hd2, 1, 1.0, vk1, 1, vk1, 1, c->stream));
        HIPCK(launch_multidot(n, 1, vk1, np, vk1, hd2 + k + 1, c->stream));   // ||w||^2
        HIPCK(hipMemcpyAsync(hh.data(), hd, 2 * (size_t)(m + 2) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCK(hipStreamSynchronize(c->stream));
        std::vector<double> h(k + 2);
        for (int i = 0; i <= k; ++i) h[i] = hh[i] + hh[(m + 2) + i];
        const double hk1 = sqrt(hh[(m + 2) + k + 1]);
        // the earlier rotations on the new column, then a new one that zeroes h[k+1]
        for (int i = 0; i < k; ++i) {
            const double a = cs[i] * h[i] + sn[i] * h[i + 1];
            h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
            h[i] = a;
        }
        const double den = hypot(h[k], hk1);
        cs[k] = den > 0 ? h[k] / den : 1.0;
        sn[k] = den > 0 ? hk1 / den : 0.0;
        h[k] = den;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = h[i];
        const bool done = fabs(g[k + 1]) <= tol_rel * beta || !(hk1 > 0) || !std::isfinite(hk1);
        if (done) {
            ++k;
            break;
        }
        HIPCK(launch_scale2d(1.0 / hk1, vk1, 1, n, 1, c->stream));
    }
    *iters_out = k;
    // y = R^{-1} g (upper triangular k x k), u = V y, d = M^{-1} u
    std::vector<double> y(std::max(k, 1), 0.0);
    for (int i = k - 1; i >= 0; --i) {
        double v = g[i];
        for (int t = i + 1; t < k; ++t) v -= H[(size_t)i * m + t] * y[t];
        y[i] = (H[(size_t)i * m + i] != 0.0) ? v / H[(size_t)i * m + i] : 0.0;
    }
    if (k > 0) {
        HIPCK(hipMemcpyAsync(hd, y.data(), k * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCK(launch_gemv_f64(n, k, 1, 1.0, V, np, OP_T, 0, hd, 1, 0.0, nullptr, 1, c->gm_w, 1, c->stream));
    } else {
        HIPCK(launch_fill2d(0.0, c->gm_w, 1, n, 1, c->stream));
    }
    // the host vector y must outlive the copy above
    HIPCK(hipStreamSynchronize(c->stream));
    return precond(c, trans, c->gm_w, d);
}

// The same cycle for the k <= 64 columns of R (n x k, row-major, ld k) at once: one Arnoldi step
// preconditions and multiplies all k basis columns together (the many-column substitutions and a
// GEMM with A instead of k vector sweeps), the Gram-Schmidt dots and updates run per column on
// the device, and each column keeps its own Hessenberg matrix, rotations and stopping test on the
// host.  A column that has met its tolerance (or broken down) stops growing: its later basis
// vectors are scaled to zero.  D (n x k, ld k) receives the corrections; its[c] the steps of
// column c.
int gmres_cycle_batched(genp_ctx* c, bool trans, int m, int k, const double* R, double* D, double tol_rel,
                        std::vector<int>& its) {
    const int n = (int)c->n;
    const long long vs = (long long)c->n_pad * k;     // block stride of the basis
    double* V = c->gmb_V;
    double* hd1 = c->gmb_h;                            // first Gram-Schmidt pass: (m + 2) x k
    double* hd2 = hd1 + (size_t)(m + 2) * k;           // second pass and the new norms
    double* fs = hd2 + (size_t)(m + 2) * k;            // k column scales
    its.assign(k, 0);
    HIPCK(hipMemcpyAsync(V, R, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCK(launch_bdot(n, k, 1, V, vs, V, hd1, c->gmb_part, GMB_PART, c->stream));
    std::vector<double> beta(k), f(k), h1((size_t)(m + 2) * k), h2((size_t)(m + 2) * k);
    HIPCK(hipMemcpyAsync(beta.data(), hd1, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    std::vector<char> active(k);
    int nact = 0;
    for (int col = 0; col < k; ++col) {
        beta[col] = sqrt(beta[col]);
        active[col] = beta[col] > 0 && std::isfinite(beta[col]);
        f[col] = active[col] ? 1.0 / beta[col] : 0.0;
        nact += active[col];
    }
    if (nact == 0) {
        HIPCK(launch_fill2d(0.0, D, k, n, k, c->stream));
        return GENP_OK;
    }
    HIPCK(hipMemcpyAsync(fs, f.data(), k * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCK(launch_colscale(n, k, fs, V, c->stream));
    std::vector<std::vector<double>> H(k, std::vector<double>((size_t)(m + 1) * m, 0.0));
    std::vector<std::vector<double>> cs(k, std::vector<double>(m)), sn(k, std::vector<double>(m));
    std::vector<std::vector<double>> g(k, std::vector<double>(m + 1, 0.0));
    for (int col = 0; col < k; ++col) g[col][0] = beta[col];
    int jmax = 0;
    for (int j = 0; j < m && nact > 0; ++j) {
        double* Vj = V + (size_t)j * vs;
        double* Vj1 = V + (size_t)(j + 1) * vs;
        if (trans) CK(solve_t_into(c, Vj, k, k, c->gmb_z, k));
        else CK(solve_into(c, Vj, k, k, c->gmb_z, k));
        CK(skinny(c, n, n, k, 1.0, c->A, c->lda, trans ? OP_T : OP_N, 0, c->gmb_z, k, 0.0, nullptr, k, Vj1, k));
        HIPCK(launch_bdot(n, k, j + 1, V, vs, Vj1, hd1, c->gmb_part, GMB_PART, c->stream));
        HIPCK(launch_bcomb(n, k, j + 1, V, vs, hd1, -1.0, 1.0, Vj1, c->stream));
        HIPCK(launch_bdot(n, k, j + 1, V, vs, Vj1, hd2, c->gmb_part, GMB_PART, c->stream));
        HIPCK(launch_bcomb(n, k, j + 1, V, vs, hd2, -1.0, 1.0, Vj1, c->stream));
        HIPCK(launch_bdot(n, k, 1, Vj1, vs, Vj1, hd2 + (size_t)(j + 1) * k, c->gmb_part, GMB_PART, c->stream));
        HIPCK(hipMemcpyAsync(h1.data(), hd1, (size_t)(j + 1) * k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCK(hipMemcpyAsync(h2.data(), hd2, (size_t)(j + 2) * k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCK(hipStreamSynchronize(c->stream));
        jmax = j + 1;
        for (int col = 0; col < k; ++col) {
            f[col] = 0.0;
            if (!active[col]) continue;
            std::vector<double> h(j + 2);
            for (int i = 0; i <= j; ++i) h[i] = h1[(size_t)i * k + col] + h2[(size_t)i * k + col];
            const double hk1 = sqrt(h2[(size_t)(j + 1) * k + col]);
            auto& C = cs[col];
            auto& S = sn[col];
            auto& gg = g[col];
            for (int i = 0; i < j; ++i) {
                const double a = C[i] * h[i] + S[i] * h[i + 1];
                h[i + 1] = -S[i] * h[i] + C[i] * h[i + 1];
                h[i] = a;
            }
            const double den = hypot(h[j], hk1);
            C[j] = den > 0 ? h[j] / den : 1.0;
            S[j] = den > 0 ? hk1 / den : 0.0;
            h[j] = den;
            gg[j + 1] = -S[j] * gg[j];
            gg[j] = C[j] * gg[j];
            for (int i = 0; i <= j; ++i) H[col][(size_t)i * m + j] = h[i];
            its[col] = j + 1;
            const bool done = fabs(gg[j + 1]) <= tol_rel * beta[col] || !(hk1 > 0) || !std::isfinite(hk1);
            if (done) {
                active[col] = 0;
                --nact;
            } else {
                f[col] = 1.0 / hk1;
            }
        }
        if (j + 1 < m && nact > 0) {
            HIPCK(hipMemcpyAsync(fs, f.data(), k * sizeof(double), hipMemcpyHostToDevice, c->stream));
            HIPCK(launch_colscale(n, k, fs, Vj1, c->stream));
        }
    }
    // per column: y = R^{-1} g over its own steps; u = V y for all columns at once; D = M^{-1} u
    std::vector<double> y((size_t)std::max(jmax, 1) * k, 0.0);
    for (int col = 0; col < k; ++col) {
        const int kc = its[col];
        for (int i = kc - 1; i >= 0; --i) {
            double v = g[col][i];
            for (int t = i + 1; t < kc; ++t) v -= H[col][(size_t)i * m + t] * y[(size_t)t * k + col];
            const double d = H[col][(size_t)i * m + i];
            y[(size_t)i * k + col] = d != 0.0 ? v / d : 0.0;
        }
    }
    if (jmax > 0) {
        HIPCK(hipMemcpyAsync(hd1, y.data(), (size_t)jmax * k * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCK(launch_bcomb(n, k, jmax, V, vs, hd1, 1.0, 0.0, c->gmb_w, c->stream));
    } else {
        HIPCK(launch_fill2d(0.0, c->gmb_w, k, n, k, c->stream));
    }
    HIPCK(hipStreamSynchronize(c->stream));   // the host vectors must outlive their copies
    if (trans) return solve_t_into(c, c->gmb_w, k, k, D, k);
    return solve_into(c, c->gmb_w, k, k, D, k);
}

int check_ctx(const genp_ctx* c) {
    if (!c) return GENP_EINVAL;
    return (hipSetDevice(c->device) == hipSuccess) ? GENP_OK : GENP_EDEVICE;
}

// Record a multiplier: dense G is borrowed; Toeplitz parameters are copied (and reversed for the
// transpose); a circulant keeps its spectrum; Householder parameters are copied with their dots.
int set_mult(genp_ctx* c, Mult& m, int kind, const double* G, int64_t ldg) {
    const int64_t n = c->n;
    m.kind = kind;
    m.G = (kind == GENP_G_DENSE) ? G : nullptr;
    m.ldg = ldg;
    if (kind == GENP_G_TOEPLITZ) {
        if (!m.p) {
            if (hipMalloc(&m.p, (2 * n - 1) * sizeof(double)) != hipSuccess ||
                hipMalloc(&m.p_rev, (2 * n - 1) * sizeof(double)) != hipSuccess)
                return GENP_ENOMEM;
        }
        HIPCK(hipMemcpyAsync(m.p, G, (2 * n - 1) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        // T^T(i, k) = T(k, i) = p[k - i + n - 1] = p_rev[i - k + n - 1] with p_rev[t] = p[2n - 2 - t]
        HIPCK(launch_copy2d(G, 1, m.p_rev + (2 * n - 2), -1, (int)(2 * n - 1), 1, c->stream));
    } else if (kind == GENP_G_CIRCULANT) {
        const int64_t N = n / 2;
        if (!c->circ_tw) {
            // twiddles of the length-N complex FFT and of the real-spectrum packing, in FP64 on the host
            std::vector<double2> tw(N / 2), wp(N + 1);
            const double pi = 3.14159265358979323846264338327950288;
            for (int64_t k = 0; k < N / 2; ++k)
                tw[k] = make_double2(cos(2.0 * pi * (double)k / (double)N), -sin(2.0 * pi * (double)k / (double)N));
            for (int64_t f = 0; f <= N; ++f)
                wp[f] = make_double2(cos(2.0 * pi * (double)f / (double)n), -sin(2.0 * pi * (double)f / (double)n));
            if (hipMalloc(&c->circ_tw, std::max<int64_t>(1, N / 2) * sizeof(double2)) != hipSuccess ||
                hipMalloc(&c->circ_wp, (N + 1) * sizeof(double2)) != hipSuccess)
                return GENP_ENOMEM;
            HIPCK(hipMemcpy(c->circ_tw, tw.data(), (N / 2) * sizeof(double2), hipMemcpyHostToDevice));
            HIPCK(hipMemcpy(c->circ_wp, wp.data(), (N + 1) * sizeof(double2), hipMemcpyHostToDevice));
        }
        if (!m.spec && hipMalloc(&m.spec, (N + 2) * sizeof(double2)) != hipSuccess) return GENP_ENOMEM;
        HIPCK(launch_circ_spectrum((int)n, G, c->circ_tw, c->circ_wp, m.spec, c->stream));
    } else if (kind == GENP_G_HOUSEHOLDER) {
        if (!m.uv && hipMalloc(&m.uv, (2 * n + 3) * sizeof(double)) != hipSuccess) return GENP_ENOMEM;
        if (!c->hw && hipMalloc(&c->hw, std::max<int64_t>(c->n_pad, 256) * sizeof(double)) != hipSuccess)
            return GENP_ENOMEM;
        HIPCK(hipMemcpyAsync(m.uv, G, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCK(launch_dot3((int)n, m.uv, m.uv + n, m.uv + 2 * n, c->stream));
    }
    return GENP_OK;
}

// C = A G (or C = A without a right multiplier), in the working precision.
// fuse_norms (circulant only): the product also forms ||A||_inf and max |C| (the slots
// R_ANORM and R_MAXC), which the caller then does not compute separately.
int right_product(genp_ctx* c, const double* A, int64_t lda, bool fuse_norms = false) {
    const int64_t n = c->n;
    const Mult& m = c->mr;
    const int lp = c->prec != GENP_F64;
    if (m.kind == GENP_G_NONE) {
        if (!lp) HIPCK(launch_copy2d(A, lda, (double*)c->C, c->ldc, (int)n, (int)n, c->stream));
        else HIPCK(launch_convert_f64_f32(A, lda, (float*)c->C, c->ldc, (int)n, (int)n, c->stream));
        return GENP_OK;
    }
    if (m.kind == GENP_G_CIRCULANT) {
        // each row of A correlated with c, by FFT
        HIPCK(launch_circ_apply((int)n, (int)n, 1, A, 1, lda, m.spec, c->circ_tw, c->circ_wp, 1.0, 0.0, nullptr, 0, 0,
                                c->C, lp, 1, c->ldc, c->stream, fuse_norms ? c->red + R_ANORM : nullptr,
                                fuse_norms ? c->red + R_MAXC : nullptr));
        return GENP_OK;
    }
    if (m.kind == GENP_G_HOUSEHOLDER) {
        // A G = A - (2 / v^T u) (A u) v^T: one product with A, one rank-1 pass
        const double* u = m.uv;
        const double* v = m.uv + n;
        HIPCK(launch_gemv_f64((int)n, (int)n, 1, 1.0, A, lda, OP_N, 0, u, 1, 0.0, nullptr, 0, c->hw, 1, c->stream));
        HIPCK(launch_rank1((int)n, (int)n, 1.0, A, lda, c->hw, v, m.uv + 2 * n, 2.0, 0.0, nullptr, 0, c->C, lp, c->ldc,
                           c->stream));
        return GENP_OK;
    }
    if (!lp) {
        GemmF64Args g{};
        g.M = g.N = g.K = (int)n;
        g.A = A;
        g.lda = lda;
        g.amode = OP_N;
        if (m.kind == GENP_G_DENSE) {
            g.B = m.G;
            g.ldb = m.ldg;
            g.bmode = OP_N;
        } else {
            g.B = m.p;
            g.ldb = n;
            g.bmode = OP_TOEP;
            g.group_m = 1;
        }
        g.alpha = 1.0;
        g.beta = 0.0;
        g.D = (double*)c->C;
        g.ldd = c->ldc;
        g.ksplit = 1;
        HIPCK(launch_gemm_f64(g, 0, c->stream));
        return GENP_OK;
    }
    if (c->lp_regs && c->prec != GENP_F32 && c->n_pad % 256 == 0) {
        // BF16 forms: A and G^T rounded once (FP64 -> FP32 -> BF16; the 2-word form also keeps
        // lo = bf16(x - hi)) into zero-padded copies, then the LDS-staged BF16 MFMA product
        const int np = (int)c->n_pad;
        const bool x3 = c->prec == GENP_BF16X3;
        const size_t sq = (size_t)np * np * sizeof(unsigned short);
        for (int w = 0; w < (x3 ? 2 : 1); ++w) {
            if (!c->Abf[w] && hipMalloc(&c->Abf[w], sq) != hipSuccess) return GENP_ENOMEM;
            if (!c->Gtbf[w] && hipMalloc(&c->Gtbf[w], sq) != hipSuccess) return GENP_ENOMEM;
        }
        const bool dense = m.kind == GENP_G_DENSE;
        HIPCK(launch_to_bf16(A, lda, (int)n, np, c->Abf[0], x3 ? c->Abf[1] : nullptr, c->stream));
        HIPCK(launch_gt_bf16(dense ? m.G : m.p, dense ? m.ldg : 0, dense ? 0 : 1, (int)n, np, c->Gtbf[0],
                             x3 ? c->Gtbf[1] : nullptr, c->stream));
        GemmBf16Args g{};
        g.M = g.N = g.K = np;
        g.A = c->Abf[0];
        g.lda = np;
        g.Bt = c->Gtbf[0];
        g.ldb = np;
        g.Alo = x3 ? c->Abf[1] : nullptr;
        g.Btlo = x3 ? c->Gtbf[1] : nullptr;
        g.D = (float*)c->C;
        g.ldd = c->ldc;
        g.alpha = 1.f;
        g.beta = 0.f;
        HIPCK(launch_gemm_bf16_nt(g, c->stream));
        return GENP_OK;
    }
    if (c->lp_regs) {
        // precision form: A and G rounded once to FP32 (BF16 form: then to BF16) into copies
        // zero-padded to n_pad, then the product over n_pad (padding rows and columns of C are
        // reset to the identity afterwards): FP32 with a Toeplitz G on the register-operand
        // kernel, otherwise the LDS-staged kernel (BF16 MFMA for the BF16 forms)
        const int np = (int)c->n_pad;
        const int bf = c->prec == GENP_BF16;
        const size_t sq = (size_t)np * np * sizeof(float);
        if (!c->A32 && hipMalloc(&c->A32, sq) != hipSuccess) return GENP_ENOMEM;
        const bool dense = m.kind == GENP_G_DENSE;
        const size_t gb = dense ? sq : (size_t)(2 * np) * sizeof(float);
        if (gb > c->g32_bytes) {
            hipFree(c->G32);
            c->G32 = nullptr;
            c->g32_bytes = 0;
            if (hipMalloc(&c->G32, gb) != hipSuccess) return GENP_ENOMEM;
            c->g32_bytes = gb;
        }
        HIPCK(launch_convert_pad(A, lda, (int)n, np, c->A32, np, bf, c->stream));
        if (dense) HIPCK(launch_convert_pad(m.G, m.ldg, (int)n, np, c->G32, np, bf, c->stream));
        else HIPCK(launch_convert_toep(m.p, (int)n, np, c->G32, bf, c->stream));
        if (!dense && c->prec == GENP_F32) {
            GemmF32Args g{};
            g.N = g.K = np;
            g.M = np;
            g.A = c->A32;
            g.lda = np;
            g.p = c->G32;
            g.ldb = np;
            g.D = (float*)c->C;
            g.ldd = c->ldc;
            HIPCK(launch_gemm_f32_toep(g, c->stream));
            return GENP_OK;
        }
        GemmLpArgs g{};
        g.M = g.N = g.K = np;
        g.A = c->A32;
        g.lda = np;
        g.amode = OP_N;
        g.a_f64 = 0;
        g.B = c->G32;
        g.ldb = np;
        g.bmode = dense ? OP_N : OP_TOEP;
        g.b_f64 = 0;
        g.alpha = 1.f;
        g.beta = 0.f;
        g.D = (float*)c->C;
        g.ldd = c->ldc;
        g.bf16 = c->prec == GENP_BF16 ? 1 : c->prec == GENP_BF16X3 ? 2 : 0;
        HIPCK(launch_gemm_lp(g, 0, c->stream));
        return GENP_OK;
    }
    // (GENP_LP_GEMM=lds) operands rounded FP64 -> FP32 (-> BF16, or 2-word BF16) in the loader
    GemmLpArgs g{};
    g.M = g.N = g.K = (int)n;
    g.A = A;
    g.lda = lda;
    g.amode = OP_N;
    g.a_f64 = 1;
    g.B = (m.kind == GENP_G_DENSE) ? (const void*)m.G : (const void*)m.p;
    g.ldb = (m.kind == GENP_G_DENSE) ? m.ldg : n;
    g.bmode = (m.kind == GENP_G_DENSE) ? OP_N : OP_TOEP;
    g.b_f64 = 1;
    g.alpha = 1.f;
    g.beta = 0.f;
    g.D = (float*)c->C;
    g.ldd = c->ldc;
    g.bf16 = c->prec == GENP_BF16 ? 1 : c->prec == GENP_BF16X3 ? 2 : 0;
    HIPCK(launch_gemm_lp(g, 0, c->stream));
    return GENP_OK;
}

// C := H C (FP64), C holding A G; from_a: there is no right multiplier, so C holds a copy of A
// and a product with a dense or Toeplitz H can read A itself.
int left_product(genp_ctx* c, const double* A, int64_t lda, bool from_a) {
    const int64_t n = c->n;
    const Mult& m = c->ml;
    double* C = (double*)c->C;
    if (m.kind == GENP_G_CIRCULANT) {
        // each column convolved with c, by FFT, in place (a column is read whole before it is written)
        HIPCK(launch_circ_apply((int)n, (int)n, 0, C, c->ldc, 1, m.spec, c->circ_tw, c->circ_wp, 1.0, 0.0, nullptr, 0,
                                0, C, 0, c->ldc, 1, c->stream));
        return GENP_OK;
    }
    if (m.kind == GENP_G_HOUSEHOLDER) {
        // H C = C - (2 / v^T u) u (C^T v)^T
        const double* u = m.uv;
        const double* v = m.uv + n;
        HIPCK(launch_gemv_t_f64((int)n, (int)n, 1, 1.0, C, c->ldc, 0, v, 1, 0.0, nullptr, 0, c->hw, 1, c->part,
                                (long long)KSPLIT_MAX * c->n_pad * c->kcap, c->stream));
        HIPCK(launch_rank1((int)n, (int)n, 1.0, C, c->ldc, u, c->hw, m.uv + 2 * n, 2.0, 0.0, nullptr, 0, C, 0, c->ldc,
                           c->stream));
        return GENP_OK;
    }
    // dense or Toeplitz H: an out-of-place product
    const double* Bsrc = A;
    int64_t ldb = lda;
    if (!from_a) {
        if (!c->w2 && hipMalloc(&c->w2, (size_t)n * n * sizeof(double)) != hipSuccess) return GENP_ENOMEM;
        HIPCK(launch_copy2d(C, c->ldc, c->w2, n, (int)n, (int)n, c->stream));
        Bsrc = c->w2;
        ldb = n;
    }
    GemmF64Args g{};
    g.M = g.N = g.K = (int)n;
    if (m.kind == GENP_G_DENSE) {
        g.A = m.G;
        g.lda = m.ldg;
        g.amode = OP_N;
    } else {
        g.A = m.p;   // H(i, k) = p[i - k + n - 1]: the Toeplitz order travels in lda
        g.lda = n;
        g.amode = OP_TOEP;
    }
    g.B = Bsrc;
    g.ldb = ldb;
    g.bmode = OP_N;
    g.alpha = 1.0;
    g.beta = 0.0;
    g.D = C;
    g.ldd = c->ldc;
    g.ksplit = 1;
    HIPCK(launch_gemm_f64(g, 0, c->stream));
    return GENP_OK;
}

}  // namespace

extern "C" {

const char* genp_strerror(int s) {
    switch (s) {
        case GENP_OK: return "ok";
        case GENP_BREAKDOWN: return "breakdown: a pivot of the elimination without pivoting failed";
        case GENP_ENOCONV: return "refinement did not reach the requested backward error";
        case GENP_EINVAL: return "invalid argument";
        case GENP_EDEVICE: return "no usable gfx950 device, or a HIP call failed";
        case GENP_ENOMEM: return "device allocation failed";
        case GENP_ESTATE: return "call out of order";
        case GENP_ENOTSUP: return "combination not supported";
        case GENP_ESINGULAR: return "the multiplier is singular to working precision";
        case GENP_ESCRATCH: return "problem too large for the fixed scratch of the allocation-free entry point";
        default: return "unknown status";
    }
}

int genp_create(genp_ctx** out, int64_t n, int prec, int nb, void* stream) {
    if (!out) return GENP_EINVAL;
    *out = nullptr;
    if (n < 1 || n > (1 << 20)) return GENP_EINVAL;
    if (prec != GENP_F64 && prec != GENP_F32 && prec != GENP_BF16 && prec != GENP_BF16X3) return GENP_EINVAL;
    if (nb == 0) nb = 256;
    if (nb != 64 && nb != 128 && nb != 256) return GENP_EINVAL;
    int dev = 0, cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt < 1) return GENP_EDEVICE;
    if (hipGetDevice(&dev) != hipSuccess) return GENP_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GENP_EDEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GENP_EDEVICE;
    genp_ctx* c = new (std::nothrow) genp_ctx();
    if (!c) return GENP_ENOMEM;
    c->device = dev;
    {
        hipDeviceProp_t prop{};
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            c->round_tiles = 2LL * prop.multiProcessorCount;
        // GENP_ROUND_CUT: "0" cuts the bulk into equal column parts; a positive number sets
        // the tiles per round (tests use small rounds to take this path at small n)
        if (const char* rc = getenv("GENP_ROUND_CUT")) {
            const long long v = atoll(rc);
            c->round_cut = v > 0;
            if (v > 1) c->round_tiles = v;
        }
    }
    c->stream = (hipStream_t)stream;
    c->n = n;
    c->nb = nb;
    c->prec = prec;
    c->n_pad = (n + nb - 1) / nb * nb;
    c->ldc = c->n_pad;
    const size_t nblk = c->n_pad / nb;
    bool ok = hipMalloc(&c->C, (size_t)c->n_pad * c->ldc * esize(prec)) == hipSuccess &&
              hipMalloc(&c->stats, nblk * sizeof(PanelStats)) == hipSuccess &&
              hipMalloc(&c->red, (R_COLS + 3 * 256) * sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&c->tsync, 2 * sizeof(unsigned)) == hipSuccess &&
              hipMemset(c->tsync, 0, 2 * sizeof(unsigned)) == hipSuccess &&
              hipMalloc(&c->tpub, (size_t)c->n_pad * 64 * sizeof(unsigned long long)) == hipSuccess;
    for (int e = 0; ok && e < EV_N; ++e)
        ok = hipEventCreate(&c->ev0[e]) == hipSuccess && hipEventCreate(&c->ev1[e]) == hipSuccess;
    for (int e = 0; ok && e < 2; ++e) ok = hipEventCreate(&c->ev_ag[e]) == hipSuccess;
    if (ok) {
        c->ev_step.assign(6 * nblk, nullptr);
        for (size_t i = 0; ok && i < c->ev_step.size(); ++i)
            ok = (i % 6 < 4 ? hipEventCreate(&c->ev_step[i])
                            : hipEventCreateWithFlags(&c->ev_step[i], hipEventDisableTiming)) == hipSuccess;
    }
    if (ok) ok = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        const char* la = getenv("GENP_LOOKAHEAD");
        c->lookahead = !(la && la[0] == '0');
        const char* gg = getenv("GENP_GROUP");  // "g" or "g_big,rows,g_small"
        if (gg) {
            int g1 = 0, g2 = 0;
            long long sw = 0;
            const int nf = sscanf(gg, "%d,%lld,%d", &g1, &sw, &g2);
            if (nf >= 1 && g1 >= 1 && g1 <= 8) c->g_big = c->g_small = g1;
            if (nf == 3 && g2 >= 1 && g2 <= 8 && sw >= 0) {
                c->g_switch = sw;
                c->g_small = g2;
            }
        }
        const char* tv = getenv("GENP_TRSV");   // "step": one launch per block instead of the chained solve
        c->trsv_chain = !(tv && strcmp(tv, "step") == 0);
        const char* dg = getenv("GENP_DIAG");   // "single": one workgroup per 256 diagonal block (any precision)
        c->diag_split = !(dg && strcmp(dg, "single") == 0);
        const char* gb = getenv("GENP_GMRES");   // "columns": one GMRES cycle per column
        c->gm_batched = !(gb && strcmp(gb, "columns") == 0);
        const char* fu = getenv("GENP_F32_UPD");   // "lp": the FP32 form's updates on the general kernel
        c->f32_upd = !(fu && strcmp(fu, "lp") == 0);
        const char* lg = getenv("GENP_LP_GEMM");   // "lds": the precision form's product from FP64 operands
        c->lp_regs = !(lg && strcmp(lg, "lds") == 0);
    }
    if (ok) ok = ensure_rhs(c, 4) == GENP_OK;
    if (!ok) {
        genp_destroy(c);
        return GENP_ENOMEM;
    }
    c->info.n = n;
    c->info.nb = nb;
    c->info.prec = prec;
    *out = c;
    return GENP_OK;
}

int genp_destroy(genp_ctx* c) {
    if (!c) return GENP_OK;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    hipFree(c->C);
    hipFree(c->stats);
    hipFree(c->red);
    hipFree(c->tsync);
    hipFree(c->tpub);
    hipFree(c->perm);
    for (Mult* m : {&c->mr, &c->ml}) {
        hipFree(m->p);
        hipFree(m->p_rev);
        hipFree(m->spec);
        hipFree(m->uv);
    }
    hipFree(c->hw);
    hipFree(c->A32);
    hipFree(c->dwork);
    for (int w = 0; w < 2; ++w) {
        hipFree(c->Abf[w]);
        hipFree(c->Gtbf[w]);
        hipFree(c->Lbf[w]);
        hipFree(c->Ubf[w]);
    }
    hipFree(c->G32);
    hipFree(c->w2);
    hipFree(c->circ_tw);
    hipFree(c->circ_wp);
    hipFree(c->Z);
    hipFree(c->R);
    hipFree(c->Dx);
    hipFree(c->Xb);
    hipFree(c->part);
    hipFree(c->gm_V);
    hipFree(c->gm_w);
    hipFree(c->gm_z);
    hipFree(c->gm_r);
    hipFree(c->gm_h);
    hipFree(c->gmb_V);
    hipFree(c->gmb_w);
    hipFree(c->gmb_z);
    hipFree(c->gmb_h);
    hipFree(c->gmb_part);
    hipFree(c->cest);
    for (int e = 0; e < EV_N; ++e) {
        if (c->ev0[e]) hipEventDestroy(c->ev0[e]);
        if (c->ev1[e]) hipEventDestroy(c->ev1[e]);
    }
    for (auto e : c->ev_ag)
        if (e) hipEventDestroy(e);
    for (auto e : c->ev_step)
        if (e) hipEventDestroy(e);
    if (c->side) hipStreamDestroy(c->side);
    delete c;
    return GENP_OK;
}

int genp_precondition(genp_ctx* c, const double* A, int64_t lda, int mult, const double* G, int64_t ldg) {
    return genp_precondition2(c, A, lda, GENP_G_NONE, nullptr, 0, mult, G, ldg);
}

int genp_precondition2(genp_ctx* c, const double* A, int64_t lda, int left, const double* H, int64_t ldh, int right,
                       const double* G, int64_t ldg) {
    CK(check_ctx(c));
    const int64_t n = c->n;
    if (!A || lda < n) return GENP_EINVAL;
    for (int kind : {left, right})
        if (kind < GENP_G_DENSE || kind > GENP_G_HOUSEHOLDER) return GENP_EINVAL;
    if ((right != GENP_G_NONE && !G) || (left != GENP_G_NONE && !H)) return GENP_EINVAL;
    if ((right == GENP_G_DENSE && ldg < n) || (left == GENP_G_DENSE && ldh < n)) return GENP_EINVAL;
    if ((right == GENP_G_CIRCULANT || left == GENP_G_CIRCULANT) && !circ_size_ok(n)) return GENP_ENOTSUP;
    if (left != GENP_G_NONE && c->prec != GENP_F64) return GENP_ENOTSUP;
    c->state = ST_CREATED;
    c->A = A;
    c->lda = lda;
    c->anorm1 = -1.0;
    c->info.anorm_1 = std::numeric_limits<double>::quiet_NaN();
    c->info.cond1_c = c->info.norm1_c = c->info.norm1_inv = std::numeric_limits<double>::quiet_NaN();
    if (right == GENP_G_HOUSEHOLDER || left == GENP_G_HOUSEHOLDER) CK(ensure_rhs(c, 4));
    ev_begin(c, EV_PRE);
    CK(set_mult(c, c->mr, right, G, ldg));
    CK(set_mult(c, c->ml, left, H, ldh));
    HIPCK(hipMemsetAsync(c->red, 0, sizeof(unsigned long long) * R_COLS, c->stream));
    HIPCK(hipEventRecord(c->ev_ag[0], c->stream));
    // a lone circulant product forms the two norms on the fly (one pass over A and C fewer)
    const bool fused = right == GENP_G_CIRCULANT && left == GENP_G_NONE;
    CK(right_product(c, A, lda, fused));
    if (left != GENP_G_NONE) CK(left_product(c, A, lda, right == GENP_G_NONE));
    HIPCK(hipEventRecord(c->ev_ag[1], c->stream));
    HIPCK(launch_pad_identity(c->prec, c->C, c->ldc, (int)n, (int)c->n_pad, c->stream));
    if (!fused) {
        HIPCK(launch_max_abs(c->prec, c->C, c->ldc, (int)n, (int)n, 0, c->red + R_MAXC, c->stream));
        HIPCK(launch_row_abs_sum_max(A, lda, (int)n, c->red + R_ANORM, c->stream));
    }
    ev_end(c, EV_PRE);
    unsigned long long h[3];
    double2 sv[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};   // circulant: (max, min) |spectrum|
    double dots[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};               // Householder: v^T u, u^T u, v^T v
    HIPCK(hipMemcpyAsync(h, c->red, sizeof h, hipMemcpyDeviceToHost, c->stream));
    const Mult* ms[2] = {&c->mr, &c->ml};
    for (int q = 0; q < 2; ++q) {
        if (ms[q]->kind == GENP_G_CIRCULANT)
            HIPCK(hipMemcpyAsync(&sv[q], ms[q]->spec + n / 2 + 1, sizeof(double2), hipMemcpyDeviceToHost, c->stream));
        if (ms[q]->kind == GENP_G_HOUSEHOLDER)
            HIPCK(hipMemcpyAsync(dots[q], ms[q]->uv + 2 * n, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCK(hipStreamSynchronize(c->stream));
    float ms_ag = 0.f;
    c->info.ms_ag = (hipEventElapsedTime(&ms_ag, c->ev_ag[0], c->ev_ag[1]) == hipSuccess) ? ms_ag : 0.0;
    c->anorm = bits_to_double(h[R_ANORM]);
    c->info.max_abs_c = bits_to_double(h[R_MAXC]);
    c->info.anorm_inf = c->anorm;
    c->info.mult = right;
    c->info.mult_left = left;
    bool singular = false;
    double conds[2];
    for (int q = 0; q < 2; ++q) {
        double& k = conds[q];
        k = std::numeric_limits<double>::quiet_NaN();
        switch (ms[q]->kind) {
            case GENP_G_NONE: k = 1.0; break;
            case GENP_G_CIRCULANT: {
                // the circulant is normal: its singular values are the moduli of its spectrum (Theorem 2.1)
                const double mx = sv[q].x, mn = sv[q].y;
                k = (mn > 0.0) ? mx / mn : std::numeric_limits<double>::infinity();
                if (mx != mx || mn != mn) k = std::numeric_limits<double>::quiet_NaN();
                if (!(mn > (double)n * 0x1p-53 * mx) || !std::isfinite(mx)) singular = true;
                break;
            }
            case GENP_G_HOUSEHOLDER: {
                // singular values 1 and a +- sqrt(a^2 - 1), a = ||u|| ||v|| / |v^T u|
                const double d = fabs(dots[q][0]), nn = sqrt(dots[q][1]) * sqrt(dots[q][2]);
                if (!(d > (double)n * 0x1p-53 * nn) || !std::isfinite(nn)) {
                    singular = true;
                    k = std::numeric_limits<double>::infinity();
                } else {
                    const double a = std::max(1.0, nn / d);
                    k = (a + sqrt(a * a - 1.0)) * (a + sqrt(a * a - 1.0));
                }
                break;
            }
            default: break;
        }
    }
    c->info.cond_g = conds[0];
    c->info.cond_h = conds[1];
    // a multiplier singular to working precision makes C singular too
    if (singular) return GENP_ESINGULAR;
    c->state = ST_PRECOND;
    c->block_ge = false;
    return GENP_OK;
}

static int factor_impl(genp_ctx* c, double pivot_tol, int64_t* breakdown_col, bool block) {
    CK(check_ctx(c));
    if (c->state != ST_PRECOND) return GENP_ESTATE;
    if (!(pivot_tol >= 0.0)) return GENP_EINVAL;
    if (block) {
        if (c->prec != GENP_F64) return GENP_ENOTSUP;
        if (!c->perm && hipMalloc(&c->perm, c->n_pad * sizeof(int)) != hipSuccess) return GENP_ENOMEM;
        HIPCK(launch_iota(c->perm, (int)c->n_pad, c->stream));
    }
    c->block_ge = block;
    const int64_t nb = c->nb, np = c->n_pad, ldc = c->ldc;
    const int lp = c->prec != GENP_F64;
    const size_t es = esize(c->prec);
    char* Cb = (char*)c->C;
    auto at = [&](int64_t r, int64_t col) -> void* { return Cb + (r * ldc + col) * es; };
    if (lp && c->diag_split && nb == 256 && !c->dwork &&
        hipMalloc(&c->dwork, (size_t)256 * 256 * sizeof(double)) != hipSuccess)
        return GENP_ENOMEM;
    if (lp && c->prec != GENP_F32 && c->lp_regs && nb == 256) {
        const size_t sz = (size_t)np * 8 * nb * sizeof(unsigned short);
        for (int w = 0; w < (c->prec == GENP_BF16X3 ? 2 : 1); ++w) {
            if (!c->Lbf[w] && hipMalloc(&c->Lbf[w], sz) != hipSuccess) return GENP_ENOMEM;
            if (!c->Ubf[w] && hipMalloc(&c->Ubf[w], sz) != hipSuccess) return GENP_ENOMEM;
        }
    }
    const double* maxc = (const double*)(c->red + R_MAXC);
    const int64_t K = np / nb;
    hipStream_t S = c->stream, P = c->side;
    auto ev = [&](int64_t b, int i) { return c->ev_step[6 * b + i]; };
    // panel j: diagonal block LU, then U12 = L11^{-1} A12 and L21 = A21 U11^{-1} by substitution
    auto diag = [&](int64_t j, hipStream_t st) -> int {
        const int64_t k = j * nb;
        const int nvalid = (int)std::max<int64_t>(0, std::min<int64_t>(nb, c->n - k));
        HIPCK(hipEventRecord(ev(j, 2), st));
        if (block) {
            // the block pivot with interchanges inside it, then the same interchanges on the
            // rest of its block row (L of earlier steps to the left, A12 to the right)
            HIPCK(launch_diag_lu_piv((double*)at(k, k), ldc, (int)nb, nvalid, k, maxc, pivot_tol, c->stats + j,
                                     c->perm + k, st));
            HIPCK(launch_block_row_perm((double*)c->C, ldc, k, (int)nb, (int)np, c->perm + k, st));
        } else if (c->diag_split && c->prec == GENP_F64 && nb == 256)
            HIPCK(launch_diag_lu_split(at(k, k), ldc, nvalid, k, maxc, pivot_tol, c->stats + j, 1, st));
        else if (c->diag_split && nb == 256) {
            // FP32 storage: the block widened into an FP64 scratch block, factored there by the
            // same two-half kernels (FP64 arithmetic), and rounded back to FP32; one scratch
            // block serves every step since the diagonal blocks run one after another on st
            HIPCK(launch_convert_f32_f64((const float*)at(k, k), ldc, c->dwork, 256, 256, 256, st));
            HIPCK(launch_diag_lu_split(c->dwork, 256, nvalid, k, maxc, pivot_tol, c->stats + j, 0, st));
            HIPCK(launch_convert_f64_f32(c->dwork, 256, (float*)at(k, k), ldc, 256, 256, st));
        } else
            HIPCK(launch_diag_lu(c->prec, at(k, k), ldc, (int)nb, nvalid, k, maxc, pivot_tol, c->stats + j, st));
        return GENP_OK;
    };
    auto solves = [&](int64_t j, hipStream_t st) -> int {
        const int64_t k = j * nb;
        const int64_t m = np - k - nb;
        if (m > 0)
            HIPCK(launch_panel_trsm(lp, !lp, at(k, k), ldc, (int)nb, at(k, k + nb), at(k + nb, k), ldc, (int)m, st));
        HIPCK(hipEventRecord(ev(j, 3), st));
        return GENP_OK;
    };
    auto panel = [&](int64_t j, hipStream_t st) -> int {
        CK(diag(j, st));
        return solves(j, st);
    };
    int64_t l21_key[4] = {-1, -1, -1, -1};   // BF16 forms: the L21 block last split into BF16 words
    // Schur update of steps j .. j+kb-1 (kb = 1 or 2: their L21 columns and U12 rows are
    // adjacent, so both updates are one product with K = kb nb), restricted to rows
    // [r0, r0 + M) x cols [c0, c0 + N) of the trailing block
    auto schur = [&](int64_t j, int64_t r0, int64_t c0, int64_t M, int64_t N, hipStream_t st, int kb = 1) -> int {
        if (M <= 0 || N <= 0) return GENP_OK;
        const int64_t k = j * nb;
        const int KK = (int)(kb * nb);
        if (lp && c->prec != GENP_F32 && c->lp_regs && nb == 256) {
            // BF16 forms: L21 and U12^T split into BF16 words (scratch), then the BF16 MFMA product
            // A22 -= L21 U12 (the 2-word form: hi hi + hi lo + lo hi)
            const bool x3 = c->prec == GENP_BF16X3;
            // the parts of one bulk update share their L21: split it once
            if (!(l21_key[0] == r0 && l21_key[1] == k && l21_key[2] == KK && l21_key[3] == M)) {
                HIPCK(launch_split_bf16((const float*)at(r0, k), ldc, (int)M, KK, 0, c->Lbf[0],
                                        x3 ? c->Lbf[1] : nullptr, KK, st));
                l21_key[0] = r0;
                l21_key[1] = k;
                l21_key[2] = KK;
                l21_key[3] = M;
            }
            HIPCK(launch_split_bf16((const float*)at(k, c0), ldc, KK, (int)N, 1, c->Ubf[0], x3 ? c->Ubf[1] : nullptr,
                                    KK, st));
            GemmBf16Args g{};
            g.M = (int)M;
            g.N = (int)N;
            g.K = KK;
            g.A = c->Lbf[0];
            g.lda = KK;
            g.Bt = c->Ubf[0];
            g.ldb = KK;
            g.Alo = x3 ? c->Lbf[1] : nullptr;
            g.Btlo = x3 ? c->Ubf[1] : nullptr;
            g.D = (float*)at(r0, c0);
            g.ldd = ldc;
            g.alpha = -1.f;
            g.beta = 1.f;
            g.Cin = (const float*)at(r0, c0);
            g.ldci = ldc;
            HIPCK(launch_gemm_bf16_nt(g, st));
            return GENP_OK;
        }
        if (lp && c->prec == GENP_F32 && c->f32_upd) {
            // FP32: the 256 x 128 LDS-staged update kernel (same k grouping and order)
            GemmF32UpdArgs g{};
            g.M = (int)M;
            g.N = (int)N;
            g.K = KK;
            g.A = (const float*)at(r0, k);
            g.lda = ldc;
            g.B = (const float*)at(k, c0);
            g.ldb = ldc;
            g.alpha = -1.f;
            g.beta = 1.f;
            g.Cin = (const float*)at(r0, c0);
            g.ldci = ldc;
            g.D = (float*)at(r0, c0);
            g.ldd = ldc;
            HIPCK(launch_gemm_f32_upd(g, st));
            return GENP_OK;
        }
        if (lp) {
            GemmLpArgs g{};
            g.M = (int)M;
            g.N = (int)N;
            g.K = KK;
            g.A = at(r0, k);             // L21 rows r0..
            g.lda = ldc;
            g.amode = OP_N;
            g.B = at(k, c0);             // U12 cols c0..
            g.ldb = ldc;
            g.bmode = OP_N;
            g.alpha = -1.f;
            g.beta = 1.f;
            g.Cin = (const float*)at(r0, c0);
            g.ldci = ldc;
            g.D = (float*)at(r0, c0);
            g.ldd = ldc;
            g.bf16 = c->prec == GENP_BF16 ? 1 : c->prec == GENP_BF16X3 ? 2 : 0;
            HIPCK(launch_gemm_lp(g, 0, st));
            return GENP_OK;
        }
        double* C = (double*)c->C;
        GemmF64Args g{};
        g.ksplit = 1;
        g.M = (int)M;
        g.N = (int)N;
        g.K = KK;
        g.A = C + r0 * ldc + k;          // L21 rows r0..
        g.lda = ldc;
        g.amode = OP_N;
        g.B = C + k * ldc + c0;          // U12 cols c0..
        g.ldb = ldc;
        g.bmode = OP_N;
        g.alpha = -1.0;
        g.beta = 1.0;
        g.Cin = C + r0 * ldc + c0;
        g.ldci = ldc;
        g.D = C + r0 * ldc + c0;
        g.ldd = ldc;
        HIPCK(launch_gemm_f64(g, 0, st));
        return GENP_OK;
    };
    // two blocks of the same update in one launch (FP64; the precision form launches twice)
    auto schur_two = [&](int64_t j, int64_t r0, int64_t c0, int64_t M, int64_t N, int64_t r1_, int64_t c1_,
                         int64_t M1, int64_t N1, hipStream_t st, int kb = 1) -> int {
        if (lp || M <= 0 || N <= 0 || M1 <= 0 || N1 <= 0) {
            CK(schur(j, r0, c0, M, N, st, kb));
            return schur(j, r1_, c1_, M1, N1, st, kb);
        }
        double* C = (double*)c->C;
        const int64_t k = j * nb;
        GemmF64Args g{};
        g.ksplit = 1;
        g.K = (int)(kb * nb);
        g.lda = g.ldb = g.ldci = g.ldd = ldc;
        g.amode = g.bmode = OP_N;
        g.alpha = -1.0;
        g.beta = 1.0;
        g.M = (int)M;
        g.N = (int)N;
        g.A = C + r0 * ldc + k;
        g.B = C + k * ldc + c0;
        g.Cin = g.D = C + r0 * ldc + c0;
        g.M2 = (int)M1;
        g.N2 = (int)N1;
        g.A2 = C + r1_ * ldc + k;
        g.B2 = C + k * ldc + c1_;
        g.Cin2 = g.D2 = C + r1_ * ldc + c1_;
        HIPCK(launch_gemm_f64(g, 0, st));
        return GENP_OK;
    };
    ev_begin(c, EV_FAC);
    // Steps go in groups of g so that the bulk of the trailing matrix takes the g Schur
    // updates as one product with K = g nb.  Invariant at the top of the loop for the group
    // of steps a .. a+g-1: their panels are factored, and the trailing block from
    // row/column (a+g) nb has every update before step a.  The next gn panels form the
    // look-ahead region.  Per group, on the main stream: updates a .. a+g-1 on the region's
    // block columns and rows; then for each region panel j, one of gn column parts of the
    // bulk update, the block solves of panel j and the update of step j on the rest of the
    // region.  The diagonal-block factorizations (one workgroup each) run on the side
    // stream, each under one part of the bulk.  The block solves need the whole GPU for a
    // short time, so they run between the parts rather than beside them.  Groups are large
    // (g_big) while the bulk is large and smaller (g_small) near the end, where the chain
    // of diagonal blocks and block solves is the critical path.  Without look-ahead the
    // same products run in the same order on one stream (identical values).
    hipStream_t PS = c->lookahead ? P : S;
    auto diag_async = [&](int64_t j, int e_after) -> int {
        // diagonal block j on the side stream once the main stream reaches this point
        if (PS != S) {
            HIPCK(hipEventRecord(ev(j, e_after), S));
            HIPCK(hipStreamWaitEvent(PS, ev(j, e_after), 0));
        }
        CK(diag(j, PS));
        if (PS != S) HIPCK(hipEventRecord(ev(j, 5), PS));
        return GENP_OK;
    };
    auto wait_diag = [&](int64_t j) -> int {
        if (PS != S) HIPCK(hipStreamWaitEvent(S, ev(j, 5), 0));
        return GENP_OK;
    };
    auto group_size = [&](int64_t a) -> int64_t {
        const int64_t g = np - a * nb >= c->g_switch ? c->g_big : c->g_small;
        return std::max<int64_t>(1, std::min<int64_t>(g, K - a));
    };
    // step j's update on the rest of the region that ends at block column e: block columns
    // j+1 .. e-1 (all rows below) and block rows j+1 .. e-1 (all columns right of the region)
    auto region_update = [&](int64_t j, int64_t e) -> int {
        const int64_t r = (j + 1) * nb, w = (e - j - 1) * nb;
        if (w <= 0) return GENP_OK;
        return schur_two(j, r, r, np - r, w, r, e * nb, w, np - e * nb, S);
    };
    std::vector<int64_t> gstart;
    int64_t a = 0, g = group_size(0);
    CK(panel(0, S));
    for (int64_t i = 1; i < g; ++i) {
        CK(region_update(i - 1, g));
        CK(panel(i, S));
    }
    while (a + g < K) {
        const int64_t a2 = a + g, gn = group_size(a2);
        const int64_t r2 = a2 * nb, m = np - r2;
        const int64_t w = gn * nb;
        const int64_t rb = r2 + w, mb = m - w;                   // the bulk: rows/cols rb.. (mb of them)
        const int64_t bb = mb / nb;                              // its block columns, split into gn parts
        HIPCK(hipEventRecord(ev(a, 0), S));
        gstart.push_back(a);
        CK(schur_two(a, r2, r2, m, w, r2, r2 + w, w, m - w, S, (int)g));
        // the bulk's column cuts: equal parts of whole blocks, or (FP64) parts of whole rounds
        // of update tiles, in 128-column steps, the last part taking what remains
        std::vector<int64_t> cut(gn + 1);
        for (int64_t i = 0; i <= gn; ++i) cut[i] = rb + (bb * i / gn) * nb;
        if (!lp && c->round_cut && mb > 0) {
            const int64_t tm = (mb + 127) / 128, tn = mb / 128;
            const int64_t rounds = (tm * tn + c->round_tiles - 1) / c->round_tiles;
            // (with fewer than two rounds a part the equal cut stays: it keeps every diagonal
            // block under some update work)
            if (rounds >= 2 * gn) {
                int64_t col = 0;
                for (int64_t i = 0; i < gn; ++i) {
                    cut[i] = rb + col * 128;
                    const int64_t ri = rounds * (i + 1) / gn - rounds * i / gn;
                    col = std::min(tn, col + ri * c->round_tiles / tm);
                }
                cut[gn] = rb + mb;   // the last part takes the rest (nb = 64: also a half tile)
            }
        }
        for (int64_t i = 0; i < gn; ++i) {
            const int64_t j = a2 + i;
            const int64_t c0 = cut[i], c1 = cut[i + 1];
            CK(diag_async(j, 4));
            CK(schur(a, rb, c0, mb, c1 - c0, S, (int)g));
            CK(wait_diag(j));
            CK(solves(j, S));
            CK(region_update(j, a2 + gn));
        }
        HIPCK(hipEventRecord(ev(a, 1), S));
        a = a2;
        g = gn;
    }
    HIPCK(launch_max_abs(c->prec, c->C, ldc, (int)c->n, (int)c->n, 1, c->red + R_MAXU, c->stream));
    ev_end(c, EV_FAC);
    const int64_t nblk = np / nb;
    std::vector<PanelStats> st(nblk);
    unsigned long long mu = 0;
    HIPCK(hipMemcpyAsync(st.data(), c->stats, nblk * sizeof(PanelStats), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipMemcpyAsync(&mu, c->red + R_MAXU, sizeof mu, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    double ms_s = 0.0, ms_p = 0.0;
    int ns = 0;
    // query only events recorded by this schedule: an unrecorded one would leave an error
    // behind for the next launch check
    for (int64_t b = 0; b < nblk; ++b) {
        float t0 = 0.f;
        if (hipEventElapsedTime(&t0, c->ev_step[6 * b + 2], c->ev_step[6 * b + 3]) == hipSuccess) ms_p += t0;
    }
    for (int64_t a : gstart) {
        float t1 = 0.f;
        if (hipEventElapsedTime(&t1, c->ev_step[6 * a], c->ev_step[6 * a + 1]) == hipSuccess) {
            ms_s += t1;
            ++ns;
        }
    }
    c->info.ms_schur = ms_s;
    c->info.ms_panel = ms_p;
    c->info.n_schur = ns;
    int64_t bad = -1;
    double mn = INFINITY, mx = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
        if (b * nb >= c->n) break;
        mn = std::min(mn, st[b].min_abs);
        mx = std::max(mx, st[b].max_abs);
        if (st[b].first_bad >= 0) {
            bad = st[b].first_bad;
            break;
        }
    }
    c->info.breakdown_col = bad >= 0 ? bad + 1 : 0;
    c->info.block_ge = block ? 1 : 0;
    c->info.row_swaps = 0;
    if (block) {
        std::vector<int> pr(np);
        HIPCK(hipMemcpy(pr.data(), c->perm, np * sizeof(int), hipMemcpyDeviceToHost));
        for (int64_t r = 0; r < np; ++r) c->info.row_swaps += pr[r] != r;
    }
    c->info.min_abs_piv = mn;
    c->info.max_abs_piv = mx;
    c->info.max_abs_u = bits_to_double(mu);
    c->info.growth = c->info.max_abs_c > 0 ? c->info.max_abs_u / c->info.max_abs_c : INFINITY;
    if (breakdown_col) *breakdown_col = c->info.breakdown_col;
    if (bad >= 0) {
        c->state = ST_BROKEN;
        return GENP_BREAKDOWN;
    }
    c->state = ST_FACTORED;
    return GENP_OK;
}

int genp_factor(genp_ctx* c, double pivot_tol, int64_t* breakdown_col) {
    return factor_impl(c, pivot_tol, breakdown_col, false);
}

int genp_factor_block(genp_ctx* c, double pivot_tol, int64_t* breakdown_col) {
    return factor_impl(c, pivot_tol, breakdown_col, true);
}

int genp_block_pivots(const genp_ctx* cc, double* out, int64_t ldo) {
    genp_ctx* c = const_cast<genp_ctx*>(cc);
    CK(check_ctx(c));
    if (c->state != ST_FACTORED) return GENP_ESTATE;
    if (c->prec != GENP_F64) return GENP_ENOTSUP;
    if (!out || ldo < c->nb) return GENP_EINVAL;
    HIPCK(launch_block_pivots((const double*)c->C, c->ldc, (int)c->n, (int)c->nb, c->block_ge ? c->perm : nullptr,
                              out, ldo, c->stream));
    return GENP_OK;
}

int genp_row_perm(const genp_ctx* cc, int32_t* perm) {
    genp_ctx* c = const_cast<genp_ctx*>(cc);
    CK(check_ctx(c));
    if (c->state != ST_FACTORED && c->state != ST_BROKEN) return GENP_ESTATE;
    if (!perm) return GENP_EINVAL;
    if (c->block_ge)
        HIPCK(hipMemcpyAsync(perm, c->perm, c->n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    else
        HIPCK(launch_iota(perm, (int)c->n, c->stream));
    return GENP_OK;
}

int genp_solve(genp_ctx* c, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx) {
    CK(check_ctx(c));
    if (c->state != ST_FACTORED) return GENP_ESTATE;
    if (!B || !X || nrhs < 1 || ldb < nrhs || ldx < nrhs) return GENP_EINVAL;
    CK(ensure_rhs(c, nrhs));
    ev_begin(c, EV_SOL);
    for (int64_t c0 = 0; c0 < nrhs; c0 += 256) {
        const int k = (int)std::min<int64_t>(256, nrhs - c0);
        CK(solve_into(c, B + c0, ldb, k, X + c0, ldx));
    }
    ev_end(c, EV_SOL);
    return GENP_OK;
}

// The chained solves record a wait that exceeded its safety limit in a sticky word;
// the next synchronizing call reports it once (the solutions computed since are invalid)
// and clears it, so later calls report only new overruns.
static int chain_status(genp_ctx* c) {
    if (!c->trsv_chain) return GENP_OK;
    unsigned err = 0;
    HIPCK(hipMemcpyAsync(&err, c->tsync + 1, sizeof err, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    if (!err) return GENP_OK;
    HIPCK(hipMemsetAsync(c->tsync + 1, 0, sizeof(unsigned), c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return GENP_EDEVICE;
}

}  // extern "C"

namespace {

// Refinement of X (n x k) against Op = A (or A^T when trans) and the right-hand sides B, in FP64:
// R = B - Op X, then the correction D = M^{-1} R (LU-IR, section 7.1) or, per column, one GMRES
// cycle for Op d = r right-preconditioned by M^{-1}; X += D.  Stops when max_j eta_j <= tol, after
// o.max_outer corrections, or once the GMRES budget o.max_inner is spent.  LU-IR also stops when a
// correction made eta worse (it is undone): the contraction factor is then above 1 and later
// steps only diverge.  GMRES-IR keeps going through such a step (a cycle shrinks the residual's
// 2-norm, which the infinity-norm eta need not follow at once) and stops after three steps in a
// row without a new best; the best iterate is kept aside and returned.  GENP_SOLVER_AUTO starts
// with LU-IR and turns to GMRES-IR (from the best iterate) at the first correction that does
// not divide eta by 4.  Status: GENP_OK when eta <= tol, or when tol = 0 (the steps were asked
// for, not a target); else GENP_ENOCONV.
int refine_core(genp_ctx* c, bool trans, const double* B, int64_t ldb, int k, double* X, int64_t ldx,
                const genp_refine_opts& o, std::vector<double>& eta, int* iters_out, int* inner_out,
                double* hist, int* n_hist) {
    const int n = (int)c->n;
    const double anorm = trans ? c->anorm1 : c->anorm;
    const int restart = o.restart > 0 ? o.restart : 50;
    const double rtol = o.inner_rtol > 0 ? o.inner_rtol : 1e-10;
    const int aop = trans ? OP_T : OP_N;
    auto residual = [&]() -> int {
        CK(skinny(c, n, n, k, -1.0, c->A, c->lda, aop, 0, X, ldx, 1.0, B, ldb, c->R, k));
        return backward_error(c, c->R, k, X, ldx, B, ldb, k, eta, anorm);
    };
    // GENP_SOLVER_AUTO: LU-IR while each correction divides eta by 4 or more, GMRES-IR after
    bool gm = o.solver == GENP_SOLVER_GMRES;
    const bool adaptive = o.solver == GENP_SOLVER_AUTO;
    int inner_total = 0;
    double best = INFINITY, prev = INFINITY;
    int it = 0, stall = 0;
    bool cur_best = true;              // X is the best iterate so far
    int status = GENP_OK;
    *n_hist = 0;
    for (;;) {
        CK(residual());
        double e = max_of(eta);
        if (*n_hist < GENP_ETA_HIST) hist[(*n_hist)++] = e;
        if (!gm && it > 0 && !(e <= best)) {
            // an LU-IR correction made things worse (or produced NaN): undo it
            HIPCK(launch_axpy2d(-1.0, c->Dx, k, X, ldx, n, k, c->stream));
            CK(residual());
            e = max_of(eta);
            if (!adaptive) {
                status = (o.tol > 0) ? GENP_ENOCONV : GENP_OK;
                break;
            }
            gm = true;   // X is the best iterate again: go on with GMRES-IR from it
        } else if (e < best || it == 0) {
            best = std::min(best, e);
            stall = 0;
            cur_best = true;
        } else {
            ++stall;
            cur_best = false;
        }
        if (adaptive && !gm && it > 0 && !(e <= 0.25 * prev)) gm = true;   // LU-IR contracts too slowly
        prev = e;
        if (gm && cur_best) HIPCK(launch_copy2d(X, ldx, c->Xb, k, n, k, c->stream));
        if (e <= o.tol) break;
        // (the many-column cycle needs one step per column; with fewer left the budget is spent)
        const bool batched = k > 1 && k <= 64 && c->gm_batched;
        const bool budget = gm && o.max_inner > 0 && o.max_inner - inner_total < (batched ? k : 1);
        if (it >= o.max_outer || budget || (gm && stall >= 3)) {
            status = (o.tol > 0) ? GENP_ENOCONV : GENP_OK;
            break;
        }
        if (!gm) {
            // Dx = M^{-1} R
            if (trans) CK(solve_t_into(c, c->R, k, k, c->Dx, k));
            else CK(solve_into(c, c->R, k, k, c->Dx, k));
        } else if (batched) {
            // all columns in one cycle; the budget counts every column's steps
            int m = restart;
            if (o.max_inner > 0) m = std::min(m, (o.max_inner - inner_total) / k);
            if (m <= 0) {
                HIPCK(launch_fill2d(0.0, c->Dx, k, n, k, c->stream));
            } else {
                CK(ensure_gmres_batched(c, m, k));
                std::vector<int> its;
                CK(gmres_cycle_batched(c, trans, m, k, c->R, c->Dx, rtol, its));
                for (int v : its) inner_total += v;
            }
        } else {
            for (int j = 0; j < k; ++j) {
                int m = restart;
                if (o.max_inner > 0) m = std::min(m, o.max_inner - inner_total);
                if (m <= 0) {
                    // budget spent: the remaining columns take no correction this step
                    HIPCK(launch_fill2d(0.0, c->Dx + j, k, n, 1, c->stream));
                    continue;
                }
                HIPCK(launch_copy2d(c->R + j, k, c->gm_r, 1, n, 1, c->stream));
                int its = 0;
                CK(gmres_cycle(c, trans, m, c->gm_r, c->gm_z, rtol, &its));
                inner_total += its;
                HIPCK(launch_copy2d(c->gm_z, 1, c->Dx + j, k, n, 1, c->stream));
            }
        }
        HIPCK(launch_axpy2d(1.0, c->Dx, k, X, ldx, n, k, c->stream));
        ++it;
    }
    if (gm && !cur_best) {
        // return the best iterate, with its eta
        HIPCK(launch_copy2d(c->Xb, k, X, ldx, n, k, c->stream));
        CK(residual());
        if (max_of(eta) <= o.tol) status = GENP_OK;
    }
    *iters_out = it;
    *inner_out = inner_total;
    return status;
}

int check_opts(const genp_refine_opts* o) {
    if (!o) return GENP_EINVAL;
    if (o->solver != GENP_SOLVER_LUIR && o->solver != GENP_SOLVER_GMRES && o->solver != GENP_SOLVER_AUTO)
        return GENP_EINVAL;
    if (o->max_outer < 0 || o->max_inner < 0 || o->restart < 0 || o->restart > GENP_GMRES_MAX_RESTART ||
        !(o->tol >= 0) || !(o->inner_rtol >= 0))
        return GENP_EINVAL;
    return GENP_OK;
}

// ||A||_1 of the borrowed A, once per precondition (the norm in the adjoint system's eta).
int ensure_anorm1(genp_ctx* c) {
    if (c->anorm1 >= 0.0) return GENP_OK;
    unsigned long long* slot = c->red + R_ANORM1;
    HIPCK(hipMemsetAsync(slot, 0, sizeof(unsigned long long), c->stream));
    HIPCK(launch_col_abs_sum_max(c->A, c->lda, (int)c->n, c->part, (long long)KSPLIT_MAX * c->n_pad * c->kcap, slot,
                                 c->stream));
    unsigned long long h = 0;
    HIPCK(hipMemcpyAsync(&h, slot, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    c->anorm1 = bits_to_double(h);
    return GENP_OK;
}

// dB = A^{-T} W (= H^T L^{-T} U^{-T} G^T W from the factors), refined against A^T per o, and
// dA = -dB X^T when dA is not NULL.
int backward_impl(genp_ctx* c, const double* W, int64_t ldw, const double* X, int64_t ldx, int64_t nrhs, double* dB,
                  int64_t lddb, double* dA, int64_t ldda, const genp_refine_opts& o, double* eta_out) {
    const int k = (int)nrhs, n = (int)c->n;
    CK(ensure_rhs(c, nrhs));
    if (o.solver != GENP_SOLVER_LUIR) CK(ensure_gmres(c, o.restart > 0 ? o.restart : 50));
    CK(ensure_anorm1(c));
    ev_begin(c, EV_BWD);
    CK(solve_t_into(c, W, ldw, k, dB, lddb));
    std::vector<double> eta;
    int it = 0, inner = 0, nh = 0;
    double hist[GENP_ETA_HIST];
    const int status = refine_core(c, true, W, ldw, k, dB, lddb, o, eta, &it, &inner, hist, &nh);
    if (status < 0) return status;
    if (dA) {
        // dA = -dB X^T
        GemmF64Args g{};
        g.M = g.N = n;
        g.K = k;
        g.A = dB;
        g.lda = lddb;
        g.amode = OP_N;
        g.B = X;
        g.ldb = ldx;
        g.bmode = OP_T;
        g.alpha = -1.0;
        g.beta = 0.0;
        g.D = dA;
        g.ldd = ldda;
        g.ksplit = 1;
        HIPCK(launch_gemm_f64(g, 0, c->stream));
    }
    ev_end(c, EV_BWD);
    HIPCK(hipStreamSynchronize(c->stream));
    CK(chain_status(c));
    c->info.bwd_iters = it;
    c->info.bwd_inner_iters = inner;
    c->info.bwd_eta = max_of(eta);
    c->info.anorm_1 = c->anorm1;
    if (eta_out)
        for (int j = 0; j < k; ++j) eta_out[j] = eta[j];
    return status;
}

int refine_impl(genp_ctx* c, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                const genp_refine_opts& o, double* eta_out) {
    CK(ensure_rhs(c, nrhs));
    if (o.solver != GENP_SOLVER_LUIR) CK(ensure_gmres(c, o.restart > 0 ? o.restart : 50));
    const int k = (int)nrhs;
    ev_begin(c, EV_REF);
    std::vector<double> eta;
    int it = 0, inner = 0, nh = 0;
    const int status = refine_core(c, false, B, ldb, k, X, ldx, o, eta, &it, &inner, c->info.eta_hist, &nh);
    c->info.n_eta = nh;
    if (status < 0) return status;
    ev_end(c, EV_REF);
    HIPCK(hipStreamSynchronize(c->stream));
    CK(chain_status(c));
    c->info.iters = it;
    c->info.inner_iters = inner;
    c->info.eta = max_of(eta);
    if (eta_out)
        for (int j = 0; j < k; ++j) eta_out[j] = eta[j];
    return status;
}

// Hager-Higham estimate of ||B||_1 for an n x n operator given by y = B x (apply) and
// y = B^T x (apply_t) on n_pad-vectors with zero padding (Higham 1988, Algorithm 4.1; at most
// five products with B^T).  On the cycling exit the larger of the last two values is kept
// (both are lower bounds of ||B||_1).
template <class F, class FT>
int hager_norm1(genp_ctx* c, F apply, FT apply_t, double* est_out) {
    const int n = (int)c->n;
    const int64_t np = c->n_pad;
    double* x = c->cest;
    double* y = x + np;
    double* xi = y + np;
    double* z = xi + np;
    double* sc = z + np;
    double hsc[3];
    auto fetch = [&](int cnt) -> int {
        HIPCK(hipMemcpyAsync(hsc, sc, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCK(hipStreamSynchronize(c->stream));
        return GENP_OK;
    };
    HIPCK(launch_fill2d(0.0, x, 1, (int)(4 * np), 1, c->stream));
    HIPCK(launch_fill2d(1.0 / n, x, 1, n, 1, c->stream));
    CK(apply(x, y));
    HIPCK(launch_cest_sign(n, y, xi, sc, c->stream));
    CK(fetch(2));
    double est = hsc[0];
    if (n == 1) {
        *est_out = est;
        return GENP_OK;
    }
    CK(apply_t(xi, z));
    HIPCK(launch_cest_argmax(n, z, -1, sc, c->stream));
    CK(fetch(2));
    int j = (int)hsc[1];
    for (int iter = 2;; ++iter) {
        HIPCK(launch_unit_vector(n, j, x, c->stream));
        CK(apply(x, y));
        HIPCK(launch_cest_sign(n, y, xi, sc, c->stream));
        CK(fetch(2));
        const double est_old = est;
        est = hsc[0];
        if (hsc[1] != 0.0 || est <= est_old) {   // repeated sign vector, or no increase
            est = std::max(est, est_old);
            break;
        }
        CK(apply_t(xi, z));
        HIPCK(launch_cest_argmax(n, z, j, sc, c->stream));
        CK(fetch(3));
        const int jlast = j;
        j = (int)hsc[1];
        (void)jlast;
        if (hsc[2] == hsc[0] || iter >= 5) break;
    }
    HIPCK(launch_cest_alt(n, x, c->stream));
    CK(apply(x, y));
    HIPCK(launch_cest_sign(n, y, xi, sc, c->stream));
    CK(fetch(1));
    const double alt = 2.0 * hsc[0] / (3.0 * n);
    *est_out = std::max(est, alt);
    return GENP_OK;
}

}  // namespace

extern "C" {

int genp_refine(genp_ctx* c, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx, int max_iter,
                double tol, int solver, double* eta_out) {
    genp_refine_opts o{};
    o.solver = solver;
    o.max_outer = max_iter;
    o.restart = 50;
    o.max_inner = 0;
    o.tol = tol;
    o.inner_rtol = 1e-10;
    return genp_refine_ex(c, B, ldb, nrhs, X, ldx, &o, eta_out);
}

int genp_refine_ex(genp_ctx* c, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                   const genp_refine_opts* o, double* eta_out) {
    CK(check_ctx(c));
    if (c->state != ST_FACTORED) return GENP_ESTATE;
    if (!B || !X || nrhs < 1 || nrhs > 256 || ldb < nrhs || ldx < nrhs) return GENP_EINVAL;
    CK(check_opts(o));
    return refine_impl(c, B, ldb, nrhs, X, ldx, *o, eta_out);
}

int genp_solve_backward(genp_ctx* c, const double* W, int64_t ldw, const double* X, int64_t ldx, int64_t nrhs,
                        double* dB, int64_t lddb, double* dA, int64_t ldda, int refine_iters) {
    if (refine_iters < 0) return GENP_EINVAL;
    genp_refine_opts o{};
    o.solver = GENP_SOLVER_LUIR;
    o.max_outer = refine_iters;
    o.tol = 0.0;
    return genp_solve_backward_ex(c, W, ldw, X, ldx, nrhs, dB, lddb, dA, ldda, &o, nullptr);
}

int genp_solve_backward_ex(genp_ctx* c, const double* W, int64_t ldw, const double* X, int64_t ldx, int64_t nrhs,
                           double* dB, int64_t lddb, double* dA, int64_t ldda, const genp_refine_opts* o,
                           double* eta_out) {
    CK(check_ctx(c));
    if (c->state != ST_FACTORED) return GENP_ESTATE;
    if (!W || !X || !dB || nrhs < 1 || nrhs > 256 || ldw < nrhs || ldx < nrhs || lddb < nrhs || (dA && ldda < c->n))
        return GENP_EINVAL;
    CK(check_opts(o));
    return backward_impl(c, W, ldw, X, ldx, nrhs, dB, lddb, dA, ldda, *o, eta_out);
}

int genp_condest(genp_ctx* c, double* kappa, double* norm_c, double* norm_inv) {
    CK(check_ctx(c));
    if (c->state != ST_FACTORED) return GENP_ESTATE;
    CK(ensure_rhs(c, 4));
    CK(ensure_gmres(c, 0));
    if (!c->cest && hipMalloc(&c->cest, (4 * (size_t)c->n_pad + 8) * sizeof(double)) != hipSuccess)
        return GENP_ENOMEM;
    const int n = (int)c->n;
    double* t1 = c->gm_w;
    double* t2 = c->gm_z;
    // (L U)^{-1} and its transpose on n_pad vectors (P and P^T included for block elimination)
    auto inv = [&](const double* x, double* y) -> int {
        HIPCK(hipMemcpyAsync(y, x, c->n_pad * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        return lu_solve_inplace(c, y, 1, 1);
    };
    auto inv_t = [&](const double* x, double* y) -> int {
        HIPCK(hipMemcpyAsync(y, x, c->n_pad * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        return lu_solve_trans_inplace(c, y, 1, 1);
    };
    // C = H A G and C^T = G^T A^T H^T, from the original FP64 A and the multipliers
    auto fwd = [&](const double* x, double* y) -> int {
        CK(apply_mult(c, c->mr, 0, 1, 1.0, x, 1, 0.0, nullptr, 0, t1, 1));
        CK(op_a(c, false, t1, t2));
        return apply_mult(c, c->ml, 0, 1, 1.0, t2, 1, 0.0, nullptr, 0, y, 1);
    };
    auto fwd_t = [&](const double* x, double* y) -> int {
        CK(apply_mult(c, c->ml, 1, 1, 1.0, x, 1, 0.0, nullptr, 0, t1, 1));
        CK(op_a(c, true, t1, t2));
        return apply_mult(c, c->mr, 1, 1, 1.0, t2, 1, 0.0, nullptr, 0, y, 1);
    };
    ev_begin(c, EV_CEST);
    double ni = 0.0, nc = 0.0;
    CK(hager_norm1(c, inv, inv_t, &ni));
    CK(hager_norm1(c, fwd, fwd_t, &nc));
    ev_end(c, EV_CEST);
    HIPCK(hipStreamSynchronize(c->stream));
    CK(chain_status(c));
    (void)n;
    c->info.norm1_c = nc;
    c->info.norm1_inv = ni;
    c->info.cond1_c = nc * ni;
    if (kappa) *kappa = nc * ni;
    if (norm_c) *norm_c = nc;
    if (norm_inv) *norm_inv = ni;
    return GENP_OK;
}

int genp_get_info(const genp_ctx* cc, genp_info* out) {
    genp_ctx* c = const_cast<genp_ctx*>(cc);
    CK(check_ctx(c));
    if (!out) return GENP_EINVAL;
    HIPCK(hipStreamSynchronize(c->stream));
    CK(chain_status(c));
    float ms;
    double* slots[EV_N] = {&c->info.ms_precond, &c->info.ms_factor, &c->info.ms_solve, &c->info.ms_refine,
                           &c->info.ms_backward, &c->info.ms_condest};
    for (int e = 0; e < EV_N; ++e)
        if (c->ev_used[e] && hipEventElapsedTime(&ms, c->ev0[e], c->ev1[e]) == hipSuccess) *slots[e] = ms;
    *out = c->info;
    return GENP_OK;
}

int genp_copy_work(const genp_ctx* cc, double* out, int64_t ldo) {
    genp_ctx* c = const_cast<genp_ctx*>(cc);
    CK(check_ctx(c));
    if (!out || ldo < c->n) return GENP_EINVAL;
    if (c->state == ST_CREATED) return GENP_ESTATE;
    HIPCK(launch_copy_work(c->prec, c->C, c->ldc, (int)c->n, out, ldo, c->stream));
    return GENP_OK;
}

}  // extern "C"
