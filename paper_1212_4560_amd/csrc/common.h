// Shared device helpers and launcher declarations of the GENP HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

// Operand access of a GEMM operand (i = row, k = column of the logical operand).
enum OpMode : int {
    OP_N = 0,     // row-major: X[i * ld + k]
    OP_T = 1,     // transposed storage: X[k * ld + i]
    OP_TOEP = 2   // Toeplitz: X(i, k) = p[i - k + t - 1], t = ld, 2t-1 parameters
};

// Working precisions (mirror of the public enum).
enum : int { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_BF16X3 = 3 };

// Per-panel pivot statistics written by the diagonal-block kernels.
struct PanelStats {
    double min_abs;       // min |u_kk| over the valid pivots of the block
    double max_abs;       // max |u_kk|
    long long first_bad;  // global 0-based index of the first failing pivot, or -1
    long long pad;
};

// Monotone encoding of a non-negative double (or NaN) for atomicMax on its bits.
__device__ inline void atomic_max_nonneg(unsigned long long* addr, double v) {
    atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

__device__ inline int xcd_remap(int bid, int total) {
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of tiles so neighbouring tiles share its L2.
    const int x = bid & 7, q = total >> 3, r = total & 7;
    return x * q + (x < r ? x : r) + (bid >> 3);
}

// ---------------------------------------------------------------- launchers ---
struct GemmF64Args {
    int M, N, K;
    const double* A; long long lda; int amode;
    const double* B; long long ldb; int bmode;
    double alpha, beta;
    const double* Cin; long long ldci;   // read only when beta != 0
    double* D; long long ldd;
    int ksplit;                          // > 1: D receives ksplit partial products
    long long split_stride;              //      at D + s * split_stride (beta ignored)
    int a_f32;                           // A operand stored as FP32 (widened on load)
    int group_m;                         // tile-rows per group of the tile order (0 = 8)
    // optional second product in the same launch (same K, modes, leading dimensions,
    // alpha, beta; no split-K): M2 x N2 into D2 from A2, B2, Cin2 (M2 = 0: none)
    int M2, N2;
    const double* A2; const double* B2; const double* Cin2; double* D2;
};
// tile: 0 = 128x128 (2x2 waves), 1 = 256x64 (4x1), 2 = 64x256 (1x4), 3 = 64x64,
//       4 = 128x64 (2x1), 5 = 64x128 (1x2)
hipError_t launch_gemm_f64(const GemmF64Args& a, int tile, hipStream_t s);

// D = alpha * sum_s P[s] + beta * Cin over an M x N block (split-K reduction)
hipError_t launch_splitk_reduce_f64(int M, int N, int ksplit, const double* P, long long ldp,
                                    long long split_stride, double alpha, double beta,
                                    const double* Cin, long long ldci, double* D, long long ldd,
                                    hipStream_t s);

// GEMM in FP32 storage: C(fp32) = A(fp64->fp32) * B(fp64->fp32) or fp32 operands.
struct GemmLpArgs {
    int M, N, K;
    const void* A; long long lda; int amode; int a_f64;   // a_f64: operand stored as FP64
    const void* B; long long ldb; int bmode; int b_f64;
    float alpha, beta;
    const float* Cin; long long ldci;
    float* D; long long ldd;
    int bf16;                            // 1: round operands to BF16, BF16 MFMA, FP32 accumulate;
                                         // 2: 2-word BF16 operands, three BF16 MFMA products
};
hipError_t launch_gemm_lp(const GemmLpArgs& a, int tile, hipStream_t s);

// FP32 product D = A G with register operands (gemm_f32.hip), A row-major M x K (FP32), G
// generated from FP32 Toeplitz parameters: G(k, j) = p[k - j + ldb - 1], K = ldb, N <= ldb.
// M, N multiples of 64, K of 16, A 16-byte aligned, lda a multiple of 4.
struct GemmF32Args {
    int M, N, K;
    const float* A; long long lda;
    const float* p; long long ldb;
    float* D; long long ldd;
};
hipError_t launch_gemm_f32_toep(const GemmF32Args& a, hipStream_t s);
// FP32 update D = alpha A B + beta Cin (row-major FP32 operands, Cin may alias D), LDS-staged,
// each MFMA over four consecutive k (gemm_f32.hip).  M, N multiples of 64, K of 16; A and B
// 16-byte aligned with leading dimensions that are multiples of 4.
struct GemmF32UpdArgs {
    int M, N, K;
    const float* A; long long lda;
    const float* B; long long ldb;
    float alpha, beta;
    const float* Cin; long long ldci;
    float* D; long long ldd;
};
hipError_t launch_gemm_f32_upd(const GemmF32UpdArgs& a, hipStream_t s);
// BF16 product D (FP32, M x N) = A Bt^T with A (M x K) and Bt (N x K) BF16 row-major (gemm_bf16.hip);
// with Alo and Btlo (the second words of 2-word BF16 operands) D = A Bt^T + A Btlo^T + Alo Bt^T.
// M, N multiples of 256, K of 32, operands 16-byte aligned, lda and ldb multiples of 8.
struct GemmBf16Args {
    int M, N, K;
    const unsigned short* A; long long lda;
    const unsigned short* Bt; long long ldb;
    const unsigned short* Alo;
    const unsigned short* Btlo;
    float* D; long long ldd;
    float alpha, beta;                  // D = alpha product + beta Cin (Cin may alias D)
    const float* Cin; long long ldci;
};
hipError_t launch_gemm_bf16_nt(const GemmBf16Args& a, hipStream_t s);
// hi / lo (rows x cols, ldo) = 2-word BF16 split of an FP32 block X (rows x cols, ldx); with trans,
// hi / lo (cols x rows) = the split of X^T; lo nullable
hipError_t launch_split_bf16(const float* X, long long ldx, int rows, int cols, int trans, unsigned short* hi,
                             unsigned short* lo, long long ldo, hipStream_t s);
// hi (n_pad x n_pad) = bf16(fp32(A)), lo (nullable) = bf16(fp32(A) - hi); zero padding
hipError_t launch_to_bf16(const double* A, long long lda, int n, int n_pad, unsigned short* hi, unsigned short* lo,
                          hipStream_t s);
// hi / lo (n_pad x n_pad): the transpose of G (dense, ldg; or Toeplitz parameters when toep) in the
// same 2-word BF16 split, zero padding
hipError_t launch_gt_bf16(const double* G, long long ldg, int toep, int n, int n_pad, unsigned short* hi,
                          unsigned short* lo, hipStream_t s);
// out (rows_pad x rows_pad, ldo) = A (n x n FP64) rounded to FP32 (bf16: then to BF16), zero padding
hipError_t launch_convert_pad(const double* A, long long lda, int n, int n_pad, float* out, long long ldo, int bf16,
                              hipStream_t s);
// out[u] = p[u - (n_pad - n)] rounded likewise for u < 2 n_pad - 1 (0 outside p's 2n - 1 entries)
hipError_t launch_convert_toep(const double* p, int n, int n_pad, float* out, int bf16, hipStream_t s);

// Diagonal block LU (no pivoting) in place, one workgroup; records PanelStats.
// FP64 256 x 256 diagonal block as two LDS-resident 128 blocks, the panel solves and one update
// (rcp: the panel solves' pivots as reciprocals, as for launch_panel_trsm)
hipError_t launch_diag_lu_split(void* Dblk, long long ldd, int nvalid, long long col0, const double* maxc,
                                double pivot_tol, PanelStats* st, int rcp, hipStream_t s);
hipError_t launch_diag_lu(int prec, void* Dblk, long long ldd, int nb, int nvalid,
                          long long col0, const double* maxc, double pivot_tol,
                          PanelStats* st, hipStream_t s);
// Block Gaussian elimination (Theorem 2.2): the FP64 diagonal block as the block pivot, rows
// interchanged inside it; perm[r] (r < nb) receives the global row that factor row r came from.
hipError_t launch_diag_lu_piv(double* Dblk, long long ldd, int nb, int nvalid, long long col0, const double* maxc,
                              double pivot_tol, PanelStats* st, int* perm, hipStream_t s);
// Rows row0 .. row0+nb-1 take the block's interchanges in the columns outside the diagonal block.
hipError_t launch_block_row_perm(double* C, long long ldc, long long row0, int nb, int ncols, const int* perm,
                                 hipStream_t s);
// out (n x ldo): the explicit block pivots P_k^T L_kk U_kk of the packed factors (perm may be null).
hipError_t launch_block_pivots(const double* C, long long ldc, int n, int nb, const int* perm, double* out,
                               long long ldo, hipStream_t s);
// dst row i = src row perm[i] (gather), or dst row perm[i] = src row i (scatter); n x k, FP64.
hipError_t launch_permute_rows(int n, int k, const double* src, long long lds, double* dst, long long ldd,
                               const int* perm, int scatter, hipStream_t s);
hipError_t launch_iota(int* p, int n, hipStream_t s);
// Fill the padding of an n_pad x n_pad working matrix: zeros off the diagonal, ones on it.
hipError_t launch_pad_identity(int prec, void* C, long long ldc, int n, int n_pad, hipStream_t s);
hipError_t launch_max_abs(int prec, const void* X, long long ldx, int rows, int cols, int upper_only,
                          unsigned long long* out_bits, hipStream_t s);
hipError_t launch_row_abs_sum_max(const double* A, long long lda, int n,
                                  unsigned long long* out_bits, hipStream_t s);
hipError_t launch_col_abs_max(const double* X, long long ldx, int rows, int cols,
                              unsigned long long* out_bits, hipStream_t s);
hipError_t launch_copy_work(int prec, const void* C, long long ldc, int n, double* out,
                            long long ldo, hipStream_t s);
hipError_t launch_copy2d(const double* src, long long lds, double* dst, long long ldd,
                         int rows, int cols, hipStream_t s);
hipError_t launch_axpy2d(double alpha, const double* X, long long ldx, double* Y, long long ldy,
                         int rows, int cols, hipStream_t s);
hipError_t launch_fill2d(double v, double* X, long long ldx, int rows, int cols, hipStream_t s);
// y (M x nrhs) = alpha A^T X + beta yin for A stored K x M (row-major, lda), nrhs <= 4, in two
// deterministic passes through part (at least M * nrhs doubles; more allows more row slices).
hipError_t launch_gemv_t_f64(int M, int K, int nrhs, double alpha, const void* A, long long lda, int a_f32,
                             const double* X, long long ldx, double beta, const double* Yin, long long ldyi,
                             double* Y, long long ldy, double* part, long long part_cap, hipStream_t s);
// Y (M x N, FP64 or FP32) = alpha (X - (factor / dot[0]) a b^T) + beta Yin; dot is a device scalar
hipError_t launch_rank1(int M, int N, double alpha, const double* X, long long ldx, const double* a, const double* b,
                        const double* dot, double factor, double beta, const double* Yin, long long ldyi, void* Y,
                        int y_f32, long long ldy, hipStream_t s);
// out[0..2] = (v^T u, u^T u, v^T v)
hipError_t launch_dot3(int n, const double* u, const double* v, double* out, hipStream_t s);

// y[i][c] = beta * yin[i][c] + alpha * sum_k op(A)(i, k) x[k][c] for nrhs <= 4 (one wave per row).
hipError_t launch_gemv_f64(int M, int K, int nrhs, double alpha,
                           const void* A, long long lda, int amode, int a_f32,
                           const double* X, long long ldx, double beta,
                           const double* Yin, long long ldyi, double* Y, long long ldy,
                           hipStream_t s);

// Triangular block solves by substitution.  T is nb x nb (nb <= 256, multiple of 16),
// X holds ncols right-hand sides and is overwritten with the solution.
enum TrsmKind : int {
    TRSM_L_UNIT = 0,    // L X = B, L unit lower (row-major T), X nb x ncols row-major
    TRSM_U = 1,         // U X = B, U upper
    TRSM_UT = 2,        // U^T X = B (T holds U)
    TRSM_LT_UNIT = 3,   // L^T X = B (T holds unit lower L)
    TRSM_RIGHT_U = 4    // X U = B with X ncols x nb row-major (rows are the right-hand sides)
};
hipError_t launch_trsm(int kind, int t_f32, int x_f32, const void* T, long long ldt, int nb, void* X,
                       long long ldx, int ncols, hipStream_t s);
// Circulant multipliers by FFT (n a power of two, 4 <= n <= 16384).  tw: e^{-2 pi i k / (n/2)},
// k < n/4; wp: e^{-2 pi i f / n}, f <= n/2; spec: the DFT of the n parameters, f <= n/2.
bool circ_size_ok(long long n);
hipError_t launch_circ_spectrum(int n, const double* c, const double2* tw, const double2* wp, double2* spec,
                                hipStream_t s);
// y_b = alpha * op(x_b) + beta * yin_b for nvec vectors b: element t of vector b is at
// x[b * bx + t * sx] (likewise y, yin); op = correlation with c (conj = 1: x^T G, G^T x)
// or convolution (conj = 0: G x).  y is FP32 when y_f32.  Optional fused reductions (device
// slots for atomic_max_nonneg, already initialized): xsum_max <- max_b sum_t |x_b[t]| (the
// infinity norm of A when the vectors are its rows), ymax <- max |y| as stored.
hipError_t launch_circ_apply(int n, int nvec, int conj, const double* x, long long sx, long long bx, const double2* spec,
                             const double2* tw, const double2* wp, double alpha, double beta, const double* yin,
                             long long syi, long long byi, void* y, int y_f32, long long sy, long long by,
                             hipStream_t s, unsigned long long* xsum_max = nullptr,
                             unsigned long long* ymax = nullptr);
// The two block solves of an elimination step in one launch: A12 <- L11^{-1} A12
// (nb x m) and A21 <- A21 U11^{-1} (m x nb), with L11 \ U11 the factored diagonal
// block D.  nb in {64, 128, 256}; f32: D, A12 and A21 are FP32 (arithmetic in FP64).
// rcp (FP64 only): the pivots applied as reciprocals taken once per 16-row tile instead of
// a division per row (faster; each result may differ in its last bit).
hipError_t launch_panel_trsm(int f32, int rcp, const void* D, long long ldd, int nb, void* A12, void* A21,
                             long long ldx, int m, hipStream_t s);
// Whole triangular solve T X = B (T = the n_pad x n_pad factor as in launch_trsm's kinds,
// except TRSM_RIGHT_U) for 1..4 right-hand sides, one launch per bs-row block.
// The same solve (T = the n_pad x n_pad factor, kinds as above except TRSM_RIGHT_U) in one
// launch of n_pad / 64 workgroups chained through the solved values published in pub
// (n_pad * nr 8-byte words of device memory) and a ticket in sync (2 words of device memory;
// word 1 is a sticky error word the caller clears once and checks).
hipError_t launch_trsv_chain(int kind, int t_f32, const void* T, long long ldt, int n_pad, double* X, long long ldx,
                             int nr, unsigned* sync, unsigned long long* pub, hipStream_t s);
// The same chained solve for 1..64 right-hand sides (MFMA block products; pub holds n_pad * 64
// 8-byte words).
hipError_t launch_trsm_chain(int kind, int t_f32, const void* T, long long ldt, int n_pad, double* X, long long ldx,
                             int ncols, unsigned* sync, unsigned long long* pub, hipStream_t s);
hipError_t launch_trsv_full(int kind, int t_f32, const void* T, long long ldt, int n_pad, int bs, double* X,
                            long long ldx, int nr, hipStream_t s);
hipError_t launch_convert_f64_f32(const double* src, long long lds, float* dst, long long ldd, int rows, int cols,
                                  hipStream_t s);
hipError_t launch_scale2d(double alpha, double* X, long long ldx, int rows, int cols, hipStream_t s);
// y (M x nrhs) = alpha T X + beta yin for the Toeplitz T(i, k) = p[i - k + t - 1] (K columns, nrhs <= 4),
// partial sums over K slices through part (part_cap doubles, at least M * nrhs), then their sum
hipError_t launch_toep_gemv(int M, int K, int nrhs, double alpha, const double* p, long long t, const double* X,
                            long long ldx, double beta, const double* Yin, long long ldyi, double* Y, long long ldy,
                            double* part, long long part_cap, hipStream_t s);
hipError_t launch_convert_f32_f64(const float* src, long long lds, double* dst, long long ldd, int rows, int cols,
                                  hipStream_t s);

// Vector kernels of GMRES and of the 1-norm estimator (krylov.hip).
// out[i] = V_i . w for i < j1, V_i = V + i * ldv (n entries each); fixed reduction order.
hipError_t launch_multidot(int n, int j1, const double* V, long long ldv, const double* w, double* out,
                           hipStream_t s);
// k columns at once (k <= 64), V_i = V + i * vs and W n x k row-major blocks:
// out[i * k + c] = V_i(:, c) . W(:, c) for i < j1; part: device scratch of part_cap doubles,
// at least (j1 + 1024) * k (fixed-order reduction over row chunks)
hipError_t launch_bdot(int n, int k, int j1, const double* V, long long vs, const double* W, double* out,
                       double* part, long long part_cap, hipStream_t s);
// W = beta W + sign sum_{i < j1} V_i diag(h[i * k .. i * k + k - 1])
hipError_t launch_bcomb(int n, int k, int j1, const double* V, long long vs, const double* h, double sign, double beta,
                        double* W, hipStream_t s);
// X(:, c) *= f[c] for an n x k block (f: device, k doubles); f[c] = 0 sets the column to zero
hipError_t launch_colscale(int n, int k, const double* f, double* X, hipStream_t s);
// out[0] = ||y||_1, out[1] = 1 if sign(y) == xi elementwise (sign(0) = +1) else 0; then xi = sign(y).
hipError_t launch_cest_sign(int n, const double* y, double* xi, double* out, hipStream_t s);
// out[0] = ||z||_inf, out[1] = first index attaining it, out[2] = z[jlast] (or -1 when jlast < 0).
hipError_t launch_cest_argmax(int n, const double* z, int jlast, double* out, hipStream_t s);
// x_i = (-1)^i (1 + i / (n - 1)), i < n.
hipError_t launch_cest_alt(int n, double* x, hipStream_t s);
// x = e_j (length n).
hipError_t launch_unit_vector(int n, int j, double* x, hipStream_t s);
// ||A||_1 = max_j sum_i |A(i, j)| of an n x n FP64 matrix into *out (bits of a non-negative
// double, atomicMax: zero it first); part: scratch of part_cap doubles (at least n).
hipError_t launch_col_abs_sum_max(const double* A, long long lda, int n, double* part, long long part_cap,
                                  unsigned long long* out, hipStream_t s);
