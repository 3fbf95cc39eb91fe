// Memory-bound kernels of the GENP path: matrix-vector products for the
// substitutions, the recovery X = G Y and the residual B - A X (few right-hand
// sides), norms for the
// backward error, and small copy/fill helpers.
//
// Row-mode matrix-vector products give one wave per row so every load of the
// matrix is a coalesced 512-byte run; transposed operands use one thread per
// row and read down the columns, which is again coalesced across the wave.
// Reductions that feed a maximum use atomicMax on the bit pattern of a
// non-negative double: the result is exact and order independent.
#include "common.h"

#include <math.h>

#include <algorithm>

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    // NaN-propagating maximum (fmax would drop a NaN)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = (w > v || isnan(w)) ? w : v;
    }
    return v;
}

template <typename T>
__global__ void pad_identity_kernel(T* C, long long ldc, int n, int n_pad) {
    // rows >= n: whole row; rows < n: columns >= n
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long padcols = n_pad - n;
    const long long top = (long long)n * padcols;
    if (idx < top) {
        const int i = (int)(idx / padcols), j = n + (int)(idx % padcols);
        C[(long long)i * ldc + j] = T(0);
        return;
    }
    const long long e = idx - top;
    if (e >= padcols * (long long)n_pad) return;
    const int i = n + (int)(e / n_pad), j = (int)(e % n_pad);
    C[(long long)i * ldc + j] = (i == j) ? T(1) : T(0);
}

__device__ inline double nanmax(double m, double a) { return (a > m || isnan(a)) ? a : m; }

// max |X(i, j)| (upper: j >= i only): one wave per row at a time, lanes across the
// row (coalesced), four independent partial maxima per lane, one atomic per wave.
template <typename T>
__global__ void max_abs_kernel(const T* __restrict__ X, long long ldx, int rows, int cols, int upper,
                               unsigned long long* out) {
    const int lane = threadIdx.x & 63;
    const int wave = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int nw = (int)(((long long)gridDim.x * blockDim.x) >> 6);
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (int i = wave; i < rows; i += nw) {
        const T* r = X + (long long)i * ldx;
        int j = (upper ? i : 0) + lane;
        for (; j + 192 < cols; j += 256) {
            m0 = nanmax(m0, fabs((double)r[j]));
            m1 = nanmax(m1, fabs((double)r[j + 64]));
            m2 = nanmax(m2, fabs((double)r[j + 128]));
            m3 = nanmax(m3, fabs((double)r[j + 192]));
        }
        for (; j < cols; j += 64) m0 = nanmax(m0, fabs((double)r[j]));
    }
    double m = nanmax(nanmax(m0, m1), nanmax(m2, m3));
    m = wave_max(m);
    if (lane == 0) atomic_max_nonneg(out, m);
}

// max_i sum_j |A(i, j)| (the infinity norm): one wave per row, one atomic per row.
// VEC: rows 16-byte aligned, pairs of entries loaded as one 16-byte load (checked by the launcher).
template <bool VEC>
__global__ void row_abs_sum_max_kernel(const double* __restrict__ A, long long lda, int n,
                                       unsigned long long* out) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n) return;
    const double* r = A + (long long)row * lda;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = lane;
    if constexpr (VEC) {
        const double2* r2 = reinterpret_cast<const double2*>(r);
        const int n2 = n >> 1;
        int k2 = lane;
        for (; k2 + 448 < n2; k2 += 512) {
            double2 a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = r2[k2 + 64 * u];
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                s0 += fabs(a[u].x);
                s1 += fabs(a[u].y);
                s2 += fabs(a[u + 1].x);
                s3 += fabs(a[u + 1].y);
            }
        }
        for (; k2 < n2; k2 += 64) {
            s0 += fabs(r2[k2].x);
            s1 += fabs(r2[k2].y);
        }
        k = (n & 1) ? ((lane == 0) ? n - 1 : n) : n;
    }
    for (; k + 192 < n; k += 256) {
        s0 += fabs(r[k]);
        s1 += fabs(r[k + 64]);
        s2 += fabs(r[k + 128]);
        s3 += fabs(r[k + 192]);
    }
    for (; k < n; k += 64) s0 += fabs(r[k]);
    const double s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) atomic_max_nonneg(out, s);
}

// out[c] = max_i |X(i, c)| for cols <= 256 columns: threads stride over rows, the
// block combines its partial maxima in LDS, one atomic per column per block.
__global__ void col_abs_max_kernel(const double* __restrict__ X, long long ldx, int rows, int cols,
                                   unsigned long long* out) {
    __shared__ double red[256];
    const int per = blockDim.x / cols;
    const int c = threadIdx.x % cols;
    const int rr = threadIdx.x / cols;
    double m = 0.0;
    if (rr < per) {
        for (int i = blockIdx.x * per + rr; i < rows; i += gridDim.x * per) m = nanmax(m, fabs(X[(long long)i * ldx + c]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    if ((int)threadIdx.x < cols) {
        double v = 0.0;
        for (int t = 0; t < per; ++t) v = nanmax(v, red[t * cols + threadIdx.x]);
        atomic_max_nonneg(out + threadIdx.x, v);
    }
}

template <typename T>
__global__ void copy_work_kernel(const T* __restrict__ C, long long ldc, int n, double* __restrict__ out,
                                 long long ldo) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    out[(long long)i * ldo + j] = (double)C[(long long)i * ldc + j];
}

__global__ void copy2d_kernel(const double* __restrict__ s, long long lds, double* __restrict__ d,
                              long long ldd, int rows, int cols) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    d[(long long)i * ldd + j] = s[(long long)i * lds + j];
}

__global__ void convert_kernel(const double* __restrict__ s, long long lds, float* __restrict__ d,
                               long long ldd, int rows, int cols) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    d[(long long)i * ldd + j] = (float)s[(long long)i * lds + j];
}

__global__ void widen_kernel(const float* __restrict__ s, long long lds, double* __restrict__ d,
                             long long ldd, int rows, int cols) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    d[(long long)i * ldd + j] = (double)s[(long long)i * lds + j];
}

__global__ void axpy2d_kernel(double alpha, const double* __restrict__ x, long long ldx,
                              double* __restrict__ y, long long ldy, int rows, int cols) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    y[(long long)i * ldy + j] += alpha * x[(long long)i * ldx + j];
}

__global__ void scale2d_kernel(double alpha, double* x, long long ldx, int rows, int cols) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    x[(long long)i * ldx + j] *= alpha;
}

__global__ void fill2d_kernel(double v, double* __restrict__ x, long long ldx, int rows, int cols) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    x[(long long)i * ldx + j] = v;
}

// Row mode: one wave per output row, NR right-hand sides (NR <= 4).
template <int NR, int AMODE, typename TA, bool VEC = false>
__global__ void __launch_bounds__(256)
gemv_row_kernel(int M, int K, double alpha, const TA* __restrict__ A, long long lda,
                const double* __restrict__ X, long long ldx, double beta, const double* Yin,
                long long ldyi, double* Y, long long ldy) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= M) return;
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    const TA* ar = (AMODE == OP_TOEP) ? A + (long long)row + lda - 1 : A + (long long)row * lda;
    int k = lane;
    if constexpr (VEC) {
        // pairs of entries as one 16-byte load, eight loads in flight per lane; the row
        // start is 16-byte aligned (checked by the launcher)
        const double2* ar2 = reinterpret_cast<const double2*>(ar);
        const int K2 = K >> 1;
        int k2 = lane;
        for (; k2 + 448 < K2; k2 += 512) {
            double2 a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = ar2[k2 + 64 * u];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const long long kk = 2LL * (k2 + 64 * u);
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    acc[c] = fma(a[u].x, X[kk * ldx + c], acc[c]);
                    acc[c] = fma(a[u].y, X[(kk + 1) * ldx + c], acc[c]);
                }
            }
        }
        for (; k2 < K2; k2 += 64) {
            const double2 a = ar2[k2];
            const long long kk = 2LL * k2;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                acc[c] = fma(a.x, X[kk * ldx + c], acc[c]);
                acc[c] = fma(a.y, X[(kk + 1) * ldx + c], acc[c]);
            }
        }
        k = (K & 1) ? ((lane == 0) ? K - 1 : K) : K;   // the odd last entry, if any, on lane 0
    }
    for (; k + 192 < K; k += 256) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            a[u] = (AMODE == OP_TOEP) ? (double)ar[-(long long)(k + 64 * u)] : (double)ar[k + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = fma(a[u], X[(long long)(k + 64 * u) * ldx + c], acc[c]);
    }
    for (; k < K; k += 64) {
        const double a = (AMODE == OP_TOEP) ? (double)ar[-(long long)k] : (double)ar[k];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = fma(a, X[(long long)k * ldx + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = wave_sum(acc[c]);
    if (lane < NR) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < NR; ++c)
            if (c == lane) v = acc[c];
        v *= alpha;
        if (beta != 0.0) v += beta * Yin[(long long)row * ldyi + lane];
        Y[(long long)row * ldy + lane] = v;
    }
}

// Column mode for transposed operands: A(i, k) = A[k * lda + i], one thread per row.
template <int NR, typename TA>
__global__ void __launch_bounds__(256)
gemv_col_kernel(int M, int K, double alpha, const TA* __restrict__ A, long long lda,
                const double* __restrict__ X, long long ldx, double beta, const double* Yin,
                long long ldyi, double* Y, long long ldy) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= M) return;
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    int k = 0;
    for (; k + 3 < K; k += 4) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = (double)A[(long long)(k + u) * lda + row];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = fma(a[u], X[(long long)(k + u) * ldx + c], acc[c]);
    }
    for (; k < K; ++k) {
        const double a = (double)A[(long long)k * lda + row];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = fma(a, X[(long long)k * ldx + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        double v = alpha * acc[c];
        if (beta != 0.0) v += beta * Yin[(long long)row * ldyi + c];
        Y[(long long)row * ldy + c] = v;
    }
}

template <int NR, typename TA>
hipError_t gemv_dispatch_t(int M, int K, double alpha, const TA* A, long long lda, int amode,
                           const double* X, long long ldx, double beta, const double* Yin,
                           long long ldyi, double* Y, long long ldy, hipStream_t s) {
    if (amode == OP_T) {
        hipLaunchKernelGGL((gemv_col_kernel<NR, TA>), dim3((M + 255) / 256), dim3(256), 0, s, M, K,
                           alpha, A, lda, X, ldx, beta, Yin, ldyi, Y, ldy);
    } else if (amode == OP_N) {
        const bool vec = std::is_same<TA, double>::value && ((uintptr_t)A % 16 == 0) && (lda % 2 == 0);
        if (vec)
            hipLaunchKernelGGL((gemv_row_kernel<NR, OP_N, TA, true>), dim3((M + 3) / 4), dim3(256), 0, s, M, K,
                               alpha, A, lda, X, ldx, beta, Yin, ldyi, Y, ldy);
        else
            hipLaunchKernelGGL((gemv_row_kernel<NR, OP_N, TA>), dim3((M + 3) / 4), dim3(256), 0, s, M, K,
                               alpha, A, lda, X, ldx, beta, Yin, ldyi, Y, ldy);
    } else {
        hipLaunchKernelGGL((gemv_row_kernel<NR, OP_TOEP, TA>), dim3((M + 3) / 4), dim3(256), 0, s, M,
                           K, alpha, A, lda, X, ldx, beta, Yin, ldyi, Y, ldy);
    }
    return hipGetLastError();
}

template <typename TA>
hipError_t gemv_dispatch(int M, int K, int nr, double alpha, const TA* A, long long lda, int amode,
                         const double* X, long long ldx, double beta, const double* Yin,
                         long long ldyi, double* Y, long long ldy, hipStream_t s) {
    switch (nr) {
        case 1: return gemv_dispatch_t<1>(M, K, alpha, A, lda, amode, X, ldx, beta, Yin, ldyi, Y, ldy, s);
        case 2: return gemv_dispatch_t<2>(M, K, alpha, A, lda, amode, X, ldx, beta, Yin, ldyi, Y, ldy, s);
        case 3: return gemv_dispatch_t<3>(M, K, alpha, A, lda, amode, X, ldx, beta, Yin, ldyi, Y, ldy, s);
        case 4: return gemv_dispatch_t<4>(M, K, alpha, A, lda, amode, X, ldx, beta, Yin, ldyi, Y, ldy, s);
        default: return hipErrorInvalidValue;
    }
}

// Transposed products y = alpha A^T X + beta yin with A stored K x M (y_j = sum_k A[k][j] X[k]),
// in two deterministic passes: partial sums over row slices, then their sum.
// Wide form (M >= 64): one thread per output j, blockIdx.y = row slice.
template <int NR, typename TA>
__global__ void __launch_bounds__(256)
gemv_tw_part_kernel(int M, int K, int slice, const TA* __restrict__ A, long long lda, const double* __restrict__ X,
                    long long ldx, double* __restrict__ part) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= M) return;
    const int k0 = blockIdx.y * slice, k1 = min(K, k0 + slice);
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    int k = k0;
    for (; k + 3 < k1; k += 4) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = (double)A[(long long)(k + u) * lda + j];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = fma(a[u], X[(long long)(k + u) * ldx + c], acc[c]);
    }
    for (; k < k1; ++k) {
        const double a = (double)A[(long long)k * lda + j];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = fma(a, X[(long long)k * ldx + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) part[((long long)blockIdx.y * M + j) * NR + c] = acc[c];
}

// Narrow form (M <= 4 outputs, one right-hand side): the block's threads stride over the rows
// of its slice, then reduce in LDS.
__global__ void __launch_bounds__(256)
gemv_tn_part_kernel(int M, int K, int slice, const double* __restrict__ A, long long lda,
                    const double* __restrict__ x, long long ldx, double* __restrict__ part) {
    __shared__ double red[4][256];
    const int t = threadIdx.x;
    const int k0 = blockIdx.x * slice, k1 = min(K, k0 + slice);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = k0 + t; k < k1; k += 256) {
        const double xv = x[(long long)k * ldx];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < M) acc[j] = fma(A[(long long)k * lda + j], xv, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[j][t] = acc[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int j = 0; j < 4; ++j) red[j][t] += red[j][t + h];
        __syncthreads();
    }
    if (t < M) part[(long long)blockIdx.x * M + t] = red[t][0];
}

// y_j = alpha sum_p part[p][j] + beta yin_j (fixed order over p)
__global__ void gemv_t_reduce_kernel(int M, int NR, int P, const double* __restrict__ part, double alpha,
                                     double beta, const double* Yin, long long ldyi, double* Y, long long ldy) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * NR) return;
    const int j = e / NR, c = e % NR;
    double s = 0.0;
    for (int q = 0; q < P; ++q) s += part[((long long)q * M + j) * NR + c];
    double v = alpha * s;
    if (beta != 0.0) v = fma(beta, Yin[(long long)j * ldyi + c], v);
    Y[(long long)j * ldy + c] = v;
}

// Toeplitz matrix-vector products y = T x, T(i, k) = p[i - k + t - 1] (M x K, 1..4 columns of x),
// with partial sums over K slices: workgroup (row block b, slice q) stages the p window of its
// 1024 rows and 256 columns (1279 values) and the 256 x-values in LDS, and thread r keeps rows
// 4 r .. 4 r + 3 with their four p values in registers: moving to the next column shifts the
// window by one entry, so each column costs one LDS read of p, one of x and four FMAs.
constexpr int TG_ROWS = 1024, TG_KC = 256;
template <int NR>
__global__ void __launch_bounds__(256)
toep_gemv_part_kernel(int M, int K, const double* __restrict__ p, long long t, const double* __restrict__ X,
                      long long ldx, int slice, double* __restrict__ part) {
    __shared__ double pw[TG_ROWS + TG_KC];
    __shared__ double xs[TG_KC][NR];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * TG_ROWS;          // first row of the block
    const int kbeg = blockIdx.y * slice, kend = min(K, kbeg + slice);
    const int ib = 4 * tid;                        // this thread's first row within the block
    double acc[4][NR];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[r][c] = 0.0;
    for (int k0 = kbeg; k0 < kend; k0 += TG_KC) {
        const int kc = min(TG_KC, kend - k0);
        __syncthreads();
        // pw[u] = T(i0 + u - (TG_KC - 1), k0) = p[i0 + u - (TG_KC - 1) - k0 + t - 1], 0 outside p
        for (int u = tid; u < TG_ROWS + TG_KC - 1; u += 256) {
            const long long idx = (long long)i0 + u - (TG_KC - 1) - k0 + t - 1;
            pw[u] = (idx >= 0 && idx < 2 * t - 1) ? p[idx] : 0.0;
        }
        for (int e = tid; e < TG_KC * NR; e += 256) {
            const int kk = e / NR, c = e % NR;
            xs[kk][c] = (kk < kc) ? X[(long long)(k0 + kk) * ldx + c] : 0.0;
        }
        __syncthreads();
        // T(i0 + ib + r, k0 + kk) = pw[ib + r - kk + TG_KC - 1]
        double w0 = pw[ib + TG_KC - 1], w1 = pw[ib + TG_KC], w2 = pw[ib + TG_KC + 1], w3 = pw[ib + TG_KC + 2];
        for (int kk = 0; kk < kc; ++kk) {
            double xv[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) xv[c] = xs[kk][c];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                acc[0][c] = fma(w0, xv[c], acc[0][c]);
                acc[1][c] = fma(w1, xv[c], acc[1][c]);
                acc[2][c] = fma(w2, xv[c], acc[2][c]);
                acc[3][c] = fma(w3, xv[c], acc[3][c]);
            }
            // next column: the window moves down one entry of p
            w3 = w2;
            w2 = w1;
            w1 = w0;
            if (kk + 1 < kc) w0 = pw[ib + TG_KC - 2 - kk];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + ib + r;
        if (i < M)
#pragma unroll
            for (int c = 0; c < NR; ++c) part[((long long)blockIdx.y * M + i) * NR + c] = acc[r][c];
    }
}

// Y = alpha (X - s a b^T) + beta Yin with s = factor / dot[0] read from device memory (the
// Householder multiplier I - 2 u v^T / (v^T u) applied as a rank-1 update).  One block per row.
template <typename TO>
__global__ void __launch_bounds__(256)
rank1_kernel(int M, int N, double alpha, const double* X, long long ldx, const double* __restrict__ a,
             const double* __restrict__ b, const double* __restrict__ dot, double factor, double beta,
             const double* Yin, long long ldyi, TO* Y, long long ldy) {
    const int i = blockIdx.x;
    if (i >= M) return;
    const double sa = factor / dot[0] * a[i];
    const double* xr = X + (long long)i * ldx;
    const double* yr = (beta != 0.0) ? Yin + (long long)i * ldyi : nullptr;
    TO* outr = Y + (long long)i * ldy;
    for (int j = threadIdx.x; j < N; j += 256) {
        double v = alpha * fma(-sa, b[j], xr[j]);
        if (yr) v = fma(beta, yr[j], v);
        outr[j] = (TO)v;
    }
}

// out = (v^T u, u^T u, v^T v), one block, fixed reduction order
__global__ void __launch_bounds__(1024) dot3_kernel(int n, const double* __restrict__ u, const double* __restrict__ v,
                                                    double* __restrict__ out) {
    __shared__ double red[3][1024];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = t; i < n; i += 1024) {
        const double ui = u[i], vi = v[i];
        a = fma(vi, ui, a);
        b = fma(ui, ui, b);
        c = fma(vi, vi, c);
    }
    red[0][t] = a;
    red[1][t] = b;
    red[2][t] = c;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] += red[1][t + h];
            red[2][t] += red[2][t + h];
        }
        __syncthreads();
    }
    if (t < 3) out[t] = red[t][0];
}

// FP64 -> FP32 (round to nearest even), then optionally FP32 -> BF16 (round to nearest even on
// the upper 16 bits, NaN kept quiet), the result held in an FP32 word.
__device__ inline float round_lp(double x, int bf16) {
    float f = (float)x;
    if (!bf16) return f;
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return __uint_as_float(u | 0x00400000u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

__global__ void convert_pad_kernel(const double* __restrict__ A, long long lda, int n, int n_pad,
                                   float* __restrict__ out, long long ldo, int bf16) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n_pad * n_pad) return;
    const int i = (int)(e / n_pad), j = (int)(e % n_pad);
    out[(long long)i * ldo + j] = (i < n && j < n) ? round_lp(A[(long long)i * lda + j], bf16) : 0.f;
}

__global__ void convert_toep_kernel(const double* __restrict__ p, int n, int n_pad, float* __restrict__ out,
                                    int bf16) {
    const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= 2LL * n_pad - 1) return;
    const long long t = u - (n_pad - n);
    out[u] = (t >= 0 && t < 2LL * n - 1) ? round_lp(p[t], bf16) : 0.f;
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_pad_identity(int prec, void* C, long long ldc, int n, int n_pad, hipStream_t s) {
    if (n_pad <= n) return hipSuccess;
    const long long tot = (long long)n * (n_pad - n) + (long long)(n_pad - n) * n_pad;
    if (prec == PREC_F64)
        hipLaunchKernelGGL(pad_identity_kernel<double>, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                           (double*)C, ldc, n, n_pad);
    else
        hipLaunchKernelGGL(pad_identity_kernel<float>, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                           (float*)C, ldc, n, n_pad);
    return hipGetLastError();
}

hipError_t launch_max_abs(int prec, const void* X, long long ldx, int rows, int cols, int upper,
                          unsigned long long* out, hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<long long>((rows + 3) / 4, 2048);
    if (prec == PREC_F64)
        hipLaunchKernelGGL(max_abs_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)X, ldx,
                           rows, cols, upper, out);
    else
        hipLaunchKernelGGL(max_abs_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)X, ldx, rows,
                           cols, upper, out);
    return hipGetLastError();
}

hipError_t launch_row_abs_sum_max(const double* A, long long lda, int n, unsigned long long* out,
                                  hipStream_t s) {
    if (((uintptr_t)A % 16 == 0) && (lda % 2 == 0))
        hipLaunchKernelGGL(row_abs_sum_max_kernel<true>, dim3((n + 3) / 4), dim3(256), 0, s, A, lda, n, out);
    else
        hipLaunchKernelGGL(row_abs_sum_max_kernel<false>, dim3((n + 3) / 4), dim3(256), 0, s, A, lda, n, out);
    return hipGetLastError();
}

hipError_t launch_col_abs_max(const double* X, long long ldx, int rows, int cols,
                              unsigned long long* out, hipStream_t s) {
    if (cols <= 0 || cols > 256 || rows <= 0) return cols > 256 ? hipErrorInvalidValue : hipSuccess;
    const int per = 256 / cols;
    const unsigned g = (unsigned)std::min<long long>((rows + per - 1) / per, 256);
    hipLaunchKernelGGL(col_abs_max_kernel, dim3(g), dim3(256), 0, s, X, ldx, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_copy_work(int prec, const void* C, long long ldc, int n, double* out, long long ldo,
                            hipStream_t s) {
    const long long tot = (long long)n * n;
    if (prec == PREC_F64)
        hipLaunchKernelGGL(copy_work_kernel<double>, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                           (const double*)C, ldc, n, out, ldo);
    else
        hipLaunchKernelGGL(copy_work_kernel<float>, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                           (const float*)C, ldc, n, out, ldo);
    return hipGetLastError();
}

hipError_t launch_copy2d(const double* src, long long lds, double* dst, long long ldd, int rows, int cols,
                         hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy2d_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, src, lds, dst, ldd,
                       rows, cols);
    return hipGetLastError();
}

hipError_t launch_axpy2d(double alpha, const double* X, long long ldx, double* Y, long long ldy, int rows,
                         int cols, hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy2d_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, alpha, X, ldx, Y, ldy,
                       rows, cols);
    return hipGetLastError();
}

hipError_t launch_fill2d(double v, double* X, long long ldx, int rows, int cols, hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill2d_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, v, X, ldx, rows, cols);
    return hipGetLastError();
}

hipError_t launch_gemv_f64(int M, int K, int nrhs, double alpha, const void* A, long long lda, int amode,
                           int a_f32, const double* X, long long ldx, double beta, const double* Yin,
                           long long ldyi, double* Y, long long ldy, hipStream_t s) {
    if (M <= 0 || nrhs <= 0) return hipSuccess;
    if (a_f32)
        return gemv_dispatch<float>(M, K, nrhs, alpha, (const float*)A, lda, amode, X, ldx, beta, Yin,
                                    ldyi, Y, ldy, s);
    return gemv_dispatch<double>(M, K, nrhs, alpha, (const double*)A, lda, amode, X, ldx, beta, Yin, ldyi,
                                 Y, ldy, s);
}

hipError_t launch_convert_f64_f32(const double* src, long long lds, float* dst, long long ldd, int rows, int cols,
                                  hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(convert_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_scale2d(double alpha, double* X, long long ldx, int rows, int cols, hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale2d_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, alpha, X, ldx, rows, cols);
    return hipGetLastError();
}

hipError_t launch_gemv_t_f64(int M, int K, int nrhs, double alpha, const void* A, long long lda, int a_f32,
                             const double* X, long long ldx, double beta, const double* Yin, long long ldyi,
                             double* Y, long long ldy, double* part, long long part_cap, hipStream_t s) {
    if (M <= 0 || nrhs <= 0) return hipSuccess;
    if (nrhs > 4 || K <= 0) return hipErrorInvalidValue;
    const bool narrow = M <= 4 && nrhs == 1 && !a_f32;
    // slices: enough blocks to fill the GPU, at least 16 rows each, partials within part_cap
    const long long cols = narrow ? 1 : (M + 255) / 256;
    long long P = std::max<long long>(1, 2048 / cols);
    P = std::min<long long>(P, std::max(1, K / 16));
    P = std::min<long long>(P, part_cap / ((long long)M * nrhs));
    if (P < 1) return hipErrorInvalidValue;
    const int slice = (int)((K + P - 1) / P);
    P = (K + slice - 1) / slice;
    if (narrow) {
        hipLaunchKernelGGL(gemv_tn_part_kernel, dim3((unsigned)P), dim3(256), 0, s, M, K, slice, (const double*)A,
                           lda, X, ldx, part);
    } else {
#define GENP_GTW(NR)                                                                                          \
    if (a_f32)                                                                                                \
        hipLaunchKernelGGL((gemv_tw_part_kernel<NR, float>), dim3((unsigned)cols, (unsigned)P), dim3(256), 0, \
                           s, M, K, slice, (const float*)A, lda, X, ldx, part);                               \
    else                                                                                                      \
        hipLaunchKernelGGL((gemv_tw_part_kernel<NR, double>), dim3((unsigned)cols, (unsigned)P), dim3(256), 0, \
                           s, M, K, slice, (const double*)A, lda, X, ldx, part)
        switch (nrhs) {
            case 1: GENP_GTW(1); break;
            case 2: GENP_GTW(2); break;
            case 3: GENP_GTW(3); break;
            default: GENP_GTW(4); break;
        }
#undef GENP_GTW
    }
    const int tot = M * nrhs;
    hipLaunchKernelGGL(gemv_t_reduce_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, M, nrhs, (int)P, part, alpha,
                       beta, Yin, ldyi, Y, ldy);
    return hipGetLastError();
}

hipError_t launch_rank1(int M, int N, double alpha, const double* X, long long ldx, const double* a, const double* b,
                        const double* dot, double factor, double beta, const double* Yin, long long ldyi, void* Y,
                        int y_f32, long long ldy, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (y_f32)
        hipLaunchKernelGGL(rank1_kernel<float>, dim3(M), dim3(256), 0, s, M, N, alpha, X, ldx, a, b, dot, factor, beta,
                           Yin, ldyi, (float*)Y, ldy);
    else
        hipLaunchKernelGGL(rank1_kernel<double>, dim3(M), dim3(256), 0, s, M, N, alpha, X, ldx, a, b, dot, factor,
                           beta, Yin, ldyi, (double*)Y, ldy);
    return hipGetLastError();
}

hipError_t launch_dot3(int n, const double* u, const double* v, double* out, hipStream_t s) {
    hipLaunchKernelGGL(dot3_kernel, dim3(1), dim3(1024), 0, s, n, u, v, out);
    return hipGetLastError();
}

hipError_t launch_convert_pad(const double* A, long long lda, int n, int n_pad, float* out, long long ldo, int bf16,
                              hipStream_t s) {
    const long long tot = (long long)n_pad * n_pad;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(convert_pad_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, A, lda, n, n_pad, out, ldo,
                       bf16);
    return hipGetLastError();
}

hipError_t launch_convert_toep(const double* p, int n, int n_pad, float* out, int bf16, hipStream_t s) {
    const long long tot = 2LL * n_pad - 1;
    hipLaunchKernelGGL(convert_toep_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, p, n, n_pad, out, bf16);
    return hipGetLastError();
}

hipError_t launch_convert_f32_f64(const float* src, long long lds, double* dst, long long ldd, int rows, int cols,
                                  hipStream_t s) {
    const long long tot = (long long)rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_toep_gemv(int M, int K, int nrhs, double alpha, const double* p, long long t, const double* X,
                            long long ldx, double beta, const double* Yin, long long ldyi, double* Y, long long ldy,
                            double* part, long long part_cap, hipStream_t s) {
    if (M <= 0 || nrhs <= 0) return hipSuccess;
    if (nrhs > 4 || K <= 0) return hipErrorInvalidValue;
    const long long rb = (M + TG_ROWS - 1) / TG_ROWS;
    // K slices of whole 256-column chunks: about 512 workgroups, partials within part_cap
    long long P = std::max<long long>(1, 512 / rb);
    P = std::min<long long>(P, (K + TG_KC - 1) / TG_KC);
    P = std::min<long long>(P, part_cap / ((long long)M * nrhs));
    if (P < 1) return hipErrorInvalidValue;
    const int slice = (int)(((K + P - 1) / P + TG_KC - 1) / TG_KC * TG_KC);
    P = (K + slice - 1) / slice;
    const dim3 grid((unsigned)rb, (unsigned)P);
    switch (nrhs) {
        case 1: hipLaunchKernelGGL(toep_gemv_part_kernel<1>, grid, dim3(256), 0, s, M, K, p, t, X, ldx, slice, part); break;
        case 2: hipLaunchKernelGGL(toep_gemv_part_kernel<2>, grid, dim3(256), 0, s, M, K, p, t, X, ldx, slice, part); break;
        case 3: hipLaunchKernelGGL(toep_gemv_part_kernel<3>, grid, dim3(256), 0, s, M, K, p, t, X, ldx, slice, part); break;
        default: hipLaunchKernelGGL(toep_gemv_part_kernel<4>, grid, dim3(256), 0, s, M, K, p, t, X, ldx, slice, part); break;
    }
    const int tot = M * nrhs;
    hipLaunchKernelGGL(gemv_t_reduce_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, M, nrhs, (int)P, part, alpha,
                       beta, Yin, ldyi, Y, ldy);
    return hipGetLastError();
}
