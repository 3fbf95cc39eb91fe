// Vector kernels of the refinement and diagnostics around the GENP solve:
//  - the Gram-Schmidt products of FP64 GMRES (dots of a vector with a block of basis
//    vectors, all on the device, so that one Arnoldi step needs one host round trip);
//  - the sign / maximum / alternating-vector steps of the Hager-Higham 1-norm estimator
//    (Higham, ACM TOMS 14 (1988), Algorithm 4.1), run on the device with the host keeping
//    only the scalar decisions;
//  - the 1-norm of A (maximum column sum), the infinity norm of A^T for the backward error
//    of the transposed (adjoint) system.
// Every reduction has a fixed order, so repeated calls give identical bits.
#include "common.h"

#include <math.h>

#include <algorithm>

namespace {

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of a 256-thread block's values (fixed order: waves, then the four wave sums).
__device__ inline double block_sum256(double v, double* red) {
    v = wsum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// out[i] = V_i . w for i < j1 (V_i = V + i * ldv, length n); one block per i, four partial
// sums per thread, 16-byte loads when both vectors allow them.
__global__ void __launch_bounds__(256)
multidot_kernel(int n, const double* __restrict__ V, long long ldv, const double* __restrict__ w,
                double* __restrict__ out) {
    __shared__ double red[4];
    const double* v = V + (long long)blockIdx.x * ldv;
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    const bool vec = ((uintptr_t)v % 16 == 0) && ((uintptr_t)w % 16 == 0);
    int i = 0;
    if (vec) {
        const double2* v2 = reinterpret_cast<const double2*>(v);
        const double2* w2 = reinterpret_cast<const double2*>(w);
        const int n2 = n >> 1;
        for (int k = t; k < n2; k += 256) {
            const double2 a = v2[k], b = w2[k];
            s0 = fma(a.x, b.x, s0);
            s1 = fma(a.y, b.y, s1);
        }
        i = 2 * n2;
    }
    for (int k = i + t; k < n; k += 256) s0 = fma(v[k], w[k], s0);
    const double s = block_sum256(s0 + s1, red);
    if (t == 0) out[blockIdx.x] = s;
}

// Hager-Higham sign step on y (length n): out[0] = ||y||_1, out[1] = 1 if sign(y) equals the
// stored sign vector xi (elementwise) else 0; then xi = sign(y) with sign(0) = +1.
__global__ void __launch_bounds__(1024)
cest_sign_kernel(int n, const double* __restrict__ y, double* __restrict__ xi, double* __restrict__ out) {
    __shared__ double red[16];
    __shared__ int diff[16];
    const int t = threadIdx.x;
    double s = 0.0;
    int d = 0;
    for (int i = t; i < n; i += 1024) {
        const double v = y[i];
        s += fabs(v);
        const double sg = (v >= 0.0) ? 1.0 : -1.0;
        d |= (sg != xi[i]);
        xi[i] = sg;
    }
    s = wsum(s);
    // any lane differs -> the wave differs
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d |= __shfl_xor(d, o, 64);
    const int w = t >> 6;
    if ((t & 63) == 0) {
        red[w] = s;
        diff[w] = d;
    }
    __syncthreads();
    if (t == 0) {
        double a = 0.0;
        int dd = 0;
        for (int q = 0; q < 16; ++q) {
            a += red[q];
            dd |= diff[q];
        }
        out[0] = a;
        out[1] = dd ? 0.0 : 1.0;
    }
}

// out[0] = ||z||_inf, out[1] = the first index attaining it (as a double),
// out[2] = z[jlast] (signed) for the previous index jlast, or -1 when jlast < 0.
__global__ void __launch_bounds__(1024)
cest_argmax_kernel(int n, const double* __restrict__ z, int jlast, double* __restrict__ out) {
    __shared__ double vm[16];
    __shared__ int im[16];
    const int t = threadIdx.x;
    double m = -1.0;
    int idx = 0x7fffffff;
    for (int i = t; i < n; i += 1024) {
        const double a = fabs(z[i]);
        if (a > m) {   // strictly greater: each thread keeps its first maximum
            m = a;
            idx = i;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double m2 = __shfl_xor(m, o, 64);
        const int i2 = __shfl_xor(idx, o, 64);
        if (m2 > m || (m2 == m && i2 < idx)) {
            m = m2;
            idx = i2;
        }
    }
    const int w = t >> 6;
    if ((t & 63) == 0) {
        vm[w] = m;
        im[w] = idx;
    }
    __syncthreads();
    if (t == 0) {
        double bm = vm[0];
        int bi = im[0];
        for (int q = 1; q < 16; ++q)
            if (vm[q] > bm || (vm[q] == bm && im[q] < bi)) {
                bm = vm[q];
                bi = im[q];
            }
        out[0] = bm;
        out[1] = (double)bi;
        out[2] = (jlast >= 0 && jlast < n) ? z[jlast] : -1.0;
    }
}

// x_i = (-1)^i (1 + i / (n - 1)), i = 0 .. n-1 (x_0 = 1 when n = 1).
__global__ void cest_alt_kernel(int n, double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m = (n > 1) ? 1.0 + (double)i / (double)(n - 1) : 1.0;
    x[i] = (i & 1) ? -m : m;
}

// x = 0 except x[j] = 1 (length n)
__global__ void unit_vector_kernel(int n, int j, double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (i == j) ? 1.0 : 0.0;
}

// Column sums of |A| over row slices: part[q * n + j] = sum_{i in slice q} |A(i, j)|.
__global__ void __launch_bounds__(256)
col_abs_sum_part_kernel(int n, const double* __restrict__ A, long long lda, int slice, double* __restrict__ part) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int i0 = blockIdx.y * slice, i1 = min(n, i0 + slice);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = i0;
    for (; i + 3 < i1; i += 4) {
        s0 += fabs(A[(long long)i * lda + j]);
        s1 += fabs(A[(long long)(i + 1) * lda + j]);
        s2 += fabs(A[(long long)(i + 2) * lda + j]);
        s3 += fabs(A[(long long)(i + 3) * lda + j]);
    }
    for (; i < i1; ++i) s0 += fabs(A[(long long)i * lda + j]);
    part[(long long)blockIdx.y * n + j] = (s0 + s1) + (s2 + s3);
}

// max_j sum_q part[q * n + j] -> one double (bits, atomicMax; order independent)
__global__ void __launch_bounds__(256)
col_abs_sum_max_kernel(int n, int P, const double* __restrict__ part, unsigned long long* out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (j < n)
        for (int q = 0; q < P; ++q) s += part[(long long)q * n + j];
    // NaN-propagating wave maximum, one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(s, o, 64);
        s = (w > s || isnan(w)) ? w : s;
    }
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, s);
}

// Many columns at once (the k right-hand sides of one refinement step, k <= 64): V_i and W
// are n x k row-major blocks, V_i = V + i * vs.  out[i * k + c] = sum_t V_i[t][c] W[t][c] in
// two passes with a fixed order: workgroup (p, i) sums the rows of chunk p (lane group c of
// 64, four row groups, two partial sums each) into part[(i P + p) k + c], then the P chunk
// sums are added in order p = 0 .. P-1.  Chunks spread a step's few basis blocks over the
// whole GPU.
__global__ void __launch_bounds__(256)
bdot_part_kernel(int n, int k, int rc, const double* __restrict__ V, long long vs, const double* __restrict__ W,
                 double* __restrict__ part) {
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int p = blockIdx.x, P = gridDim.x, i = blockIdx.y;
    const double* v = V + (long long)i * vs;
    const int r0 = p * rc, r1 = min(n, r0 + rc);
    double s0 = 0.0, s1 = 0.0;
    if (c < k) {
        int t = r0 + rg;
        for (; t + 4 < r1; t += 8) {
            s0 = fma(v[(long long)t * k + c], W[(long long)t * k + c], s0);
            s1 = fma(v[(long long)(t + 4) * k + c], W[(long long)(t + 4) * k + c], s1);
        }
        for (; t < r1; t += 4) s0 = fma(v[(long long)t * k + c], W[(long long)t * k + c], s0);
    }
    red[rg][c] = s0 + s1;
    __syncthreads();
    if (rg == 0 && c < k) part[((long long)i * P + p) * k + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

__global__ void bdot_sum_kernel(int k, int P, int j1, const double* __restrict__ part, double* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= j1 * k) return;
    const int i = e / k, c = e % k;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += part[((long long)i * P + p) * k + c];
    out[e] = s;
}

// W[t][c] = beta W[t][c] + sign sum_{i < j1} V_i[t][c] h[i * k + c] (beta = 0: W not read)
__global__ void __launch_bounds__(256)
bcomb_kernel(int n, int k, int j1, const double* __restrict__ V, long long vs, const double* __restrict__ h,
             double sign, double beta, double* __restrict__ W) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * k) return;
    const int c = (int)(e % k);
    double s = 0.0;
    for (int i = 0; i < j1; ++i) s = fma(V[(long long)i * vs + e], h[(long long)i * k + c], s);
    W[e] = (beta != 0.0 ? beta * W[e] : 0.0) + sign * s;
}

// X[t][c] *= f[c] (column scaling of an n x k block); f[c] = 0 clears the column, NaN included
__global__ void colscale_kernel(int n, int k, const double* __restrict__ f, double* __restrict__ X) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * k) return;
    const double fc = f[e % k];
    X[e] = fc != 0.0 ? X[e] * fc : 0.0;
}

}  // namespace

int bdot_chunks(int n, int j1) {
    // about 1024 workgroups in all, chunks of 256 rows at least
    const int by_rows = std::max(1, (n + 255) / 256);
    return std::max(1, std::min(by_rows, (1024 + j1 - 1) / j1));
}

hipError_t launch_bdot(int n, int k, int j1, const double* V, long long vs, const double* W, double* out,
                       double* part, long long part_cap, hipStream_t s) {
    if (j1 <= 0) return hipSuccess;
    if (k < 1 || k > 64 || n <= 0) return hipErrorInvalidValue;
    const int P = bdot_chunks(n, j1);
    if ((long long)j1 * P * k > part_cap) return hipErrorInvalidValue;
    const int rc = (n + P - 1) / P;
    hipLaunchKernelGGL(bdot_part_kernel, dim3(P, j1), dim3(256), 0, s, n, k, rc, V, vs, W, part);
    hipLaunchKernelGGL(bdot_sum_kernel, dim3((j1 * k + 255) / 256), dim3(256), 0, s, k, P, j1, part, out);
    return hipGetLastError();
}

hipError_t launch_bcomb(int n, int k, int j1, const double* V, long long vs, const double* h, double sign, double beta,
                        double* W, hipStream_t s) {
    const long long tot = (long long)n * k;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(bcomb_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, j1, V, vs, h, sign,
                       beta, W);
    return hipGetLastError();
}

hipError_t launch_colscale(int n, int k, const double* f, double* X, hipStream_t s) {
    const long long tot = (long long)n * k;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(colscale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, f, X);
    return hipGetLastError();
}

hipError_t launch_multidot(int n, int j1, const double* V, long long ldv, const double* w, double* out,
                           hipStream_t s) {
    if (j1 <= 0) return hipSuccess;
    hipLaunchKernelGGL(multidot_kernel, dim3(j1), dim3(256), 0, s, n, V, ldv, w, out);
    return hipGetLastError();
}

hipError_t launch_cest_sign(int n, const double* y, double* xi, double* out, hipStream_t s) {
    hipLaunchKernelGGL(cest_sign_kernel, dim3(1), dim3(1024), 0, s, n, y, xi, out);
    return hipGetLastError();
}

hipError_t launch_cest_argmax(int n, const double* z, int jlast, double* out, hipStream_t s) {
    hipLaunchKernelGGL(cest_argmax_kernel, dim3(1), dim3(1024), 0, s, n, z, jlast, out);
    return hipGetLastError();
}

hipError_t launch_cest_alt(int n, double* x, hipStream_t s) {
    hipLaunchKernelGGL(cest_alt_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, x);
    return hipGetLastError();
}

hipError_t launch_unit_vector(int n, int j, double* x, hipStream_t s) {
    hipLaunchKernelGGL(unit_vector_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, j, x);
    return hipGetLastError();
}

hipError_t launch_col_abs_sum_max(const double* A, long long lda, int n, double* part, long long part_cap,
                                  unsigned long long* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long cols = (n + 255) / 256;
    long long P = std::max<long long>(1, 2048 / cols);
    P = std::min<long long>(P, std::max(1, n / 64));
    P = std::min<long long>(P, part_cap / n);
    if (P < 1) return hipErrorInvalidValue;
    const int slice = (int)((n + P - 1) / P);
    P = (n + slice - 1) / slice;
    hipLaunchKernelGGL(col_abs_sum_part_kernel, dim3((unsigned)cols, (unsigned)P), dim3(256), 0, s, n, A, lda, slice,
                       part);
    hipLaunchKernelGGL(col_abs_sum_max_kernel, dim3((unsigned)cols), dim3(256), 0, s, n, (int)P, part, out);
    return hipGetLastError();
}
