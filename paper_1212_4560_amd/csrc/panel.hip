// Diagonal-block factorization of the blocked elimination.
//
// GENP (section 1.1) on an nb x nb diagonal block, in place, with no pivot
// search and no row exchanges: right-looking, 32 columns at a time.  Each
// 32-column panel is factored in LDS with one thread per row (the pivot row is
// read by every thread as an LDS broadcast); the 32-row block of U to its right
// is a unit-lower substitution (one thread per column); the rest of the block
// takes the rank-32 Schur update (Fact 2.1).  Pivot statistics and the first
// failing pivot (non-finite, or |u_kk| <= pivot_tol * max|C|) are recorded.
#include "common.h"

#include <math.h>

namespace {

constexpr int PW = 32;    // inner panel width
constexpr int MAXNB = 256;

template <typename T>
__global__ void __launch_bounds__(512)
diag_lu_kernel(T* __restrict__ D, long long ldd, int nb, int nvalid, long long col0,
               const double* __restrict__ maxc, double pivot_tol, PanelStats* __restrict__ st) {
    __shared__ T P[MAXNB][PW + 1];
    __shared__ T R[PW][MAXNB - PW + 1];
    __shared__ double s_min, s_max;
    __shared__ long long s_bad;
    const int tid = threadIdx.x;
    const double tol_abs = pivot_tol * maxc[0];
    if (tid == 0) {
        s_min = INFINITY;
        s_max = 0.0;
        s_bad = -1;
    }
    for (int kb = 0; kb < nb; kb += PW) {
        const int rows = nb - kb;
        for (int e = tid; e < rows * PW; e += blockDim.x) {
            const int r = e / PW, c = e % PW;
            P[r][c] = D[(long long)(kb + r) * ldd + kb + c];
        }
        __syncthreads();
        for (int k = 0; k < PW; ++k) {
            const T piv = P[k][k];
            if (tid == 0 && kb + k < nvalid) {
                const double a = fabs((double)piv);
                if (s_bad < 0 && (!isfinite(a) || a <= tol_abs)) s_bad = col0 + kb + k;
                if (s_bad < 0) {
                    s_min = fmin(s_min, a);
                    s_max = fmax(s_max, a);
                }
            }
            if (tid > k && tid < rows) {
                const T l = P[tid][k] / piv;
                P[tid][k] = l;
#pragma unroll 8
                for (int c = k + 1; c < PW; ++c) P[tid][c] = fma(-l, P[k][c], P[tid][c]);
            }
            __syncthreads();
        }
        for (int e = tid; e < rows * PW; e += blockDim.x) {
            const int r = e / PW, c = e % PW;
            D[(long long)(kb + r) * ldd + kb + c] = P[r][c];
        }
        const int ncols = nb - kb - PW;
        if (ncols > 0) {
            // rows kb..kb+31 right of the panel: x <- L_kk^{-1} x (unit lower)
            if (tid < ncols) {
                T x[PW];
#pragma unroll
                for (int i = 0; i < PW; ++i) x[i] = D[(long long)(kb + i) * ldd + kb + PW + tid];
#pragma unroll
                for (int i = 1; i < PW; ++i) {
                    T v = x[i];
#pragma unroll
                    for (int t = 0; t < i; ++t) v = fma(-P[i][t], x[t], v);
                    x[i] = v;
                }
#pragma unroll
                for (int i = 0; i < PW; ++i) {
                    D[(long long)(kb + i) * ldd + kb + PW + tid] = x[i];
                    R[i][tid] = x[i];
                }
            }
            __syncthreads();
            // trailing rows/cols: A22 -= L21 * U12 (rank 32)
            const int trows = rows - PW;
            const int j = tid & 255, rg = tid >> 8;
            if (j < ncols) {
                T rj[PW];
#pragma unroll
                for (int t = 0; t < PW; ++t) rj[t] = R[t][j];
                for (int r = rg; r < trows; r += 2) {
                    T* dp = D + (long long)(kb + PW + r) * ldd + kb + PW + j;
                    T acc = *dp;
#pragma unroll
                    for (int t = 0; t < PW; ++t) acc = fma(-P[PW + r][t], rj[t], acc);
                    *dp = acc;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        st->min_abs = s_min;
        st->max_abs = s_max;
        st->first_bad = s_bad;
    }
}

}  // namespace

hipError_t launch_diag_lu(int prec, void* Dblk, long long ldd, int nb, int nvalid, long long col0,
                          const double* maxc, double pivot_tol, PanelStats* st, hipStream_t s) {
    if (nb <= 0 || nb > MAXNB || nb % PW) return hipErrorInvalidValue;
    if (prec == PREC_F64)
        hipLaunchKernelGGL(diag_lu_kernel<double>, dim3(1), dim3(512), 0, s, (double*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st);
    else
        hipLaunchKernelGGL(diag_lu_kernel<float>, dim3(1), dim3(512), 0, s, (float*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st);
    return hipGetLastError();
}
