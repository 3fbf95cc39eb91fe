// Diagonal-block factorization of the blocked elimination.
//
// GENP (section 1.1) on an nb x nb diagonal block, in place, with no pivot
// search and no row exchanges: right-looking, 16 columns at a time, each step
// replacing the trailing block by its Schur complement (Fact 2.1).  Pivot
// statistics and the first failing pivot (non-finite, or
// |u_kk| <= pivot_tol * max|C|) are recorded.
#include "common.h"

#include <math.h>

#include <algorithm>

namespace {

constexpr int PW = 16;    // inner panel width
constexpr int MAXNB = 256;
constexpr int TB = 8;     // 16x16 tiles per batch of the trailing update

__device__ inline double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One workgroup of 256 threads (one wave per SIMD), FP64 arithmetic for either
// storage type.  For each 16-column panel:
//  1. wave 0 factors the panel alone, with no barrier: lane l holds rows
//     l, l+64, l+128, l+192 of it in registers and the pivot row is broadcast
//     with readlane;
//  2. one thread per column solves the 16 rows of U right of the panel with the
//     unit lower 16 x 16 block (column sweep);
//  3. the trailing block takes the rank-16 Schur update (Fact 2.1) on the
//     matrix cores: 16 x 16 tiles, 8 per wave per batch of loads, operands from
//     LDS (the panel below the diagonal and the new rows of U).
template <typename T>
__global__ void __launch_bounds__(256)
diag_lu_kernel(T* __restrict__ D, long long ldd, int nb, int nvalid, long long col0,
               const double* __restrict__ maxc, double pivot_tol, PanelStats* __restrict__ st) {
    __shared__ double Ls[MAXNB][PW + 1];        // panel rows kb.. (row r - kb), 16 columns
    __shared__ double Rs[PW][MAXNB - PW + 1];   // rows kb..kb+15 of U right of the panel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double tol_abs = pivot_tol * maxc[0];
    double s_min = INFINITY, s_max = 0.0;
    long long s_bad = -1;
    for (int kb = 0; kb < nb; kb += PW) {
        const int rows = nb - kb;
        if (wave == 0) {
            double p[4][PW];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int r = s * 64 + lane;
#pragma unroll
                for (int c = 0; c < PW; ++c) p[s][c] = (r < rows) ? (double)D[(long long)(kb + r) * ldd + kb + c] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                // pivot row c is row c of the panel: lane c, slot 0 (its first c entries are L)
                double prow[PW];
#pragma unroll
                for (int t = 0; t < PW; ++t) prow[t] = (t >= c) ? readlane_d(p[0][t], c) : 0.0;
                const double piv = prow[c];
                if (lane == 0 && kb + c < nvalid) {
                    const double a = fabs(piv);
                    if (s_bad < 0 && (!isfinite(a) || a <= tol_abs)) s_bad = col0 + kb + c;
                    if (s_bad < 0) {
                        s_min = fmin(s_min, a);
                        s_max = fmax(s_max, a);
                    }
                }
                const double rp = 1.0 / piv;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int r = s * 64 + lane;
                    if (r > c && r < rows) {
                        const double l = p[s][c] * rp;
                        p[s][c] = l;
#pragma unroll
                        for (int t = 0; t < PW; ++t)
                            if (t > c) p[s][t] = fma(-l, prow[t], p[s][t]);
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int r = s * 64 + lane;
                if (r < rows) {
#pragma unroll
                    for (int c = 0; c < PW; ++c) {
                        D[(long long)(kb + r) * ldd + kb + c] = (T)p[s][c];
                        Ls[r][c] = p[s][c];
                    }
                }
            }
        }
        __syncthreads();
        const int ncols = rows - PW;
        if (ncols > 0) {
            if (tid < ncols) {
                // rows kb..kb+15, column kb+16+tid: x <- L11^{-1} x (unit lower, column sweep)
                double x[PW];
#pragma unroll
                for (int i = 0; i < PW; ++i) x[i] = (double)D[(long long)(kb + i) * ldd + kb + PW + tid];
#pragma unroll
                for (int t = 0; t < PW; ++t)
#pragma unroll
                    for (int i = 0; i < PW; ++i)
                        if (i > t) x[i] = fma(-Ls[i][t], x[t], x[i]);
#pragma unroll
                for (int i = 0; i < PW; ++i) {
                    D[(long long)(kb + i) * ldd + kb + PW + tid] = (T)x[i];
                    Rs[i][tid] = x[i];
                }
            }
            __syncthreads();
            // trailing block rows/cols kb+16..: 16 x 16 tiles, A22 -= L21 U12 on the matrix cores.
            // f64 16x16x4 layout: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
            // accumulator lane l, element r -> (row l/16 + 4r, col l%16).
            const int nt = ncols / PW, ntiles = nt * nt;
            const int lr = lane & 15, lq = lane >> 4;
            for (int t0 = wave * TB; t0 < ntiles; t0 += 4 * TB) {
                f64x4 acc[TB];
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    const int tile = t0 + b;
                    const int ti = tile / nt, tj = tile % nt;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = kb + PW + ti * 16 + lq + 4 * r, col = kb + PW + tj * 16 + lr;
                        acc[b][r] = (tile < ntiles) ? (double)D[(long long)row * ldd + col] : 0.0;
                    }
                }
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    const int tile = t0 + b;
                    if (tile < ntiles) {
                        const int ti = tile / nt, tj = tile % nt;
#pragma unroll
                        for (int kk = 0; kk < PW; kk += 4) {
                            const double a = Ls[PW + ti * 16 + lr][kk + lq];
                            const double bb = Rs[kk + lq][tj * 16 + lr];
                            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, bb, acc[b], 0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    const int tile = t0 + b;
                    if (tile < ntiles) {
                        const int ti = tile / nt, tj = tile % nt;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = kb + PW + ti * 16 + lq + 4 * r, col = kb + PW + tj * 16 + lr;
                            D[(long long)row * ldd + col] = (T)acc[b][r];
                        }
                    }
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

// GENP of a 128 x 128 FP64 block held in LDS for the whole elimination (the same steps as
// diag_lu_kernel, 16 columns at a time: panel by wave 0 with readlane broadcasts, the 16 rows of
// U right of the panel by a column sweep, the rank-16 Schur update on the matrix cores), so
// the only global traffic is one read and one write of the block.  merge: combine the pivot
// statistics with those already in *st (the second diagonal quadrant of a 256 block).
constexpr int Q = 128;
__global__ void __launch_bounds__(256)
lu128_lds_kernel(double* __restrict__ D, long long ldd, int nvalid, long long col0, const double* __restrict__ maxc,
                 double pivot_tol, PanelStats* __restrict__ st, int merge) {
    __shared__ double L[Q][Q + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double tol_abs = pivot_tol * maxc[0];
    // load: 64 elements per thread, rows coalesced
#pragma unroll 8
    for (int e = tid; e < Q * Q; e += 256) L[e / Q][e % Q] = D[(long long)(e / Q) * ldd + e % Q];
    __syncthreads();
    double s_min = INFINITY, s_max = 0.0;
    long long s_bad = -1;
    for (int kb = 0; kb < Q; kb += PW) {
        const int rows = Q - kb;
        if (wave == 0) {
            double p[2][PW];
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int r = sl * 64 + lane;
#pragma unroll
                for (int c = 0; c < PW; ++c) p[sl][c] = (r < rows) ? L[kb + r][kb + c] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                double prow[PW];
#pragma unroll
                for (int t = 0; t < PW; ++t) prow[t] = (t >= c) ? readlane_d(p[0][t], c) : 0.0;
                const double piv = prow[c];
                if (lane == 0 && kb + c < nvalid) {
                    const double a = fabs(piv);
                    if (s_bad < 0 && (!isfinite(a) || a <= tol_abs)) s_bad = col0 + kb + c;
                    if (s_bad < 0) {
                        s_min = fmin(s_min, a);
                        s_max = fmax(s_max, a);
                    }
                }
                const double rp = 1.0 / piv;
#pragma unroll
                for (int sl = 0; sl < 2; ++sl) {
                    const int r = sl * 64 + lane;
                    if (r > c && r < rows) {
                        const double l = p[sl][c] * rp;
                        p[sl][c] = l;
#pragma unroll
                        for (int t = 0; t < PW; ++t)
                            if (t > c) p[sl][t] = fma(-l, prow[t], p[sl][t]);
                    }
                }
            }
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int r = sl * 64 + lane;
                if (r < rows)
#pragma unroll
                    for (int c = 0; c < PW; ++c) L[kb + r][kb + c] = p[sl][c];
            }
        }
        __syncthreads();
        const int ncols = rows - PW;
        if (ncols > 0) {
            if (tid < ncols) {
                // rows kb..kb+15 of U right of the panel: x <- L11^{-1} x (unit lower, column sweep)
                const int col = kb + PW + tid;
                double x[PW];
#pragma unroll
                for (int i = 0; i < PW; ++i) x[i] = L[kb + i][col];
#pragma unroll
                for (int t = 0; t < PW; ++t)
#pragma unroll
                    for (int i = 0; i < PW; ++i)
                        if (i > t) x[i] = fma(-L[kb + i][kb + t], x[t], x[i]);
#pragma unroll
                for (int i = 0; i < PW; ++i) L[kb + i][col] = x[i];
            }
            __syncthreads();
            // trailing block: 16 x 16 tiles, A22 -= L21 U12 on the matrix cores, operands and
            // accumulators in LDS (accumulator lane l, element r: row l/16 + 4r, column l%16)
            const int nt = ncols / PW, ntiles = nt * nt;
            const int lr = lane & 15, lq = lane >> 4;
            for (int tile = wave; tile < ntiles; tile += 4) {
                const int r0 = kb + PW + (tile / nt) * 16, c0 = kb + PW + (tile % nt) * 16;
                f64x4 acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = L[r0 + lq + 4 * r][c0 + lr];
#pragma unroll
                for (int kk = 0; kk < PW; kk += 4)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-L[r0 + lr][kb + kk + lq], L[kb + kk + lq][c0 + lr], acc,
                                                               0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) L[r0 + lq + 4 * r][c0 + lr] = acc[r];
            }
        }
        __syncthreads();
    }
#pragma unroll 8
    for (int e = tid; e < Q * Q; e += 256) D[(long long)(e / Q) * ldd + e % Q] = L[e / Q][e % Q];
    if (tid == 0) {
        if (merge) {
            const PanelStats o = *st;
            if (o.first_bad >= 0) s_bad = o.first_bad;
            s_min = fmin(s_min, o.min_abs);
            s_max = fmax(s_max, o.max_abs);
        }
        st->min_abs = s_min;
        st->max_abs = s_max;
        st->first_bad = s_bad;
    }
}

}  // namespace

hipError_t launch_diag_lu(int prec, void* Dblk, long long ldd, int nb, int nvalid, long long col0,
                          const double* maxc, double pivot_tol, PanelStats* st, hipStream_t s) {
    if (nb <= 0 || nb > MAXNB || nb % PW) return hipErrorInvalidValue;   // nb: multiple of 16, <= 256
    if (prec == PREC_F64)
        hipLaunchKernelGGL(diag_lu_kernel<double>, dim3(1), dim3(256), 0, s, (double*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st);
    else
        hipLaunchKernelGGL(diag_lu_kernel<float>, dim3(1), dim3(256), 0, s, (float*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st);
    return hipGetLastError();
}

// A 256 x 256 FP64 diagonal block as four steps on one stream: GENP of the leading 128 block in
// LDS; U12 = L11^{-1} A12 and L21 = A21 U11^{-1} on the matrix cores (the panel solves of the
// blocked elimination with nb = 128); A22 -= L21 U12; GENP of A22 in LDS.  This is block
// Gaussian elimination (Theorem 2.2) on the block itself, with the same pivots.
hipError_t launch_diag_lu_split(void* Dblk, long long ldd, int nvalid, long long col0, const double* maxc,
                                double pivot_tol, PanelStats* st, hipStream_t s) {
    double* D = (double*)Dblk;
    hipLaunchKernelGGL(lu128_lds_kernel, dim3(1), dim3(256), 0, s, D, ldd, std::min(nvalid, 128), col0, maxc,
                       pivot_tol, st, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_panel_trsm(0, D, ldd, 128, D + 128, D + 128 * ldd, ldd, 128, s);
    if (e != hipSuccess) return e;
    GemmF64Args g{};
    g.M = g.N = g.K = 128;
    g.A = D + 128 * ldd;
    g.lda = ldd;
    g.amode = OP_N;
    g.B = D + 128;
    g.ldb = ldd;
    g.bmode = OP_N;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.Cin = D + 128 * ldd + 128;
    g.ldci = ldd;
    g.D = D + 128 * ldd + 128;
    g.ldd = ldd;
    g.ksplit = 1;
    e = launch_gemm_f64(g, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lu128_lds_kernel, dim3(1), dim3(256), 0, s, D + 128 * ldd + 128, ldd, std::max(0, nvalid - 128),
                       col0 + 128, maxc, pivot_tol, st, 1);
    return hipGetLastError();
}
