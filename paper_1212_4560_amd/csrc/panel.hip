// Diagonal-block factorization of the blocked elimination.
//
// GENP (section 1.1) on an nb x nb diagonal block, in place, with no pivot
// search and no row exchanges: right-looking, 32 columns at a time, each step
// replacing the trailing block by its Schur complement (Fact 2.1).  Pivot
// statistics and the first failing pivot (non-finite, or
// |u_kk| <= pivot_tol * max|C|) are recorded.
#include "common.h"

#include <math.h>

namespace {

constexpr int PW = 32;    // inner panel width
constexpr int MAXNB = 256;

// One workgroup of 256 threads (one wave per SIMD) whose registers and LDS fit
// in the footprint of one Schur-GEMM workgroup, so the factorization of the
// next diagonal block can run beside the trailing update.
//
// For each 32-column panel: thread r keeps row r of the panel in registers;
// the pivot row is published through a double-buffered LDS row, so each
// elimination step costs one barrier.  The factored panel goes to LDS (XOR
// swizzled: the writes of a wave spread over the banks, the broadcast reads
// of the update hit one address).  Thread j then solves column j of the
// 32-row block of U to its right by a column sweep (critical path 31 FMAs)
// and applies the rank-32 Schur update to column j of the trailing block,
// 8 rows per batch of loads.
template <typename T>
__global__ void __launch_bounds__(256)
diag_lu_kernel(T* __restrict__ D, long long ldd, int nb, int nvalid, long long col0,
               const double* __restrict__ maxc, double pivot_tol, PanelStats* __restrict__ st) {
    __shared__ double P[MAXNB][PW];
    __shared__ double prow[2][PW];
    const int tid = threadIdx.x;
    const double tol_abs = pivot_tol * maxc[0];
    double s_min = INFINITY, s_max = 0.0;
    long long s_bad = -1;
    for (int kb = 0; kb < nb; kb += PW) {
        const int rows = nb - kb;
        // an opaque copy of the thread index: keeps the compiler from hoisting the
        // 32 per-step comparisons out of this loop (that exhausts the registers)
        int me = tid;
        asm volatile("" : "+v"(me));
        double p[PW];
#pragma unroll
        for (int c = 0; c < PW; ++c) p[c] = (me < rows) ? (double)D[(long long)(kb + me) * ldd + kb + c] : 0.0;
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < PW; ++c) prow[0][c] = p[c];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const double* pr = prow[k & 1];
            const double piv = pr[k];
            if (tid == 0 && kb + k < nvalid) {
                const double a = fabs((double)piv);
                if (s_bad < 0 && (!isfinite(a) || a <= tol_abs)) s_bad = col0 + kb + k;
                if (s_bad < 0) {
                    s_min = fmin(s_min, a);
                    s_max = fmax(s_max, a);
                }
            }
            if (me > k && me < rows) {
                const double l = p[k] / piv;
                p[k] = l;
#pragma unroll
                for (int c = k + 1; c < PW; ++c) p[c] = fma(-l, pr[c], p[c]);
            }
            if (k + 1 < PW && me == k + 1) {
#pragma unroll
                for (int c = 0; c < PW; ++c) prow[(k + 1) & 1][c] = p[c];
            }
            __syncthreads();
        }
        if (me < rows) {
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                D[(long long)(kb + me) * ldd + kb + c] = (T)p[c];
                P[me][c ^ (me & 31)] = p[c];
            }
        }
        __syncthreads();
        const int ncols = nb - kb - PW;
        if (ncols > 0 && me < ncols) {
            const int j = me;
            // x <- L_kk^{-1} x for column j of the 32 rows right of the panel (unit lower)
            double x[PW];
#pragma unroll
            for (int i = 0; i < PW; ++i) x[i] = (double)D[(long long)(kb + i) * ldd + kb + PW + j];
#pragma unroll
            for (int t = 0; t < PW; ++t) {
#pragma unroll
                for (int i = t + 1; i < PW; ++i) x[i] = fma(-P[i][t ^ (i & 31)], x[t], x[i]);
                __builtin_amdgcn_sched_barrier(0);   // bound the loads the scheduler hoists
            }
#pragma unroll
            for (int i = 0; i < PW; ++i) D[(long long)(kb + i) * ldd + kb + PW + j] = (T)x[i];
            // trailing block, column j: A22 -= L21 * U12 (rank 32); rows in batches of 16
            // whose loads are issued one batch ahead
            const int trows = rows - PW;
            constexpr int RB = 16;
            double va[RB], vb[RB];
            auto ld_batch = [&](double* v, int r0) {
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const int r = r0 + u;
                    v[u] = (r < trows) ? (double)D[(long long)(kb + PW + r) * ldd + kb + PW + j] : 0.0;
                }
            };
            auto do_batch = [&](const double* v, int r0) {
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const int r = r0 + u;
                    if (r < trows) {
                        const int pr = PW + r;
                        double acc = v[u];
#pragma unroll
                        for (int t = 0; t < PW; ++t) acc = fma(-P[pr][t ^ (pr & 31)], x[t], acc);
                        D[(long long)(kb + PW + r) * ldd + kb + PW + j] = (T)acc;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            if (trows > 0) ld_batch(va, 0);
            for (int r0 = 0; r0 < trows; r0 += 2 * RB) {
                if (r0 + RB < trows) ld_batch(vb, r0 + RB);
                do_batch(va, r0);
                if (r0 + RB < trows) {
                    if (r0 + 2 * RB < trows) ld_batch(va, r0 + 2 * RB);
                    do_batch(vb, r0 + RB);
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
        hipLaunchKernelGGL(diag_lu_kernel<double>, dim3(1), dim3(256), 0, s, (double*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st);
    else
        hipLaunchKernelGGL(diag_lu_kernel<float>, dim3(1), dim3(256), 0, s, (float*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st);
    return hipGetLastError();
}
