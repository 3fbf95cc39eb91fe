// Triangular solves with an nb x nb triangular block by substitution (no
// explicit inverse): the two block solves of each elimination step,
// L21 = A21 U11^{-1} and U12 = L11^{-1} A12, and the diagonal-block solves of
// the substitutions Y = U^{-1} L^{-1} B and of the adjoint (U^T, L^T).
//
// Every case is written as a left solve T X = B with an nb x nb triangular T
// and the right-hand sides as the columns of X.  A workgroup owns CB columns of
// X, staged in LDS, and sweeps the rows of T: at step i every row r below
// (above) i subtracts T(r, i) / T(i, i) times the unscaled row i; the rows are
// divided by the diagonal at the end.  Columns of T are staged in LDS 16 at a
// time (coalesced loads: by rows of T, or down its columns when T is accessed
// transposed).  Right solves X U = B become U^T X^T = B^T with both operands
// accessed transposed.  Substitution keeps the backward error of the block
// solves at the level of the elimination itself; multiplying by a computed
// inverse would add a factor of the block's condition number.
#include "common.h"

namespace {

constexpr int CB = 16;   // right-hand sides per workgroup
constexpr int TC = 16;   // columns of T staged per LDS chunk
constexpr int MAXNB = 256;

template <bool LOWER, bool UNIT, bool TT, bool XT, typename TF, typename TX>
__global__ void __launch_bounds__(256)
trsm_left_kernel(const TF* __restrict__ T, long long ldt, int nb, TX* X, long long ldx, int ncols) {
    __shared__ double Xs[MAXNB][CB + 1];
    __shared__ double Ts[MAXNB][TC + 1];
    __shared__ double Tinv[TC];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * CB;
    const int cb = min(CB, ncols - c0);
    auto xat = [&](int r, int c) -> long long {
        return XT ? (long long)(c0 + c) * ldx + r : (long long)r * ldx + c0 + c;
    };
    auto tat = [&](int r, int c) -> long long {
        return TT ? (long long)c * ldt + r : (long long)r * ldt + c;
    };
    // stage X: for XT the rows of X^T are contiguous in r
    for (int e = tid; e < nb * CB; e += blockDim.x) {
        int r, c;
        if (XT) { c = e / nb; r = e % nb; }
        else { r = e / CB; c = e % CB; }
        Xs[r][c] = (c < cb) ? (double)X[xat(r, c)] : 0.0;
    }
    const int r = tid;
    for (int step = 0; step < nb; step += TC) {
        // chunk of T columns [i0, i0 + TC) in sweep order
        const int i0 = LOWER ? step : nb - step - TC;
        __syncthreads();
        for (int e = tid; e < nb * TC; e += blockDim.x) {
            int rr, t;
            if (TT) { t = e / nb; rr = e % nb; }
            else { rr = e / TC; t = e % TC; }
            Ts[rr][t] = (double)T[tat(rr, i0 + t)];
        }
        __syncthreads();
        if (!UNIT && tid < TC) Tinv[tid] = 1.0 / Ts[i0 + tid][tid];
        __syncthreads();
        for (int u = 0; u < TC; ++u) {
            const int t = LOWER ? u : TC - 1 - u;
            const int i = i0 + t;
            if (r < nb && (LOWER ? r > i : r < i)) {
                double m = Ts[r][t];
                if (!UNIT) m *= Tinv[t];
#pragma unroll
                for (int c = 0; c < CB; ++c) Xs[r][c] = fma(-m, Xs[i][c], Xs[r][c]);
            }
            __syncthreads();
        }
    }
    if (!UNIT) {
        // x_r = y_r / T(r, r)
        if (r < nb) {
            const double d = 1.0 / (double)T[tat(r, r)];
#pragma unroll
            for (int c = 0; c < CB; ++c) Xs[r][c] *= d;
        }
    }
    __syncthreads();
    for (int e = tid; e < nb * CB; e += blockDim.x) {
        int rr, c;
        if (XT) { c = e / nb; rr = e % nb; }
        else { rr = e / CB; c = e % CB; }
        if (c < cb) X[xat(rr, c)] = (TX)Xs[rr][c];
    }
}

template <bool LOWER, bool UNIT, bool TT, bool XT, typename TF, typename TX>
hipError_t go(const void* T, long long ldt, int nb, void* X, long long ldx, int ncols, hipStream_t s) {
    hipLaunchKernelGGL((trsm_left_kernel<LOWER, UNIT, TT, XT, TF, TX>), dim3((ncols + CB - 1) / CB), dim3(256), 0,
                       s, (const TF*)T, ldt, nb, (TX*)X, ldx, ncols);
    return hipGetLastError();
}

template <typename TF, typename TX>
hipError_t dispatch(int kind, const void* T, long long ldt, int nb, void* X, long long ldx, int ncols,
                    hipStream_t s) {
    switch (kind) {
        case TRSM_L_UNIT: return go<true, true, false, false, TF, TX>(T, ldt, nb, X, ldx, ncols, s);
        case TRSM_U: return go<false, false, false, false, TF, TX>(T, ldt, nb, X, ldx, ncols, s);
        case TRSM_UT: return go<true, false, true, false, TF, TX>(T, ldt, nb, X, ldx, ncols, s);
        case TRSM_LT_UNIT: return go<false, true, true, false, TF, TX>(T, ldt, nb, X, ldx, ncols, s);
        case TRSM_RIGHT_U: return go<true, false, true, true, TF, TX>(T, ldt, nb, X, ldx, ncols, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_trsm(int kind, int t_f32, int x_f32, const void* T, long long ldt, int nb, void* X,
                       long long ldx, int ncols, hipStream_t s) {
    if (nb <= 0 || nb > MAXNB || nb % TC) return hipErrorInvalidValue;
    if (ncols <= 0) return hipSuccess;
    if (!t_f32 && !x_f32) return dispatch<double, double>(kind, T, ldt, nb, X, ldx, ncols, s);
    if (t_f32 && !x_f32) return dispatch<float, double>(kind, T, ldt, nb, X, ldx, ncols, s);
    if (t_f32 && x_f32) return dispatch<float, float>(kind, T, ldt, nb, X, ldx, ncols, s);
    return hipErrorInvalidValue;
}
