// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4_f64), LDS double-buffered.
//
// D = alpha * op(A) op(B) + beta * Cin with M x N output, K reduction.  Used for
// the multiplier product C = A G (section 1.1; G dense or generated from its
// Toeplitz parameters, section 2.3), the triangular-block products
// L21 = A21 U11^{-1}, U12 = L11^{-1} A12 and the Schur complement update
// A22 -= L21 U12 (Fact 2.1) of the blocked elimination, and the skinny
// products of substitution, recovery and refinement (split-K).
//
// Each wave owns a 64 x 64 output tile = 4 x 4 MFMA tiles of 16 x 16.
// The 16x16x4 f64 MFMA takes a 16x4 A fragment (lane l: A[l%16][l/16]), a
// 4x16 B fragment (lane l: B[l/16][l%16]) and accumulates a 16x16 tile held
// as 4 doubles per lane (lane l, element r: row l/16 + 4r, column l%16 -- the
// f64 form interleaves rows, unlike the 4-consecutive-rows layout of the f32 forms).
#include "common.h"

namespace {

constexpr int BK = 16;

template <int MODE, typename TA>
__device__ inline double load_op(const TA* __restrict__ X, long long ld, int i, int k,
                                 int rows, int cols) {
    // element (i, k) of an operand of logical size rows x cols; 0 outside
    if (i >= rows || k >= cols) return 0.0;
    if (MODE == OP_N) return (double)X[(long long)i * ld + k];
    if (MODE == OP_T) return (double)X[(long long)k * ld + i];
    return 0.0;
}

template <int WM, int WN, int AMODE, int BMODE, bool AF32 = false>
__global__ void __launch_bounds__(64 * WM * WN, 2)
gemm_f64_kernel(GemmF64Args g) {
    constexpr int T = 64 * WM * WN;
    constexpr int BMt = 64 * WM, BNt = 64 * WN;
    constexpr int PADA = 1, PADB = 1;
    constexpr int LA = (AMODE == OP_TOEP) ? 1 : (BMt * BK) / T;           // per-thread loads
    constexpr int LB = (BMODE == OP_TOEP) ? 1 : (BNt * BK) / T;
    constexpr int PA = BMt + BK - 1, PB = BNt + BK - 1;                   // Toeplitz windows
    constexpr int LPA = (PA + T - 1) / T, LPB = (PB + T - 1) / T;

    __shared__ double As[2][(AMODE == OP_TOEP) ? 1 : BK][(AMODE == OP_TOEP) ? PA : BMt + PADA];
    __shared__ double Bs[2][(BMODE == OP_TOEP) ? 1 : BK][(BMODE == OP_TOEP) ? PB : BNt + PADB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    // which product this block computes (the optional second one follows the first's tiles)
    int bid = blockIdx.x;
    int gM = g.M, gN = g.N;
    const double* gA = g.A;
    const double* gB = g.B;
    const double* gCin = g.Cin;
    double* gD = g.D;
    {
        const int t1 = ((g.M + BMt - 1) / BMt) * ((g.N + BNt - 1) / BNt);
        if (g.M2 > 0 && bid >= t1) {
            bid -= t1;
            gM = g.M2;
            gN = g.N2;
            gA = g.A2;
            gB = g.B2;
            gCin = g.Cin2;
            gD = g.D2;
        }
    }
    const int ntm = (gM + BMt - 1) / BMt, ntn = (gN + BNt - 1) / BNt;
    const int total = ntm * ntn;
    const int pid = xcd_remap(bid, total);
    // tile order: groups of GROUP tile-rows, column-major inside a group.  With a generated
    // (Toeplitz) B the only streamed operand is A, so GROUP = 1 lets all concurrent blocks of
    // an XCD share each chunk of one A row-panel in its L2.
    const int GROUP = g.group_m > 0 ? g.group_m : 8;
    const int group = pid / (GROUP * ntn);
    const int first_m = group * GROUP;
    const int gsz = min(ntm - first_m, GROUP);
    const int tm = first_m + (pid % (GROUP * ntn)) % gsz;
    const int tn = (pid % (GROUP * ntn)) / gsz;
    const int m0 = tm * BMt, n0 = tn * BNt;

    // K range of this split
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        const int chunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
        kbeg = blockIdx.y * chunk;
        kend = min(g.K, kbeg + chunk);
    }
    const int nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;

    double ra[(AMODE == OP_TOEP) ? LPA : LA];
    double rb[(BMODE == OP_TOEP) ? LPB : LB];

    auto gload = [&](int k0) {
        if constexpr (AMODE == OP_TOEP) {
            // A(i, k) = p[i - k + t - 1]; window over i - k in [m0 - k0 - BK + 1, m0 + BMt - 1 - k0]
            const long long base = (long long)m0 - k0 - (BK - 1) + g.lda - 1;
#pragma unroll
            for (int r = 0; r < LPA; ++r) {
                const int e = tid + r * T;
                const long long idx = base + e;
                ra[r] = (e < PA && idx >= 0 && idx < 2 * g.lda - 1) ? gA[idx] : 0.0;
            }
        } else {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int e = tid + r * T;
                int i, k;
                if constexpr (AMODE == OP_N) { i = e / BK; k = e % BK; }
                else { k = e / BMt; i = e % BMt; }
                if constexpr (AF32) ra[r] = load_op<AMODE>((const float*)gA, g.lda, m0 + i, k0 + k, gM, kend);
                else ra[r] = load_op<AMODE>(gA, g.lda, m0 + i, k0 + k, gM, kend);
            }
        }
        if constexpr (BMODE == OP_TOEP) {
            // B(k, j) = p[k - j + t - 1]; window over k - j in [k0 - n0 - BNt + 1, k0 + BK - 1 - n0]
            const long long base = (long long)k0 - n0 - (BNt - 1) + g.ldb - 1;
#pragma unroll
            for (int r = 0; r < LPB; ++r) {
                const int e = tid + r * T;
                const long long idx = base + e;
                rb[r] = (e < PB && idx >= 0 && idx < 2 * g.ldb - 1) ? gB[idx] : 0.0;
            }
        } else {
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int e = tid + r * T;
                int k, j;
                if constexpr (BMODE == OP_N) { k = e / BNt; j = e % BNt; }
                else { j = e / BK; k = e % BK; }
                // B(k, j): OP_N -> B[k*ld + j]; OP_T -> B[j*ld + k]
                double v = 0.0;
                if (k0 + k < kend && n0 + j < gN)
                    v = (BMODE == OP_N) ? gB[(long long)(k0 + k) * g.ldb + n0 + j]
                                        : gB[(long long)(n0 + j) * g.ldb + k0 + k];
                rb[r] = v;
            }
        }
    };
    auto sstore = [&](int buf, int k0) {
        if constexpr (AMODE == OP_TOEP) {
#pragma unroll
            for (int r = 0; r < LPA; ++r) {
                const int e = tid + r * T;
                if (e < PA) As[buf][0][e] = ra[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int e = tid + r * T;
                int i, k;
                if constexpr (AMODE == OP_N) { i = e / BK; k = e % BK; }
                else { k = e / BMt; i = e % BMt; }
                As[buf][k][i] = ra[r];
            }
        }
        if constexpr (BMODE == OP_TOEP) {
#pragma unroll
            for (int r = 0; r < LPB; ++r) {
                const int e = tid + r * T;
                if (e < PB) Bs[buf][0][e] = rb[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int e = tid + r * T;
                int k, j;
                if constexpr (BMODE == OP_N) { k = e / BNt; j = e % BNt; }
                else { j = e / BK; k = e % BK; }
                Bs[buf][k][j] = rb[r];
            }
        }
        (void)k0;
    };

    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int lr = lane & 15, lq = lane >> 4;
    if (nk > 0) {
        gload(kbeg);
        sstore(0, kbeg);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            const int k0 = kbeg + kt * BK;
            if (kt + 1 < nk) gload(k0 + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                double af[4], bf[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) {
                    const int i = wm * 64 + mi * 16 + lr;
                    if constexpr (AMODE == OP_TOEP) af[mi] = As[cur][0][i - (kk + lq) + BK - 1];
                    else af[mi] = As[cur][kk + lq][i];
                }
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const int j = wn * 64 + ni * 16 + lr;
                    if constexpr (BMODE == OP_TOEP) bf[ni] = Bs[cur][0][(kk + lq) - j + BNt - 1];
                    else bf[ni] = Bs[cur][kk + lq][j];
                }
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
            }
            if (kt + 1 < nk) sstore(cur ^ 1, k0 + BK);
            __syncthreads();
        }
    }

    // epilogue.  Cin may alias D (in-place Schur update), so the compiler cannot move
    // a load above an earlier store: the loads of each 16-row strip are issued as a
    // batch before its stores.
    double* D = gD;
    const bool split = g.ksplit > 1;
    if (split) D += (long long)blockIdx.y * g.split_stride;
    const bool rd = !split && g.beta != 0.0;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        double cv[4][4];
        if (rd) {
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const int col = n0 + wn * 64 + ni * 16 + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * 64 + mi * 16 + lq + 4 * r;
                    cv[ni][r] = (row < gM && col < gN) ? gCin[(long long)row * g.ldci + col] : 0.0;
                }
            }
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int col = n0 + wn * 64 + ni * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + mi * 16 + lq + 4 * r;
                if (row < gM && col < gN) {
                    double v = g.alpha * acc[mi][ni][r];
                    if (rd) v = fma(g.beta, cv[ni][r], v);
                    D[(long long)row * g.ldd + col] = v;
                }
            }
        }
    }
}

// C = A G with G the Toeplitz matrix of parameters p (G(k, j) = p[k - j + K - 1]):
// the plain product on interior tiles only (M, N multiples of 128, K of 32), with no
// bounds checks and a 32-deep K chunk per barrier (the generated operand needs only a
// window of BNt + 31 parameters in LDS, so two blocks still fit on a CU).  Same tile
// layout and tile order as gemm_f64_kernel with one tile-row per group.
__global__ void __launch_bounds__(256, 2)
gemm_ag_toep_kernel(int M, int N, int K, const double* __restrict__ A, long long lda,
                    const double* __restrict__ p, double* __restrict__ D, long long ldd) {
    constexpr int BKT = 32, BMt = 128, BNt = 128, T = 256;
    constexpr int LA = BMt * BKT / T, PB = BNt + BKT - 1;
    __shared__ double As[2][BKT][BMt + 1];
    __shared__ double Bs[2][PB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int ntn = N / BNt, total = (M / BMt) * ntn;
    const int pid = xcd_remap(blockIdx.x, total);
    const int m0 = (pid / ntn) * BMt, n0 = (pid % ntn) * BNt;
    const int nk = K / BKT;
    const int lr = lane & 15, lq = lane >> 4;
    double ra[LA], rb;
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = tid + r * T;
            ra[r] = A[(long long)(m0 + e / BKT) * lda + k0 + e % BKT];
        }
        // window of p over k - j in [k0 - n0 - BNt + 1, k0 + BKT - 1 - n0]
        const long long idx = (long long)k0 - n0 - (BNt - 1) + K - 1 + tid;
        rb = (tid < PB && idx >= 0 && idx < 2LL * K - 1) ? p[idx] : 0.0;
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = tid + r * T;
            As[buf][e % BKT][e / BKT] = ra[r];
        }
        if (tid < PB) Bs[buf][tid] = rb;
    };
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    gload(0);
    sstore(0);
    __syncthreads();
    auto mfma_chunk = [&](int cur, int kk0, int kk1) {
#pragma unroll
        for (int kk = kk0; kk < kk1; kk += 4) {
            double af[4], bf[4];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) af[mi] = As[cur][kk + lq][wm * 64 + mi * 16 + lr];
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) bf[ni] = Bs[cur][(kk + lq) - (wn * 64 + ni * 16 + lr) + BNt - 1];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
        }
    };
    // Per chunk: issue the next chunk's loads, run half the MFMAs, write the next chunk to
    // LDS (its loads have had half a chunk to land), run the other half.  The wave runs
    // at raised priority through the MFMA stream and drops it before the barrier.
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BKT);
        __builtin_amdgcn_s_setprio(1);
        mfma_chunk(cur, 0, BKT / 2);
        if (kt + 1 < nk) sstore(cur ^ 1);
        mfma_chunk(cur, BKT / 2, BKT);
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                D[(long long)(m0 + wm * 64 + mi * 16 + lq + 4 * r) * ldd + n0 + wn * 64 + ni * 16 + lr] =
                    acc[mi][ni][r];
}

__global__ void splitk_reduce_kernel(int M, int N, int ks, const double* __restrict__ P, long long ldp,
                                     long long ss, double alpha, double beta, const double* Cin,
                                     long long ldci, double* D, long long ldd) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)M * N) return;
    const int i = (int)(idx / N), j = (int)(idx % N);
    double s = 0.0;
    for (int t = 0; t < ks; ++t) s += P[t * ss + (long long)i * ldp + j];
    double v = alpha * s;
    if (beta != 0.0) v += beta * Cin[(long long)i * ldci + j];
    D[(long long)i * ldd + j] = v;
}

template <int WM, int WN, int AM, int BMd, bool AF32 = false>
hipError_t launch_t(const GemmF64Args& a, hipStream_t s) {
    const int ntm = (a.M + 64 * WM - 1) / (64 * WM), ntn = (a.N + 64 * WN - 1) / (64 * WN);
    int tiles = ntm * ntn;
    if (a.M2 > 0) tiles += ((a.M2 + 64 * WM - 1) / (64 * WM)) * ((a.N2 + 64 * WN - 1) / (64 * WN));
    dim3 grid(tiles, a.ksplit > 1 ? a.ksplit : 1);
    hipLaunchKernelGGL((gemm_f64_kernel<WM, WN, AM, BMd, AF32>), grid, dim3(64 * WM * WN), 0, s, a);
    return hipGetLastError();
}

template <int WM, int WN>
hipError_t dispatch_modes(const GemmF64Args& a, hipStream_t s) {
    const int am = a.amode, bm = a.bmode;
    if (am == OP_N && bm == OP_N) return launch_t<WM, WN, OP_N, OP_N>(a, s);
    if (am == OP_N && bm == OP_T) return launch_t<WM, WN, OP_N, OP_T>(a, s);
    if (am == OP_N && bm == OP_TOEP) return launch_t<WM, WN, OP_N, OP_TOEP>(a, s);
    if (am == OP_T && bm == OP_N) return launch_t<WM, WN, OP_T, OP_N>(a, s);
    if (am == OP_TOEP && bm == OP_N) return launch_t<WM, WN, OP_TOEP, OP_N>(a, s);
    if (am == OP_T && bm == OP_T) return launch_t<WM, WN, OP_T, OP_T>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gemm_f64(const GemmF64Args& a, int tile, hipStream_t s) {
    if (a.M2 > 0 && (a.N2 <= 0 || a.ksplit > 1 || a.a_f32)) return hipErrorInvalidValue;
    if (a.M <= 0 || a.N <= 0) {
        if (a.M2 <= 0) return hipSuccess;
        // only the second product is non-empty
        GemmF64Args b = a;
        b.M = a.M2;
        b.N = a.N2;
        b.A = a.A2;
        b.B = a.B2;
        b.Cin = a.Cin2;
        b.D = a.D2;
        b.M2 = 0;
        return launch_gemm_f64(b, tile, s);
    }
    if (a.a_f32) {
        // FP32 factors times FP64 right-hand sides (the correction solves of the precision form)
        if (tile != 4 || a.bmode != OP_N) return hipErrorInvalidValue;
        if (a.amode == OP_N) return launch_t<2, 1, OP_N, OP_N, true>(a, s);
        if (a.amode == OP_T) return launch_t<2, 1, OP_T, OP_N, true>(a, s);
        return hipErrorInvalidValue;
    }
    if (tile == 0 && a.M2 <= 0 && a.amode == OP_N && a.bmode == OP_TOEP && a.ksplit <= 1 && a.alpha == 1.0 &&
        a.beta == 0.0 &&
        a.M % 128 == 0 && a.N % 128 == 0 && a.K % 32 == 0 && a.K == a.ldb) {
        // the multiplier product on full tiles (ldb carries the Toeplitz order, which is K)
        hipLaunchKernelGGL(gemm_ag_toep_kernel, dim3((a.M / 128) * (a.N / 128)), dim3(256), 0, s, a.M, a.N, a.K, a.A,
                           a.lda, a.B, a.D, a.ldd);
        return hipGetLastError();
    }
    switch (tile) {
        case 0: return dispatch_modes<2, 2>(a, s);
        case 1: return dispatch_modes<4, 1>(a, s);
        case 2: return dispatch_modes<1, 4>(a, s);
        case 3: return dispatch_modes<1, 1>(a, s);
        case 4: return dispatch_modes<2, 1>(a, s);
        case 5: return dispatch_modes<1, 2>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_splitk_reduce_f64(int M, int N, int ks, const double* P, long long ldp, long long ss,
                                    double alpha, double beta, const double* Cin, long long ldci,
                                    double* D, long long ldd, hipStream_t s) {
    const long long tot = (long long)M * N;
    if (tot <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s,
                       M, N, ks, P, ldp, ss, alpha, beta, Cin, ldci, D, ldd);
    return hipGetLastError();
}
