// GEMM into FP32 storage on the CDNA matrix cores, for the precision form of
// the method: C = A G and the Schur updates in FP32 (v_mfma_f32_16x16x4_f32), with
// BF16 operands and FP32 accumulation (v_mfma_f32_16x16x32_bf16), or with 2-word BF16
// operands: x = hi + lo, hi = bf16(x), lo = bf16(x - hi) (exact in FP32: hi shares x's
// leading bits), and a b taken as hi_a hi_b + hi_a lo_b + lo_a hi_b, three BF16 MFMAs
// per tile (about 16 significand bits instead of 8).
//
// D(fp32) = alpha * op(A) op(B) + beta * Cin(fp32).  Operands are FP64 (the
// caller's A, G or Toeplitz parameters) or FP32 (the working matrix); the
// loader rounds them to FP32 (round to nearest even) and, in BF16 mode, the
// FP32 value to BF16 (round to nearest even on the upper 16 bits, NaN kept
// quiet) -- the same two-step rounding the oracle's mirror uses.
//
// Tiling: a wave owns 64 x 64 outputs = 4 x 4 MFMA tiles of 16 x 16; a block is
// 2 x 2 waves (128 x 128); K is staged through LDS in chunks of 32, double
// buffered.  f32/bf16 16 x 16 accumulators hold 4 consecutive rows per lane
// group: lane l, element r -> row 4 (l / 16) + r, column l % 16.
#include "common.h"

#include <type_traits>

namespace {

constexpr int BKL = 32;

__device__ inline unsigned short f32_to_bf16_rne(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x0040u);   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <int MODE, bool F64>
__device__ inline float ld_op(const void* X, long long ld, int i, int k, int rows, int cols) {
    if (i >= rows || k >= cols) return 0.f;
    const long long idx = (MODE == OP_N) ? (long long)i * ld + k : (long long)k * ld + i;
    return F64 ? (float)((const double*)X)[idx] : ((const float*)X)[idx];
}

__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <bool F64>
__device__ inline float ld_lin(const void* X, long long idx) {
    return F64 ? (float)((const double*)X)[idx] : ((const float*)X)[idx];
}

// BF16: tiles in LDS as bf16 with k contiguous (As[i][k], Bs[j][k]) so a lane reads
// its 8 consecutive k values with one 16-byte load.  FP32: As[k][i], Bs[k][j].
// X3 (with BF16): 2-word operands, the lo words in their own LDS tiles.
// One workgroup per CU with X3 (its three products and lo tiles need more than half the registers).
template <int WM, int WN, int AMODE, int BMODE, bool AF64, bool BF64, bool BF16, bool X3 = false>
__global__ void __launch_bounds__(64 * WM * WN, X3 ? 1 : 2)
gemm_lp_kernel(GemmLpArgs g) {
    constexpr int T = 64 * WM * WN;
    constexpr int BMt = 64 * WM, BNt = 64 * WN;
    constexpr int LA = (BMt * BKL) / T, LBB = (BNt * BKL) / T;   // per-thread loads
    // LDS: bf16 -> [row][k] with 8 bf16 of padding; fp32 -> [k][row] with 4 floats of padding
    constexpr int A_LD = BF16 ? BKL + 8 : BMt + 4;
    constexpr int B_LD = BF16 ? BKL + 8 : BNt + 4;
    constexpr int A_SZ = BF16 ? BMt * A_LD : BKL * A_LD;
    constexpr int B_SZ = BF16 ? BNt * B_LD : BKL * B_LD;
    using ET = typename std::conditional<BF16, unsigned short, float>::type;
    __shared__ __attribute__((aligned(16))) ET As[2][A_SZ];
    __shared__ __attribute__((aligned(16))) ET Bs[2][B_SZ];
    __shared__ __attribute__((aligned(16))) ET As_lo[X3 ? 2 : 1][X3 ? A_SZ : 8];
    __shared__ __attribute__((aligned(16))) ET Bs_lo[X3 ? 2 : 1][X3 ? B_SZ : 8];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    const int ntm = (g.M + BMt - 1) / BMt, ntn = (g.N + BNt - 1) / BNt;
    const int total = ntm * ntn;
    const int pid = xcd_remap(blockIdx.x, total);
    constexpr int GROUP = 8;
    const int group = pid / (GROUP * ntn);
    const int first_m = group * GROUP;
    const int gsz = min(ntm - first_m, GROUP);
    const int tm = first_m + (pid % (GROUP * ntn)) % gsz;
    const int tn = (pid % (GROUP * ntn)) / gsz;
    const int m0 = tm * BMt, n0 = tn * BNt;
    const int K = g.K;
    const int nk = (K + BKL - 1) / BKL;

    static_assert(AMODE != OP_TOEP, "Toeplitz A operand not used in the precision form");
    float ra[LA], rb[LBB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = tid + r * T;
            int i, k;
            if (AMODE == OP_N) { i = e / BKL; k = e % BKL; }
            else { k = e / BMt; i = e % BMt; }
            ra[r] = ld_op<AMODE, AF64>(g.A, g.lda, m0 + i, k0 + k, g.M, K);
        }
#pragma unroll
        for (int r = 0; r < LBB; ++r) {
            const int e = tid + r * T;
            int k, j;
            if (BMODE == OP_T) { j = e / BKL; k = e % BKL; }
            else { k = e / BNt; j = e % BNt; }
            // B(k, j): OP_N -> B[k*ld + j]; OP_T -> B[j*ld + k]; Toeplitz -> p[k - j + t - 1]
            float v = 0.f;
            if (k0 + k < K && n0 + j < g.N) {
                long long idx;
                if (BMODE == OP_N) idx = (long long)(k0 + k) * g.ldb + n0 + j;
                else if (BMODE == OP_T) idx = (long long)(n0 + j) * g.ldb + k0 + k;
                else idx = (long long)(k0 + k) - (n0 + j) + g.ldb - 1;
                v = ld_lin<BF64>(g.B, idx);
            }
            rb[r] = v;
        }
    };
    auto put = [&](ET* arr, ET* arr_lo, int idx, float v) {
        if constexpr (BF16) {
            const unsigned short h = f32_to_bf16_rne(v);
            arr[idx] = h;
            if constexpr (X3) arr_lo[idx] = f32_to_bf16_rne(v - bf16_to_f32(h));
        } else {
            arr[idx] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = tid + r * T;
            int i, k;
            if (AMODE == OP_N) { i = e / BKL; k = e % BKL; }
            else { k = e / BMt; i = e % BMt; }
            put(As[buf], As_lo[X3 ? buf : 0], BF16 ? i * A_LD + k : k * A_LD + i, ra[r]);
        }
#pragma unroll
        for (int r = 0; r < LBB; ++r) {
            const int e = tid + r * T;
            int k, j;
            if (BMODE == OP_T) { j = e / BKL; k = e % BKL; }
            else { k = e / BNt; j = e % BNt; }
            put(Bs[buf], Bs_lo[X3 ? buf : 0], BF16 ? j * B_LD + k : k * B_LD + j, rb[r]);
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int lr = lane & 15, lq = lane >> 4;
    if (nk > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            const int k0 = kt * BKL;
            if (kt + 1 < nk) gload(k0 + BKL);
            if constexpr (BF16) {
                // one 16x16x32 step covers the whole chunk
                bf16x8 af[4], bfr[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) {
                    const int i = wm * 64 + mi * 16 + lr;
                    af[mi] = *reinterpret_cast<const bf16x8*>(&As[cur][i * A_LD + lq * 8]);
                }
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const int j = wn * 64 + ni * 16 + lr;
                    bfr[ni] = *reinterpret_cast<const bf16x8*>(&Bs[cur][j * B_LD + lq * 8]);
                }
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mi], bfr[ni], acc[mi][ni], 0, 0, 0);
                if constexpr (X3) {
                    // hi_a lo_b, then lo_a hi_b
                    bf16x8 xf[4];
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni) {
                        const int j = wn * 64 + ni * 16 + lr;
                        xf[ni] = *reinterpret_cast<const bf16x8*>(&Bs_lo[cur][j * B_LD + lq * 8]);
                    }
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 4; ++ni)
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mi], xf[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi) {
                        const int i = wm * 64 + mi * 16 + lr;
                        xf[mi] = *reinterpret_cast<const bf16x8*>(&As_lo[cur][i * A_LD + lq * 8]);
                    }
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 4; ++ni)
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xf[mi], bfr[ni], acc[mi][ni], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < BKL; kk += 4) {
                    float af[4], bfr[4];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi) af[mi] = As[cur][(kk + lq) * A_LD + wm * 64 + mi * 16 + lr];
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni) bfr[ni] = Bs[cur][(kk + lq) * B_LD + wn * 64 + ni * 16 + lr];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 4; ++ni)
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mi], bfr[ni], acc[mi][ni], 0, 0, 0);
                }
            }
            if (kt + 1 < nk) sstore(cur ^ 1);
            __syncthreads();
        }
    }

    const bool rd = g.beta != 0.f;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        float cv[4][4];
        if (rd) {
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const int col = n0 + wn * 64 + ni * 16 + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * 64 + mi * 16 + lq * 4 + r;
                    cv[ni][r] = (row < g.M && col < g.N) ? g.Cin[(long long)row * g.ldci + col] : 0.f;
                }
            }
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int col = n0 + wn * 64 + ni * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + mi * 16 + lq * 4 + r;
                if (row < g.M && col < g.N) {
                    float v = g.alpha * acc[mi][ni][r];
                    if (rd) v = fmaf(g.beta, cv[ni][r], v);
                    g.D[(long long)row * g.ldd + col] = v;
                }
            }
        }
    }
}

template <int AM, int BMd, bool AF64, bool BF64, bool BF16, bool X3>
hipError_t launch_t(const GemmLpArgs& a, hipStream_t s) {
    const int ntm = (a.M + 127) / 128, ntn = (a.N + 127) / 128;
    hipLaunchKernelGGL((gemm_lp_kernel<2, 2, AM, BMd, AF64, BF64, BF16, X3>), dim3(ntm * ntn), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <bool BF16, bool X3 = false>
hipError_t dispatch(const GemmLpArgs& a, hipStream_t s) {
    // the combinations the path uses: A G (FP64 or FP32 A, dense or Toeplitz G of the same
    // type) and the Schur update (FP32 L21, FP32 U12)
    if (a.amode == OP_N && a.a_f64 && a.bmode == OP_N && a.b_f64) return launch_t<OP_N, OP_N, true, true, BF16, X3>(a, s);
    if (a.amode == OP_N && a.a_f64 && a.bmode == OP_TOEP && a.b_f64)
        return launch_t<OP_N, OP_TOEP, true, true, BF16, X3>(a, s);
    if (a.amode == OP_N && !a.a_f64 && a.bmode == OP_N && !a.b_f64)
        return launch_t<OP_N, OP_N, false, false, BF16, X3>(a, s);
    if (a.amode == OP_N && !a.a_f64 && a.bmode == OP_TOEP && !a.b_f64)
        return launch_t<OP_N, OP_TOEP, false, false, BF16, X3>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gemm_lp(const GemmLpArgs& a, int tile, hipStream_t s) {
    (void)tile;
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    if (a.bf16 == 2) return dispatch<true, true>(a, s);
    return a.bf16 ? dispatch<true>(a, s) : dispatch<false>(a, s);
}
