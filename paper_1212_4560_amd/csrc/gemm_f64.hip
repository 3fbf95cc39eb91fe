// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4_f64): an LDS double-buffered
// kernel for every shape, and a register-operand kernel for the two dominant products.
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

// Operands loaded straight into MFMA registers (no LDS, no barriers), for the two
// products that dominate the solve: the multiplier product C = A G with a Toeplitz G
// generated from its parameters, and the Schur complement updates A22 -= L21 U12.
//
// A workgroup of 2 x WMW waves covers (64 WMW) x 128 outputs, each wave an independent
// 64 x 64 tile (4 x 4 MFMA tiles).  The 16x16x4 MFMA sums over its 4 k-slots, and any fixed
// assignment of actual k indices to the slots gives the same sum, so lane group q
// (lanes 16q .. 16q+15) takes the k pair k0 + 2q, k0 + 2q + 1 of each 8-deep chunk:
// its A fragment of a row is one 16-byte load, its B fragment two 8-byte loads from rows
// of B, 16 consecutive columns per lane group.  Two register buffers alternate: the next
// chunk's loads are issued before the current chunk's 32 MFMAs.  An FP64 MFMA of this
// shape occupies the matrix unit for 64 cycles, so a chunk is about 2k cycles of MFMA per
// wave and about 4k with two waves per SIMD: enough to cover the load latency from L2
// without staging through LDS.  The loop body has no branches, so the waits the compiler
// places before each MFMA only cover the buffer that MFMA reads.
//
// DEPTH register buffers rotate: C = A G (K = n) keeps two chunks of loads in flight (three
// buffers, 248 VGPRs; 0.7 % faster than two at n = 16384), the Schur updates (K <= 768) one.
//
// WMW = 4 (8 waves, one workgroup per CU) keeps the waves that share a CU's matrix units in
// one workgroup.  With two 4-wave workgroups per CU the older one takes the units first, the
// two drift apart along K, and the workgroups of a tile-row stop meeting in L2: for C = A G
// at n = 16384 the fetch counter read 2.1x more (the 8-wave form is 0.7 % slower).
//
// Requirements (checked by the launcher): M, N multiples of 64 (a wave whose quadrant lies
// outside the output returns at once; there is no barrier to miss), K a multiple of 16,
// A 16-byte aligned with an even leading dimension.  Toeplitz B: G(k, j) = p[k - j + ldb - 1],
// K = ldb, N <= K.
typedef const double __attribute__((address_space(1)))* gcd_ptr;   // global (not flat) loads
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef const f64x2 __attribute__((address_space(1)))* gcd2_ptr;

template <bool TOEP, int WMW, int DEPTH = 2>
__device__ __forceinline__ void gemm_regs_body(const GemmF64Args& g) {
    constexpr int BMt = 64 * WMW;
    constexpr int KS = 2;   // k values per lane group per chunk; chunk depth 4 * KS = 8
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int bid = blockIdx.x;
    int gM = g.M, gN = g.N;
    const double* gA = g.A;
    const double* gB = g.B;
    const double* gCin = g.Cin;
    double* gD = g.D;
    {
        const int t1 = ((g.M + BMt - 1) / BMt) * ((g.N + 127) / 128);
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
    const int ntm = (gM + BMt - 1) / BMt, ntn = (gN + 127) / 128;
    const int pid = xcd_remap(bid, ntm * ntn);
    const int GROUP = g.group_m > 0 ? g.group_m : 8;
    const int first_m = (pid / (GROUP * ntn)) * GROUP;
    const int gsz = min(ntm - first_m, GROUP);
    const int tm = first_m + (pid % (GROUP * ntn)) % gsz;
    const int tn = (pid % (GROUP * ntn)) / gsz;
    const int m0 = tm * BMt + wm * 64, n0 = tn * 128 + wn * 64;
    if (m0 >= gM || n0 >= gN) return;
    const int lr = lane & 15, lq = lane >> 4;
    const long long lda = g.lda, ldb = g.ldb;
    const gcd_ptr Ab = (gcd_ptr)(gA + (long long)(m0 + lr) * lda + lq * KS);
    const gcd_ptr Bb = (gcd_ptr)(TOEP ? gB + (long long)lq * KS - (n0 + lr) + ldb - 1
                                      : gB + (long long)lq * KS * ldb + n0 + lr);
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    double ra[DEPTH][4][KS], rb[DEPTH][4][KS];
    auto load = [&](int buf, int k0) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            const f64x2 v = *(gcd2_ptr)(Ab + (long long)mi * 16 * lda + k0);
            ra[buf][mi][0] = v.x;
            ra[buf][mi][1] = v.y;
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int s = 0; s < KS; ++s)
                rb[buf][ni][s] = TOEP ? Bb[k0 + s - ni * 16] : Bb[(long long)(k0 + s) * ldb + ni * 16];
    };
    auto mma = [&](int buf) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[buf][mi][s], rb[buf][ni][s], acc[mi][ni], 0, 0, 0);
    };
    // The empty asm statements keep the compiler from sinking each batch of loads down to
    // its first use; the scheduling barriers keep the MFMAs from moving above the loads.
    const int nk = g.K / (4 * KS);   // even
    if constexpr (DEPTH == 3) {
        // three buffers in rotation (buffer c % 3 holds chunk c): two chunks of loads in flight
        load(0, 0);
        load(1, 4 * KS);
        int c = 0;
        for (; c + 5 <= nk; c += 3) {
            load(2, (c + 2) * 4 * KS);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(0);
            __builtin_amdgcn_sched_barrier(0);
            load(0, (c + 3) * 4 * KS);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(1);
            __builtin_amdgcn_sched_barrier(0);
            load(1, (c + 4) * 4 * KS);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(2);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (c + t < nk) {
                if (c + t + 2 < nk) load((t + 2) % 3, (c + t + 2) * 4 * KS);
                mma(t % 3);
            }
        }
    } else {
        load(0, 0);
        for (int c = 0; c < nk - 2; c += 2) {
            load(1, (c + 1) * 4 * KS);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(0);
            __builtin_amdgcn_sched_barrier(0);
            load(0, (c + 2) * 4 * KS);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(1);
            __builtin_amdgcn_sched_barrier(0);
        }
        load(1, (nk - 1) * 4 * KS);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mma(0);
        __builtin_amdgcn_sched_barrier(0);
    }
    // Epilogue: D = alpha acc + beta Cin, one 16-row strip at a time, with the loads of the
    // next strip of Cin in flight while a strip is stored: the first strip's loads go out
    // before the last chunk's MFMAs, into the registers the first buffer has freed.  Each
    // element is read before it is written and the strips are disjoint, so Cin may alias D.
    const bool rd = g.beta != 0.0;
    double cv[2][4][4];
    auto load_c = [&](int buf, int mi) {
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                cv[buf][ni][r] = ((gcd_ptr)gCin)[(long long)(m0 + mi * 16 + lq + 4 * r) * g.ldci + n0 + ni * 16 + lr];
    };
    if (rd) load_c(0, 0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DEPTH == 2) mma(1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        if (mi + 1 < 4 && rd) load_c((mi + 1) & 1, mi + 1);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = g.alpha * acc[mi][ni][r];
                if (rd) v = fma(g.beta, cv[mi & 1][ni][r], v);
                ((double __attribute__((address_space(1)))*)gD)[(long long)(m0 + mi * 16 + lq + 4 * r) * g.ldd + n0 + ni * 16 + lr] = v;
            }
    }
}

// C = A G with the Toeplitz G generated from its parameters
__global__ void __launch_bounds__(512, 1) gemm_ag_toep_kernel(GemmF64Args g) { gemm_regs_body<true, 4, 3>(g); }

// D = alpha A B + beta Cin, A and B row-major (the Schur complement updates), 128 x 128
// workgroups.  (256 x 128 workgroups run a lone update 6 % faster at M = N = 15872, but
// inside the factorization they fill whole CUs, and the diagonal-block kernel on the side
// stream then waits for a CU to drain and leaves half of it idle: the factorization took
// 64.0 ms against 62.8.)
__global__ void __launch_bounds__(256, 2) gemm_regs_kernel(GemmF64Args g) { gemm_regs_body<false, 2>(g); }

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

// shapes the register-operand kernels take (see gemm_regs_body)
static bool regs_ok(const GemmF64Args& a) {
    auto al = [](const double* p, long long ld) { return ((uintptr_t)p & 15) == 0 && (ld & 1) == 0; };
    if (a.ksplit > 1 || a.a_f32 || a.K <= 0 || a.K % 16) return false;
    if (a.M % 64 || a.N % 64 || !al(a.A, a.lda)) return false;
    if (a.M2 > 0 && (a.M2 % 64 || a.N2 % 64 || !al(a.A2, a.lda))) return false;
    return true;
}

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
    if (tile == 0 && regs_ok(a) && a.amode == OP_N && (a.bmode == OP_N || a.bmode == OP_TOEP)) {
        const bool toep = a.bmode == OP_TOEP;
        if (!toep || (a.M2 <= 0 && a.K == a.ldb && a.N <= a.K)) {
            const int bm = toep ? 256 : 128;   // workgroup rows (gemm_ag_toep_kernel: 8 waves)
            int tiles = ((a.M + bm - 1) / bm) * ((a.N + 127) / 128);
            if (a.M2 > 0) tiles += ((a.M2 + bm - 1) / bm) * ((a.N2 + 127) / 128);
            if (toep) hipLaunchKernelGGL(gemm_ag_toep_kernel, dim3(tiles), dim3(512), 0, s, a);
            else hipLaunchKernelGGL(gemm_regs_kernel, dim3(tiles), dim3(256), 0, s, a);
            return hipGetLastError();
        }
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
