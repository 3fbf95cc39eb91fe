// FP32 product C = A G on the CDNA matrix cores with register operands (v_mfma_f32_16x16x4_f32),
// for the FP32 precision form of the method (section 1.1) with a Gaussian Toeplitz multiplier
// (section 2.3): A is an FP32 copy of the caller's A, G is generated in the loader from an FP32
// copy of its parameters, G(k, j) = p[k - j + ldb - 1], and never stored.
//
// Each wave owns a 64 x 64 output tile = 4 x 4 MFMA tiles of 16 x 16 and reads its operands
// straight from global memory (L2 / MALL) into registers, three chunks of 16 k-values in rotation
// (two chunks of loads in flight while one is multiplied); 256 x 128 workgroups of eight waves,
// one per CU.  The 16x16x4 f32 MFMA takes lane l's A value at (row l % 16, k slot l / 16) and B
// value at (k slot l / 16, column l % 16); lane group q's k slot s of a chunk is k0 + 4q + s, so
// each lane reads four consecutive A values with one 16-byte load.  (The MFMA adds its four
// products with one rounding step whose result depends on which k meet in it; with the
// structured operands of the elimination -- large multipliers in a few columns -- grouping four
// consecutive k as the LDS-staged kernel does keeps the Schur updates about three times more
// accurate, so those updates stay on that kernel.)  Accumulator lane l, element r: row
// 4 (l / 16) + r, column l % 16.
//
// Requirements (checked by the launcher): M, N multiples of 64, K = ldb a multiple of 16,
// N <= ldb, A 16-byte aligned with a leading dimension that is a multiple of 4.
#include "common.h"

namespace {

typedef const float __attribute__((address_space(1)))* gcf_ptr;
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef const f32x4v __attribute__((address_space(1)))* gcf4_ptr;

__global__ void __launch_bounds__(512, 1) gemm_f32_toep_kernel(GemmF32Args g) {
    constexpr int BMt = 256;
    constexpr int KS = 4;            // k values per lane group per chunk; chunk depth 16
    constexpr int CH = 4 * KS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int ntm = (g.M + BMt - 1) / BMt, ntn = (g.N + 127) / 128;
    // tiles in column-major order within each XCD's contiguous range: the blocks running
    // together on an XCD share one row panel of A in its L2 (the only streamed operand)
    const int pid = xcd_remap(blockIdx.x, ntm * ntn);
    const int tm = pid % ntm, tn = pid / ntm;
    const int m0 = tm * BMt + wm * 64, n0 = tn * 128 + wn * 64;
    if (m0 >= g.M || n0 >= g.N) return;   // no barrier in this kernel: a wave may leave early
    const int lr = lane & 15, lq = lane >> 4;
    const long long lda = g.lda, ldb = g.ldb;
    const gcf_ptr Ab = (gcf_ptr)(g.A + (long long)(m0 + lr) * lda + lq * KS);
    const gcf_ptr Bb = (gcf_ptr)(g.p + (long long)lq * KS - (n0 + lr) + ldb - 1);
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float ra[3][4][KS], rb[3][4][KS];
    auto load = [&](int buf, int k0) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            const f32x4v v = *(gcf4_ptr)(Ab + (long long)mi * 16 * lda + k0);
            ra[buf][mi][0] = v.x;
            ra[buf][mi][1] = v.y;
            ra[buf][mi][2] = v.z;
            ra[buf][mi][3] = v.w;
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int s = 0; s < KS; ++s) rb[buf][ni][s] = Bb[k0 + s - ni * 16];
    };
    auto mma = [&](int buf) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[buf][mi][s], rb[buf][ni][s], acc[mi][ni], 0, 0, 0);
    };
    // Three buffers in rotation, buffer c % 3 holding chunk c; a load is issued only for a
    // chunk that exists.  The empty asm statements keep the compiler from sinking a batch of
    // loads down to its first use; the scheduling barriers keep the MFMAs below the loads.
    const int nk = g.K / CH;
    load(0, 0);
    if (nk > 1) load(1, CH);
    int c = 0;
    for (; c + 5 <= nk; c += 3) {
        load(2, (c + 2) * CH);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mma(0);
        __builtin_amdgcn_sched_barrier(0);
        load(0, (c + 3) * CH);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mma(1);
        __builtin_amdgcn_sched_barrier(0);
        load(1, (c + 4) * CH);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mma(2);
        __builtin_amdgcn_sched_barrier(0);
    }
    // the last one to four chunks: c + t < nk runs chunk c + t from buffer (c + t) % 3 = t % 3
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (c + t < nk) {
            if (c + t + 2 < nk) load((t + 2) % 3, (c + t + 2) * CH);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            mma(t % 3);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // Epilogue: D = acc, one 16-row strip at a time
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ((float __attribute__((address_space(1)))*)g.D)[(long long)(m0 + mi * 16 + lq * 4 + r) * g.ldd + n0 +
                                                            ni * 16 + lr] = acc[mi][ni][r];
}

}  // namespace

hipError_t launch_gemm_f32_toep(const GemmF32Args& a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0 || a.M % 64 || a.N % 64 || a.K % 16 || a.K != a.ldb || a.N > a.ldb ||
        ((uintptr_t)a.A & 15) || (a.lda & 3))
        return hipErrorInvalidValue;
    const int tiles = ((a.M + 255) / 256) * ((a.N + 127) / 128);
    hipLaunchKernelGGL(gemm_f32_toep_kernel, dim3(tiles), dim3(512), 0, s, a);
    return hipGetLastError();
}
