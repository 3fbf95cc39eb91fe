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

// Schur update of the FP32 precision form, D = alpha A B + beta Cin (A: L21, M x K; B: U12,
// K x N; FP32 row-major; Cin may alias D), LDS-staged: 256 x 128 workgroups of eight 64 x 64
// waves, 16-deep K chunks in two LDS buffers, 16-byte global loads (the next chunk in flight
// while the current one is multiplied).  Each MFMA takes four consecutive k (lane group q of
// step s: k0 + 4 s + q), in increasing k, the grouping and order of the general LDS-staged
// kernel, so the products are the same.  The epilogue reads each 16-row strip of Cin before
// storing it.
template <int BK>
__global__ void __launch_bounds__(512, 1) gemm_f32_upd_kernel(GemmF32UpdArgs g) {
    constexpr int BM = 256, BN = 128;
    constexpr int NA = BK / 8, NB = BK / 16;   // 16-byte loads per thread per chunk (A, B)
    __shared__ __attribute__((aligned(16))) float As[2][BK][BM + 4];   // [k][row]
    __shared__ __attribute__((aligned(16))) float Bs[2][BK][BN + 4];   // [k][col]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int ntm = (g.M + BM - 1) / BM, ntn = (g.N + BN - 1) / BN;
    const int pid = xcd_remap(blockIdx.x, ntm * ntn);
    constexpr int GROUP = 8;
    const int first_m = (pid / (GROUP * ntn)) * GROUP;
    const int gsz = min(ntm - first_m, GROUP);
    const int tm = first_m + (pid % (GROUP * ntn)) % gsz;
    const int tn = (pid % (GROUP * ntn)) / gsz;
    const int m0 = tm * BM, n0 = tn * BN;
    const int lr = lane & 15, lq = lane >> 4;
    // global -> registers, 16 bytes a load: A element f = tid + 512 r covers row f / (BK / 4) and
    // k 4 (f % (BK / 4)) .. + 3; B element f covers row k = f / 32 and columns 4 (f % 32) .. + 3
    f32x4v ra[NA], rb[NB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const int f = tid + 512 * r, row = m0 + f / (BK / 4), kq = f % (BK / 4);
            ra[r] = row < g.M ? *(gcf4_ptr)(g.A + (long long)row * g.lda + k0 + 4 * kq) : f32x4v{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid + 512 * r, k = f / 32, col = n0 + 4 * (f % 32);
            rb[r] = col < g.N ? *(gcf4_ptr)(g.B + (long long)(k0 + k) * g.ldb + col) : f32x4v{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const int f = tid + 512 * r, row = f / (BK / 4), kq = f % (BK / 4);
            As[buf][4 * kq + 0][row] = ra[r].x;
            As[buf][4 * kq + 1][row] = ra[r].y;
            As[buf][4 * kq + 2][row] = ra[r].z;
            As[buf][4 * kq + 3][row] = ra[r].w;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid + 512 * r;
            *reinterpret_cast<f32x4v*>(&Bs[buf][f / 32][4 * (f % 32)]) = rb[r];
        }
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool live = wm * 64 < g.M - m0 && wn * 64 < g.N - n0;   // this wave has outputs
    const int nk = g.K / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        if (live) {
#pragma unroll
            for (int st = 0; st < BK / 4; ++st) {
                float af[4], bf[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) af[mi] = As[cur][4 * st + lq][wm * 64 + mi * 16 + lr];
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) bf[ni] = Bs[cur][4 * st + lq][wn * 64 + ni * 16 + lr];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
            }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    if (!live) return;
    float __attribute__((address_space(1)))* D = (float __attribute__((address_space(1)))*)g.D;
    const float __attribute__((address_space(1)))* Ci = (const float __attribute__((address_space(1)))*)g.Cin;
    const bool rd = g.beta != 0.f;
    const int mw = m0 + wm * 64, nw = n0 + wn * 64;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        float cv[4][4];
        if (rd) {
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    cv[ni][r] = Ci[(long long)(mw + mi * 16 + lq * 4 + r) * g.ldci + nw + ni * 16 + lr];
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = g.alpha * acc[mi][ni][r];
                if (rd) v = fmaf(g.beta, cv[ni][r], v);
                D[(long long)(mw + mi * 16 + lq * 4 + r) * g.ldd + nw + ni * 16 + lr] = v;
            }
    }
}

}  // namespace

constexpr int F32_UPD_BK = 16;   // K chunk of the FP32 update kernel (16 or 32)

hipError_t launch_gemm_f32_upd(const GemmF32UpdArgs& a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    auto al = [](const float* p, long long ld) { return ((uintptr_t)p & 15) == 0 && (ld & 3) == 0; };
    if (a.M % 64 || a.N % 64 || a.K <= 0 || a.K % 16 || !a.A || !a.B || !a.D || !al(a.A, a.lda) ||
        !al(a.B, a.ldb) || (a.beta != 0.f && !a.Cin))
        return hipErrorInvalidValue;
    const int tiles = ((a.M + 255) / 256) * ((a.N + 127) / 128);
    if (a.K % 32 == 0 && F32_UPD_BK == 32) hipLaunchKernelGGL(gemm_f32_upd_kernel<32>, dim3(tiles), dim3(512), 0, s, a);
    else hipLaunchKernelGGL(gemm_f32_upd_kernel<16>, dim3(tiles), dim3(512), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm_f32_toep(const GemmF32Args& a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0 || a.M % 64 || a.N % 64 || a.K % 16 || a.K != a.ldb || a.N > a.ldb ||
        ((uintptr_t)a.A & 15) || (a.lda & 3))
        return hipErrorInvalidValue;
    const int tiles = ((a.M + 255) / 256) * ((a.N + 127) / 128);
    hipLaunchKernelGGL(gemm_f32_toep_kernel, dim3(tiles), dim3(512), 0, s, a);
    return hipGetLastError();
}
