// BF16 product on the CDNA matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) for the
// BF16 precision form of the method: C = A G (section 1.1) from BF16 copies of A and of the
// multiplier made once per precondition (the Toeplitz multiplier of section 2.3 is written out
// transposed, so that both operands are K-contiguous).  The 2-word BF16 form (x = hi + lo)
// takes three products per tile pair, hi hi + hi lo + lo hi, from the hi and lo copies.
//
// D (FP32, M x N) = A (BF16, M x K, row-major) * Bt^T (Bt: BF16, N x K, row-major).
// Workgroups of four waves own 256 x 256 outputs (each wave 128 x 128 = 8 x 8 MFMA tiles of
// 16 x 16) and stage 256 x 32 tiles of A and of Bt through LDS, two buffers: the next k-chunk
// is fetched from global memory into registers while the current one is multiplied, then
// written to the other buffer.  The 16x16x32 bf16 MFMA takes lane l's eight A values at row
// l % 16, k 8 (l / 16) .. + 7 and its eight B values at column l % 16, the same k: one 16-byte
// LDS read each.  Accumulator lane l, element r: row 4 (l / 16) + r, column l % 16.
//
// Requirements (checked by the launcher): M, N multiples of 256, K of 32, both operands
// 16-byte aligned with leading dimensions that are multiples of 8 elements.
#include "common.h"

namespace {

constexpr int BT = 256;      // workgroup tile (rows and columns)
constexpr int BKB = 32;      // k-chunk
constexpr int LDB = BKB + 8; // LDS row stride in bf16 (80 bytes: 16-byte aligned rows)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet)
__device__ inline unsigned short bf16_bits(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
typedef const u32x4 __attribute__((address_space(1)))* gu4_ptr;

template <bool X3>
__global__ void __launch_bounds__(256, 1)
gemm_bf16_nt_kernel(GemmBf16Args g) {
    // X3: the lo copies take their own LDS tiles
    __shared__ __attribute__((aligned(16))) unsigned short As[2][BT * LDB];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][BT * LDB];
    __shared__ __attribute__((aligned(16))) unsigned short Al[X3 ? 2 : 1][X3 ? BT * LDB : 8];
    __shared__ __attribute__((aligned(16))) unsigned short Bl[X3 ? 2 : 1][X3 ? BT * LDB : 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int ntm = g.M / BT, ntn = g.N / BT;
    // each XCD takes a contiguous range of tiles, walked down the columns of tiles so that the
    // workgroups running together share rows of A and columns of B in that XCD's L2
    const int pid = xcd_remap(blockIdx.x, ntm * ntn);
    const int tm = pid % ntm, tn = pid / ntm;
    const int m0 = tm * BT, n0 = tn * BT;
    // global -> LDS staging: thread t moves 16 bytes (8 bf16) of rows r = t / 4 + 64 i,
    // chunk t % 4 of the 32-wide k-chunk, for i = 0..3, for each operand
    const int sr = tid >> 2, sc = tid & 3;
    const unsigned short* Ag = g.A + (long long)(m0 + sr) * g.lda + sc * 8;
    const unsigned short* Bg = g.Bt + (long long)(n0 + sr) * g.ldb + sc * 8;
    const unsigned short* Alg = X3 ? g.Alo + (long long)(m0 + sr) * g.lda + sc * 8 : nullptr;
    const unsigned short* Blg = X3 ? g.Btlo + (long long)(n0 + sr) * g.ldb + sc * 8 : nullptr;
    constexpr int NR = X3 ? 16 : 8;
    u32x4 st[NR];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            st[i] = *(gu4_ptr)(Ag + (long long)(64 * i) * g.lda + k0);
            st[4 + i] = *(gu4_ptr)(Bg + (long long)(64 * i) * g.ldb + k0);
            if constexpr (X3) {
                st[8 + i] = *(gu4_ptr)(Alg + (long long)(64 * i) * g.lda + k0);
                st[12 + i] = *(gu4_ptr)(Blg + (long long)(64 * i) * g.ldb + k0);
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int off = (sr + 64 * i) * LDB + sc * 8;
            *reinterpret_cast<u32x4*>(&As[buf][off]) = st[i];
            *reinterpret_cast<u32x4*>(&Bs[buf][off]) = st[4 + i];
            if constexpr (X3) {
                *reinterpret_cast<u32x4*>(&Al[buf][off]) = st[8 + i];
                *reinterpret_cast<u32x4*>(&Bl[buf][off]) = st[12 + i];
            }
        }
    };
    f32x4 acc[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lq = lane >> 4;
    const int nk = g.K / BKB;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BKB);
        bf16x8 bf[8];
#pragma unroll
        for (int ni = 0; ni < 8; ++ni)
            bf[ni] = *reinterpret_cast<const bf16x8*>(&Bs[cur][(wn * 128 + ni * 16 + lr) * LDB + lq * 8]);
#pragma unroll
        for (int mi = 0; mi < 8; ++mi) {
            const bf16x8 af = *reinterpret_cast<const bf16x8*>(&As[cur][(wm * 128 + mi * 16 + lr) * LDB + lq * 8]);
#pragma unroll
            for (int ni = 0; ni < 8; ++ni)
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[ni], acc[mi][ni], 0, 0, 0);
        }
        if constexpr (X3) {
            // hi_a lo_b, then lo_a hi_b
            bf16x8 bl[8];
#pragma unroll
            for (int ni = 0; ni < 8; ++ni)
                bl[ni] = *reinterpret_cast<const bf16x8*>(&Bl[cur][(wn * 128 + ni * 16 + lr) * LDB + lq * 8]);
#pragma unroll
            for (int mi = 0; mi < 8; ++mi) {
                const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&As[cur][(wm * 128 + mi * 16 + lr) * LDB + lq * 8]);
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(&Al[cur][(wm * 128 + mi * 16 + lr) * LDB + lq * 8]);
#pragma unroll
                for (int ni = 0; ni < 8; ++ni) {
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ni], acc[mi][ni], 0, 0, 0);
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bf[ni], acc[mi][ni], 0, 0, 0);
                }
            }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    // D = alpha acc + beta Cin (row 4 lq + r, column lr of each 16 x 16 tile); each element is
    // read before it is written, by the same lane, so Cin may alias D.  The reads of a 16-row
    // strip are issued together before its stores: with Cin possibly aliasing D the compiler
    // keeps every read after the stores that precede it, and one read-then-store per element
    // made the update's epilogue some 250 memory round trips long.
    float __attribute__((address_space(1)))* D = (float __attribute__((address_space(1)))*)g.D;
    const float __attribute__((address_space(1)))* Ci = (const float __attribute__((address_space(1)))*)g.Cin;
    const bool rd = g.beta != 0.f;
#pragma unroll
    for (int mi = 0; mi < 8; ++mi) {
        const long long row0 = m0 + wm * 128 + mi * 16 + lq * 4;
        float cv[8][4];
        if (rd) {
#pragma unroll
            for (int ni = 0; ni < 8; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) cv[ni][r] = Ci[(row0 + r) * g.ldci + n0 + wn * 128 + ni * 16 + lr];
        }
#pragma unroll
        for (int ni = 0; ni < 8; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = g.alpha * acc[mi][ni][r];
                if (rd) v = fmaf(g.beta, cv[ni][r], v);
                D[(row0 + r) * g.ldd + n0 + wn * 128 + ni * 16 + lr] = v;
            }
    }
}

// hi / lo = 2-word BF16 split of an FP32 block (trans: of its transpose), 32 x 32 tiles via LDS
__global__ void __launch_bounds__(256)
split_bf16_kernel(const float* __restrict__ X, long long ldx, int rows, int cols, int trans,
                  unsigned short* __restrict__ hi, unsigned short* __restrict__ lo, long long ldo) {
    __shared__ float t[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = r0 + r, j = c0 + tx;
        t[r][tx] = (i < rows && j < cols) ? X[(long long)i * ldx + j] : 0.f;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        // output row: trans ? column c0 + r of X : row r0 + r; output column likewise
        const int oi = trans ? c0 + r : r0 + r, oj = trans ? r0 + tx : c0 + tx;
        const float v = trans ? t[tx][r] : t[r][tx];
        if (oi < (trans ? cols : rows) && oj < (trans ? rows : cols)) {
            const unsigned short h = bf16_bits(v);
            hi[(long long)oi * ldo + oj] = h;
            if (lo) lo[(long long)oi * ldo + oj] = bf16_bits(v - __uint_as_float((unsigned int)h << 16));
        }
    }
}

// FP64 -> FP32 -> BF16, round to nearest even at each step; with lo, also lo = bf16(x32 - hi)
// (exact in FP32: hi carries x32's leading bits)

__device__ inline void split_bf16(double x, unsigned short& hi, unsigned short& lo) {
    const float f = (float)x;
    hi = bf16_bits(f);
    lo = bf16_bits(f - __uint_as_float((unsigned int)hi << 16));
}

// out (n_pad x n_pad, row-major) = bf16 of A (n x n FP64), zero padding; lo: the second words
__global__ void to_bf16_kernel(const double* __restrict__ A, long long lda, int n, int n_pad,
                               unsigned short* __restrict__ hi, unsigned short* __restrict__ lo) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n_pad * n_pad) return;
    const int i = (int)(e / n_pad), j = (int)(e % n_pad);
    unsigned short h = 0, l = 0;
    if (i < n && j < n) split_bf16(A[(long long)i * lda + j], h, l);
    hi[e] = h;
    if (lo) lo[e] = l;
}

// Gt (n_pad x n_pad): Gt[j][k] = G(k, j) in BF16; G dense (ldg) or Toeplitz (p, 2n - 1
// parameters, G(k, j) = p[k - j + n - 1]); zero outside n x n.  32 x 32 tiles through LDS so
// that both the dense reads and the writes are coalesced.
__global__ void __launch_bounds__(256)
gt_bf16_kernel(const double* __restrict__ G, long long ldg, int toep, int n, int n_pad,
               unsigned short* __restrict__ hi, unsigned short* __restrict__ lo) {
    __shared__ double t[32][33];
    const int k0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int k = k0 + r, j = j0 + tx;
        double v = 0.0;
        if (k < n && j < n) v = toep ? G[(long long)k - j + n - 1] : G[(long long)k * ldg + j];
        t[r][tx] = v;   // t[k - k0][j - j0]
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + r, k = k0 + tx;
        unsigned short h, l;
        split_bf16(t[tx][r], h, l);
        const long long o = (long long)j * n_pad + k;
        hi[o] = h;
        if (lo) lo[o] = l;
    }
}

}  // namespace

hipError_t launch_gemm_bf16_nt(const GemmBf16Args& a, hipStream_t s) {
    auto al = [](const void* p, long long ld) { return ((uintptr_t)p & 15) == 0 && (ld & 7) == 0; };
    if (a.M <= 0 || a.N <= 0 || a.M % BT || a.N % BT || a.K <= 0 || a.K % BKB || !al(a.A, a.lda) ||
        !al(a.Bt, a.ldb))
        return hipErrorInvalidValue;
    const bool x3 = a.Alo != nullptr;
    if (x3 && (!a.Btlo || !al(a.Alo, a.lda) || !al(a.Btlo, a.ldb))) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.M / BT) * (a.N / BT)));
    if (x3) hipLaunchKernelGGL(gemm_bf16_nt_kernel<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(gemm_bf16_nt_kernel<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const double* A, long long lda, int n, int n_pad, unsigned short* hi, unsigned short* lo,
                          hipStream_t s) {
    const long long tot = (long long)n_pad * n_pad;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A, lda, n, n_pad, hi, lo);
    return hipGetLastError();
}

hipError_t launch_gt_bf16(const double* G, long long ldg, int toep, int n, int n_pad, unsigned short* hi,
                          unsigned short* lo, hipStream_t s) {
    const dim3 grid((unsigned)((n_pad + 31) / 32), (unsigned)((n_pad + 31) / 32));
    hipLaunchKernelGGL(gt_bf16_kernel, grid, dim3(256), 0, s, G, ldg, toep, n, n_pad, hi, lo);
    return hipGetLastError();
}

hipError_t launch_split_bf16(const float* X, long long ldx, int rows, int cols, int trans, unsigned short* hi,
                             unsigned short* lo, long long ldo, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(split_bf16_kernel, grid, dim3(256), 0, s, X, ldx, rows, cols, trans, hi, lo, ldo);
    return hipGetLastError();
}
