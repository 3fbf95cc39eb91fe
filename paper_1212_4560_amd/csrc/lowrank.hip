// Randomized low-rank approximation (Proto-Algorithm 5.1 with the orthogonal basis of
// Remark 5.4):
//   Stage 1  T' = A^T G                 (n x rho_+; the FP64 GEMM, split over K)
//   Stage 2  rank-revealing QR of T'     (Gram-Schmidt with column pivoting, each projection
//                                         applied twice; stops at the least s with
//                                         ||remaining columns||_F <= tau ||A||_F)
//   Stage 3  W = A T, A_hat = W T^T       (Theorem 5.1 with an orthogonal basis T), and
//            ||A - W T^T||_F for the check ||A - A_hat||_F <= tau2 ||A||_F.
// The pivoting loop runs on the device: a small state record carries the pivot, the scale
// and the stop decision from one launch to the next, so the host waits once, at the end.
#include "../../include/genp.h"
#include "common.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

namespace {

constexpr int LR_MAXK = 64;   // rho_+ <= 64
constexpr int CG_T = 256;     // threads: 4 row groups x 64 columns

struct LrState {
    int done;      // stop decision taken
    int rank;      // s
    int p;         // pivot column of the current step
    int pad;
    double scale;  // 1 / ||pivot column||
    double tail;   // ||remaining columns||_F when stopped
};

// out[0] = sum of the np partials (one block, fixed order)
__global__ void __launch_bounds__(256) sum_kernel(int np, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// G[i][j] = p[i - j + k - 1] (m x k)
__global__ void toeplitz_expand_kernel(int m, int k, const double* __restrict__ p, double* __restrict__ G) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)m * k) return;
    const int i = (int)(e / k), j = (int)(e % k);
    G[e] = p[i - j + k - 1];
}

// ---------------------------------------------------------------------------------------
// Skinny FP64 products on the matrix cores with register operands (no LDS): each wave owns a
// 64 x 64 output tile (4 x 4 MFMA tiles of 16 x 16, accumulator lane l / element r: row
// l/16 + 4r, column l%16), the k slots of lane group q are k0 + 2q and k0 + 2q + 1 of each
// 8-deep chunk, and two register buffers alternate.  Bounds are checked (any M, N, K).
//   AT: the A operand is stored transposed (element (i, k) at A[k * lda + i]);
//   BT: the B operand is stored transposed (element (k, j) at B[j * ldb + k]).
// B is scratch owned by the caller: zero beyond K in the k direction up to the next multiple
// of 16 (so a partial chunk adds nothing), and N <= 64 columns are available in it.
//   EPI 0: D = A B over the K range of blockIdx.y (split-K partial: D + y * M * ldd);
//   EPI 1: residual: the tile of R - A B is squared and summed into part[block], and A B is
//          stored into D (ld ldd) when D is not null.
// Workgroup: WGM x WGN waves.
//   SQ (EPI 0, with the whole of N in one tile column, so each element of A is loaded once
//       over the grid): the squares of the A entries the workgroup multiplies are summed into
//       sq[blockIdx.y * gridDim.x + blockIdx.x] (the Frobenius norm of A in the same pass).
template <bool AT, bool BT, int EPI, int WGM, int WGN, int NT = 4, int DEPTH = 2, bool SQ = false>
__global__ void __launch_bounds__(64 * WGM * WGN, NT >= 4 ? 1 : 2)   // two waves per SIMD where they fit
lr_mfma_kernel(int M, int N, int K, int kchunk, const double* __restrict__ A, long long lda,
               const double* __restrict__ B, long long ldb, double* __restrict__ D, long long ldd,
               const double* __restrict__ R, long long ldr, double* __restrict__ part, double* __restrict__ sq) {
    // NT: 16-column MFMA tiles per wave (a wave covers 64 x 16 NT outputs)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int m0 = (blockIdx.x / ((N + 16 * NT * WGN - 1) / (16 * NT * WGN))) * 64 * WGM + wm * 64;
    const int n0 = (blockIdx.x % ((N + 16 * NT * WGN - 1) / (16 * NT * WGN))) * 16 * NT * WGN + wn * 16 * NT;
    const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
    const int lr = lane & 15, lq = lane >> 4;
    f64x4 acc[4][NT];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // Rows of A past M and columns of B past N are read at clamped indices and feed only
    // outputs that are not stored.  Full 8-deep chunks use plain base-plus-offset loads; a
    // final partial chunk clamps k on A and relies on B being zero past K (the caller pads B).
    // DEPTH register buffers: DEPTH - 1 chunks of loads in flight while one is multiplied
    double ra[DEPTH][4][2], rb[DEPTH][NT][2];
    int ic[4], jc[NT];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) ic[mi] = min(m0 + mi * 16 + lr, M - 1);
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) jc[ni] = min(n0 + ni * 16 + lr, N - 1);
    const int kl = kb + 2 * lq;   // this lane group's first k
    auto load = [&](int buf, int koff) {
        const int k = kl + koff;
        if (AT) {
            const double* r0 = A + (long long)k * lda;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                ra[buf][mi][0] = r0[ic[mi]];
                ra[buf][mi][1] = r0[lda + ic[mi]];
            }
        } else {
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                const double* q = A + (long long)ic[mi] * lda + k;
                ra[buf][mi][0] = q[0];
                ra[buf][mi][1] = q[1];
            }
        }
        if (BT) {
#pragma unroll
            for (int ni = 0; ni < NT; ++ni) {
                const double* q = B + (long long)jc[ni] * ldb + k;
                rb[buf][ni][0] = q[0];
                rb[buf][ni][1] = q[1];
            }
        } else {
            const double* r0 = B + (long long)k * ldb;
#pragma unroll
            for (int ni = 0; ni < NT; ++ni) {
                rb[buf][ni][0] = r0[jc[ni]];
                rb[buf][ni][1] = r0[ldb + jc[ni]];
            }
        }
    };
    auto load_tail = [&](int koff) {   // into buffer 0, k clamped on A
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int k = kl + koff + s;
            const int ka = min(k, K - 1);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                ra[0][mi][s] = AT ? A[(long long)ka * lda + ic[mi]] : A[(long long)ic[mi] * lda + ka];
#pragma unroll
            for (int ni = 0; ni < NT; ++ni) rb[0][ni][s] = BT ? B[(long long)jc[ni] * ldb + k] : B[(long long)k * ldb + jc[ni]];
        }
    };
    double ss = 0.0;   // SQ: sum of squares of the A entries of this lane (unclamped only)
    auto mma = [&](int buf, bool tail = false, int koff = 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < NT; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[buf][mi][s], rb[buf][ni][s], acc[mi][ni], 0, 0, 0);
        if (SQ) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) {
                    const bool ok = m0 + mi * 16 + lr < M && (!tail || kl + koff + s < ke);
                    const double x = ra[buf][mi][s];
                    ss = ok ? fma(x, x, ss) : ss;
                }
        }
    };
    const bool live = m0 < M && n0 < N;
    // EPI 1: the tile of R is loaded first, so that its latency hides behind the products
    double rt[4][NT][4];
    if (EPI == 1 && live) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < NT; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = min(m0 + mi * 16 + lq + 4 * r, M - 1), j = jc[ni];
                    rt[mi][ni][r] = R[(long long)i * ldr + j];
                }
    }
    if (live) {
        // full chunks: branch-free steady state (the waits before each MFMA then cover only
        // its own buffer), DEPTH register buffers in rotation: buffer b % DEPTH holds chunk b
        const int nf = (ke - kb) / 8;
        if constexpr (DEPTH == 2) {
            if (nf > 0) load(0, 0);
            int c = 0;
            for (; c + 3 <= nf; c += 2) {
                load(1, (c + 1) * 8);
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                mma(0);
                __builtin_amdgcn_sched_barrier(0);
                load(0, (c + 2) * 8);
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                mma(1);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (c + 2 == nf) {
                load(1, (c + 1) * 8);
                mma(0);
                mma(1);
            } else if (c + 1 == nf) {
                mma(0);
            }
        } else {
#pragma unroll
            for (int b = 0; b + 1 < DEPTH; ++b)
                if (b < nf) load(b, b * 8);
            int c = 0;
            for (; c + 2 * DEPTH - 1 <= nf; c += DEPTH) {
#pragma unroll
                for (int b = 0; b < DEPTH; ++b) {
                    load((b + DEPTH - 1) % DEPTH, (c + b + DEPTH - 1) * 8);
                    asm volatile("" ::: "memory");
                    __builtin_amdgcn_sched_barrier(0);
                    mma(b);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // the last (fewer than 2 DEPTH - 1) chunks, each load only if its chunk exists
#pragma unroll
            for (int t = 0; t < 2 * DEPTH - 2; ++t) {
                if (c + t < nf) {
                    if (c + t + DEPTH - 1 < nf) load((t + DEPTH - 1) % DEPTH, (c + t + DEPTH - 1) * 8);
                    mma(t % DEPTH);
                }
            }
        }
        if ((ke - kb) % 8) {
            load_tail(nf * 8);
            mma(0, true, nf * 8);
        }
    }
    if (EPI == 0) {
        if (SQ) {
            __shared__ double sqs[WGM * WGN];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off);
            if (lane == 0) sqs[wave] = ss;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
                for (int w = 0; w < WGM * WGN; ++w) t += sqs[w];
                sq[(long long)blockIdx.y * gridDim.x + blockIdx.x] = t;
            }
        }
        if (!live) return;
        double* Dp = D + (long long)blockIdx.y * M * ldd;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < NT; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + mi * 16 + lq + 4 * r, j = n0 + ni * 16 + lr;
                    if (i < M && j < N) Dp[(long long)i * ldd + j] = acc[mi][ni][r];
                }
    } else {
        __shared__ double red[64 * WGM * WGN];
        double ss = 0.0;
        if (live) {
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < NT; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = m0 + mi * 16 + lq + 4 * r, j = n0 + ni * 16 + lr;
                        if (i < M && j < N) {
                            const double e = rt[mi][ni][r] - acc[mi][ni][r];
                            ss = fma(e, e, ss);
                            if (D) D[(long long)i * ldd + j] = acc[mi][ni][r];
                        }
                    }
        }
        red[tid] = ss;
        __syncthreads();
        for (int h = 32 * WGM * WGN; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        if (tid == 0) part[blockIdx.x] = red[0];
    }
}

// ---------------------------------------------------------------------------------------
// Gram-Schmidt with column pivoting on T' (n x 64, zero-padded), three launches per step.
// A workgroup owns 64 rows; thread (ty, c) handles column c of rows ty, ty + 4, ...  Every
// workgroup reduces the previous launch's per-workgroup partials itself, in the same fixed
// order, so all of them take the same pivot and stop decisions.
constexpr int CG_ROWS = 64;   // rows per workgroup (at most 256)

// sum over the np per-workgroup partials of column c, four threads per column, fixed order
__device__ inline void cg_reduce(int np, const double* __restrict__ part, double* out /* LDS[64] */,
                                 double* scratch /* LDS[4][64] */) {
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    double s = 0.0;
    int p = q;
    // partials q, q + 4, q + 8, ... summed in that order, eight loads in flight at a time
    for (; p + 28 < np; p += 32) {
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = part[(long long)(p + 4 * i) * LR_MAXK + c];
#pragma unroll
        for (int i = 0; i < 8; ++i) s += v[i];
    }
    for (; p < np; p += 4) s += part[(long long)p * LR_MAXK + c];
    scratch[q * LR_MAXK + c] = s;
    __syncthreads();
    if (q == 0) out[c] = (scratch[c] + scratch[LR_MAXK + c]) + (scratch[2 * LR_MAXK + c] + scratch[3 * LR_MAXK + c]);
    __syncthreads();
}

// the partial column sums of this workgroup's rows: v(r, c) summed over its 64 rows
template <typename F>
__device__ inline void cg_partial(int n, F v, double* __restrict__ part, double* scratch) {
    const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int r0 = blockIdx.x * CG_ROWS;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < CG_ROWS / 4; ++t) {
        const int r = r0 + ty + 4 * t;
        if (r < n) acc += v(r, c);
    }
    scratch[ty * LR_MAXK + c] = acc;
    __syncthreads();
    if (ty == 0)
        part[(long long)blockIdx.x * LR_MAXK + c] =
            (scratch[c] + scratch[LR_MAXK + c]) + (scratch[2 * LR_MAXK + c] + scratch[3 * LR_MAXK + c]);
}

// squared column norms (all columns) of the starting matrix
__global__ void __launch_bounds__(256) cg_norms0_kernel(int n, const double* __restrict__ T, double* __restrict__ part) {
    __shared__ double scr[4 * LR_MAXK];
    cg_partial(n, [&](int r, int c) { const double v = T[(long long)r * LR_MAXK + c]; return v * v; }, part, scr);
}

// step k, part 1: pivot choice and stop test (from the norm partials), column swap and
// scaling of this workgroup's rows, first-pass dot partials of column k with columns > k.
__global__ void __launch_bounds__(256) cg_step_a_kernel(int n, int np, int k, int kmax, double* __restrict__ T,
                                                        const double* __restrict__ pnorm, const double* __restrict__ anorm2,
                                                        double tau, int* __restrict__ perm, LrState* __restrict__ st,
                                                        double* __restrict__ pdot) {
    if (st->done) return;
    __shared__ double nrm[LR_MAXK];
    __shared__ double scr[4 * LR_MAXK];
    __shared__ int piv;
    __shared__ int stop;
    cg_reduce(np, pnorm, nrm, scr);
    if (threadIdx.x == 0) {
        double tail2 = 0.0;
        for (int j = k; j < kmax; ++j) tail2 += nrm[j];
        const double thr = tau * sqrt(anorm2[0]);
        stop = (k >= kmax || sqrt(tail2) <= thr || !(tail2 > 0.0)) ? 1 : 0;
        int p = k;
        if (!stop)
            for (int j = k + 1; j < kmax; ++j)
                if (nrm[j] > nrm[p]) p = j;
        piv = p;
        if (blockIdx.x == 0) {
            if (stop) {
                st->done = 1;
                st->rank = k;
                st->tail = (k >= kmax) ? 0.0 : sqrt(tail2);
            } else {
                st->p = p;
                const int t = perm[k];
                perm[k] = perm[p];
                perm[p] = t;
            }
        }
    }
    __syncthreads();
    if (stop) return;
    const int p = piv;
    const double scale = 1.0 / sqrt(nrm[p]);
    // swap and scale this workgroup's rows (one thread per row)
    const int r = blockIdx.x * CG_ROWS + threadIdx.x;
    if (threadIdx.x < CG_ROWS && r < n) {
        double* row = T + (long long)r * LR_MAXK;
        const double a = row[p], b = row[k];
        row[k] = a * scale;
        if (p != k) row[p] = b;
    }
    __syncthreads();
    cg_partial(n, [&](int rr, int c) {
        const double* row = T + (long long)rr * LR_MAXK;
        return (c > k && c < kmax) ? row[k] * row[c] : 0.0;
    }, pdot, scr);
}

// step k, projection pass: coefficients from the dot partials, update of this workgroup's
// rows, then either the next pass's dot partials (NORMS false) or the squared norms of the
// remaining columns for step k + 1 (NORMS true).
template <bool NORMS>
__global__ void __launch_bounds__(256) cg_step_b_kernel(int n, int np, int k, int kmax, double* __restrict__ T,
                                                        const double* __restrict__ pdot, const LrState* __restrict__ st,
                                                        double* __restrict__ pout) {
    if (st->done) return;
    __shared__ double d[LR_MAXK];
    __shared__ double scr[4 * LR_MAXK];
    cg_reduce(np, pdot, d, scr);
    const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (c > k && c < kmax) {
        const double dc = d[c];
        const int r0 = blockIdx.x * CG_ROWS;
#pragma unroll
        for (int t = 0; t < CG_ROWS / 4; ++t) {
            const int r = r0 + ty + 4 * t;
            if (r < n) {
                double* row = T + (long long)r * LR_MAXK;
                row[c] = fma(-row[k], dc, row[c]);
            }
        }
    }
    __syncthreads();
    cg_partial(n, [&](int rr, int cc) {
        const double* row = T + (long long)rr * LR_MAXK;
        if (NORMS) return (cc > k && cc < kmax) ? row[cc] * row[cc] : 0.0;
        return (cc > k && cc < kmax) ? row[k] * row[cc] : 0.0;
    }, pout, scr);
}

// columns >= rank set to zero (so that W = A T and W T^T only see the basis)
__global__ void cg_zero_tail_kernel(int n, double* __restrict__ T, const LrState* __restrict__ st) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * LR_MAXK) return;
    if ((int)(e % LR_MAXK) >= st->rank) T[e] = 0.0;
}

// dst (rows x cols, ldd) = src (rows x cols of a 64-column array)
__global__ void copy_cols_kernel(int rows, int cols, const double* __restrict__ src, double* __restrict__ dst,
                                 long long ldd) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const int i = (int)(e / cols), j = (int)(e % cols);
    dst[(long long)i * ldd + j] = src[(long long)i * LR_MAXK + j];
}

// dst (rows x 64) = src (rows x cols, lds) padded with zero columns
__global__ void pad_cols_kernel(int rows, int cols, const double* __restrict__ src, long long lds,
                                double* __restrict__ dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * LR_MAXK) return;
    const int i = (int)(e / LR_MAXK), j = (int)(e % LR_MAXK);
    dst[e] = (j < cols) ? src[(long long)i * lds + j] : 0.0;
}

__global__ void lr_init_kernel(int k, int* perm, LrState* st) {
    const int c = threadIdx.x;
    if (c < k) perm[c] = c;
    if (c == 0) {
        st->done = 0;
        st->rank = 0;
        st->p = 0;
        st->scale = 1.0;
        st->tail = 0.0;
    }
}

// D (M x 64, ld 64) = op(A) (M x K) * B (K x 64, ld 64) on the matrix cores, split over K so that
// about 1024 workgroups run; partials in `part` (ks x M x 64), then their fixed-order sum.
// With sq (AT only): the sum of squares of A's entries in *nsq per-workgroup partials at sq
// (at most 16 ceil(M / 256)).
template <bool AT>
hipError_t skinny_mfma(int M, int K, int N, const double* A, long long lda, const double* B, double* D, double* part,
                       long long part_cap, hipStream_t s, double* sq = nullptr, int* nsq = nullptr) {
    // N <= 64 columns of B and D (ld 64) in 16-column MFMA tiles
    const int tiles = (M + 255) / 256;
    long long ks = std::max(1, std::min(16, (1024 + tiles - 1) / tiles));
    ks = std::min<long long>(ks, std::max(1, K / 512));
    ks = std::max<long long>(1, std::min<long long>(ks, part_cap / ((long long)M * LR_MAXK)));
    int kchunk = (int)((K + ks - 1) / ks);
    kchunk = (kchunk + 15) / 16 * 16;
    ks = (K + kchunk - 1) / kchunk;
    const int nt = (N + 15) / 16;
#define LR_SKINNY(NTV)                                                                                              \
    if (AT && sq)                                                                                                   \
        hipLaunchKernelGGL((lr_mfma_kernel<AT, false, 0, 4, 1, NTV, (NTV <= 2 ? 4 : 2), true>),                     \
                           dim3(tiles, (unsigned)ks), dim3(256), 0, s, M, N, K, kchunk, A, lda, B, (long long)LR_MAXK, \
                           part, (long long)LR_MAXK, (const double*)nullptr, 0LL, (double*)nullptr, sq);            \
    else                                                                                                            \
        hipLaunchKernelGGL((lr_mfma_kernel<AT, false, 0, 4, 1, NTV, (NTV <= 2 ? 4 : 2)>), dim3(tiles, (unsigned)ks), \
                           dim3(256), 0, s, M, N, K, kchunk, A, lda, B, (long long)LR_MAXK, part, (long long)LR_MAXK, \
                           (const double*)nullptr, 0LL, (double*)nullptr, (double*)nullptr)
    switch (nt) {
        case 1: LR_SKINNY(1); break;
        case 2: LR_SKINNY(2); break;
        case 3: LR_SKINNY(3); break;
        default: LR_SKINNY(4); break;
    }
#undef LR_SKINNY
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nsq) *nsq = tiles * (int)ks;
    return launch_splitk_reduce_f64(M, N, (int)ks, part, LR_MAXK, (long long)M * LR_MAXK, 1.0, 0.0, nullptr, 0, D,
                                    LR_MAXK, s);
}

// ---------------------------------------------------------------------------------------
// Numerical rank without pivoting or orthogonalization (Proto-Algorithm B.1): bisection over
// s (Remark B.4) on the conditioning of B_s = A^T G_s, the first s columns of the sketch.
// COND (Remark B.2): Lanczos on the leading s x s block of the Gram matrix S = B^T B, no
// reorthogonalization, 6 s steps; the extreme eigenvalues of the tridiagonal by multisection
// on Sturm counts (64 trial points per round, one per lane); kappa_2 = sqrt(lmax / lmin).
// One wave does everything: lane i holds component i of the Lanczos vectors.
constexpr int NR_STEPS = 6;                       // Lanczos steps per column
constexpr int NR_MAXT = NR_STEPS * LR_MAXK;       // tridiagonal order

struct NrOut {
    int rank, tests;
    double cond_at_rank, cond_above;
};

// Sum over the 64 lanes (all active) with DPP moves, the same in every lane: shifts by 1, 2, 4, 8
// inside each row of 16 lanes (a lane with no source adds 0) leave each row's sum in its lane
// 15; the row broadcasts of lanes 15 and 31 then carry the totals into lane 63, which is read.
template <int CTRL, int ROWS>
__device__ inline double dpp_or_zero(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double wave_sum64(double v) {
    v += dpp_or_zero<0x111, 0xf>(v);
    v += dpp_or_zero<0x112, 0xf>(v);
    v += dpp_or_zero<0x114, 0xf>(v);
    v += dpp_or_zero<0x118, 0xf>(v);
    v += dpp_or_zero<0x142, 0xa>(v);
    v += dpp_or_zero<0x143, 0xc>(v);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// eigenvalues < x of the tridiagonal (al[0..k), be[0..k-1)) from the pivots of T - x I
__device__ int nr_sturm(const double* al, const double* be, int k, double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
        d = (al[i] - x) - (i ? be[i - 1] * be[i - 1] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        cnt += d < 0.0;
    }
    return cnt;
}

// the target-th smallest eigenvalue (target 1 or k) by multisection in [lo, hi]
__device__ double nr_eig(const double* al, const double* be, int k, int target, double lo, double hi) {
    const int lane = threadIdx.x;
    for (int round = 0; round < 16; ++round) {
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const bool ge = nr_sturm(al, be, k, x) >= target;
        const unsigned long long m = __ballot(ge);
        const int first = m ? __ffsll((long long)m) - 1 : 64;   // first trial point at or past the eigenvalue
        const double nlo = lo + (hi - lo) * (double)first / 65.0;
        const double nhi = (first < 64) ? lo + (hi - lo) * (double)(first + 1) / 65.0 : hi;
        if (!(nhi - nlo < hi - lo)) break;
        lo = nlo;
        hi = nhi;
    }
    return 0.5 * (lo + hi);
}

__global__ void __launch_bounds__(64) nr_search_kernel(int lo, int hi, const double* __restrict__ S,
                                                       const double* __restrict__ v0src, double cond_max,
                                                       NrOut* __restrict__ out) {
    __shared__ double Ss[LR_MAXK][LR_MAXK + 1];
    __shared__ double vs[LR_MAXK];
    __shared__ double al[NR_MAXT], be[NR_MAXT];
    const int lane = threadIdx.x;
    for (int e = lane; e < LR_MAXK * LR_MAXK; e += 64) Ss[e / LR_MAXK][e % LR_MAXK] = S[e];
    __syncthreads();
    // this lane's row of the Gram matrix in registers for all tests: the Lanczos vector is zero
    // past s, so the product over all 64 columns equals the product with the leading s x s block
    // (only the leading hi x hi block of S is defined: the rest is read as zero)
    double srow[LR_MAXK];
#pragma unroll
    for (int j = 0; j < LR_MAXK; ++j) srow[j] = (j < hi && lane < hi) ? Ss[lane][j] : 0.0;
    int tests = 0;
    double cond_rank = -1.0, cond_above = -1.0;   // -1: not tested
    while (lo < hi) {
        const int s = (lo + hi + 1) / 2;
        // Lanczos on S_s from the first s entries of the multiplier's first column
        const bool on = lane < s;
        double v = on ? v0src[(long long)lane * LR_MAXK] : 0.0;
        v /= sqrt(wave_sum64(v * v));
        double vp = 0.0, b = 0.0;
        int k = 0;
        for (; k < NR_STEPS * s; ++k) {
            vs[lane] = v;
            __syncthreads();
            // four independent partial sums over the 64 columns (v is zero past s)
            double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int j = 0; j < LR_MAXK; ++j) w4[j & 3] = fma(srow[j], vs[j], w4[j & 3]);
            double w = on ? (w4[0] + w4[1]) + (w4[2] + w4[3]) : 0.0;
            __syncthreads();
            w -= b * vp;
            const double a = wave_sum64(v * w);
            w -= a * v;
            al[k] = a;   // every lane writes the same value
            b = sqrt(wave_sum64(w * w));
            if (!(b > 1e-300)) {
                ++k;
                break;
            }
            be[k] = b;
            vp = v;
            v = w / b;
        }
        __syncthreads();
        // Gershgorin interval, then the extreme eigenvalues
        double glo = 1e300, ghi = -1e300;
        for (int i = 0; i < k; ++i) {
            const double r = (i ? fabs(be[i - 1]) : 0.0) + (i + 1 < k ? fabs(be[i]) : 0.0);
            glo = fmin(glo, al[i] - r);
            ghi = fmax(ghi, al[i] + r);
        }
        const double lmin = nr_eig(al, be, k, 1, glo, ghi);
        const double lmax = nr_eig(al, be, k, k, glo, ghi);
        const double kap = (lmin > 0.0) ? sqrt(lmax / lmin) : __builtin_inf();
        const bool ok = kap <= cond_max;
        ++tests;
        if (ok) {
            lo = s;
            cond_rank = kap;
        } else {
            hi = s - 1;
            cond_above = kap;
        }
        __syncthreads();
    }
    if (lane == 0) {
        out->rank = lo;
        out->tests = tests;
        out->cond_at_rank = cond_rank;
        out->cond_above = cond_above;
    }
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) hipFree(p);
    }
    template <typename X>
    bool get(X** p, size_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(X)) != hipSuccess) return false;
        ptrs.push_back(q);
        *p = (X*)q;
        return true;
    }
};

}  // namespace

#define LR_HIP(x)                                              \
    do {                                                       \
        if ((x) != hipSuccess) return GENP_EDEVICE;            \
    } while (0)

extern "C" int genp_lowrank(const double* A, int64_t m, int64_t n, int64_t lda, int mult, const double* G,
                            int64_t ldg, int64_t rho_plus, double tau, double tau2, double* T, int64_t ldt,
                            double* W, int64_t ldw, double* Ahat, int64_t ldah, int32_t* perm_out,
                            genp_lr_info* info, void* stream) {
    if (!A || !G || !T || !W || !info || m < 1 || n < 1 || lda < n || rho_plus < 1 || rho_plus > LR_MAXK ||
        rho_plus > std::min(m, n) || ldt < rho_plus || ldw < rho_plus || (Ahat && ldah < n) || !(tau >= 0.0) ||
        !(tau2 >= 0.0) || m > (int64_t)1 << 30 || n > (int64_t)1 << 30)
        return GENP_EINVAL;
    if (mult != GENP_G_DENSE && mult != GENP_G_TOEPLITZ) return GENP_ENOTSUP;
    if (mult == GENP_G_DENSE && ldg < rho_plus) return GENP_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return GENP_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int M = (int)m, N = (int)n, K = (int)rho_plus;
    Scratch sc;
    double *G64 = nullptr, *T64 = nullptr, *W64 = nullptr, *part = nullptr, *cpart = nullptr, *rpart = nullptr,
           *scal = nullptr, *Gx = nullptr;
    int* perm = nullptr;
    LrState* st = nullptr;
    const long long part_cap = 16LL * std::max(M, N) * LR_MAXK;
    const int np = (N + CG_ROWS - 1) / CG_ROWS;
    const int rt_m = (M + 127) / 128, rt_n = (N + 63) / 64;   // residual: 128 x 64 workgroup tiles
    const long long nres = (long long)rt_m * rt_n;
    const long long nsq = 16LL * ((N + 255) / 256);   // sum-of-squares partials of the sketch
    // G64 and T64 are B operands: rows padded with zeros to a multiple of 16
    const size_t Mp = ((size_t)M + 15) / 16 * 16, Np = ((size_t)N + 15) / 16 * 16;
    if (!sc.get(&G64, Mp * LR_MAXK) || !sc.get(&T64, Np * LR_MAXK) || !sc.get(&W64, (size_t)M * LR_MAXK) ||
        !sc.get(&part, part_cap) || !sc.get(&cpart, (size_t)3 * np * LR_MAXK) ||
        !sc.get(&rpart, std::max<long long>(nres, nsq)) || !sc.get(&scal, 2) || !sc.get(&perm, LR_MAXK) ||
        !sc.get(&st, 1))
        return GENP_ENOMEM;
    if (mult == GENP_G_TOEPLITZ && !sc.get(&Gx, (size_t)M * K)) return GENP_ENOMEM;
    double* pn = cpart;                    // norm partials
    double* pd1 = cpart + np * LR_MAXK;    // dot partials, pass 1
    double* pd2 = cpart + 2 * np * LR_MAXK;
    hipEvent_t ev[5];
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return GENP_EDEVICE;
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int i = 0; i < 5; ++i) hipEventDestroy(e[i]);
        }
    } eg{ev};
    auto blocks = [](long long tot) { return dim3((unsigned)((tot + 255) / 256)); };
    LR_HIP(hipEventRecord(ev[0], s));
    // Stage 1: T' = A^T G (64 columns, zero beyond rho_+), and ||A||_F^2 from the same pass
    const double* Gs = G;
    long long ldgs = ldg;
    if (mult == GENP_G_TOEPLITZ) {
        hipLaunchKernelGGL(toeplitz_expand_kernel, blocks((long long)M * K), dim3(256), 0, s, M, K, G, Gx);
        Gs = Gx;
        ldgs = K;
    }
    LR_HIP(hipMemsetAsync(G64, 0, Mp * LR_MAXK * sizeof(double), s));
    hipLaunchKernelGGL(pad_cols_kernel, blocks((long long)M * LR_MAXK), dim3(256), 0, s, M, K, Gs, ldgs, G64);
    LR_HIP(hipMemsetAsync(T64, 0, Np * LR_MAXK * sizeof(double), s));
    LR_HIP(hipMemsetAsync(W64, 0, (size_t)M * LR_MAXK * sizeof(double), s));
    int nsqp = 0;
    LR_HIP(skinny_mfma<true>(N, M, K, A, lda, G64, T64, part, part_cap, s, rpart, &nsqp));
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, nsqp, rpart, scal);
    LR_HIP(hipEventRecord(ev[1], s));
    // Stage 2: pivoted Gram-Schmidt, each projection applied twice
    hipLaunchKernelGGL(lr_init_kernel, dim3(1), dim3(LR_MAXK), 0, s, K, perm, st);
    hipLaunchKernelGGL(cg_norms0_kernel, dim3(np), dim3(256), 0, s, N, T64, pn);
    for (int k = 0; k <= K; ++k) {
        hipLaunchKernelGGL(cg_step_a_kernel, dim3(np), dim3(256), 0, s, N, np, k, K, T64, pn, scal, tau, perm, st, pd1);
        if (k == K) break;
        hipLaunchKernelGGL((cg_step_b_kernel<false>), dim3(np), dim3(256), 0, s, N, np, k, K, T64, pd1, st, pd2);
        hipLaunchKernelGGL((cg_step_b_kernel<true>), dim3(np), dim3(256), 0, s, N, np, k, K, T64, pd2, st, pn);
    }
    hipLaunchKernelGGL(cg_zero_tail_kernel, blocks((long long)N * LR_MAXK), dim3(256), 0, s, N, T64, st);
    LR_HIP(hipGetLastError());
    LR_HIP(hipEventRecord(ev[2], s));
    // the rank sizes Stage 3's products: one wait for the stream here
    LrState hs0;
    LR_HIP(hipMemcpyAsync(&hs0, st, sizeof hs0, hipMemcpyDeviceToHost, s));
    LR_HIP(hipStreamSynchronize(s));
    const int rk = hs0.rank;
    const int kres = std::max(8, (rk + 7) / 8 * 8);   // columns beyond the rank are zero
    // Stage 3: W = A T, then ||A - W T^T||_F (and A_hat)
    if (rk > 0) LR_HIP(skinny_mfma<false>(M, N, rk, A, lda, T64, W64, part, part_cap, s));
    LR_HIP(hipEventRecord(ev[3], s));
    {
        const int ntn = (N + 63) / 64;
        const unsigned g = (unsigned)((long long)((M + 127) / 128) * ntn);
        hipLaunchKernelGGL((lr_mfma_kernel<false, true, 1, 2, 2, 2>), dim3(g, 1), dim3(256), 0, s, M, N, kres, kres, W64,
                           (long long)LR_MAXK, T64, (long long)LR_MAXK, Ahat, (long long)ldah, A, (long long)lda, rpart,
                           (double*)nullptr);
    }
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, (int)nres, rpart, scal + 1);   // nres = rt_m * rt_n
    hipLaunchKernelGGL(copy_cols_kernel, blocks((long long)N * K), dim3(256), 0, s, N, K, T64, T, (long long)ldt);
    hipLaunchKernelGGL(copy_cols_kernel, blocks((long long)M * K), dim3(256), 0, s, M, K, W64, W, (long long)ldw);
    LR_HIP(hipGetLastError());
    LR_HIP(hipEventRecord(ev[4], s));
    LrState hs;
    double hsc[2];
    int32_t hp[LR_MAXK];
    LR_HIP(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s));
    LR_HIP(hipMemcpyAsync(hsc, scal, sizeof hsc, hipMemcpyDeviceToHost, s));
    LR_HIP(hipMemcpyAsync(hp, perm, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s));
    LR_HIP(hipStreamSynchronize(s));
    *info = genp_lr_info{};
    info->m = m;
    info->n = n;
    info->rho_plus = rho_plus;
    info->rank = hs.rank;
    info->a_fro = sqrt(hsc[0]);
    info->tail_fro = hs.tail;
    info->resid_fro = sqrt(hsc[1]);
    info->failed = !(info->resid_fro <= tau2 * info->a_fro);
    float ms = 0.f;
    double* slots[4] = {&info->ms_sketch, &info->ms_basis, &info->ms_project, &info->ms_resid};
    for (int i = 0; i < 4; ++i)
        if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) *slots[i] = ms;
    if (hipEventElapsedTime(&ms, ev[0], ev[4]) == hipSuccess) info->ms_total = ms;
    if (perm_out)
        for (int i = 0; i < K; ++i) perm_out[i] = hp[i];
    return GENP_OK;
}

namespace {

// Scratch of one numerical-rank call: the padded multiplier and sketch (rows to a multiple of
// 16, 64 columns), the Gram matrix, the split-K partials and the result record.
struct NrBufs {
    double* G64;
    double* T64;
    double* Sg;
    double* part;
    long long part_cap;
    NrOut* od;
};

int nrank_args_ok(const double* A, int64_t m, int64_t n, int64_t lda, const double* G, int64_t ldg,
                  int64_t rho_minus, int64_t rho_plus, double cond_max, const double* B, int64_t ldb,
                  const genp_nrank_info* info) {
    return A && G && B && info && m >= 1 && n >= 1 && lda >= n && rho_minus >= 0 && rho_plus > rho_minus &&
           rho_plus <= LR_MAXK && rho_plus <= std::min(m, n) && ldg >= rho_plus && ldb >= rho_plus &&
           cond_max >= 1.0 && m <= (int64_t)1 << 30 && n <= (int64_t)1 << 30;
}

int gfx950_current() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return -1;
    return dev;
}

// The steps of genp_numerical_rank on the given scratch: B = A^T G (split over K), S = B^T B,
// the bisection with COND on the device, the copy of B out; one wait at the end.  ev: four
// events for the stage times, or null (times reported as NaN).
int nrank_core(const double* A, int64_t m, int64_t n, int64_t lda, const double* G, int64_t ldg, int64_t rho_minus,
               int64_t rho_plus, double cond_max, double* B, int64_t ldb, genp_nrank_info* info, hipStream_t s,
               const NrBufs& b, hipEvent_t* ev) {
    const int M = (int)m, N = (int)n, K = (int)rho_plus;
    const int Mp = (M + 15) / 16 * 16, Np = (N + 15) / 16 * 16;
    auto blocks = [](long long tot) { return dim3((unsigned)((tot + 255) / 256)); };
    if (ev) LR_HIP(hipEventRecord(ev[0], s));
    // zero padding by kernels (also safe where a caller captures the stream into a graph)
    LR_HIP(launch_fill2d(0.0, b.G64, LR_MAXK, Mp, LR_MAXK, s));
    LR_HIP(launch_fill2d(0.0, b.T64, LR_MAXK, Np, LR_MAXK, s));
    LR_HIP(launch_fill2d(0.0, b.Sg, LR_MAXK, LR_MAXK, LR_MAXK, s));
    hipLaunchKernelGGL(pad_cols_kernel, blocks((long long)M * LR_MAXK), dim3(256), 0, s, M, K, G, (long long)ldg,
                       b.G64);
    LR_HIP(skinny_mfma<true>(N, M, K, A, lda, b.G64, b.T64, b.part, b.part_cap, s));        // B = A^T G
    if (ev) LR_HIP(hipEventRecord(ev[1], s));
    LR_HIP(skinny_mfma<true>(K, N, K, b.T64, LR_MAXK, b.T64, b.Sg, b.part, b.part_cap, s));   // S = B^T B
    if (ev) LR_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL(nr_search_kernel, dim3(1), dim3(64), 0, s, (int)rho_minus, K, b.Sg, b.G64, cond_max, b.od);
    hipLaunchKernelGGL(copy_cols_kernel, blocks((long long)N * K), dim3(256), 0, s, N, K, b.T64, B, (long long)ldb);
    LR_HIP(hipGetLastError());
    if (ev) LR_HIP(hipEventRecord(ev[3], s));
    NrOut ho;
    LR_HIP(hipMemcpyAsync(&ho, b.od, sizeof ho, hipMemcpyDeviceToHost, s));
    LR_HIP(hipStreamSynchronize(s));
    *info = genp_nrank_info{};
    info->m = m;
    info->n = n;
    info->rho_minus = rho_minus;
    info->rho_plus = rho_plus;
    info->rank = ho.rank;
    info->tests = ho.tests;
    const double nan = __builtin_nan("");
    info->cond_at_rank = ho.cond_at_rank < 0 ? nan : ho.cond_at_rank;
    info->cond_above = ho.cond_above < 0 ? nan : ho.cond_above;
    double* slots[3] = {&info->ms_sketch, &info->ms_gram, &info->ms_search};
    info->ms_total = nan;
    for (int i = 0; i < 3; ++i) *slots[i] = nan;
    if (ev) {
        float ms = 0.f;
        for (int i = 0; i < 3; ++i)
            if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) *slots[i] = ms;
        if (hipEventElapsedTime(&ms, ev[0], ev[3]) == hipSuccess) info->ms_total = ms;
    }
    return GENP_OK;
}

}  // namespace

extern "C" int genp_numerical_rank(const double* A, int64_t m, int64_t n, int64_t lda, const double* G, int64_t ldg,
                                   int64_t rho_minus, int64_t rho_plus, double cond_max, double* B, int64_t ldb,
                                   genp_nrank_info* info, void* stream) {
    if (!nrank_args_ok(A, m, n, lda, G, ldg, rho_minus, rho_plus, cond_max, B, ldb, info)) return GENP_EINVAL;
    if (gfx950_current() < 0) return GENP_EDEVICE;
    const int M = (int)m, N = (int)n;
    const size_t Mp = ((size_t)M + 15) / 16 * 16, Np = ((size_t)N + 15) / 16 * 16;
    Scratch sc;
    NrBufs b{};
    b.part_cap = 16LL * std::max(M, N) * LR_MAXK;
    if (!sc.get(&b.G64, Mp * LR_MAXK) || !sc.get(&b.T64, Np * LR_MAXK) || !sc.get(&b.Sg, (size_t)LR_MAXK * LR_MAXK) ||
        !sc.get(&b.part, b.part_cap) || !sc.get(&b.od, 1))
        return GENP_ENOMEM;
    hipEvent_t ev[4];
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return GENP_EDEVICE;
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int i = 0; i < 4; ++i) hipEventDestroy(e[i]);
        }
    } eg{ev};
    return nrank_core(A, m, n, lda, G, ldg, rho_minus, rho_plus, cond_max, B, ldb, info, (hipStream_t)stream, b, ev);
}

// ---------------------------------------------------------------------------------------
// Allocation-free numerical rank: the scratch of genp_numerical_rank taken from one fixed
// device array instead of hipMalloc.  In host code the array's name is only a stand-in for the
// symbol; its device address (one per GPU) comes from hipGetSymbolAddress on the first call
// with that GPU current, and only that address is handed to kernels.

namespace {

constexpr size_t NR_SCRATCH_BYTES = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int NR_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[NR_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_dev[NR_MAX_DEVICES] = {};

// The device address of `scratch` on device dev (current), looked up once per device.
void* scratch_on(int dev) {
    if (dev < 0 || dev >= NR_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_dev[dev] = p;
    }
    return g_scratch_dev[dev];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" int genp_numerical_rank_noalloc(const double* A, int64_t m, int64_t n, int64_t lda, const double* G,
                                           int64_t ldg, int64_t rho_minus, int64_t rho_plus, double cond_max,
                                           double* B, int64_t ldb, genp_nrank_info* info, void* stream) {
    if (!nrank_args_ok(A, m, n, lda, G, ldg, rho_minus, rho_plus, cond_max, B, ldb, info)) return GENP_EINVAL;
    const int M = (int)m, N = (int)n;
    const size_t Mp = ((size_t)M + 15) / 16 * 16, Np = ((size_t)N + 15) / 16 * 16;
    // fixed parts, then the split-K partials (at least one slice of the sketch: N x 64, and of
    // the Gram matrix: 64 x 64) in what is left
    const size_t fixed = align256(Mp * LR_MAXK * sizeof(double)) + align256(Np * LR_MAXK * sizeof(double)) +
                         align256((size_t)LR_MAXK * LR_MAXK * sizeof(double)) + align256(sizeof(NrOut));
    const size_t part_min = (size_t)std::max(N, LR_MAXK) * LR_MAXK * sizeof(double);
    if (fixed + part_min > NR_SCRATCH_BYTES) return GENP_ESCRATCH;
    const int dev = gfx950_current();
    if (dev < 0) return GENP_EDEVICE;
    unsigned char* base = (unsigned char*)scratch_on(dev);
    if (!base) return GENP_EDEVICE;
    NrBufs b{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        void* p = base + off;
        off += align256(bytes);
        return p;
    };
    b.G64 = (double*)carve(Mp * LR_MAXK * sizeof(double));
    b.T64 = (double*)carve(Np * LR_MAXK * sizeof(double));
    b.Sg = (double*)carve((size_t)LR_MAXK * LR_MAXK * sizeof(double));
    b.od = (NrOut*)carve(sizeof(NrOut));
    b.part = (double*)(base + off);
    // as many partial slices as genp_numerical_rank would use, if they fit
    b.part_cap = std::min<long long>(16LL * std::max(M, N) * LR_MAXK,
                                     (long long)((NR_SCRATCH_BYTES - off) / sizeof(double)));
    return nrank_core(A, m, n, lda, G, ldg, rho_minus, rho_plus, cond_max, B, ldb, info, (hipStream_t)stream, b,
                      nullptr);
}
