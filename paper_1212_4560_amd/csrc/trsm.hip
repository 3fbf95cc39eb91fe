// Triangular solves by substitution (no
// explicit inverse): the two block solves of each elimination step,
// L21 = A21 U11^{-1} and U12 = L11^{-1} A12, and the diagonal-block solves of
// the substitutions Y = U^{-1} L^{-1} B and of the adjoint (U^T, L^T).
//
// Every case is a left solve T X = B with an nb x nb triangular T and the
// right-hand sides as the columns of X (right solves X U = B become
// U^T X^T = B^T, both operands accessed transposed).  Substitution keeps the
// backward error of the block solves at the level of the elimination itself;
// multiplying by a computed inverse would add a factor of the block's
// condition number.
//
// trsm_cols_kernel (many right-hand sides): a workgroup owns 16 columns of X;
// thread (c, g) keeps rows 16g..16g+15 of column c in registers.  T is swept
// in 16 x 16 blocks: the owner group solves its diagonal block thread-locally,
// publishes the 16 values through LDS, and the groups below (above) subtract
// the off-diagonal block times them.  One LDS stage of a 16-column strip of T
// and two barriers per 16 rows; the footprint (256 threads, 37 KB LDS) lets it
// run beside a Schur-GEMM workgroup.
//
// panel_trsm_kernel (the two block solves of an elimination step, one launch):
// lower-triangular solves T Y = Z, 16 x 16 blocks, right-looking.  A wave owns
// 16 right-hand sides and keeps all NB / 16 of its 16 x 16 tiles of Y in MFMA
// accumulators; the diagonal block is solved by substitution (one lane per
// right-hand side), the update of the blocks below by v_mfma_f64_16x16x4_f64.
//
// trsv_step_kernel (1..4 right-hand sides, one launch per block), trsv_chain_kernel
// (1..4, the whole triangle in one launch) and trsm_chain_kernel (5..64, the whole
// triangle in one launch, MFMA block products): see below.
#include "common.h"

#include <type_traits>

namespace {

constexpr int MAXNB = 256;
constexpr int SB = 16;       // sub-block of the sweep and columns per workgroup

template <bool TT>
__device__ inline long long tat(int r, int c, long long ld) {
    return TT ? (long long)c * ld + r : (long long)r * ld + c;
}

template <bool LOWER, bool UNIT, bool TT, bool XT, typename TF, typename TX>
__global__ void __launch_bounds__(256)
trsm_cols_kernel(const TF* __restrict__ T, long long ldt, int nb, TX* X, long long ldx, int ncols) {
    __shared__ double Ts[MAXNB][SB + 1];   // strip of T: all rows, 32 columns
    __shared__ double Xs[SB][SB + 1];      // the 32 solved rows of the current block
    const int tid = threadIdx.x;
    const int c = tid % SB, g = tid / SB;  // column within the workgroup, row group
    const int ng = nb / SB;
    const int col = blockIdx.x * SB + c;
    const bool act = g < ng && col < ncols;
    auto xat = [&](int r) -> long long {
        return XT ? (long long)col * ldx + r : (long long)r * ldx + col;
    };
    double x[SB];
#pragma unroll
    for (int i = 0; i < SB; ++i) x[i] = act ? (double)X[xat(g * SB + i)] : 0.0;

    for (int s = 0; s < ng; ++s) {
        const int ib = LOWER ? s : ng - 1 - s;
        const int c0 = ib * SB;
        // rows of the strip that are used: the diagonal block and the rows still to update
        const int r_lo = LOWER ? c0 : 0, r_hi = LOWER ? nb : c0 + SB;
        __syncthreads();
        {
            // at most MAXNB * SB / 256 = 16 elements per thread: issue every load first
            const int nrow = r_hi - r_lo;
            double v[MAXNB * SB / 256];
#pragma unroll
            for (int q = 0; q < MAXNB * SB / 256; ++q) {
                const int e = tid + q * 256;
                int r, t;
                if (TT) { t = e / nrow; r = r_lo + e % nrow; }
                else { r = r_lo + e / SB; t = e % SB; }
                v[q] = (e < nrow * SB) ? (double)T[tat<TT>(r, c0 + t, ldt)] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < MAXNB * SB / 256; ++q) {
                const int e = tid + q * 256;
                int r, t;
                if (TT) { t = e / nrow; r = r_lo + e % nrow; }
                else { r = r_lo + e / SB; t = e % SB; }
                if (e < nrow * SB) Ts[r][t] = v[q];
            }
        }
        __syncthreads();
        if (g == ib && act) {
            // x <- T_bb^{-1} x, thread-local column sweep (critical path SB FMAs)
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int t = LOWER ? u : SB - 1 - u;
                if (!UNIT) x[t] /= Ts[c0 + t][t];
#pragma unroll
                for (int w = 0; w < SB; ++w) {
                    if (LOWER ? (w > t) : (w < t)) x[w] = fma(-Ts[c0 + w][t], x[t], x[w]);
                }
            }
        }
        if (g == ib) {
#pragma unroll
            for (int i = 0; i < SB; ++i) Xs[i][c] = x[i];
        }
        __syncthreads();
        if (act && (LOWER ? g > ib : g < ib)) {
            double xb[SB];
#pragma unroll
            for (int t = 0; t < SB; ++t) xb[t] = Xs[t][c];
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                double v = x[i];
                const double* trow = &Ts[g * SB + i][0];
#pragma unroll
                for (int t = 0; t < SB; ++t) v = fma(-trow[t], xb[t], v);
                x[i] = v;
            }
        }
    }
    if (act) {
#pragma unroll
        for (int i = 0; i < SB; ++i) X[xat(g * SB + i)] = (TX)x[i];
    }
}

__device__ inline double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lower-triangular solve T Y = Z by 16 x 16 blocks, T = L (unit, TT = false) or U^T
// (TT = true, T(i, k) = U[k][i]).  Y(i, c): XT = false -> X[i * ldx + c] (the columns
// of X are the right-hand sides), XT = true -> X[c * ldx + i] (its rows are).
// The wave owning right-hand sides c0..c0+15 holds tile b of Y in acc[b]: lane l,
// element r = Y(16 b + l / 16 + 4 r, c0 + l % 16).  With that layout, element q of
// acc[b] is exactly the B operand of the 16x16x4 MFMA for rows 16 b + 4 q .. + 3 of
// Y (lane l: k = l / 16, column l % 16), so the solved tiles feed the update of the
// tiles below with no data movement.  The diagonal blocks are solved by
// substitution in the same order as a column sweep, scaled by the pivot's reciprocal
// (RCP) or divided by the pivot,
// in place in the accumulators (cross-lane broadcast of each solved row).
// T is staged through LDS one 16-column strip at a time (rows 16 b .. NB - 1),
// prefetched one strip ahead through registers.  Only LDS traffic is fenced at the
// barriers, so the prefetch stays in flight across them.
template <int NBLK, bool TT, bool UNIT, bool XT, bool RCP, typename TF, typename TX>
__device__ __forceinline__ void blk_lower_solve(double (*Ts)[NBLK * 16][17], const TF* __restrict__ T,
                                                long long ldt, TX* X, long long ldx, int ncols, int wg) {
    constexpr int NB = NBLK * 16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int cc = wg * 64 + w * 16 + lr;
    const bool cok = cc < ncols;
    // Y(i, cc) with i = 16 b + lq + 4 r: one per-lane base pointer plus a uniform offset
    // (an immediate when the rows of X are the right-hand sides)
    TX* const xb = XT ? X + (long long)(cok ? cc : 0) * ldx + lq : X + (long long)lq * ldx + (cok ? cc : 0);
    const long long xs = XT ? 1 : ldx;
    auto xat = [&](int b, int r) -> TX& { return xb[(long long)(16 * b + 4 * r) * xs]; };
    auto tload = [&](int i, int k) -> double {
        return (double)(TT ? T[(long long)k * ldt + i] : T[(long long)i * ldt + k]);
    };
    // strip b: T(i, 16 b + k), i in [16 b, NB), k in [0, 16): NBLK - b elements per thread
    auto strip_ik = [&](int b, int e, int& i, int& k) {
        const int rows = NB - 16 * b;
        if (TT) { k = e / rows; i = 16 * b + e % rows; }
        else { i = 16 * b + e / 16; k = e % 16; }
    };
    auto lds_barrier = []() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    };

    f64x4 acc[NBLK];
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[b][r] = cok ? (double)xat(b, r) : 0.0;

#pragma unroll
    for (int q = 0; q < NBLK; ++q) {
        int i, k;
        strip_ik(0, tid + q * 256, i, k);
        Ts[0][i][k] = tload(i, k);
    }
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        const int cur = b & 1;
        // strip b + 1 -> registers now, -> LDS at the end of this step
        double pf[NBLK];
        if (b + 1 < NBLK) {
#pragma unroll
            for (int q = 0; q < NBLK - b - 1; ++q) {
                int i, k;
                strip_ik(b + 1, tid + q * 256, i, k);
                pf[q] = tload(i, 16 * (b + 1) + k);
            }
        }
        // diagonal block, in place in the accumulator layout: row s of every right-hand
        // side sits in lane group s % 4, element s / 4; the owner scales it by the pivot,
        // the value is broadcast to the other three lane groups of the same column, and
        // each lane updates its rows below s (a column sweep: the operations and their
        // order per element are those of substitution)
        // RCP: the pivots' reciprocals, one per lane (lane l: row l % 16 of the tile), taken
        // once per tile so that no division sits on the substitution's chain; otherwise a
        // division per row
        const double rdv = (UNIT || !RCP) ? 1.0 : 1.0 / Ts[cur][16 * b + lr][lr];
#pragma unroll
        for (int s_ = 0; s_ < 16; ++s_) {
            double v = acc[b][s_ >> 2];
            if (!UNIT) v = RCP ? v * readlane_d(rdv, s_) : v / Ts[cur][16 * b + s_][s_];
            const double ys = __shfl(v, (s_ & 3) * 16 + lr, 64);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = lq + 4 * r;
                const double nv = fma(-Ts[cur][16 * b + i][s_], ys, acc[b][r]);
                acc[b][r] = (i > s_) ? nv : ((i == s_) ? ys : acc[b][r]);
            }
        }
        // Y_bb -= T(bb, b) Y_b for the tiles below, the next one first
#pragma unroll
        for (int bb = b + 1; bb < NBLK; ++bb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double a = -Ts[cur][16 * bb + lr][4 * q + lq];
                acc[bb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, acc[b][q], acc[bb], 0, 0, 0);
            }
        if (b + 1 < NBLK) {
#pragma unroll
            for (int q = 0; q < NBLK - b - 1; ++q) {
                int i, k;
                strip_ik(b + 1, tid + q * 256, i, k);
                Ts[cur ^ 1][i][k] = pf[q];
            }
        }
        lds_barrier();
    }
    if (cok) {
#pragma unroll
        for (int b = 0; b < NBLK; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) xat(b, r) = (TX)acc[b][r];
    }
}

// Both block solves of step k in one launch (they depend only on the diagonal block):
// workgroups [0, nwg) compute U12 = L11^{-1} A12 in place (the columns of A12 are the
// right-hand sides), workgroups [nwg, 2 nwg) compute L21 = A21 U11^{-1}, i.e.
// U11^T L21^T = A21^T (the rows of A21 are the right-hand sides).
template <int NBLK, typename TF, typename TX, bool RCP>
__global__ void __launch_bounds__(256, 2)
panel_trsm_kernel(const TF* __restrict__ D, long long ldd, TX* A12, TX* A21, long long ldx, int m, int nwg) {
    __shared__ double Ts[2][NBLK * 16][17];
    if ((int)blockIdx.x < nwg) blk_lower_solve<NBLK, false, true, false, RCP>(Ts, D, ldd, A12, ldx, m, blockIdx.x);
    else blk_lower_solve<NBLK, true, false, true, RCP>(Ts, D, ldd, A21, ldx, m, blockIdx.x - nwg);
}

template <int NBLK, typename TF, typename TX, bool RCP = false>
hipError_t panel_go(const void* D, long long ldd, void* A12, void* A21, long long ldx, int m, hipStream_t s) {
    const int nwg = (m + 63) / 64;
    hipLaunchKernelGGL((panel_trsm_kernel<NBLK, TF, TX, RCP>), dim3(2 * nwg), dim3(256), 0, s, (const TF*)D, ldd,
                       (TX*)A12, (TX*)A21, ldx, m, nwg);
    return hipGetLastError();
}

// One elimination step of the blocked substitution for 1..4 right-hand sides,
// block size BS.  Block t is solved here; the block p solved by the previous
// launch (p = t-1 forward, t+1 backward) is applied first.  Workgroup 0 stages
// the diagonal block t in LDS (one round of loads), applies x_p to the rows of
// block t, and then wave 0 sweeps the triangle: lane l holds rows l + 64 s,
// x_i is broadcast with readlane, the column of T is read from LDS.  The other
// workgroups apply x_p to every row beyond block t (one wave per row, the row
// read as one coalesced run).  One launch per block.
template <bool LOWER, bool UNIT, bool TT, int NR, int BS, typename TF>
__global__ void __launch_bounds__(256)
trsv_step_kernel(const TF* __restrict__ T, long long ldt, int n_pad, int t, double* X, long long ldx) {
    constexpr int NS = BS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = n_pad / BS;
    const int p = LOWER ? t - 1 : t + 1;
    const bool has_p = p >= 0 && p < nblk;
    const int pc0 = p * BS;   // first column of block p
    // x_p (BS x NR) is read by every wave: lane l holds rows l + 64 s of it
    double xp[NS][NR];
    if (has_p) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < NR; ++c) xp[s][c] = X[(long long)(pc0 + s * 64 + lane) * ldx + c];
    }
    // z_r -= T(r, block p) x_p for RPW rows r = rf, rf + rstep, ... (< r_end), one wave;
    // the loads of all RPW rows are issued before the arithmetic
    constexpr int RPW = 16;
    auto apply_rows = [&](int rf, int rstep, int r_end) {
        double a[RPW][NS];
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int r = rf + q * rstep;
#pragma unroll
            for (int s = 0; s < NS; ++s)
                a[q][s] = (r < r_end) ? (double)T[tat<TT>(r, pc0 + s * 64 + lane, ldt)] : 0.0;
        }
        // all RPW dot products first; then the read-modify-write of X as one batch of
        // loads followed by the stores (a load of X cannot move above an earlier store to X)
        double res[RPW];
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                acc[c] = 0.0;
#pragma unroll
                for (int s = 0; s < NS; ++s) acc[c] = fma(a[q][s], xp[s][c], acc[c]);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
            }
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c == lane) v = acc[c];
            res[q] = v;
        }
        if (lane < NR) {
            double old[RPW];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int r = rf + q * rstep;
                old[q] = (r < r_end) ? X[(long long)r * ldx + lane] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int r = rf + q * rstep;
                if (r < r_end) X[(long long)r * ldx + lane] = old[q] - res[q];
            }
        }
    };
    if (blockIdx.x > 0) {
        if (!has_p) return;
        const int base = (LOWER ? (t + 1) * BS : 0) + (blockIdx.x - 1) * 4 * RPW;
        const int r_end = LOWER ? n_pad : t * BS;
        apply_rows(base + wave, 4, r_end);
        return;
    }
    __shared__ double Ts[BS][BS + 1];
    __shared__ double rdiag[BS];
    const int r0 = t * BS;
    constexpr int LPT = BS * BS / 256;   // staged elements per thread, all loads issued together
    constexpr int LB = LPT < 64 ? LPT : 64;
#pragma unroll
    for (int q0 = 0; q0 < LPT; q0 += LB) {
        double v[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + (q0 + q) * 256;
            int r, c;
            if (TT) { c = e / BS; r = e % BS; }
            else { r = e / BS; c = e % BS; }
            v[q] = (double)T[tat<TT>(r0 + r, r0 + c, ldt)];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + (q0 + q) * 256;
            int r, c;
            if (TT) { c = e / BS; r = e % BS; }
            else { r = e / BS; c = e % BS; }
            Ts[r][c] = v[q];
        }
    }
    if (has_p) {
        for (int rf = wave; rf < BS; rf += 4 * RPW) apply_rows(r0 + rf, 4, r0 + BS);
    }
    __syncthreads();
    if (!UNIT && tid < BS) rdiag[tid] = 1.0 / Ts[tid][tid];
    __syncthreads();
    if (wave != 0) return;
    double x[NS][NR];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < NR; ++c) x[s][c] = X[(long long)(r0 + s * 64 + lane) * ldx + c];
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
        const int sblk = LOWER ? sb : NS - 1 - sb;   // the 64-row slice holding the pivots
        for (int u = 0; u < 64; ++u) {
            const int li = LOWER ? u : 63 - u;
            const int i = sblk * 64 + li;
            double xi[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                xi[c] = readlane_d(x[sblk][c], li);
                if (!UNIT) xi[c] *= rdiag[i];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (LOWER ? s < sblk : s > sblk) continue;   // these rows are final
                const int r = s * 64 + lane;
                const double m = Ts[r][i];
                const bool upd = (s != sblk) || (LOWER ? lane > li : lane < li);
                const bool own = (s == sblk) && lane == li;
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    const double nv = fma(-m, xi[c], x[s][c]);
                    x[s][c] = own ? xi[c] : (upd ? nv : x[s][c]);
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < NR; ++c) X[(long long)(r0 + s * 64 + lane) * ldx + c] = x[s][c];
}

// Whole triangular solve T x = b for 1..4 right-hand sides in ONE launch, 64-row
// blocks.  Workgroups take their position in the elimination order from an atomic
// ticket, so a workgroup only ever waits for blocks owned by workgroups that started
// before it: the chain always progresses, whether or not every workgroup is resident.
// Block t: stage the diagonal block in LDS; for every earlier block p (in solve
// order) wait for its published solution x_p, accumulate T(t, p) x_p (the 64 x 64
// block is prefetched one step ahead through registers into LDS); then substitute
// with the diagonal block (one wave, readlane broadcast), store x_t, and publish it.
// Publication: each solved value is its own flag.  pub (n_pad x NR, row-major) holds
// a signalling-NaN bit pattern (kUnset) before the launch; the writer stores x_t into
// it with device-scope relaxed atomic stores, and a reader polls the values it needs
// with device-scope relaxed atomic loads until none is kUnset (the first request for a
// block goes out one block ahead, during the products with the block before it).
// Arithmetic never produces kUnset (a NaN result is quiet), and each 8-byte value is
// written and read whole, so no fence or separate flag sits on the chain.  sync[0]: ticket, sync[1]:
// sticky error word (a wait exceeded spin_limit polls: the result is invalid).  The
// caller resets sync[0] and pub before every launch.
constexpr unsigned long long kUnset = 0x7ff4a5a5a5a5a5a5ull;

template <bool LOWER, bool UNIT, bool TT, int NR, typename TF>
__global__ void __launch_bounds__(256)
trsv_chain_kernel(const TF* __restrict__ T, long long ldt, int nblk, double* X, long long ldx,
                  unsigned* sync, unsigned long long* pub, unsigned spin_limit) {
    constexpr int BS = 64;
    __shared__ double Td[BS][BS + 1];
    __shared__ double To[2][BS][BS + 1];
    __shared__ double xs[BS][NR];
    __shared__ double zs[BS][NR];
    __shared__ int s_q;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_q = (int)atomicAdd(&sync[0], 1u);
    __syncthreads();
    const int q = s_q;
    const int t = LOWER ? q : nblk - 1 - q;
    const long long r0 = (long long)t * BS;
    // 64 x 64 block (rb, cb) of the operator, 16 elements per thread, coalesced for either access
    auto load_blk = [&](int rb, int cb, double (&v)[16]) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int i = TT ? (e & 63) : (e >> 6), j = TT ? (e >> 6) : (e & 63);
            v[k] = (double)T[tat<TT>((long long)rb * BS + i, (long long)cb * BS + j, ldt)];
        }
    };
    auto store_blk = [&](double (*dst)[BS + 1], const double (&v)[16]) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int i = TT ? (e & 63) : (e >> 6), j = TT ? (e >> 6) : (e & 63);
            dst[i][j] = v[k];
        }
    };
    auto order = [&](int s_) { return LOWER ? s_ : nblk - 1 - s_; };
    {
        double v[16];
        load_blk(t, t, v);
        store_blk(Td, v);
    }
    double vn[16];
    if (q > 0) {
        load_blk(t, order(0), vn);
        store_blk(To[0], vn);
    }
    __syncthreads();
    // wave 0's row of the diagonal block and its pivot's reciprocal, read before the waits
    // so that only the substitution itself follows the last one; the row's entries that do
    // not update this lane (the diagonal, and the solved side) are zeroed
    double trow[BS];
    double rd = 1.0;
    if (wave == 0) {
        if (!UNIT) rd = 1.0 / Td[lane][lane];
#pragma unroll
        for (int i = 0; i < BS; ++i) trow[i] = (LOWER ? lane > i : lane < i) ? Td[lane][i] : 0.0;
    }
    const int ri = tid >> 2, part = tid & 3;   // row and column quarter of the block products
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    // the right-hand side of this block's rows, read before the waits (only this workgroup
    // writes them, at the end)
    double bv[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) bv[c] = (part == 0) ? X[(r0 + ri) * ldx + c] : 0.0;
    // this thread's published value of a block is requested one block ahead (in flight during
    // the products with the block before it) and polled again while it is unset
    unsigned long long pnext = (q > 0 && tid < BS * NR)
                                   ? __hip_atomic_load(pub + (long long)order(0) * BS * NR + tid, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)
                                   : 0ull;
    for (int s_ = 0; s_ < q; ++s_) {
        const int p = order(s_);
        const int buf = s_ & 1;
        if (s_ + 1 < q) load_blk(t, order(s_ + 1), vn);
        if (tid < BS * NR) {
            unsigned long long* src = pub + (long long)p * BS * NR + tid;
            unsigned long long v = pnext;
            if (s_ + 1 < q)
                pnext = __hip_atomic_load(pub + (long long)order(s_ + 1) * BS * NR + tid, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            unsigned it = 0;
            while (v == kUnset) {
                if (++it > spin_limit) {
                    __hip_atomic_fetch_or(&sync[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            xs[tid / NR][tid % NR] = __longlong_as_double((long long)v);
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = part * 16 + jj;
            const double a = To[buf][ri][j];
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = fma(a, xs[j][c], acc[c]);
        }
        if (s_ + 1 < q) store_blk(To[buf ^ 1], vn);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        acc[c] += __shfl_xor(acc[c], 1, 64);
        acc[c] += __shfl_xor(acc[c], 2, 64);
    }
    if (part == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c) zs[ri][c] = bv[c] - acc[c];
    }
    __syncthreads();
    if (wave == 0) {
        double z[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) z[c] = zs[lane][c];
        // step i: x_i = z_i / T_ii formed on every lane (lane i's is the one broadcast), then
        // z_j -= T_ji x_i on the lanes still to solve (the others' T_ji are zero); one product,
        // one broadcast and one FMA on the chain per step.  Lane j's z_j is final after its
        // own step, so its x_j is the same product once more.
#pragma unroll
        for (int u = 0; u < BS; ++u) {
            const int i = LOWER ? u : BS - 1 - u;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const double xi = readlane_d(UNIT ? z[c] : z[c] * rd, i);
                z[c] = fma(-trow[i], xi, z[c]);
            }
        }
        if (!UNIT) {
#pragma unroll
            for (int c = 0; c < NR; ++c) z[c] *= rd;
        }
#pragma unroll
        for (int c = 0; c < NR; ++c)
            __hip_atomic_store(pub + (r0 + lane) * NR + c, (unsigned long long)__double_as_longlong(z[c]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int c = 0; c < NR; ++c) X[(r0 + lane) * ldx + c] = z[c];
    }
}

// Whole triangular solve T X = B for 5..64 right-hand sides in ONE launch: the many-column
// form of trsv_chain_kernel, with the same ticket order and the same publication (every solved
// value its own flag; pub is n_pad x 64, row-major).  64-row blocks, 256 threads; wave w owns
// columns 16 w .. 16 w + 15 and keeps the block's 64 x 16 slab of Y in four MFMA accumulators
// (tile b: lane l, element r = Y(16 b + l / 16 + 4 r, 16 w + l % 16)), so element u of tile b
// is the B operand of v_mfma_f64_16x16x4_f64 for rows 16 b + 4 u .. + 3.  For every earlier
// block p in solve order, T(t, p) is staged through LDS (prefetched one block ahead through
// registers) and the values of X_p are polled straight into B operands, one 16-row tile of p
// at a time in the order p solves its tiles: the product with a block overlaps the end of
// that block's own solve; a lane's sixteen values of p are requested in one go, one block
// ahead, and only the ones still unset are polled again.  Then the diagonal block is solved
// in place in the accumulators, tile by tile: substitution row by row with a cross-lane
// broadcast of each solved row (pivots applied as reciprocals taken when the block is
// loaded, so no division sits on the chain), then the MFMA update of the tiles still to be
// solved.  Each tile is published as soon as it is final.
template <bool LOWER, bool UNIT, bool TT, typename TF>
__global__ void __launch_bounds__(256)
trsm_chain_kernel(const TF* __restrict__ T, long long ldt, int nblk, double* X, long long ldx, int ncols,
                  unsigned* sync, unsigned long long* pub, unsigned spin_limit) {
    constexpr int BS = 64;
    __shared__ double Td[BS][BS + 1];
    __shared__ double To[2][BS][BS + 1];
    __shared__ double rdg[BS];         // reciprocals of the diagonal block's pivots
    __shared__ int s_q;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int cc = w * 16 + lr;
    const bool cok = cc < ncols;
    if (tid == 0) s_q = (int)atomicAdd(&sync[0], 1u);
    __syncthreads();
    const int q = s_q;
    const int t = LOWER ? q : nblk - 1 - q;
    const long long r0 = (long long)t * BS;
    auto load_blk = [&](int rb, int cb, double (&v)[16]) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int i = TT ? (e & 63) : (e >> 6), j = TT ? (e >> 6) : (e & 63);
            v[k] = (double)T[tat<TT>((long long)rb * BS + i, (long long)cb * BS + j, ldt)];
        }
    };
    auto store_blk = [&](double (*dst)[BS + 1], const double (&v)[16]) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int i = TT ? (e & 63) : (e >> 6), j = TT ? (e >> 6) : (e & 63);
            dst[i][j] = v[k];
        }
    };
    auto order = [&](int s_) { return LOWER ? s_ : nblk - 1 - s_; };
    auto tord = [](int j) { return LOWER ? j : 3 - j; };   // tiles of a block in solve order
    {
        double v[16];
        load_blk(t, t, v);
        store_blk(Td, v);
        if (!UNIT) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int e = tid + 256 * k;
                if ((e >> 6) == (e & 63)) rdg[e & 63] = 1.0 / v[k];
            }
        }
    }
    double vn[16];
    if (q > 0) {
        load_blk(t, order(0), vn);
        store_blk(To[0], vn);
    }
    f64x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[b][r] = cok ? X[(r0 + 16 * b + lq + 4 * r) * ldx + cc] : 0.0;
    __syncthreads();
    // the sixteen values of this lane for a block are requested one block ahead (in flight
    // during the products with the block before it); those still unset when their tile is
    // reached are polled again before its products
    auto request = [&](int pblk, unsigned long long (&v)[4][4]) {
        const unsigned long long* src = pub + (long long)pblk * BS * 64 + (long long)lq * 64 + cc;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                v[j][u] = cok ? __hip_atomic_load(src + (16 * tord(j) + 4 * u) * 64, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : 0ull;
    };
    unsigned long long pv[4][4], pvn[4][4];
    if (q > 0) request(order(0), pv);
    for (int s_ = 0; s_ < q; ++s_) {
        const int p = order(s_);
        const int buf = s_ & 1;
        if (s_ + 1 < q) {
            load_blk(t, order(s_ + 1), vn);
            request(order(s_ + 1), pvn);
        }
        const unsigned long long* srcp = pub + (long long)p * BS * 64 + (long long)lq * 64 + cc;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pb = tord(j);
            unsigned it = 0;
            while (pv[j][0] == kUnset || pv[j][1] == kUnset || pv[j][2] == kUnset || pv[j][3] == kUnset) {
                if (++it > spin_limit) {
                    __hip_atomic_fetch_or(&sync[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (pv[j][u] == kUnset)
                        pv[j][u] = __hip_atomic_load(srcp + (16 * pb + 4 * u) * 64, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            }
            double bq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) bq[u] = cok ? __longlong_as_double((long long)pv[j][u]) : 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-To[buf][16 * b + lr][16 * pb + 4 * u + lq], bq[u],
                                                                  acc[b], 0, 0, 0);
        }
        if (s_ + 1 < q) {
            store_blk(To[buf ^ 1], vn);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int u = 0; u < 4; ++u) pv[jj][u] = pvn[jj][u];
        }
        __syncthreads();
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int b = tord(jb);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int sr = LOWER ? j : 15 - j;
            double v = acc[b][sr >> 2];
            if (!UNIT) v = v * rdg[16 * b + sr];
            const double ys = __shfl(v, (sr & 3) * 16 + lr, 64);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = lq + 4 * r;
                const double nv = fma(-Td[16 * b + i][16 * b + sr], ys, acc[b][r]);
                const bool upd = LOWER ? i > sr : i < sr;
                acc[b][r] = upd ? nv : ((i == sr) ? ys : acc[b][r]);
            }
        }
        if (cok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = r0 + 16 * b + lq + 4 * r;
                __hip_atomic_store(pub + row * 64 + cc, (unsigned long long)__double_as_longlong(acc[b][r]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) X[(r0 + 16 * b + lq + 4 * r) * ldx + cc] = acc[b][r];
        }
#pragma unroll
        for (int jj = jb + 1; jj < 4; ++jj) {
            const int bb = tord(jj);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[bb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-Td[16 * bb + lr][16 * b + 4 * u + lq], acc[b][u],
                                                               acc[bb], 0, 0, 0);
        }
    }
}

__global__ void trsv_chain_reset_kernel(unsigned* sync, unsigned long long* pub, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) sync[0] = 0u;
    if (i < count) pub[i] = kUnset;
}

template <bool LOWER, bool UNIT, bool TT, bool XT, typename TF, typename TX>
hipError_t go(const void* T, long long ldt, int nb, void* X, long long ldx, int ncols, hipStream_t s) {
    hipLaunchKernelGGL((trsm_cols_kernel<LOWER, UNIT, TT, XT, TF, TX>), dim3((ncols + SB - 1) / SB), dim3(256),
                       0, s, (const TF*)T, ldt, nb, (TX*)X, ldx, ncols);
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
    if (nb <= 0 || nb > MAXNB || nb % SB) return hipErrorInvalidValue;
    if (ncols <= 0) return hipSuccess;
    if (!t_f32 && !x_f32) return dispatch<double, double>(kind, T, ldt, nb, X, ldx, ncols, s);
    if (t_f32 && !x_f32) return dispatch<float, double>(kind, T, ldt, nb, X, ldx, ncols, s);
    if (t_f32 && x_f32) return dispatch<float, float>(kind, T, ldt, nb, X, ldx, ncols, s);
    return hipErrorInvalidValue;
}

hipError_t launch_panel_trsm(int f32, int rcp, const void* D, long long ldd, int nb, void* A12, void* A21,
                             long long ldx, int m, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    if (f32) {
        switch (nb) {
            case 64: return panel_go<4, float, float>(D, ldd, A12, A21, ldx, m, s);
            case 128: return panel_go<8, float, float>(D, ldd, A12, A21, ldx, m, s);
            case 256: return panel_go<16, float, float>(D, ldd, A12, A21, ldx, m, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (nb) {
        case 64: return rcp ? panel_go<4, double, double, true>(D, ldd, A12, A21, ldx, m, s)
                            : panel_go<4, double, double>(D, ldd, A12, A21, ldx, m, s);
        case 128: return rcp ? panel_go<8, double, double, true>(D, ldd, A12, A21, ldx, m, s)
                             : panel_go<8, double, double>(D, ldd, A12, A21, ldx, m, s);
        case 256: return rcp ? panel_go<16, double, double, true>(D, ldd, A12, A21, ldx, m, s)
                             : panel_go<16, double, double>(D, ldd, A12, A21, ldx, m, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {

template <bool LOWER, bool UNIT, bool TT, int BS, typename TF>
hipError_t trsv_go(const void* T, long long ldt, int n_pad, double* X, long long ldx, int nr, hipStream_t s) {
    const int nblk = n_pad / BS;
    for (int q = 0; q < nblk; ++q) {
        const int t = LOWER ? q : nblk - 1 - q;
        const int rows_rest = LOWER ? n_pad - (t + 1) * BS : t * BS;
        const int has_p = LOWER ? t > 0 : t < nblk - 1;
        const unsigned grid = 1 + (has_p ? (unsigned)((rows_rest + 63) / 64) : 0u);
        switch (nr) {
#define GENP_TRSV_CASE(NR)                                                                                  \
    case NR:                                                                                                \
        hipLaunchKernelGGL((trsv_step_kernel<LOWER, UNIT, TT, NR, BS, TF>), dim3(grid), dim3(256), 0, s,     \
                           (const TF*)T, ldt, n_pad, t, X, ldx);                                            \
        break;
            GENP_TRSV_CASE(1)
            GENP_TRSV_CASE(2)
            GENP_TRSV_CASE(3)
            GENP_TRSV_CASE(4)
#undef GENP_TRSV_CASE
            default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int BS, typename TF>
hipError_t trsv_kind(int kind, const void* T, long long ldt, int n_pad, double* X, long long ldx, int nr,
                     hipStream_t s) {
    switch (kind) {
        case TRSM_L_UNIT: return trsv_go<true, true, false, BS, TF>(T, ldt, n_pad, X, ldx, nr, s);
        case TRSM_U: return trsv_go<false, false, false, BS, TF>(T, ldt, n_pad, X, ldx, nr, s);
        case TRSM_UT: return trsv_go<true, false, true, BS, TF>(T, ldt, n_pad, X, ldx, nr, s);
        case TRSM_LT_UNIT: return trsv_go<false, true, true, BS, TF>(T, ldt, n_pad, X, ldx, nr, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

namespace {

template <bool LOWER, bool UNIT, bool TT, typename TF>
hipError_t chain_go(const void* T, long long ldt, int nblk, double* X, long long ldx, int nr, unsigned* sync,
                    unsigned long long* pub, hipStream_t s) {
    constexpr unsigned kSpin = 1u << 20;   // polls (about 1 s in all): a safety limit a running chain never reaches
    const int count = nblk * 64 * nr;
    hipLaunchKernelGGL(trsv_chain_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, sync, pub, count);
    switch (nr) {
#define GENP_CHAIN_CASE(NR)                                                                                      \
    case NR:                                                                                                     \
        hipLaunchKernelGGL((trsv_chain_kernel<LOWER, UNIT, TT, NR, TF>), dim3(nblk), dim3(256), 0, s, (const TF*)T, \
                           ldt, nblk, X, ldx, sync, pub, kSpin);                                                      \
        break;
        GENP_CHAIN_CASE(1)
        GENP_CHAIN_CASE(2)
        GENP_CHAIN_CASE(3)
        GENP_CHAIN_CASE(4)
#undef GENP_CHAIN_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool LOWER, bool UNIT, bool TT, typename TF>
hipError_t mchain_go(const void* T, long long ldt, int nblk, double* X, long long ldx, int ncols, unsigned* sync,
                     unsigned long long* pub, hipStream_t s) {
    constexpr unsigned kSpin = 1u << 20;
    const int count = nblk * 64 * 64;
    hipLaunchKernelGGL(trsv_chain_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, sync, pub, count);
    hipLaunchKernelGGL((trsm_chain_kernel<LOWER, UNIT, TT, TF>), dim3(nblk), dim3(256), 0, s, (const TF*)T, ldt,
                       nblk, X, ldx, ncols, sync, pub, kSpin);
    return hipGetLastError();
}

template <typename TF>
hipError_t mchain_kind(int kind, const void* T, long long ldt, int nblk, double* X, long long ldx, int ncols,
                       unsigned* sync, unsigned long long* pub, hipStream_t s) {
    switch (kind) {
        case TRSM_L_UNIT: return mchain_go<true, true, false, TF>(T, ldt, nblk, X, ldx, ncols, sync, pub, s);
        case TRSM_U: return mchain_go<false, false, false, TF>(T, ldt, nblk, X, ldx, ncols, sync, pub, s);
        case TRSM_UT: return mchain_go<true, false, true, TF>(T, ldt, nblk, X, ldx, ncols, sync, pub, s);
        case TRSM_LT_UNIT: return mchain_go<false, true, true, TF>(T, ldt, nblk, X, ldx, ncols, sync, pub, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename TF>
hipError_t chain_kind(int kind, const void* T, long long ldt, int nblk, double* X, long long ldx, int nr,
                      unsigned* sync, unsigned long long* pub, hipStream_t s) {
    switch (kind) {
        case TRSM_L_UNIT: return chain_go<true, true, false, TF>(T, ldt, nblk, X, ldx, nr, sync, pub, s);
        case TRSM_U: return chain_go<false, false, false, TF>(T, ldt, nblk, X, ldx, nr, sync, pub, s);
        case TRSM_UT: return chain_go<true, false, true, TF>(T, ldt, nblk, X, ldx, nr, sync, pub, s);
        case TRSM_LT_UNIT: return chain_go<false, true, true, TF>(T, ldt, nblk, X, ldx, nr, sync, pub, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_trsv_chain(int kind, int t_f32, const void* T, long long ldt, int n_pad, double* X, long long ldx,
                             int nr, unsigned* sync, unsigned long long* pub, hipStream_t s) {
    if (nr < 1 || nr > 4 || n_pad % 64) return hipErrorInvalidValue;
    const int nblk = n_pad / 64;
    return t_f32 ? chain_kind<float>(kind, T, ldt, nblk, X, ldx, nr, sync, pub, s)
                 : chain_kind<double>(kind, T, ldt, nblk, X, ldx, nr, sync, pub, s);
}

hipError_t launch_trsm_chain(int kind, int t_f32, const void* T, long long ldt, int n_pad, double* X, long long ldx,
                             int ncols, unsigned* sync, unsigned long long* pub, hipStream_t s) {
    if (ncols < 1 || ncols > 64 || n_pad % 64) return hipErrorInvalidValue;
    const int nblk = n_pad / 64;
    return t_f32 ? mchain_kind<float>(kind, T, ldt, nblk, X, ldx, ncols, sync, pub, s)
                 : mchain_kind<double>(kind, T, ldt, nblk, X, ldx, ncols, sync, pub, s);
}

hipError_t launch_trsv_full(int kind, int t_f32, const void* T, long long ldt, int n_pad, int bs, double* X,
                            long long ldx, int nr, hipStream_t s) {
    if (nr < 1 || nr > 4 || (bs != 64 && bs != 128) || n_pad % bs) return hipErrorInvalidValue;
    if (bs == 128)
        return t_f32 ? trsv_kind<128, float>(kind, T, ldt, n_pad, X, ldx, nr, s)
                     : trsv_kind<128, double>(kind, T, ldt, n_pad, X, ldx, nr, s);
    return t_f32 ? trsv_kind<64, float>(kind, T, ldt, n_pad, X, ldx, nr, s)
                 : trsv_kind<64, double>(kind, T, ldt, n_pad, X, ldx, nr, s);
}
