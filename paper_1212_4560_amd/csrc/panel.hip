// Diagonal-block factorization of the blocked elimination.
//
// GENP (section 1.1) on an nb x nb diagonal block, in place, with no pivot
// search and no row exchanges: right-looking, 16 columns at a time, each step
// replacing the trailing block by its Schur complement (Fact 2.1).  Pivot
// statistics and the first failing pivot (non-finite, or
// |u_kk| <= pivot_tol * max|C|) are recorded.
#include "common.h"

#include <math.h>

#include <algorithm>

namespace {

constexpr int PW = 16;    // inner panel width
constexpr int MAXNB = 256;
constexpr int TB = 8;     // 16x16 tiles per batch of the trailing update

__device__ inline double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide max (doubles) and min (ints) with DPP moves: shifts by 1, 2, 4, 8 inside each row
// of 16 lanes leave a row's result in its lane 15; the row broadcasts of lanes 15 and 31 then
// bring the whole wave's into lane 63, which is read out.  A lane with no source keeps its own
// value.
template <int CTRL, int ROWS>
__device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ inline double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, ROWS>((int)(b & 0xffffffffLL)), hi = dpp_i<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double wave_max_d(double v) {
    v = fmax(v, dpp_d<0x111, 0xf>(v));
    v = fmax(v, dpp_d<0x112, 0xf>(v));
    v = fmax(v, dpp_d<0x114, 0xf>(v));
    v = fmax(v, dpp_d<0x118, 0xf>(v));
    v = fmax(v, dpp_d<0x142, 0xa>(v));
    v = fmax(v, dpp_d<0x143, 0xc>(v));
    return readlane_d(v, 63);
}
__device__ inline int wave_min_i(int v) {
    v = min(v, dpp_i<0x111, 0xf>(v));
    v = min(v, dpp_i<0x112, 0xf>(v));
    v = min(v, dpp_i<0x114, 0xf>(v));
    v = min(v, dpp_i<0x118, 0xf>(v));
    v = min(v, dpp_i<0x142, 0xa>(v));
    v = min(v, dpp_i<0x143, 0xc>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// One workgroup of 256 threads (one wave per SIMD), FP64 arithmetic for either
// storage type.  For each 16-column panel:
//  1. wave 0 factors the panel alone, with no barrier: lane l holds rows
//     l, l+64, l+128, l+192 of it in registers and the pivot row is broadcast
//     with readlane;
//  2. one thread per column solves the 16 rows of U right of the panel with the
//     unit lower 16 x 16 block (column sweep);
//  3. the trailing block takes the rank-16 Schur update (Fact 2.1) on the
//     matrix cores: 16 x 16 tiles, 8 per wave per batch of loads, operands from
//     LDS (the panel below the diagonal and the new rows of U).
// Steps 3 and 1 overlap (look-ahead): wave 0 updates the next panel's column of tiles first,
// keeps it in LDS and factors it while waves 1-3 update the rest of the trailing block; the
// panel's L goes to the other of two LDS buffers.  Every tile takes the same operations in the
// same order as without the overlap (the next panel staged at the storage precision), so the
// factors are the same.
//
// PIV: block Gaussian elimination with the diagonal block as the block pivot (Theorem 2.2):
// rows are interchanged inside the block, at each column the row with the largest |entry|
// among the block's remaining rows (the first on ties) becomes the pivot row.  The panel's
// interchanges are made in wave 0's registers, then on the block's other columns (net row
// movement, all loads before any store, one column per thread), and the block's net
// permutation is written to perm: factor row r comes from row perm[r] (global index).
template <typename T, bool PIV>
__global__ void __launch_bounds__(256)
diag_lu_kernel(T* __restrict__ D, long long ldd, int nb, int nvalid, long long col0,
               const double* __restrict__ maxc, double pivot_tol, PanelStats* __restrict__ st,
               int* __restrict__ perm) {
    __shared__ double Ls[2][MAXNB][PW + 1];     // two panels: rows kb.. (row r - kb), 16 columns
    __shared__ double Rs[PW][MAXNB - PW + 1];   // rows kb..kb+15 of U right of the panel
    __shared__ int sw[MAXNB];                   // PIV: row interchanged with row r at step r
    __shared__ int ptmp[MAXNB];                 // PIV: the current panel's net row movement
    __shared__ int bperm[MAXNB];                // PIV: the block's net permutation so far
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const double tol_abs = pivot_tol * maxc[0];
    double s_min = INFINITY, s_max = 0.0;
    long long s_bad = -1;
    if (PIV) {
        bperm[tid] = tid;
        __syncthreads();
    }
    // wave 0: factor the panel at columns kb..kb+15, rows kb..nb-1, read from D or (from_lds)
    // from Lp, written to D and Lp
    auto factor_panel = [&](int kb, double (*Lp)[PW + 1], bool from_lds) {
        const int rows = nb - kb;
        double p[4][PW];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = s * 64 + lane;
#pragma unroll
            for (int c = 0; c < PW; ++c)
                    p[s][c] = (r < rows) ? (from_lds ? Lp[r][c] : (double)D[(long long)(kb + r) * ldd + kb + c]) : 0.0;
        }
        // PIV: the panel's rows stay in their registers; pos[s] is the current position of
        // the row in slot s (LAPACK's interchange order: at step c the chosen row takes
        // position c and the row that held position c takes the chosen row's place) and
        // done[s] marks rows already taken as pivot rows.  Rows are written back at their
        // final positions.  Without PIV, pos[s] = r and pivot row c sits in lane c, slot 0.
        int pos[4];
        bool done[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            pos[s] = s * 64 + lane;
            done[s] = false;
        }
#pragma unroll
        for (int c = 0; c < PW; ++c) {
            double prow[PW];
            double rp;
            if (PIV) {
                // pivot: the largest |entry| of column c among the rows not yet taken (valid
                // rows only; a NaN counts below every number), the smallest position on ties
                int q = c, qpos = c;   // pad columns: the pad row at position c, never moved
                if (kb + c < nvalid) {
                    double best = -1.0;
                    int bp = 1 << 30, bi = c;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        if (s * 64 >= rows) break;   // no rows of the block in this slot (uniform)
                        const int r = s * 64 + lane;
                        const double a = fabs(p[s][c]);
                        const double key = a == a ? a : -0.5;
                        // one basic block: the conditions evaluated in full, the result selected
                        const bool take =
                            (!done[s]) & (kb + r < nvalid) & ((key > best) | ((key == best) & (pos[s] < bp)));
                        best = take ? key : best;
                        bp = take ? pos[s] : bp;
                        bi = take ? r : bi;
                    }
                    const double m = wave_max_d(best);
                    unsigned long long hold = __ballot(best == m);
                    if (__popcll(hold) > 1) {
                        // several lanes hold the maximum: keep those with the smallest position
                        const int mp = wave_min_i(best == m ? bp : 1 << 30);
                        hold = __ballot(best == m && bp == mp);
                    }
                    const int wl = __builtin_ctzll(hold);
                    q = __builtin_amdgcn_readlane(bi, wl);
                    qpos = __builtin_amdgcn_readlane(bp, wl);
                }
                if (lane == 0) sw[kb + c] = kb + qpos;
                const int qs = q >> 6, ql = q & 63;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    if (pos[s] == c) pos[s] = qpos;
                    if (s == qs && lane == ql) {
                        pos[s] = c;
                        done[s] = true;
                    }
                }
                auto get = [&](const double (&row)[PW]) {
                    // the pivot first: its reciprocal is under way while the rest of the row is read
                    const double pv = readlane_d(row[c], ql);
                    rp = 1.0 / pv;
#pragma unroll
                    for (int t = 0; t < PW; ++t) prow[t] = (t > c) ? readlane_d(row[t], ql) : (t == c ? pv : 0.0);
                };
                switch (qs) {
                    case 0: get(p[0]); break;
                    case 1: get(p[1]); break;
                    case 2: get(p[2]); break;
                    default: get(p[3]); break;
                }
            } else {
                // pivot row c is row c of the panel: lane c, slot 0 (its first c entries are L)
                const double pv = readlane_d(p[0][c], c);
                rp = 1.0 / pv;
#pragma unroll
                for (int t = 0; t < PW; ++t) prow[t] = (t > c) ? readlane_d(p[0][t], c) : (t == c ? pv : 0.0);
            }
            const double piv = prow[c];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (s * 64 >= rows) break;   // the whole slot below the block (uniform)
                const int r = s * 64 + lane;
                if ((PIV ? !done[s] : r > c) && r < rows) {
                    const double l = p[s][c] * rp;
                    p[s][c] = l;
#pragma unroll
                    for (int t = 0; t < PW; ++t)
                        if (t > c) p[s][t] = fma(-l, prow[t], p[s][t]);
                }
            }
            if (lane == 0 && kb + c < nvalid) {
                const double a = fabs(piv);
                if (s_bad < 0 && (!isfinite(a) || a <= tol_abs)) s_bad = col0 + kb + c;
                if (s_bad < 0) {
                    s_min = fmin(s_min, a);
                    s_max = fmax(s_max, a);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = s * 64 + lane;
            if (r < rows) {
#pragma unroll
                for (int c = 0; c < PW; ++c) {
                    D[(long long)(kb + pos[s]) * ldd + kb + c] = (T)p[s][c];
                    Lp[pos[s]][c] = p[s][c];
                }
            }
        }
        if (PIV) {
            // the panel's net row movement (ptmp: new position -> old position) and the
            // block's permutation so far, from the rows' final positions
            int ob[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) ob[s] = s * 64 + lane < rows ? bperm[kb + s * 64 + lane] : 0;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int r = s * 64 + lane;
                if (r < rows) {
                    ptmp[kb + pos[s]] = kb + r;
                    bperm[kb + pos[s]] = ob[s];
                }
            }
        }
    };
    // trailing block at row and column kb+16: A22 -= L21 U12 on 16 x 16 tiles, TB per batch of
    // loads; this wave's tiles are entries first, first + 1, ... of a list of total tiles, TB at
    // a time every stride entries, entry e being tile tile_of(e) = (ti, tj).  f64 16x16x4
    // layout: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16); accumulator
    // lane l, element r -> (row l/16 + 4r, col l%16).  to_lds: the tiles (which form the next
    // panel) go to Ln at the storage precision instead of D.
    auto update_tiles = [&](int kb, const double (*Lc)[PW + 1], int total, int first, int stride, auto tile_of,
                            double (*Ln)[PW + 1]) {
        for (int t0 = first; t0 < total; t0 += stride) {
            f64x4 acc[TB];
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const int e = t0 + b;
                const int2 tt = tile_of(e < total ? e : t0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = kb + PW + tt.x * 16 + lq + 4 * r, col = kb + PW + tt.y * 16 + lr;
                    acc[b][r] = (e < total) ? (double)D[(long long)row * ldd + col] : 0.0;
                }
            }
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const int e = t0 + b;
                if (e < total) {
                    const int2 tt = tile_of(e);
#pragma unroll
                    for (int kk = 0; kk < PW; kk += 4) {
                        const double a = Lc[PW + tt.x * 16 + lr][kk + lq];
                        const double bb = Rs[kk + lq][tt.y * 16 + lr];
                        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, bb, acc[b], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const int e = t0 + b;
                if (e < total) {
                    const int2 tt = tile_of(e);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = kb + PW + tt.x * 16 + lq + 4 * r, col = kb + PW + tt.y * 16 + lr;
                        if (Ln)
                            Ln[tt.x * 16 + lq + 4 * r][lr] = (double)(T)acc[b][r];
                        else
                            D[(long long)row * ldd + col] = (T)acc[b][r];
                    }
                }
            }
        }
    };
    if (wave == 0) factor_panel(0, Ls[0], false);
    for (int kb = 0; kb < nb; kb += PW) {
        const int rows = nb - kb;
        double (*Lc)[PW + 1] = Ls[(kb / PW) & 1];
        double (*Ln)[PW + 1] = Ls[((kb / PW) & 1) ^ 1];
        __syncthreads();   // the panel at kb factored; the previous trailing update stored
        const int ncols = rows - PW;
        // one thread per column j of the block outside the panel.  PIV: rows kb..kb+15 and the
        // rows they were exchanged with take the panel's net movement (all loads before any
        // store).  Right of the panel (j >= kb+16) rows kb..kb+15 of column j then take
        // x <- L11^{-1} x (unit lower, column sweep): the rows of U12, also kept in Rs.
        {
            const int j = tid;
            const bool right = j >= kb + PW && j < nb;
            if (PIV && j < nb && (j < kb || j >= kb + PW)) {
                double v[2 * PW];
#pragma unroll
                for (int i = 0; i < 2 * PW; ++i) {
                    const int q = i < PW ? kb + i : sw[kb + i - PW];
                    const int src = ptmp[q];
                    v[i] = (src != q || (right && i < PW)) ? (double)D[(long long)src * ldd + j] : 0.0;
                }
                if (right) {
#pragma unroll
                    for (int t = 0; t < PW; ++t)
#pragma unroll
                        for (int i = 0; i < PW; ++i)
                            if (i > t) v[i] = fma(-Lc[i][t], v[t], v[i]);
#pragma unroll
                    for (int i = 0; i < PW; ++i) {
                        D[(long long)(kb + i) * ldd + j] = (T)v[i];
                        Rs[i][j - kb - PW] = v[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 2 * PW; ++i) {
                    // right of the panel rows kb..kb+15 already hold their rows of U12, also
                    // where one is named again as an exchange partner
                    const int q = i < PW ? kb + i : sw[kb + i - PW];
                    const bool done_u = right && q >= kb && q < kb + PW;
                    if (ptmp[q] != q && !done_u) D[(long long)q * ldd + j] = (T)v[i];
                }
            } else if (!PIV && right) {
                double x[PW];
#pragma unroll
                for (int i = 0; i < PW; ++i) x[i] = (double)D[(long long)(kb + i) * ldd + j];
#pragma unroll
                for (int t = 0; t < PW; ++t)
#pragma unroll
                    for (int i = 0; i < PW; ++i)
                        if (i > t) x[i] = fma(-Lc[i][t], x[t], x[i]);
#pragma unroll
                for (int i = 0; i < PW; ++i) {
                    D[(long long)(kb + i) * ldd + j] = (T)x[i];
                    Rs[i][j - kb - PW] = x[i];
                }
            }
        }
        if (ncols > 0) {
            __syncthreads();
            const int nt = ncols / PW;
            if (wave == 0) {
                // the next panel's column of tiles, then that panel, while waves 1-3 update the rest
                update_tiles(kb, Lc, nt, 0, TB, [](int e) { return make_int2(e, 0); }, Ln);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                factor_panel(kb + PW, Ln, true);
            } else if (nt > 1) {
                const int w1 = nt - 1;
                update_tiles(kb, Lc, nt * w1, (wave - 1) * TB, 3 * TB,
                             [w1](int e) { return make_int2(e / w1, 1 + e % w1); }, nullptr);
            }
        }
    }
    if (tid == 0) {
        st->min_abs = s_min;
        st->max_abs = s_max;
        st->first_bad = s_bad;
    }
    if (PIV && tid < nb) perm[tid] = (int)(col0 + bperm[tid]);
}

// GENP of a 128 x 128 FP64 block held in LDS for the whole elimination (the same steps as
// diag_lu_kernel, 16 columns at a time: panel by wave 0 with readlane broadcasts, the 16 rows of
// U right of the panel by a column sweep, the rank-16 Schur update on the matrix cores), so
// the only global traffic is one read and one write of the block.  merge: combine the pivot
// statistics with those already in *st (the second diagonal quadrant of a 256 block).
constexpr int Q = 128;
__global__ void __launch_bounds__(256)
lu128_lds_kernel(double* __restrict__ D, long long ldd, int nvalid, long long col0, const double* __restrict__ maxc,
                 double pivot_tol, PanelStats* __restrict__ st, int merge) {
    __shared__ double L[Q][Q + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double tol_abs = pivot_tol * maxc[0];
    // load: 64 elements per thread, rows coalesced
#pragma unroll 8
    for (int e = tid; e < Q * Q; e += 256) L[e / Q][e % Q] = D[(long long)(e / Q) * ldd + e % Q];
    __syncthreads();
    double s_min = INFINITY, s_max = 0.0;
    long long s_bad = -1;
    for (int kb = 0; kb < Q; kb += PW) {
        const int rows = Q - kb;
        if (wave == 0) {
            double p[2][PW];
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int r = sl * 64 + lane;
#pragma unroll
                for (int c = 0; c < PW; ++c) p[sl][c] = (r < rows) ? L[kb + r][kb + c] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                double prow[PW];
#pragma unroll
                for (int t = 0; t < PW; ++t) prow[t] = (t >= c) ? readlane_d(p[0][t], c) : 0.0;
                const double piv = prow[c];
                if (lane == 0 && kb + c < nvalid) {
                    const double a = fabs(piv);
                    if (s_bad < 0 && (!isfinite(a) || a <= tol_abs)) s_bad = col0 + kb + c;
                    if (s_bad < 0) {
                        s_min = fmin(s_min, a);
                        s_max = fmax(s_max, a);
                    }
                }
                const double rp = 1.0 / piv;
#pragma unroll
                for (int sl = 0; sl < 2; ++sl) {
                    const int r = sl * 64 + lane;
                    if (r > c && r < rows) {
                        const double l = p[sl][c] * rp;
                        p[sl][c] = l;
#pragma unroll
                        for (int t = 0; t < PW; ++t)
                            if (t > c) p[sl][t] = fma(-l, prow[t], p[sl][t]);
                    }
                }
            }
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int r = sl * 64 + lane;
                if (r < rows)
#pragma unroll
                    for (int c = 0; c < PW; ++c) L[kb + r][kb + c] = p[sl][c];
            }
        }
        __syncthreads();
        const int ncols = rows - PW;
        if (ncols > 0) {
            if (tid < ncols) {
                // rows kb..kb+15 of U right of the panel: x <- L11^{-1} x (unit lower, column sweep)
                const int col = kb + PW + tid;
                double x[PW];
#pragma unroll
                for (int i = 0; i < PW; ++i) x[i] = L[kb + i][col];
#pragma unroll
                for (int t = 0; t < PW; ++t)
#pragma unroll
                    for (int i = 0; i < PW; ++i)
                        if (i > t) x[i] = fma(-L[kb + i][kb + t], x[t], x[i]);
#pragma unroll
                for (int i = 0; i < PW; ++i) L[kb + i][col] = x[i];
            }
            __syncthreads();
            // trailing block: 16 x 16 tiles, A22 -= L21 U12 on the matrix cores, operands and
            // accumulators in LDS (accumulator lane l, element r: row l/16 + 4r, column l%16)
            const int nt = ncols / PW, ntiles = nt * nt;
            const int lr = lane & 15, lq = lane >> 4;
            for (int tile = wave; tile < ntiles; tile += 4) {
                const int r0 = kb + PW + (tile / nt) * 16, c0 = kb + PW + (tile % nt) * 16;
                f64x4 acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = L[r0 + lq + 4 * r][c0 + lr];
#pragma unroll
                for (int kk = 0; kk < PW; kk += 4)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-L[r0 + lr][kb + kk + lq], L[kb + kk + lq][c0 + lr], acc,
                                                               0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) L[r0 + lq + 4 * r][c0 + lr] = acc[r];
            }
        }
        __syncthreads();
    }
#pragma unroll 8
    for (int e = tid; e < Q * Q; e += 256) D[(long long)(e / Q) * ldd + e % Q] = L[e / Q][e % Q];
    if (tid == 0) {
        if (merge) {
            const PanelStats o = *st;
            if (o.first_bad >= 0) s_bad = o.first_bad;
            s_min = fmin(s_min, o.min_abs);
            s_max = fmax(s_max, o.max_abs);
        }
        st->min_abs = s_min;
        st->max_abs = s_max;
        st->first_bad = s_bad;
    }
}

}  // namespace

hipError_t launch_diag_lu(int prec, void* Dblk, long long ldd, int nb, int nvalid, long long col0,
                          const double* maxc, double pivot_tol, PanelStats* st, hipStream_t s) {
    if (nb <= 0 || nb > MAXNB || nb % PW) return hipErrorInvalidValue;   // nb: multiple of 16, <= 256
    if (prec == PREC_F64)
        hipLaunchKernelGGL((diag_lu_kernel<double, false>), dim3(1), dim3(256), 0, s, (double*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st, nullptr);
    else
        hipLaunchKernelGGL((diag_lu_kernel<float, false>), dim3(1), dim3(256), 0, s, (float*)Dblk, ldd, nb,
                           nvalid, col0, maxc, pivot_tol, st, nullptr);
    return hipGetLastError();
}

hipError_t launch_diag_lu_piv(double* Dblk, long long ldd, int nb, int nvalid, long long col0, const double* maxc,
                              double pivot_tol, PanelStats* st, int* perm, hipStream_t s) {
    if (nb <= 0 || nb > MAXNB || nb % PW || !perm) return hipErrorInvalidValue;
    hipLaunchKernelGGL((diag_lu_kernel<double, true>), dim3(1), dim3(256), 0, s, Dblk, ldd, nb, nvalid, col0, maxc,
                       pivot_tol, st, perm);
    return hipGetLastError();
}

namespace {

// Rows row0 .. row0 + nb - 1 of C take their block's interchanges in every column outside the
// diagonal block: row r becomes the former row perm[r] (global index, inside the block).  One
// workgroup per 32 columns: the block's rows are staged in LDS, then written back permuted.
constexpr int RP_COLS = 32;
__global__ void __launch_bounds__(256)
block_row_perm_kernel(double* __restrict__ C, long long ldc, long long row0, int nb, int ncols,
                      const int* __restrict__ perm) {
    __shared__ double tile[MAXNB][RP_COLS + 1];
    const long long c0 = (long long)blockIdx.x * RP_COLS;
    if (c0 >= row0 && c0 + RP_COLS <= row0 + nb) return;   // inside the diagonal block: nothing to do
    const int cl = threadIdx.x & (RP_COLS - 1), rg = threadIdx.x / RP_COLS;
    const long long col = c0 + cl;
    const bool in = col < ncols && !(col >= row0 && col < row0 + nb);
    for (int r = rg; r < nb; r += 256 / RP_COLS) tile[r][cl] = in ? C[(row0 + r) * ldc + col] : 0.0;
    __syncthreads();
    for (int r = rg; r < nb; r += 256 / RP_COLS) {
        const int src = (int)(perm[r] - row0);
        if (in && src != r) C[(row0 + r) * ldc + col] = tile[src][cl];
    }
}

// The explicit block pivots B_k = P_k^T L_kk U_kk: factor row i of block k (rows k0 .. k0+w-1,
// w = min(nb, n - k0)) gives row perm[i] of the output (row i when perm is null).  One
// workgroup per row, one thread per column; columns w .. nb-1 of a ragged last block are 0.
__global__ void __launch_bounds__(256)
block_pivots_kernel(const double* __restrict__ C, long long ldc, int n, int nb, const int* __restrict__ perm,
                    double* __restrict__ out, long long ldo) {
    const int i = blockIdx.x;
    const int k0 = (i / nb) * nb, r = i - k0, w = min(nb, n - k0);
    const int j = threadIdx.x;
    if (j >= nb) return;
    double s = 0.0;
    if (j < w) {
        // (L U)(r, j) = sum over t <= min(r, j) of L(r, t) U(t, j), with L(r, r) = 1
        const double* Lr = C + (long long)(k0 + r) * ldc + k0;
        const double* Ub = C + (long long)k0 * ldc + k0 + j;
        const int tmax = r <= j ? r : j + 1;
        for (int t = 0; t < tmax; ++t) s = fma(Lr[t], Ub[(long long)t * ldc], s);
        if (r <= j) s += Lr[j];
    }
    const long long orow = perm ? perm[i] : i;
    out[orow * ldo + j] = s;
}

__global__ void permute_rows_kernel(int n, int k, const double* __restrict__ src, long long lds,
                                    double* __restrict__ dst, long long ldd, const int* __restrict__ perm,
                                    int scatter) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * k) return;
    const int i = (int)(idx / k), b = (int)(idx % k);
    if (scatter) dst[(long long)perm[i] * ldd + b] = src[(long long)i * lds + b];
    else dst[(long long)i * ldd + b] = src[(long long)perm[i] * lds + b];
}

__global__ void iota_kernel(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

}  // namespace

hipError_t launch_block_row_perm(double* C, long long ldc, long long row0, int nb, int ncols, const int* perm,
                                 hipStream_t s) {
    if (nb <= 0 || nb > MAXNB || ncols <= 0 || row0 < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_row_perm_kernel, dim3((ncols + RP_COLS - 1) / RP_COLS), dim3(256), 0, s, C, ldc, row0,
                       nb, ncols, perm);
    return hipGetLastError();
}

hipError_t launch_block_pivots(const double* C, long long ldc, int n, int nb, const int* perm, double* out,
                               long long ldo, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nb <= 0 || nb > MAXNB || ldo < nb) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_pivots_kernel, dim3(n), dim3((nb + 63) / 64 * 64), 0, s, C, ldc, n, nb, perm, out, ldo);
    return hipGetLastError();
}

hipError_t launch_permute_rows(int n, int k, const double* src, long long lds, double* dst, long long ldd,
                               const int* perm, int scatter, hipStream_t s) {
    const long long tot = (long long)n * k;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, src, lds,
                       dst, ldd, perm, scatter);
    return hipGetLastError();
}

hipError_t launch_iota(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// A 256 x 256 FP64 diagonal block as four steps on one stream: GENP of the leading 128 block in
// LDS; U12 = L11^{-1} A12 and L21 = A21 U11^{-1} on the matrix cores (the panel solves of the
// blocked elimination with nb = 128); A22 -= L21 U12; GENP of A22 in LDS.  This is block
// Gaussian elimination (Theorem 2.2) on the block itself, with the same pivots.
hipError_t launch_diag_lu_split(void* Dblk, long long ldd, int nvalid, long long col0, const double* maxc,
                                double pivot_tol, PanelStats* st, int rcp, hipStream_t s) {
    double* D = (double*)Dblk;
    hipLaunchKernelGGL(lu128_lds_kernel, dim3(1), dim3(256), 0, s, D, ldd, std::min(nvalid, 128), col0, maxc,
                       pivot_tol, st, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_panel_trsm(0, rcp, D, ldd, 128, D + 128, D + 128 * ldd, ldd, 128, s);
    if (e != hipSuccess) return e;
    GemmF64Args g{};
    g.M = g.N = g.K = 128;
    g.A = D + 128 * ldd;
    g.lda = ldd;
    g.amode = OP_N;
    g.B = D + 128;
    g.ldb = ldd;
    g.bmode = OP_N;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.Cin = D + 128 * ldd + 128;
    g.ldci = ldd;
    g.D = D + 128 * ldd + 128;
    g.ldd = ldd;
    g.ksplit = 1;
    e = launch_gemm_f64(g, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lu128_lds_kernel, dim3(1), dim3(256), 0, s, D + 128 * ldd + 128, ldd, std::max(0, nvalid - 128),
                       col0 + 128, maxc, pivot_tol, st, 1);
    return hipGetLastError();
}
