// Circulant multipliers applied by FFT (the DFT diagonalizes every circulant matrix,
// Theorem 2.1; circulant multipliers, Definition 3.2).
//
// G[i][j] = c[(i - j) mod n], n = 2N a power of two, 4 <= n <= 16384.
//   row correlation   (x^T G)[j] = sum_k x[k] c[(k - j) mod n]  <->  X conj(C)   (A G, G^T y)
//   column convolution  (G y)[i] = sum_j c[(i - j) mod n] y[j]  <->  Y C         (G y)
// with X, Y, C the DFTs of length n.
//
// One workgroup per vector.  The real vector of length n = 2N is packed as N complex
// numbers z[k] = x[2k] + i x[2k+1] and transformed in place in LDS (radix-2 butterflies,
// three stages per pass over LDS, length N: decimation in time from bit-reversed order, so
// the spectrum comes out in natural order).  The spectrum of the real vector follows from Z[f] and Z[N-f]:
//   E[f] = (Z[f] + conj Z[N-f]) / 2,  O[f] = (Z[f] - conj Z[N-f]) / (2i),
//   X[f] = E[f] + W^f O[f]  (W = e^{-2 pi i / n}),  f = 0..N.
// After the product R = X S (S = C or conj C), the inverse runs the same relations
// backwards:
//   E'[f] = (R[f] + conj R[N-f]) / 2,  O'[f] = (R[f] - conj R[N-f]) W^{-f} / 2,
//   Z'[f] = E'[f] + i O'[f],
// an inverse FFT of length N (decimation in frequency: natural order in, bit-reversed
// order out), and the unpacking r[2k] = Re z'[k] / N, r[2k+1] = Im z'[k] / N.
// Each pair (f, N - f) is handled by one thread, so the unpack, product and repack need
// no barrier between them.
#include "common.h"

namespace {

constexpr int CIRC_MAXN2 = 8192;   // largest N = n / 2: N complex doubles = 128 KB of LDS
constexpr int CIRC_THREADS = 1024;
constexpr int FFT_R = 3;           // radix-2 stages per pass over LDS

struct cplx {
    double re, im;
};

// LDS slot of element i.  A row of the 64 four-byte banks holds 16 complex doubles, so the
// power-of-two strides of the radix-2 passes and of the bit-reversed load and store would put
// every lane of a wave on the same banks; XOR-ing the low four index bits with bits 4..7 and
// 9..12 spreads each of those access patterns over all 16 bank groups (a bijection: only bits
// 0..3 change, as a function of the bits above them).
__device__ inline int sw(int i) { return i ^ (((i >> 4) ^ (i >> 9)) & 15); }

__device__ inline double nanmax_d(double m, double a) { return (a > m || a != a) ? a : m; }
__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max_nan(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = nanmax_d(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ inline cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }

// Twiddle factors W_N^e, 0 <= e < N/2, from two 64-entry tables in LDS: Tf[j] = W_N^j and
// Tc[j] = W_N^(64 j), so W_N^e = Tc[e / 64] Tf[e mod 64] (one complex product; exact for e < 64,
// where Tc[0] = 1).  Both tables hold the correctly rounded values of the twiddle table in
// global memory.
struct Twid {
    const double2* Tf;
    const double2* Tc;
    __device__ inline cplx operator()(int e) const {
        const double2 a = Tc[e >> 6], b = Tf[e & 63];
        return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
    }
};

// r consecutive radix-2 stages (r <= 4) of a length-N FFT in place in L.  Forward (decimation
// in time): stages of halves q, 2q, .., q 2^(r-1), q = 2^qlog; inverse (decimation in
// frequency, conjugate twiddles): stages of halves q 2^(r-1), .., 2q, q.  Each thread owns the
// 2^r elements base + m q of aligned blocks of 2^r q (registers: r is a template parameter, so
// every index into v is a constant).  In the stage of half h the pair (m, m + 2^sb) takes the
// twiddle of its lower element's offset p = pos + j q in its block of 2h, j = m mod 2^sb, i.e.
// W_N^(p N / 2h): 2^sb distinct factors per stage, computed once each.
template <bool INV, int RL>
__device__ inline void fft_pass_r(cplx* L, int N, int qlog, int tid, const Twid& W) {
    constexpr int R = 1 << RL;
    const int q = 1 << qlog;
    for (int g = tid; g < (N >> RL); g += CIRC_THREADS) {
        const int pos = g & (q - 1);
        const int base = (g - pos) * R + pos;
        cplx v[R];
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = L[sw(base + m * q)];
#pragma unroll
        for (int t = 0; t < RL; ++t) {
            const int sb = INV ? RL - 1 - t : t;   // pairs m, m + 2^sb (compile-time after unrolling)
            const int h = q << sb;                 // the stage's half
            const int step = N / (2 * h);
            cplx w[R / 2];   // 2^sb <= R / 2 of them used
#pragma unroll
            for (int j = 0; j < (1 << sb); ++j) {
                const cplx x = W((pos + j * q) * step);
                w[j] = INV ? cconj(x) : x;
            }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (m & (1 << sb)) continue;
                const int mm = m + (1 << sb);
                const cplx wm = w[m & ((1 << sb) - 1)];
                if (!INV) {
                    const cplx tt = cmul(wm, v[mm]);
                    const cplx a = v[m];
                    v[m] = cadd(a, tt);
                    v[mm] = csub(a, tt);
                } else {
                    const cplx a = v[m], c = v[mm];
                    v[m] = cadd(a, c);
                    v[mm] = cmul(csub(a, c), wm);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < R; ++m) L[sw(base + m * q)] = v[m];
    }
}

// (only the stage counts up to FFT_R are instantiated: the largest sets the register budget)
template <bool INV>
__device__ inline void fft_pass(cplx* L, int N, int qlog, int r, int tid, const Twid& W) {
    if constexpr (FFT_R >= 4) {
        if (r == 4) return fft_pass_r<INV, 4>(L, N, qlog, tid, W);
    }
    if constexpr (FFT_R >= 3) {
        if (r == 3) return fft_pass_r<INV, 3>(L, N, qlog, tid, W);
    }
    if constexpr (FFT_R >= 2) {
        if (r == 2) return fft_pass_r<INV, 2>(L, N, qlog, tid, W);
    }
    fft_pass_r<INV, 1>(L, N, qlog, tid, W);
}

// MODE 0: y = alpha * (x correlated / convolved with c) + beta * yin.
// MODE 1: the spectrum X[0..N] of x itself (the multiplier's spectrum, once per multiplier),
// and in spec_out[N + 1] the pair (max_f |X[f]|, min_f |X[f]|): the extreme singular values
// of the circulant, which is normal (Theorem 2.1).  A NaN modulus makes both NaN.
template <int MODE, bool CONJ, typename TO>
__global__ void __launch_bounds__(CIRC_THREADS)
circ_kernel(int n, int logN, const double* x, long long sx, long long bx,
            const double2* __restrict__ spec, const double2* __restrict__ tw, const double2* __restrict__ wp,
            double alpha, double beta, const double* yin, long long syi, long long byi, TO* y, long long sy,
            long long by, double2* __restrict__ spec_out, unsigned long long* xsum_max, unsigned long long* ymax) {
    __shared__ cplx L[CIRC_MAXN2];
    __shared__ double2 Tf[64], Tc[64];
    __shared__ double red[CIRC_THREADS / 64];
    const int N = n >> 1;
    const int tid = threadIdx.x;
    const long long b = blockIdx.x;
    const double* xv = x + b * bx;
    // the twiddle tables (entries past N/2 are never used)
    if (tid < 64) {
        Tf[tid] = tid < (N >> 1) ? tw[tid] : make_double2(1.0, 0.0);
        Tc[tid] = 64 * tid < (N >> 1) ? tw[64 * tid] : make_double2(1.0, 0.0);
    }
    Twid W;   // (assigned, not brace-initialized: no constant initializer from LDS addresses)
    W.Tf = Tf;
    W.Tc = Tc;
    // packed, bit-reversed load: every global load issued before the first LDS store
    {
        constexpr int KL = CIRC_MAXN2 / CIRC_THREADS;
        cplx ld[KL];
        if (sx == 1 && ((uintptr_t)xv & 15) == 0) {
            // contiguous vector: one 16-byte load per complex element
            const double2* x2 = reinterpret_cast<const double2*>(xv);
#pragma unroll
            for (int i = 0; i < KL; ++i) {
                const int k = tid + i * CIRC_THREADS;
                if (k < N) {
                    const double2 v = x2[k];
                    ld[i] = {v.x, v.y};
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < KL; ++i) {
                const int k = tid + i * CIRC_THREADS;
                if (k < N) ld[i] = {xv[(2LL * k) * sx], xv[(2LL * k + 1) * sx]};
            }
        }
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int k = tid + i * CIRC_THREADS;
            if (k < N) L[sw((int)(__brev((unsigned)k) >> (32 - logN)))] = ld[i];
        }
        if (MODE == 0 && xsum_max) {
            // sum of |x| over the vector: per thread, per wave, then the waves in order
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < KL; ++i)
                if (tid + i * CIRC_THREADS < N) a += fabs(ld[i].re) + fabs(ld[i].im);
            a = wave_sum_d(a);
            if ((tid & 63) == 0) red[tid >> 6] = a;
        }
    }
    __syncthreads();
    if (MODE == 0 && xsum_max && tid == 0) {
        double a = 0.0;
        for (int w = 0; w < CIRC_THREADS / 64; ++w) a += red[w];
        atomic_max_nonneg(xsum_max, a);
    }
    // forward FFT of length N, decimation in time: the radix-2 stages of halves 1, 2, .., N/2
    // taken FFT_R at a time.  In a pass whose first stage has half q, a thread owns the 2^r
    // elements base + m q of one aligned block of 2^r q and runs the pass's stages on them in
    // registers: stage s pairs m and m + 2^s (bit s of m clear) at distance h = q 2^s, with the
    // twiddle of the lower element's offset pos + (m mod 2^s) q in its block of 2h -- the same
    // butterflies, in the same order per element, as one stage at a time, with a fraction of the
    // LDS passes and barriers.
    for (int s0 = 0; s0 < logN;) {
        const int r = min(FFT_R, logN - s0);
        fft_pass<false>(L, N, s0, r, tid, W);
        __syncthreads();
        s0 += r;
    }
    // spectrum of the real vector, product with the multiplier's spectrum, repack
    double smax = 0.0, smin = __builtin_inf();   // MODE 1: extreme moduli (NaN sticks)
    auto upd_max = [&](double v) { smax = (v != v || v > smax) ? v : smax; };
    auto upd_min = [&](double v) { smin = (v != v || v < smin) ? v : smin; };
    auto track = [&](double v) {
        upd_max(v);
        upd_min(v);
    };
    constexpr int KS = CIRC_MAXN2 / 2 / CIRC_THREADS + 1;   // pairs per thread at most
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        const int f = tid + i * CIRC_THREADS;
        if (f > (N >> 1)) continue;
        if (f == 0) {
            const cplx z0 = L[sw(0)];
            const double x0 = z0.re + z0.im, xN = z0.re - z0.im;   // X[0], X[N] (real)
            if (MODE == 1) {
                spec_out[0] = make_double2(x0, 0.0);
                spec_out[N] = make_double2(xN, 0.0);
                track(fabs(x0));
                track(fabs(xN));
                continue;
            }
            const cplx r0 = cmul({x0, 0.0}, CONJ ? cconj({spec[0].x, spec[0].y}) : cplx{spec[0].x, spec[0].y});
            const cplx rN = cmul({xN, 0.0}, CONJ ? cconj({spec[N].x, spec[N].y}) : cplx{spec[N].x, spec[N].y});
            // E'[0] = (R[0] + conj R[N]) / 2, O'[0] = (R[0] - conj R[N]) / 2
            const cplx e = cscale(cadd(r0, cconj(rN)), 0.5), o = cscale(csub(r0, cconj(rN)), 0.5);
            L[sw(0)] = {e.re - o.im, e.im + o.re};
            continue;
        }
        const int g = N - f;
        const cplx zf = L[sw(f)], zg = L[sw(g)];
        const double2 wf2 = wp[f], wg2 = wp[g];
        const cplx wf = {wf2.x, wf2.y}, wg = {wg2.x, wg2.y};
        // E = (Z[f] + conj Z[N-f]) / 2; O = (Z[f] - conj Z[N-f]) / (2i) = -i (Z[f] - conj Z[N-f]) / 2
        const cplx ef = cscale(cadd(zf, cconj(zg)), 0.5), df = cscale(csub(zf, cconj(zg)), 0.5);
        const cplx of = {df.im, -df.re};
        const cplx eg = cscale(cadd(zg, cconj(zf)), 0.5), dg = cscale(csub(zg, cconj(zf)), 0.5);
        const cplx og = {dg.im, -dg.re};
        const cplx xf = cadd(ef, cmul(wf, of)), xg = cadd(eg, cmul(wg, og));
        if (MODE == 1) {
            spec_out[f] = make_double2(xf.re, xf.im);
            spec_out[g] = make_double2(xg.re, xg.im);
            track(hypot(xf.re, xf.im));
            track(hypot(xg.re, xg.im));
            continue;
        }
        const cplx sf = {spec[f].x, spec[f].y}, sg = {spec[g].x, spec[g].y};
        const cplx rf = cmul(xf, CONJ ? cconj(sf) : sf), rg = cmul(xg, CONJ ? cconj(sg) : sg);
        // E' = (R[f] + conj R[N-f]) / 2, O' = (R[f] - conj R[N-f]) W^{-f} / 2, Z' = E' + i O'
        const cplx ef2 = cscale(cadd(rf, cconj(rg)), 0.5);
        const cplx of2 = cmul(cscale(csub(rf, cconj(rg)), 0.5), cconj(wf));
        const cplx eg2 = cscale(cadd(rg, cconj(rf)), 0.5);
        const cplx og2 = cmul(cscale(csub(rg, cconj(rf)), 0.5), cconj(wg));
        L[sw(f)] = {ef2.re - of2.im, ef2.im + of2.re};
        if (g != f) L[sw(g)] = {eg2.re - og2.im, eg2.im + og2.re};
    }
    if constexpr (MODE == 1) {
        // block reduction of the extreme moduli: within each wave, then across the 8 waves
        for (int o = 32; o >= 1; o >>= 1) {
            const double a = __shfl_xor(smax, o, 64), b = __shfl_xor(smin, o, 64);
            upd_max(a);
            upd_min(b);
        }
        __shared__ double red2[2][CIRC_THREADS / 64];
        const int wv = tid >> 6;
        if ((tid & 63) == 0) {
            red2[0][wv] = smax;
            red2[1][wv] = smin;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 0; w < CIRC_THREADS / 64; ++w) {
                upd_max(red2[0][w]);
                upd_min(red2[1][w]);
            }
            spec_out[N + 1] = make_double2(smax, smin);
        }
        return;
    }
    __syncthreads();
    // inverse FFT of length N, decimation in frequency (bit-reversed output): the stages of
    // halves N/2, N/4, .., 1, FFT_R at a time in the same way (a pass whose last stage has half
    // q: elements base + m q, stage t pairs m and m + 2^(r-1-t))
    for (int sh = logN - 1; sh >= 0;) {
        const int r = min(FFT_R, sh + 1);
        fft_pass<true>(L, N, sh - r + 1, r, tid, W);
        __syncthreads();
        sh -= r;
    }
    const double s = alpha / (double)N;
    TO* yv = y + b * by;
    const double* yiv = (beta != 0.0) ? yin + b * byi : nullptr;
    // contiguous output: the pair of results as one store (16 bytes, or 8 for FP32)
    const bool pair = sy == 1 && ((uintptr_t)yv % (2 * sizeof(TO))) == 0;
    double ym = 0.0;   // max |y| as stored (a NaN sticks)
    for (int k = tid; k < N; k += CIRC_THREADS) {
        const int r = (int)(__brev((unsigned)k) >> (32 - logN));
        const cplx z = L[sw(r)];
        double v0 = s * z.re, v1 = s * z.im;
        if (yiv) {
            v0 = fma(beta, yiv[(2LL * k) * syi], v0);
            v1 = fma(beta, yiv[(2LL * k + 1) * syi], v1);
        }
        if (pair) {
            if constexpr (sizeof(TO) == 8) reinterpret_cast<double2*>(yv)[k] = make_double2(v0, v1);
            else reinterpret_cast<float2*>(yv)[k] = make_float2((float)v0, (float)v1);
        } else {
            yv[(2LL * k) * sy] = (TO)v0;
            yv[(2LL * k + 1) * sy] = (TO)v1;
        }
        if (ymax) ym = nanmax_d(nanmax_d(ym, fabs((double)(TO)v0)), fabs((double)(TO)v1));
    }
    if (ymax) {
        // red was last read before the first FFT pass's barrier: free to reuse
        ym = wave_max_nan(ym);
        if ((tid & 63) == 0) red[tid >> 6] = ym;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int w = 0; w < CIRC_THREADS / 64; ++w) m = nanmax_d(m, red[w]);
            atomic_max_nonneg(ymax, m);
        }
    }
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

bool circ_size_ok(long long n) {
    return n >= 4 && n <= 2LL * CIRC_MAXN2 && (n & (n - 1)) == 0;
}

hipError_t launch_circ_spectrum(int n, const double* c, const double2* tw, const double2* wp, double2* spec,
                                hipStream_t s) {
    if (!circ_size_ok(n)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((circ_kernel<1, false, double>), dim3(1), dim3(CIRC_THREADS), 0, s, n, ilog2(n / 2), c, 1LL,
                       0LL, (const double2*)nullptr, tw, wp, 1.0, 0.0, (const double*)nullptr, 0LL, 0LL,
                       (double*)nullptr, 0LL, 0LL, spec, (unsigned long long*)nullptr, (unsigned long long*)nullptr);
    return hipGetLastError();
}

hipError_t launch_circ_apply(int n, int nvec, int conj, const double* x, long long sx, long long bx, const double2* spec,
                             const double2* tw, const double2* wp, double alpha, double beta, const double* yin,
                             long long syi, long long byi, void* y, int y_f32, long long sy, long long by,
                             hipStream_t s, unsigned long long* xsum_max, unsigned long long* ymax) {
    if (!circ_size_ok(n)) return hipErrorInvalidValue;
    if (nvec <= 0) return hipSuccess;
    const int lg = ilog2(n / 2);
#define GENP_CIRC_GO(CJ, TO)                                                                                   \
    hipLaunchKernelGGL((circ_kernel<0, CJ, TO>), dim3(nvec), dim3(CIRC_THREADS), 0, s, n, lg, x, sx, bx, spec, \
                       tw, wp, alpha, beta, yin, syi, byi, (TO*)y, sy, by, (double2*)nullptr, xsum_max, ymax)
    if (conj) {
        if (y_f32) GENP_CIRC_GO(true, float);
        else GENP_CIRC_GO(true, double);
    } else {
        if (y_f32) GENP_CIRC_GO(false, float);
        else GENP_CIRC_GO(false, double);
    }
#undef GENP_CIRC_GO
    return hipGetLastError();
}
