// Sub-quadratic shared-seed hash: the Toeplitz product as a middle product
// computed with double-precision FFTs (the fast route for CPUs and GPUs that
// Sec. I mentions), exact by construction of the bound and checked per output.
//
// With T[r][c] = s[c - r + M - 1] and xr_j the reversal of x_j,
//     K_j[r] = (s * xr_j)[n_j + M - 2 - r]  mod 2,
// a linear convolution of 0/1 sequences.  With L >= seed_bits a cyclic
// convolution of length L gives those entries unaliased.  Two sub-blocks ride
// in one complex transform (xr_a real, xr_b imaginary): the seed is real, so
// the product with its spectrum keeps them apart and the inverse returns
// (s * xr_a) + i (s * xr_b).
//
// Exactness: entries are integers in [0, n_j]; for 0/1 data the
// double-precision FFT error is of order eps log2 L |x| |s| (about 1e-8 at
// L = 2^18, a few 1e-6 at 2^31), far from 1/2.  L is the smallest of 2^k and
// 3 * 2^k (k >= 12) that holds the seed.  Every output entry is rounded and
// its distance to the integer is checked (> 1/4 sets SSBH_E_PRECISION), so a
// result is never silently wrong.
//
// Transform (four-step, N1 = 64, N2 = L / 64; natural input, transposed
// frequency order Z[N2 k1 + k2] = X[k1 + 64 k2], which the pointwise product
// does not mind):
//   k_fft_cols   64-point FFTs down the columns of a 64-column tile (bits
//                loaded and expanded on the fly), times w_L^(n2 k1), store.
//   k_fft_mid    (L > 2^18) the same split applied again to every row, once
//                for three levels (64 x 64 x L/4096), twice for four
//                (64 x 64 x 64 x L/2^18, L > 3 * 2^23), forward and inverse.
//   k_fft_rows   row FFT (64 .. 8192 points), times the seed spectrum,
//                inverse FFT, times the inverse of the row's twiddle, store
//                (one pass over the data; radix-16 stages, the last forward
//                stage and the first inverse one share registers).
//   k_fft_out    inverse 64-point FFTs down the columns, 1/L, round, parity;
//                64 consecutive output rows per wavefront ballot.
// Independent seeds (seed stride S > 0): transform j carries z_j = s_j +
// i xr_j, sub-block j's own seed window s_j[q] = s[jS + q] in the real part
// and its reversed bits in the imaginary part.  For real u and v,
//     (u + i v) (*) (u + i v) = u (*) u - v (*) v + 2 i (u (*) v),
// so squaring the spectrum pointwise (no second spectrum, no pairing of the
// frequencies k and L - k) and inverting gives 2 (s_j * xr_j) as the
// imaginary part: one transform per sub-block, no separate seed spectra.
// A single sub-block with a shared seed (S = 0, j = 0) takes the same joint
// transform: one transform instead of the seed spectrum's forward passes
// plus a transform of the sub-block.  With a shared seed and several
// sub-blocks the seed spectrum comes from the same forward passes.
// LDS FFTs are Stockham autosort stages with radix-8 (columns) or radix-16 (rows)
// butterflies in registers, then one smaller stage for the rest of the
// length; one twiddle-table read per butterfly group, the other powers by
// squaring and products.  The first stage of each pass reads global memory
// (or bits) and the last one writes its result straight out (spectrum
// product, twiddle, or parity ballot fused in).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include <stdio.h>

#include <hip/hip_ext.h>

#include "ssbh_internal.hpp"

namespace ssbh {

ssbh_status plan_only(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                      hipStream_t stream);

namespace {

constexpr int kN1 = 64;        // column FFT length (and columns per tile)
constexpr int kThreads = 512;

struct FftArgs {
    const uint64_t *sub;
    const uint64_t *len, *woff, *mlen, *ooff;
    const uint64_t *seed;
    uint64_t seed_bits;
    uint64_t mcap;
    uint32_t ns;
    uint32_t n2;               // L / 64 (level-1 columns)
    uint32_t nr;               // row FFT length: L / 64, L / 4096 or
                               // L / 2^18 (two, three or four levels)
    uint64_t L;
    uint32_t pair0;            // first pair of this chunk
    double2 *work;             // [pairs in chunk][L]
    double2 *spec;             // [L], transposed frequency order
    const double2 *tw64;       // w_64^k, k < 64 (column FFTs)
    const double2 *twr;        // w_N2^k, k < N2 (row FFTs)
    const double2 *tlo, *thi;  // w_L^e = thi[e >> 9] * tlo[e & 511]
    const double2 *rlo, *rhi;  // w_(64 nr)^e, same split (the parent of a
                               // row: w_L, w_(L/64) or w_(L/4096))
    const double2 *wlo[3], *whi[3];  // w_(L/64^d)^e for level d, same split
    int lvl;                   // level of a middle pass (1 or 2)
    int per;                   // sub-blocks per transform: 1 (independent
                               // seeds: transform t is sub-block t alone),
                               // 2 (real, imaginary part) or 4 (two per
                               // part, x_lo + 2^18 x_hi)
    uint64_t seed_off;         // first seed bit of the spectrum's seed
    uint64_t stride;           // seed stride S (independent seeds)
    uint64_t *qbuf;            // parity words by transform index q (k_fft_out
                               // writes, k_fft_emit reorders into `out`)
    uint64_t *out;
    int32_t *status;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 conj2(double2 a) {
    return make_double2(a.x, -a.y);
}
// Transform data between passes: complex doubles, or (independent seeds,
// short transforms) complex floats, rounded to nearest on the way out and
// widened exactly on the way in; every butterfly computes in double.
template <class W> __device__ __forceinline__ W to_work(double2 v);
template <> __device__ __forceinline__ double2 to_work<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 to_work<float2>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ double2 from_work(double2 v) { return v; }
__device__ __forceinline__ double2 from_work(float2 v) {
    return make_double2((double)v.x, (double)v.y);
}

// Multiply by -i (forward) or +i (inverse).
template <bool INV>
__device__ __forceinline__ double2 rot90(double2 a) {
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

template <bool INV>
__device__ __forceinline__ void dft2(double2 (&v)[2]) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(double2 (&v)[4]) {
    const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const double2 a2 = cadd(v[1], v[3]), a3 = rot90<INV>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
}

// 8-point DFT, natural order in and out (radix-2 decimation in frequency,
// then the bit-reversal permutation).
template <bool INV>
__device__ __forceinline__ void dft8(double2 (&v)[8]) {
    const double h = 0.70710678118654752440;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double2 a = v[r], b = v[r + 4];
        v[r] = cadd(a, b);
        v[r + 4] = csub(a, b);
    }
    v[5] = cmul(v[5], make_double2(h, INV ? h : -h));
    v[6] = rot90<INV>(v[6]);
    v[7] = cmul(v[7], make_double2(-h, INV ? h : -h));
#pragma unroll
    for (int base = 0; base < 8; base += 4) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const double2 a = v[base + r], b = v[base + r + 2];
            v[base + r] = cadd(a, b);
            v[base + r + 2] = csub(a, b);
        }
    }
    v[3] = rot90<INV>(v[3]);
    v[7] = rot90<INV>(v[7]);
#pragma unroll
    for (int p = 0; p < 8; p += 2) {
        const double2 a = v[p], b = v[p + 1];
        v[p] = cadd(a, b);
        v[p + 1] = csub(a, b);
    }
    double2 t = v[1]; v[1] = v[4]; v[4] = t;
    t = v[3]; v[3] = v[6]; v[6] = t;
}

// 3-point DFT: with w = exp(-+2 pi i / 3), X1,2 = v0 - (v1 + v2)/2 -+ i (sqrt(3)/2)(v1 - v2).
template <bool INV>
__device__ __forceinline__ void dft3(double2 (&v)[3]) {
    const double hs = 0.86602540378443864676;
    const double2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    const double2 m = make_double2(fma(-0.5, t1.x, v[0].x), fma(-0.5, t1.y, v[0].y));
    const double2 r = rot90<INV>(make_double2(hs * t2.x, hs * t2.y));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(double2 (&v)[R]);

// x * w_12^q (q taken mod 12; w_12 = exp(-2 pi i / 12), conjugated for the
// inverse).  q is a compile-time constant after unrolling, so the trivial
// cases cost nothing and the others are one complex multiply by constants.
template <bool INV>
__device__ __forceinline__ double2 mul_w12(double2 x, int q) {
    const double c = 0.86602540378443864676;   // cos 30 deg
    q %= 12;
    if (q == 0) return x;
    if (q == 3) return rot90<INV>(x);
    if (q == 6) return make_double2(-x.x, -x.y);
    if (q == 9) return rot90<!INV>(x);
    const double cs[12] = {1, c, 0.5, 0, -0.5, -c, -1, -c, -0.5, 0, 0.5, c};
    const double sn[12] = {0, 0.5, c, 1, c, 0.5, 0, -0.5, -c, -1, -c, -0.5};
    return cmul(x, make_double2(cs[q], INV ? sn[q] : -sn[q]));
}

// x * w_16^q (q taken mod 16), as mul_w12: cos and sin of multiples of
// 22.5 degrees.
template <bool INV>
__device__ __forceinline__ double2 mul_w16(double2 x, int q) {
    const double c1 = 0.92387953251128675613;  // cos 22.5 deg
    const double s1 = 0.38268343236508977173;  // sin 22.5 deg
    const double h = 0.70710678118654752440;   // cos 45 deg
    q %= 16;
    if (q == 0) return x;
    if (q == 4) return rot90<INV>(x);
    if (q == 8) return make_double2(-x.x, -x.y);
    if (q == 12) return rot90<!INV>(x);
    const double cs[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
    const double sn[16] = {0, s1, h, c1, 1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1};
    return cmul(x, make_double2(cs[q], INV ? sn[q] : -sn[q]));
}

// x * w_R^q for R dividing 12 or R = 16.
template <int R, bool INV>
__device__ __forceinline__ double2 mul_wR(double2 x, int q) {
    if constexpr (R == 16) return mul_w16<INV>(x, q);
    else return mul_w12<INV>(x, q * (12 / R));
}

// R1 * R2-point DFT (R1 R2 divides 12, or is 16), natural order in and out,
// by one Cooley-Tukey split: R2 DFTs of R1 points on the stride-R2
// subsequences, the constant twiddles w_R^(n2 k1), then R1 DFTs of R2 points.
template <int R1, int R2, bool INV>
__device__ __forceinline__ void dft_ct(double2 (&v)[R1 * R2]) {
    constexpr int R = R1 * R2;
    double2 u[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        double2 t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
        dftR<R1, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1)
            u[n2][k1] = mul_wR<R, INV>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        double2 t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) t[n2] = u[n2][k1];
        dftR<R2, INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(double2 (&v)[R]) {
    if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 6) dft_ct<2, 3, INV>(v);
    else if constexpr (R == 12) dft_ct<4, 3, INV>(v);
    else if constexpr (R == 16) dft_ct<4, 4, INV>(v);
    else dft2<INV>(v);
}

// LDS address of element e of FFT f: F interleaved FFTs (e * F + f; lanes
// walk f, so every access is contiguous), or one FFT with the element index
// XOR-swizzled inside blocks of 8 (contiguous and stride-8 accesses of 8
// lanes then cover all banks).
template <int F>
__device__ __forceinline__ int lds_addr(int f, int e) {
    if constexpr (F > 1) return e * F + f;
    else return e ^ ((e >> 3) & 7);
}

// Stage radices of an N-point FFT, N = 2^a or 3 * 2^a: radix 8 while it
// divides the power of two; the remaining 2 or 4 is merged with the 3 into
// one radix-6 or radix-12 stage, or is a stage of its own when there is no 3.
constexpr int two_part(int n) { return n % 3 == 0 ? n / 3 : n; }
constexpr int pow2_bits(int n) { return ilog2c(two_part(n)); }
constexpr int num_stages(int n) {
    return pow2_bits(n) / 3 + (n % 3 == 0 ? 1 : (pow2_bits(n) % 3 ? 1 : 0));
}
constexpr int radix_of(int n, int s) {
    return s < pow2_bits(n) / 3 ? 8
         : (n % 3 == 0 ? 3 : 1) * (1 << (pow2_bits(n) % 3));
}
// Span (product of the radices before it) of stage s.
constexpr int span_of(int n, int s) {
    return s == 0 ? 1 : span_of(n, s - 1) * radix_of(n, s - 1);
}
// The powers w^(2^b), b < tw_bits(R), give every twiddle w^r with r < R.
constexpr int tw_bits(int r) { return ilog2c(r - 1) + 1; }

// Work of one stage: item g = threadIdx.x + kThreads * i (i < PER) is group
// j = g / F of FFT f = g % F, if g < TOTAL.
template <int N, int R, int F> struct StageShape {
    static constexpr int G = N / R;
    static constexpr int TOTAL = F * G;
    static constexpr int PER = (TOTAL + kThreads - 1) / kThreads;
    static constexpr bool active(int g) { return TOTAL % kThreads == 0 || g < TOTAL; }
};

__device__ __forceinline__ double2 csq(double2 a) {
    return make_double2(fma(a.x, a.x, -a.y * a.y), 2.0 * a.x * a.y);
}

// Twiddles of stage S (S >= 1) for group j: v[r] *= w^r, r < R, with
// w = w_(SPAN R)^(j mod SPAN) = w_N^base, base = (j mod SPAN) N / (SPAN R),
// from the table of w_N^k (conjugated for the inverse).  One table read per
// group: w^(2^b) by repeated squaring, every other power as w^(2^b) w^rest
// (r = 2^b + rest); a few roundings more than reading every power, and one
// vector-memory instruction instead of several.  With F >= 64 interleaved
// FFTs j is the same on a whole wavefront.
template <int N, int F, int S, bool INV, int R>
__device__ __forceinline__ void twiddle(double2 (&v)[R], int j,
                                        const double2 *tw) {
    constexpr int SPAN = span_of(N, S);
    int base = (j % SPAN) * (N / (SPAN * R));
    if constexpr (F % 64 == 0) base = __builtin_amdgcn_readfirstlane(base);
    double2 pw[tw_bits(R)];
    pw[0] = tw[base];
    if (INV) pw[0] = conj2(pw[0]);
#pragma unroll
    for (int b = 1; b < tw_bits(R); ++b) pw[b] = csq(pw[b - 1]);
    double2 wr[R];
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const int hb = ilog2c(r);
        const int rest = r - (1 << hb);
        wr[r] = rest ? cmul(pw[hb], wr[rest]) : pw[hb];
        v[r] = cmul(v[r], wr[r]);
    }
}

// Stage S (radix R, span Ns) of F Stockham FFTs of length N.  Group j of an
// FFT takes elements j + r N/R (from `ld`), twiddles them by w_{Ns R}^(r (j
// mod Ns)), transforms, and hands its R results to `st(f, d, Ns, v)`: v[r]
// is element d + r Ns, d = (j / Ns) Ns R + (j mod Ns).  Barrier between all
// loads and all stores (they share the LDS buffer); END: barrier after the
// stores (the next stage reads them).
template <int N, int F, bool INV, int S, bool END, class Ld, class St>
__device__ __forceinline__ void fft_stage(const double2 *tw, Ld ld, St st) {
    constexpr int R = radix_of(N, S), SPAN = span_of(N, S);
    using SH = StageShape<N, R, F>;
    double2 v[SH::PER][R];
#pragma unroll
    for (int i = 0; i < SH::PER; ++i) {
        const int g = threadIdx.x + kThreads * i;
        if (SH::active(g)) {
            const int f = g % F, j = g / F;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = ld(f, j + r * SH::G);
            if constexpr (S > 0) twiddle<N, F, S, INV>(v[i], j, tw);
            dftR<R, INV>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SH::PER; ++i) {
        const int g = threadIdx.x + kThreads * i;
        if (SH::active(g)) {
            const int f = g % F, j = g / F;
            st(f, (j / SPAN) * SPAN * R + (j % SPAN), SPAN, v[i]);
        }
    }
    if (END) __syncthreads();
}

template <int N, int F, bool INV, int S, class Ld, class St, class LL, class LS>
__device__ __forceinline__ void fft_stages(const double2 *tw, Ld first_ld,
                                           St last_st, LL lds_ld, LS lds_st) {
    constexpr int NST = num_stages(N);
    if constexpr (S == NST - 1) {
        fft_stage<N, F, INV, S, false>(tw, lds_ld, last_st);
    } else {
        if constexpr (S == 0)
            fft_stage<N, F, INV, S, true>(tw, first_ld, lds_st);
        else
            fft_stage<N, F, INV, S, true>(tw, lds_ld, lds_st);
        fft_stages<N, F, INV, S + 1>(tw, first_ld, last_st, lds_ld, lds_st);
    }
}

// Number of elements of a group handed to a store functor.
template <class V> constexpr int group_size(const V &) {
    return sizeof(V) / sizeof(double2);
}

// A whole FFT of length N (2^a or 3 * 2^a, N >= 64) over F transforms, with
// the twiddle table of w_N^k: the first stage reads with `first_ld`, the last
// stage writes its groups with `last_st`, the stages between go through the
// LDS buffer.  Every stage has a barrier between its loads and stores
// (first_ld and last_st may touch the same buffer) and the inner ones one
// after the stores.
template <int N, int F, bool INV, class Ld, class St>
__device__ __forceinline__ void fft_run(double2 *buf, const double2 *tw,
                                        Ld first_ld, St last_st) {
    static_assert(num_stages(N) >= 2, "at least two stages");
    auto lds_ld = [&](int f, int e) { return buf[lds_addr<F>(f, e)]; };
    auto lds_st = [&](int f, int d, int span, auto &v) {
#pragma unroll
        for (int r = 0; r < group_size(v); ++r)
            buf[lds_addr<F>(f, d + r * span)] = v[r];
    };
    fft_stages<N, F, INV, 0>(tw, first_ld, last_st, lds_ld, lds_st);
}

// Hands v[r] w0 w^r to put(r, .) for the group's r = 0, 1, ..: the powers of
// w by repeated multiplication (at most 11 factors, a few roundings).
template <int R, class Put>
__device__ __forceinline__ void twiddle_run(const double2 (&v)[R], double2 w0,
                                            double2 w, Put put) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        put(r, cmul(v[r], w0));
        if (r + 1 < R) w0 = cmul(w0, w);
    }
}

// 64-point FFTs down the 64 columns of a tile, 512 threads: column f =
// lane, butterfly group j = wavefront.  Two radix-8 stages (the first's
// group j writes elements 8j .. 8j+7, the second's group j reads j + 8k and
// is twiddled by w_64^(k j)); the transposition between them goes through
// LDS in two halves, real parts then imaginary parts, so `x` holds 64 x 64
// doubles (32 KiB) instead of complex values.  `ld(f, e)` gives element e of
// column f; `st(f, j, 8, v)` takes the second stage's group j (elements
// j + 8r).
template <bool INV, class Ld, class St>
__device__ __forceinline__ void fft64_cols(double *x, const double2 *tw, Ld ld,
                                           St st) {
    const int f = threadIdx.x & 63, j = threadIdx.x >> 6;
    double2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = ld(f, j + 8 * r);
    dft8<INV>(v);
    double2 u[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[(8 * j + r) * kN1 + f] = v[r].x;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k].x = x[(j + 8 * k) * kN1 + f];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) x[(8 * j + r) * kN1 + f] = v[r].y;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k].y = x[(j + 8 * k) * kN1 + f];
    twiddle<kN1, kN1, 1, INV>(u, j, tw);
    dft8<INV>(u);
    st(f, j, 8, u);
}

__device__ __forceinline__ double2 omega_l(const FftArgs &a, uint64_t e) {
    return cmul(a.thi[e >> 9], a.tlo[e & 511]);
}
__device__ __forceinline__ double2 omega_r(const FftArgs &a, uint64_t e) {
    return cmul(a.rhi[e >> 9], a.rlo[e & 511]);
}

// Bits b0 .. b0+63 of a bit string of nbits bits at words w (0 outside).
__device__ __forceinline__ uint64_t window64(const uint64_t *w, int64_t nbits,
                                             int64_t b0) {
    if (b0 >= nbits || b0 <= -64) return 0ull;
    const int64_t wi = b0 >> 6;                 // floor division
    const int sh = (int)(b0 & 63);
    const uint64_t lo = (wi >= 0) ? w[wi] : 0ull;
    const uint64_t hi = ((wi + 1) * 64 < nbits) ? w[wi + 1] : 0ull;
    uint64_t v = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
    const int64_t valid = nbits - b0;
    if (valid < 64) v &= (1ull << valid) - 1ull;
    return v;
}

// Scale of the high sub-block of a part when four share a transform: the
// middle product of a low sub-block is at most its length n_j < 2^18 (the
// largest sub-block length the library accepts is far below), so the part's
// integer result lo + 2^18 hi gives both back.
constexpr double kPackScale = 262144.0;
constexpr int kPackBits = 18;

// Sub-block in slot `slot` of transform pl of the chunk; a.ns when there is
// none.  Slots: per = 1: 0 only; per = 2: 0 real, 1 imaginary; per = 4: 0 / 1
// the low / high sub-block of the real part, 2 / 3 of the imaginary part.
__device__ __forceinline__ uint64_t sub_of(const FftArgs &a, uint32_t pl, int slot) {
    if (slot >= a.per) return a.ns;
    const uint64_t j = (uint64_t)a.per * (a.pair0 + pl) + (uint64_t)slot;
    return j < a.ns ? j : (uint64_t)a.ns;
}

// Forward column pass.  SEED: the input is the seed from bit seed_off on
// (u[q] = s[seed_off + q], real); JOINT: transform p is sub-block j = pair0 +
// p with its own seed window s[jS + q] real and xr_j imaginary; else
// transform p's reversed sub-blocks (PACK: xr_0 + 2^18 xr_1 real, xr_2 +
// 2^18 xr_3 imaginary; else xr_0 real, xr_1 imaginary).  The first stage
// reads bits, the last stage stores times w_L^(n2 k1).  A sub-block whose
// n_j + m_cap - 1 exceeds L (possible only with a seed stride below n_max +
// m_cap - 1) sets SSBH_E_UNSUPPORTED.
template <bool SEED, bool PACK, bool JOINT = false, class W = double2>
__global__ __launch_bounds__(kThreads) void k_fft_cols(FftArgs a) {
    constexpr int SLOTS = PACK ? 4 : 2;
    __shared__ double buf[kN1 * kN1];
    __shared__ uint64_t win[SLOTS][kN1];
    if (*a.status) return;
    const uint32_t n2 = a.n2;
    const uint32_t c0 = blockIdx.x * kN1;
    const uint32_t pl = blockIdx.y;
    const int t = threadIdx.x;
    // 64-bit windows: thread (n1, slot) for the 64 columns of this tile.
    if (t < SLOTS * kN1) {
        const int n1 = t & (kN1 - 1), part = t >> 6;
        uint64_t v = 0ull;
        if (SEED) {
            if (part == 0)
                v = window64(a.seed, (int64_t)a.seed_bits,
                             (int64_t)(a.seed_off + (uint64_t)n2 * n1 + c0));
        } else if (JOINT && part == 0) {
            const uint64_t j = sub_of(a, pl, 0);
            if (j < a.ns)
                v = window64(a.seed, (int64_t)a.seed_bits,
                             (int64_t)(j * a.stride + (uint64_t)n2 * n1 + c0));
        } else {
            const uint64_t j = sub_of(a, pl, JOINT ? 0 : part);
            if (j < a.ns) {
                const int64_t n = (int64_t)a.len[j];
                if (n1 == 0 && blockIdx.x == 0 &&
                    ((uint64_t)n + a.mcap - 1 > a.L || (PACK && n >> kPackBits)))
                    atomicCAS(a.status, 0, (int32_t)SSBH_E_UNSUPPORTED);
                // xr[q] = x[n-1-q] for q = n2*n1 + c0 + i, i < 64.
                const int64_t b0 = n - 1 - ((int64_t)n2 * n1 + c0) - 63;
                v = __brevll(window64(a.sub + a.woff[j], n, b0));
            }
        }
        win[part][n1] = v;
    }
    __syncthreads();
    W *y = reinterpret_cast<W *>(a.work) + (size_t)pl * a.L;
    // Element (column i = f, row n1 = e).
    auto ld = [&](int f, int e) {
        const double b0 = (double)((win[0][e] >> f) & 1ull);
        const double b1 = (double)((win[1][e] >> f) & 1ull);
        if constexpr (PACK)
            return make_double2(fma(kPackScale, b1, b0),
                                fma(kPackScale, (double)((win[3][e] >> f) & 1ull),
                                    (double)((win[2][e] >> f) & 1ull)));
        else
            return make_double2(b0, b1);
    };
    // Output k1 of column n2i = c0 + f gets w_L^(n2i k1); a group's outputs
    // k1 = k0 + r span take w_L^(n2i k0) (w_L^(n2i span))^r.
    auto st = [&](int f, int k0, int span, auto &v) {
        const uint64_t n2i = c0 + f;
        twiddle_run(v, omega_l(a, n2i * k0), omega_l(a, n2i * span),
                    [&](int r, double2 x) {
                        y[(size_t)(k0 + r * span) * n2 + n2i] = to_work<W>(x);
                    });
    };
    fft64_cols<false>(buf, a.tw64, ld, st);
}

// ------------------------------------------------------------ row pass ---
//
// Stockham stages with radix-16 butterflies where the length allows.  The
// last forward stage keeps its results in registers: they are multiplied by
// the seed spectrum there and fed straight into the inverse, which runs the
// forward stages in reverse order, each as its exact inverse (read where the
// forward stage wrote, inverse DFT, conjugate twiddles, write where it
// read).  Per row that is 2 S - 2 LDS writes and as many reads for S stages,
// one LDS round trip and its barriers fewer than a second forward-style pass.
//
// A workgroup holds RPW rows of TPR threads each: TPR covers the widest
// stage (groups beyond it loop), and short rows are packed so that the
// workgroup has up to 256 threads and at most 48 KiB of LDS.

struct RowPlan {
    int ns;        // stages
    int r[4];      // radices, first to last
};
// Radix plan per row length: few stages, and for short rows stages whose
// group counts are alike (idle threads are what packing cannot recover).
constexpr RowPlan rp_plan(int n) {
    switch (n) {
    case 64: return {2, {8, 8, 0, 0}};
    case 128: return {2, {16, 8, 0, 0}};
    case 192: return {2, {16, 12, 0, 0}};
    case 256: return {2, {16, 16, 0, 0}};
    case 384: return {3, {8, 8, 6, 0}};
    case 512: return {3, {8, 8, 8, 0}};
    case 768: return {3, {16, 8, 6, 0}};
    case 1024: return {3, {16, 8, 8, 0}};
    case 1536: return {3, {16, 16, 6, 0}};
    case 2048: return {3, {16, 16, 8, 0}};
    case 3072: return {3, {16, 16, 12, 0}};
    case 4096: return {3, {16, 16, 16, 0}};
    case 6144: return {4, {16, 16, 4, 6}};
    default: return {4, {2, 16, 16, 16}};   // 8192
    }
}
constexpr int rp_stages(int n) { return rp_plan(n).ns; }
constexpr int rp_radix(int n, int s) { return rp_plan(n).r[s]; }
constexpr int rp_span(int n, int s) {
    return s == 0 ? 1 : rp_span(n, s - 1) * rp_radix(n, s - 1);
}
constexpr int rp_maxg(int n, int s = 0) {
    return s == rp_stages(n) ? 0 : std::max(n / rp_radix(n, s), rp_maxg(n, s + 1));
}
constexpr int pow2_ceil(int x) { return x <= 1 ? 1 : 2 * pow2_ceil((x + 1) / 2); }
constexpr int pow2_floor(int x) { return x <= 1 ? 1 : 2 * pow2_floor(x / 2); }
// Threads per row and rows per workgroup.
constexpr int rp_tpr(int n) {
    return n >= 6144 ? 512 : std::min(256, pow2_ceil(rp_maxg(n)));
}
constexpr int rp_rpw(int n) {
    return pow2_floor(std::max(1, std::min(256 / std::min(256, rp_tpr(n)),
                                           (48 * 1024) / (16 * n))));
}
constexpr int rp_threads(int n) { return rp_tpr(n) * rp_rpw(n); }

// Stage S of the row plan: group j < G reads elements in(j, k) = j + k G
// (k < R) and writes out(j, r) = (j / span) span R + (j mod span) + r span.
// Group j = lt + TPR i (i < PER) belongs to the row's thread lt.
template <int N, int S> struct RowStage {
    static constexpr int R = rp_radix(N, S), SPAN = rp_span(N, S), G = N / R;
    static constexpr int TPR = rp_tpr(N);
    static constexpr int PER = (G + TPR - 1) / TPR;
    static __device__ bool active(int g) { return G % TPR == 0 || g < G; }
    static __device__ int in(int j, int k) { return j + k * G; }
    static __device__ int out(int j, int r) {
        return (j / SPAN) * SPAN * R + (j % SPAN) + r * SPAN;
    }
    static __device__ int base(int j) { return (j % SPAN) * (N / (SPAN * R)); }
};

// LDS address of row element e: the index XOR-swizzled inside blocks of 8
// by bits 4..6, so that stride-16 accesses (a radix-16 first stage) and
// contiguous ones of 8 lanes both touch every bank once.
__device__ __forceinline__ int rsw(int e) { return e ^ ((e >> 4) & 7); }

// w^r, r < R, from w (wr[0] = 1): w^(2^b) by squaring, the others as
// w^(2^b) w^rest.
template <int R>
__device__ __forceinline__ void tw_powers(double2 (&wr)[R], double2 w) {
    double2 pw[tw_bits(R)];
    pw[0] = w;
#pragma unroll
    for (int b = 1; b < tw_bits(R); ++b) pw[b] = csq(pw[b - 1]);
    wr[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const int hb = ilog2c(r);
        const int rest = r - (1 << hb);
        wr[r] = rest ? cmul(pw[hb], wr[rest]) : pw[hb];
    }
}

// Forward stage S < last of the row at `buf` (thread lt of the row): read
// (global `ld` for S = 0, else LDS), twiddle, DFT, write LDS.  Barrier
// before the writes (S > 0: other groups may still read those places) and
// after them.
template <int N, int S, class Ld>
__device__ __forceinline__ void row_fwd(double2 *buf, const double2 *tw, int lt,
                                        Ld ld) {
    using T = RowStage<N, S>;
    double2 v[T::PER][T::R];
#pragma unroll
    for (int i = 0; i < T::PER; ++i) {
        const int g = lt + T::TPR * i;
        if (T::active(g)) {
#pragma unroll
            for (int k = 0; k < T::R; ++k)
                v[i][k] = S == 0 ? ld(T::in(g, k)) : buf[rsw(T::in(g, k))];
            if constexpr (S > 0) {
                double2 wr[T::R];
                tw_powers(wr, tw[T::base(g)]);
#pragma unroll
                for (int k = 1; k < T::R; ++k) v[i][k] = cmul(v[i][k], wr[k]);
            }
            dftR<T::R, false>(v[i]);
        }
    }
    if constexpr (S > 0) __syncthreads();
#pragma unroll
    for (int i = 0; i < T::PER; ++i) {
        const int g = lt + T::TPR * i;
        if (T::active(g)) {
#pragma unroll
            for (int r = 0; r < T::R; ++r) buf[rsw(T::out(g, r))] = v[i][r];
        }
    }
    __syncthreads();
}

// Inverse of forward stage S (0 < S < last): read LDS where it wrote,
// inverse DFT, conjugate twiddles, write where it read.
template <int N, int S>
__device__ __forceinline__ void row_inv(double2 *buf, const double2 *tw, int lt) {
    using T = RowStage<N, S>;
    double2 v[T::PER][T::R];
#pragma unroll
    for (int i = 0; i < T::PER; ++i) {
        const int g = lt + T::TPR * i;
        if (T::active(g)) {
#pragma unroll
            for (int r = 0; r < T::R; ++r) v[i][r] = buf[rsw(T::out(g, r))];
            dftR<T::R, true>(v[i]);
            double2 wr[T::R];
            tw_powers(wr, conj2(tw[T::base(g)]));
#pragma unroll
            for (int k = 1; k < T::R; ++k) v[i][k] = cmul(v[i][k], wr[k]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < T::PER; ++i) {
        const int g = lt + T::TPR * i;
        if (T::active(g)) {
#pragma unroll
            for (int k = 0; k < T::R; ++k) buf[rsw(T::in(g, k))] = v[i][k];
        }
    }
    __syncthreads();
}

template <int N, int S, class Ld>
__device__ __forceinline__ void row_fwd_all(double2 *buf, const double2 *tw,
                                            int lt, Ld ld) {
    if constexpr (S + 1 < rp_stages(N)) {
        row_fwd<N, S>(buf, tw, lt, ld);
        row_fwd_all<N, S + 1>(buf, tw, lt, ld);
    }
}
template <int N, int S>
__device__ __forceinline__ void row_inv_all(double2 *buf, const double2 *tw, int lt) {
    if constexpr (S >= 1) {
        row_inv<N, S>(buf, tw, lt);
        row_inv_all<N, S - 1>(buf, tw, lt);
    }
}

// Row pass over rows of N2 (= nr) points.  SPEC: forward only, the result is
// the seed spectrum; else forward, times the spectrum, inverse, times
// w_(64 N2)^(-e (row mod 64)) -- the inverse of the twiddle of the column
// pass that made the row (k_fft_cols with two levels, the last k_fft_mid
// with three or four).  Workgroup x holds rows x RPW .. x RPW + RPW - 1.
// SQ (independent seeds): the spectrum is squared instead (see the top of
// the file); the seed spectrum is not read.
template <int N2, bool SPEC, bool SQ = false, class W = double2>
__global__ __launch_bounds__(rp_threads(N2)) void k_fft_rows(FftArgs a) {
    constexpr int TPR = rp_tpr(N2), RPW = rp_rpw(N2);
    __shared__ double2 lds[N2 * RPW];
    if (*a.status) return;
    constexpr int NS = rp_stages(N2);
    static_assert(NS >= 2, "at least two stages");
    using TL = RowStage<N2, NS - 1>;
    using T0 = RowStage<N2, 0>;
    const int lt = threadIdx.x % TPR;
    const uint32_t row = blockIdx.x * RPW + threadIdx.x / TPR;
    const uint32_t pl = SPEC ? 0u : blockIdx.y;
    const uint64_t k1 = row & 63u;
    double2 *buf = lds + (threadIdx.x / TPR) * N2;
    W *y = reinterpret_cast<W *>(a.work) + (size_t)pl * a.L + (size_t)row * N2;
    double2 *sp = a.spec + (size_t)row * N2;
    const double2 *tw = a.twr;
    row_fwd_all<N2, 0>(buf, tw, lt, [&](int e) { return from_work(y[e]); });

    // Last stage: forward DFT in registers, spectrum product, inverse DFT.
    double2 v[TL::PER][TL::R], wr[TL::PER][TL::R];
#pragma unroll
    for (int i = 0; i < TL::PER; ++i) {
        const int g = lt + TPR * i;
        if (TL::active(g)) {
#pragma unroll
            for (int k = 0; k < TL::R; ++k) v[i][k] = buf[rsw(TL::in(g, k))];
            tw_powers(wr[i], tw[TL::base(g)]);
#pragma unroll
            for (int k = 1; k < TL::R; ++k) v[i][k] = cmul(v[i][k], wr[i][k]);
            dftR<TL::R, false>(v[i]);
            if (SPEC) {
#pragma unroll
                for (int r = 0; r < TL::R; ++r) sp[TL::out(g, r)] = v[i][r];
                continue;
            }
            if constexpr (SQ) {
#pragma unroll
                for (int r = 0; r < TL::R; ++r) v[i][r] = csq(v[i][r]);
            } else {
#pragma unroll
                for (int r = 0; r < TL::R; ++r) v[i][r] = cmul(v[i][r], sp[TL::out(g, r)]);
            }
            dftR<TL::R, true>(v[i]);
            // The same group's places: no other thread reads them, no barrier.
#pragma unroll
            for (int k = 0; k < TL::R; ++k)
                buf[rsw(TL::in(g, k))] = k ? cmul(v[i][k], conj2(wr[i][k])) : v[i][k];
        }
    }
    if (SPEC) return;
    __syncthreads();
    row_inv_all<N2, NS - 2>(buf, tw, lt);

    // Inverse of stage 0 (no twiddle), element e = g + k G0 times
    // conj(w^(g k1)) conj(w^(G0 k1))^k, w = w_(64 N2), to global memory.
    double2 u[T0::PER][T0::R];
#pragma unroll
    for (int i = 0; i < T0::PER; ++i) {
        const int g = lt + TPR * i;
        if (T0::active(g)) {
#pragma unroll
            for (int r = 0; r < T0::R; ++r) u[i][r] = buf[rsw(T0::out(g, r))];
            dftR<T0::R, true>(u[i]);
            twiddle_run(u[i], conj2(omega_r(a, (uint64_t)g * k1)),
                        conj2(omega_r(a, (uint64_t)T0::G * k1)),
                        [&](int k, double2 x) { y[T0::in(g, k)] = to_work<W>(x); });
        }
    }
}

__device__ __forceinline__ double2 omega_d(const FftArgs &a, int d, uint64_t e) {
    return cmul(a.whi[d][e >> 9], a.wlo[d][e & 511]);
}

// Middle column pass at level d (1 or 2) of a transform with three or four
// levels.  Each row of level d (P = L / 64^d points; row index p < 64^d,
// its index in its parent kp = p mod 64) is viewed as 64 x C, C = P / 64,
// and transformed by 64-point FFTs down 64-column tiles.  Forward: times
// w_P^(m l) (m the column, l the output of the 64-point FFT), which makes
// the rows of level d + 1.  Inverse (INV): the rows of level d + 1 are
// already back in place; after the inverse FFT the twiddle of the level
// above is undone, times w_(64 P)^(-q kp) with q = C k + m the element of
// this row.
template <bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_mid(FftArgs a) {
    __shared__ double buf[kN1 * kN1];
    if (*a.status) return;
    const int d = a.lvl;
    const uint64_t P = a.L >> (6 * d);
    const uint32_t C = (uint32_t)(P >> 6);
    const uint32_t c0 = blockIdx.x * kN1;
    const uint64_t p = blockIdx.y;
    const uint64_t kp = p & 63u;
    const uint32_t pl = blockIdx.z;
    double2 *y = a.work + (size_t)pl * a.L + (size_t)p * P;
    auto ld = [&](int f, int e) { return y[(size_t)e * C + c0 + f]; };
    // A group's outputs k = k0 + r span: the twiddle's exponent grows by a
    // fixed step per r, so it is a running product.
    auto st = [&](int f, int k0, int span, auto &v) {
        const uint64_t m = c0 + f;
        const double2 w0 = INV ? conj2(omega_d(a, d - 1, ((uint64_t)k0 * C + m) * kp))
                               : omega_d(a, d, m * (uint64_t)k0);
        const double2 ws = INV ? conj2(omega_d(a, d - 1, (uint64_t)span * C * kp))
                               : omega_d(a, d, m * (uint64_t)span);
        twiddle_run(v, w0, ws, [&](int r, double2 x) {
            y[(size_t)(k0 + r * span) * C + m] = x;
        });
    };
    fft64_cols<INV>(buf, a.tw64, ld, st);
}

// Where the parities of sub-block j go.  Output row r of the sub-block is
// entry q = Q0 - r of its convolution, Q0 = n_j + m_cap - 2, so its m_j rows
// are q in [qlo, Q0], qlo = Q0 - m_j + 1.  The words of that range (64
// q values each, aligned to multiples of 64) sit at qbuf[qoff + q / 64 -
// qlo / 64], qoff = ooff_j / 64 + 3 j: the regions of consecutive sub-blocks
// do not overlap, and all of them fit out_cap_bits / 64 + 3 n_sub words.
struct QRange {
    int64_t q0, qlo;     // needed entries [qlo, q0]; q0 = -1 when none
    int64_t widx;        // qbuf index of entry 0's word: qoff - qlo / 64
};
__device__ __forceinline__ QRange q_range(const FftArgs &a, uint64_t j, int64_t n,
                                          int64_t m, uint64_t o) {
    if (n == 0 || m == 0) return QRange{-1, 0, 0};    // rows are all zero
    QRange r;
    r.q0 = n + (int64_t)a.mcap - 2;
    r.qlo = r.q0 - m + 1;                             // >= n - 1 >= 0
    r.widx = (int64_t)(o >> 6) + 3 * (int64_t)j - (r.qlo >> 6);
    return r;
}

// Inverse column pass.  The last stage hands the wavefront the 64 columns of
// one row n1 (lane = column): 64 consecutive entries q, one aligned parity
// word per sub-block (ballot), stored with a plain store (each word has one
// writer); k_fft_emit then places them.  PACK: a part's integer is
// lo + 2^18 hi, the low sub-block's parity is its bit 0, the high one's its
// bit 18.  JOINT: the imaginary part is 2 (s_j * xr_j); its half is rounded
// and checked like any other entry, and the real part carries no sub-block.
template <bool PACK, bool JOINT = false, class W = double2>
__global__ __launch_bounds__(kThreads) void k_fft_out(FftArgs a) {
    constexpr int SLOTS = PACK ? 4 : JOINT ? 1 : 2;
    constexpr int PER_PART = PACK ? 2 : 1;
    __shared__ double2 buf[kN1 * kN1];
    if (*a.status) return;
    const uint32_t n2 = a.n2;
    const uint32_t c0 = blockIdx.x * kN1;
    const uint32_t pl = blockIdx.y;
    const W *w = reinterpret_cast<const W *>(a.work) + (size_t)pl * a.L;
    const int lane = threadIdx.x & 63;
    const double scale = 1.0 / (double)a.L;
    // The same for the whole workgroup: kept in scalar registers.
    auto uni = [](int64_t x) {
        const uint64_t u = (uint64_t)x;
        return (int64_t)((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)u) |
                         ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32)) << 32));
    };
    QRange qr[SLOTS];
#pragma unroll
    for (int slot = 0; slot < SLOTS; ++slot) {
        const uint64_t j = sub_of(a, pl, slot);
        const QRange r = j < a.ns ? q_range(a, j, (int64_t)a.len[j], (int64_t)a.mlen[j], a.ooff[j])
                                  : QRange{-1, 0, 0};
        qr[slot] = QRange{uni(r.q0), uni(r.qlo), uni(r.widx)};
    }
    bool bad = false;
    auto ld = [&](int f, int e) { return from_work(w[(size_t)e * n2 + c0 + f]); };
    // Parity of an integer-valued double below 2^53, exactly.
    auto parity = [](double x) { return x != 2.0 * floor(0.5 * x); };
    // Called with the same row n1 on all 64 lanes: entries q = qb + lane.
    auto st1 = [&](int n1, double2 x) {
        const int64_t qb = (int64_t)n2 * n1 + c0;
        const int64_t q = qb + lane;
#pragma unroll
        for (int part = JOINT ? 1 : 0; part < 2; ++part) {
            // JOINT: half the imaginary part is the entry.
            const double v = (part ? x.y : x.x) * (JOINT ? 0.5 * scale : scale);
            const double rv = rint(v);
            const bool off = fabs(v - rv) > 0.25 || rv < -0.25;
            // PACK: rv = lo + 2^18 hi, lo < 2^18; parity(lo) = parity(rv).
            const double hi = PACK ? floor(rv * (1.0 / kPackScale)) : 0.0;
#pragma unroll
            for (int h = 0; h < PER_PART; ++h) {
                const QRange &r = qr[JOINT ? 0 : PER_PART * part + h];
                if (qb > r.q0 || qb + 63 < r.qlo) continue;  // uniform
                // Only the needed entries [qlo, q0] count as off.
                if (off && q >= r.qlo && q <= r.q0) bad = true;
                const uint64_t word = ballot64(parity(h ? hi : rv));
                if (lane == 0) a.qbuf[r.widx + (qb >> 6)] = word;
            }
        }
    };
    auto st = [&](int f, int n0, int span, auto &v) {
        (void)f;
#pragma unroll
        for (int r = 0; r < group_size(v); ++r) st1(n0 + r * span, v[r]);
    };
    fft_run<kN1, kN1, true>(buf, a.tw64, ld, st);
    if (bad && lane == 0) atomicCAS(a.status, 0, (int32_t)SSBH_E_PRECISION);
}

// Output: sub-block j (blockIdx.x) writes its m_j rows at bit o_j of the
// output.  Output word W holds rows R0 .. R0 + 63, R0 = 64 W - o_j, that is
// entries q = Q0 - R0 - t: the 64-entry window from qa = Q0 - R0 - 63 taken
// from its one or two parity words, bit-reversed.  Words wholly inside the
// sub-block's range have no other writer (plain store); the two at its ends
// are shared with the neighbours (atomic XOR into the zeroed output).
__global__ __launch_bounds__(256) void k_fft_emit(FftArgs a) {
    if (*a.status) return;
    const uint64_t j = blockIdx.x;
    const int64_t n = (int64_t)a.len[j], m = (int64_t)a.mlen[j];
    if (n == 0 || m == 0) return;                   // all-zero rows
    const uint64_t o = a.ooff[j];
    const QRange r = q_range(a, j, n, m, o);
    const uint64_t w0 = o >> 6, w1 = (o + (uint64_t)m - 1) >> 6;
    for (uint64_t W = w0 + (uint64_t)blockIdx.y * 2048 + threadIdx.x;
         W <= w1 && W < w0 + (uint64_t)(blockIdx.y + 1) * 2048; W += 256) {
        const int64_t R0 = (int64_t)(64 * W) - (int64_t)o;
        const int64_t tlo = R0 < 0 ? -R0 : 0;                  // first row bit
        const int64_t thi = R0 + 63 < m ? 63 : m - 1 - R0;     // last row bit
        // Needed entries of this word: q in [Q0 - R0 - thi, Q0 - R0 - tlo].
        const int64_t qa = r.q0 - R0 - 63;
        const int64_t qmin = r.q0 - R0 - thi, qmax = r.q0 - R0 - tlo;
        const int64_t wa = qa >= 0 ? qa >> 6 : -1;
        auto word_at = [&](int64_t qw) -> uint64_t {
            return (qw >= (qmin >> 6) && qw <= (qmax >> 6)) ? a.qbuf[r.widx + qw] : 0ull;
        };
        const uint64_t lo = word_at(wa), hi = word_at(wa + 1);
        const int sh = (int)(qa - 64 * wa);            // 0 .. 63
        const uint64_t win = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
        // Bit k of win is entry qa + k, row R0 + 63 - k.
        uint64_t bits = __brevll(win);                 // bit t = row R0 + t
        bits &= (~0ull >> (63 - (thi - tlo))) << tlo;
        if (tlo == 0 && thi == 63) a.out[W] = bits;
        else if (bits) atomicXor((unsigned long long *)&a.out[W],
                                 (unsigned long long)bits);
    }
}

// Twiddle tables, computed once per transform length on the host in long
// double and kept by the context.
struct FftTables {
    DevBuf tw64, twr, lo[3], hi[3];   // lo/hi[d]: w_(L/64^d), 512 + P/512 entries
};
std::mutex g_tab_mu;
std::map<std::pair<int, uint64_t>, FftTables *> g_tables;   // (device, L)

// Levels of the transform: 64 x (L/64) up to 2^19 (rows of up to 8192
// points), 64 x 64 x (L/4096) up to 3 * 2^23, 64 x 64 x 64 x (L/2^18) above.
int fft_levels(uint64_t L) {
    return L <= (1ull << 19) ? 2 : L <= (3ull << 23) ? 3 : 4;
}
// Row FFT length.
uint64_t row_length(uint64_t L) { return L >> (6 * (fft_levels(L) - 1)); }

ssbh_status get_tables(int device, uint64_t L, FftTables **out) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tables.find({device, L});
    if (it != g_tables.end()) {
        *out = it->second;
        return SSBH_OK;
    }
    const long double two_pi = 6.283185307179586476925286766559L;
    auto unit = [&](uint64_t k, uint64_t n) {
        const long double ang = -two_pi * (long double)k / (long double)n;
        return make_double2((double)cosl(ang), (double)sinl(ang));
    };
    const int levels = fft_levels(L);
    const uint64_t nr = row_length(L);
    std::vector<std::vector<double2>> src;
    std::vector<DevBuf *> bufs;
    auto *t = new FftTables();
    src.emplace_back(kN1);
    for (uint64_t k = 0; k < (uint64_t)kN1; ++k) src.back()[k] = unit(k, kN1);
    bufs.push_back(&t->tw64);
    src.emplace_back(nr);
    for (uint64_t k = 0; k < nr; ++k) src.back()[k] = unit(k, nr);
    bufs.push_back(&t->twr);
    for (int d = 0; d <= levels - 2; ++d) {       // w_P for the parents of rows
        const uint64_t P = L >> (6 * d);
        src.emplace_back(512);
        for (uint64_t k = 0; k < 512; ++k) src.back()[k] = unit(k, P);
        bufs.push_back(&t->lo[d]);
        src.emplace_back(P / 512);
        for (uint64_t k = 0; k < P / 512; ++k) src.back()[k] = unit(k * 512, P);
        bufs.push_back(&t->hi[d]);
    }
    for (size_t b = 0; b < bufs.size(); ++b) {
        ssbh_status st = bufs[b]->reserve(src[b].size() * sizeof(double2));
        if (st == SSBH_OK &&
            hipMemcpy(bufs[b]->ptr, src[b].data(), src[b].size() * sizeof(double2),
                      hipMemcpyHostToDevice) != hipSuccess) {
            set_error("twiddle table upload failed");
            st = SSBH_E_DEVICE;
        }
        if (st != SSBH_OK) {
            for (DevBuf *d : bufs) d->release();
            delete t;
            return st;
        }
    }
    g_tables[{device, L}] = t;
    *out = t;
    return SSBH_OK;
}

// Launch `kernel`; with the workspace's timer on, through
// hipExtLaunchKernelGGL so that its events mark the kernel's own start and
// end (not the dispatch around it, as events recorded on the stream would).
template <class K, class... A>
void launch_timed(Workspace *ws, const char *name, K kernel, dim3 grid, dim3 block,
                  hipStream_t stream, A... args) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ws && ws->timer) ws->timer->begin_ext(name, &e0, &e1);
    if (e0 && e1)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, e0, e1, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, stream, args...);
}

template <int N2>
void launch_rows(const FftArgs &a, uint32_t pairs, bool spec, bool sq,
                 bool narrow, hipStream_t stream, Workspace *ws) {
    // Rows per transform (64, 4096 or 2^18) are a multiple of the rows per
    // workgroup (a power of two up to 32).
    const uint32_t rows = (uint32_t)(a.L / N2);
    static_assert(64 % rp_rpw(N2) == 0, "rows per workgroup divide 64");
    const dim3 grid(rows / rp_rpw(N2), spec ? 1u : pairs);
    if (spec)
        hipLaunchKernelGGL((k_fft_rows<N2, true>), grid, dim3(rp_threads(N2)),
                           0, stream, a);
    else if (sq && narrow) {
        if constexpr (N2 <= 4096)   // L <= 2^18
            launch_timed(ws, "k_fft_rows", k_fft_rows<N2, false, true, float2>, grid,
                         dim3(rp_threads(N2)), stream, a);
    }
    else if (sq)
        launch_timed(ws, "k_fft_rows", k_fft_rows<N2, false, true>, grid,
                     dim3(rp_threads(N2)), stream, a);
    else
        launch_timed(ws, "k_fft_rows", k_fft_rows<N2, false>, grid,
                     dim3(rp_threads(N2)), stream, a);
}

void rows(const FftArgs &a, uint32_t pairs, bool spec, hipStream_t stream,
          Workspace *ws = nullptr, bool sq = false, bool narrow = false) {
    switch (a.nr) {
    case 64: launch_rows<64>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 128: launch_rows<128>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 192: launch_rows<192>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 256: launch_rows<256>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 384: launch_rows<384>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 512: launch_rows<512>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 768: launch_rows<768>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 1024: launch_rows<1024>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 1536: launch_rows<1536>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 2048: launch_rows<2048>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 3072: launch_rows<3072>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 4096: launch_rows<4096>(a, pairs, spec, sq, narrow, stream, ws); break;
    case 6144: launch_rows<6144>(a, pairs, spec, sq, narrow, stream, ws); break;
    default: launch_rows<8192>(a, pairs, spec, sq, narrow, stream, ws); break;
    }
}

}  // namespace

// Transform length: the smallest supported L that holds the seed, 2^k or
// 3 * 2^k, 4096 <= L <= 2^31, with two, three or four levels and row FFTs of
// 64 .. 8192 points; kMaxFftLength + 1 when none holds it.
uint64_t fft_length(uint64_t seed_bits) {
    // Every row length is a multiple of 64: 3 * 2^11 (two levels, rows of
    // 96 points) is left out.
    for (uint64_t L = 4096; L <= kMaxFftLength;) {
        if (L >= seed_bits) return L;
        L = (L % 3 == 0) ? L / 3 * 4 : L / 2 * 3;   // 2^k, 3 * 2^(k-1), 2^(k+1)
        if (L == 6144) L = 8192;
    }
    return kMaxFftLength + 1;
}

// Sub-blocks per transform with a shared seed: four (two per part, the high
// one scaled by 2^18) when every sub-block is shorter than 2^18 bits (the
// plan rejects n_j > seed_bits + 1 - m_cap) and L <= 2^20, else two.  The
// scale multiplies the inputs' norm by 2^18; the usual bound on the
// rounding error of an FFT convolution, a few eps log2(L) |x|_2 |s|_2
// (Percival, Math. Comp. 72, 2003), stays below 1/100 for such L even for
// all-one inputs, against the 1/4 every output is checked for.
// Transforms of length L in `mib` MiB (at least one).  A chunk's transforms
// are written by one pass and read by the next: below the 256 MB
// last-level cache much of that traffic stays on chip.  With two chunks in
// flight (see FftSchedule::overlap) 96 MiB chunks measured best at the
// batched length.
uint32_t fft_chunk_of_bytes(uint64_t L, uint64_t mib, uint64_t point_bytes) {
    return (uint32_t)std::max<uint64_t>(1, (mib << 20) / (L * point_bytes));
}

// Complex floats between the passes (8 bytes a point instead of 16) for the
// joint transform (independent seeds, or a single sub-block) and L <= 2^18.  Rounding the column pass's output Y1 and
// the row pass's output Y2 to float (relative error u = 2^-24 per entry)
// moves the result c = z (*) z of the transform of z = s_j + i xr_j by at
// most (2u + u^2) |z|^2 through Y1 (the spectrum error, sqrt(L) u |z|_2 in
// 2-norm, meets the spectrum, sqrt(L) |z|_2, in the squaring; the 1/L of the
// inverse cancels the two square roots) and by at most 8 u |z|^2 through Y2
// (a column's 64 entries of Y2 are L/64 times the DFT of 64 entries of c,
// each at most |z|^2 in size).  The entry s_j * xr_j is half the imaginary
// part, so its error stays below 5 u |z|^2 + (double rounding), and
// |z|^2 <= L + n_j < 2 L (L seed bits in the real part, n_j input bits in
// the imaginary part): at L = 2^18 that is 5/32 < 1/4,
// the distance every entry is checked for.  With a shared seed the second
// sub-block of a part is scaled by 2^18, far beyond what floats carry.
constexpr uint64_t kNarrowMaxLength = 1ull << 18;
bool fft_narrow(const HashRequest &q, uint64_t L, int storage) {
    return storage != 64 && (q.stride != 0 || q.n_sub == 1) &&
           L <= kNarrowMaxLength;
}
uint64_t fft_point_bytes(const HashRequest &q, uint64_t L, int storage) {
    return fft_narrow(q, L, storage) ? sizeof(float2) : sizeof(double2);
}

bool fft_can_pack(const HashRequest &q, uint64_t L) {
    return q.stride == 0 && q.seed_bits + 1 < q.m_cap + (1ull << kPackBits) &&
           L <= (1ull << 20);
}
// One sub-block per transform (the joint transform) with a seed stride, and
// for a single sub-block with a shared seed unless packing is forced.
int fft_per_transform(const ssbh_ctx *ctx, const HashRequest &q, uint64_t L) {
    if (q.stride) return 1;
    if (ctx->forced_fft_pack) return 2 * ctx->forced_fft_pack;
    if (q.n_sub == 1) return 1;
    return fft_can_pack(q, L) ? 4 : 2;
}

ssbh_status launch_hash_fft(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                            const FftSchedule &s, hipStream_t stream) {
    // Transform length: the whole seed when it is shared, one stride of it
    // (the seed of one sub-block) otherwise.
    const uint64_t L = fft_length(q.stride ? q.stride : q.seed_bits);
    if (L > kMaxFftLength) {
        set_error("the FFT hash supports seeds (or seed strides) of at most "
                  "%llu bits", (unsigned long long)kMaxFftLength);
        return SSBH_E_UNSUPPORTED;
    }
    ssbh_status st = plan_only(ctx, ws, q, stream);
    if (st != SSBH_OK) return st;
    // Two chunks in flight on two streams (see FftSchedule::overlap).  The
    // second stream and its events belong to the context: only calls on the
    // context's own workspace, which hold its lock, use them (a pipeline's
    // eager run and serving jobs have workspaces of their own).
    const bool may_fork = s.overlap && &ws == &ctx->ws && !ws.timer;
    const int per = fft_per_transform(ctx, q, L);
    // Seed and data in one transform (see the top of the file).
    const bool joint = per == 1;
    if (s.storage == 32 && !(joint && L <= kNarrowMaxLength)) {
        set_error("float transform storage needs one sub-block per transform "
                  "(a seed stride, or a single sub-block) and a transform "
                  "length of at most 2^18");
        return SSBH_E_UNSUPPORTED;
    }
    const bool narrow = joint && L <= kNarrowMaxLength && s.storage != 64;
    const uint64_t pb = narrow ? sizeof(float2) : sizeof(double2);
    // Default chunk: 96 MiB of transforms when two are in flight (both fit
    // the 256 MB last-level cache), else 160 MiB.
    uint32_t chunk = s.chunk_pairs ? s.chunk_pairs
                                   : fft_chunk_of_bytes(L, may_fork ? 96 : 160, pb);
    // At most 512 MiB of transforms per chunk.
    chunk = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(chunk, (1ull << 29) / (L * pb)));
    if (per == 4 && !fft_can_pack(q, L)) {
        set_error("four sub-blocks per transform need a shared seed, "
                  "seed_bits + 1 - m_cap < 2^18 and L <= 2^20");
        return SSBH_E_UNSUPPORTED;
    }
    snprintf(ws.last_schedule, sizeof ws.last_schedule, "fft:%u:x%d:L%llu%s",
             s.chunk_pairs, per, (unsigned long long)L, narrow ? ":f32" : "");
    if (!q.n_sub) return SSBH_OK;
    FftTables *tab = nullptr;
    if ((st = get_tables(ctx->device, L, &tab)) != SSBH_OK) return st;
    // Transforms ("pairs"): one per sub-block with independent seeds, else
    // one per two or four sub-blocks.
    const uint64_t pairs = (q.n_sub + per - 1ull) / per;
    // Equal chunks of at most `chunk` transforms (no short last chunk).
    const uint64_t nchunks = (pairs + chunk - 1) / chunk;
    const uint32_t cp = (uint32_t)((pairs + nchunks - 1) / nchunks);
    if (!joint && (st = ws.fft_spec.reserve(L * sizeof(double2))) != SSBH_OK)
        return st;
    bool fork = may_fork && nchunks > 1;
    if (fork) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess ||
            cs != hipStreamCaptureStatusNone) {
            (void)hipGetLastError();
            fork = false;
        }
    }
    if (fork && !ctx->fft_side) {
        if (hipStreamCreateWithFlags(&ctx->fft_side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->fft_ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->fft_ev[1], hipEventDisableTiming) != hipSuccess) {
            set_error("FFT hash: second stream or events could not be created");
            return SSBH_E_DEVICE;
        }
    }
    const size_t work_b = (size_t)cp * L * pb;
    if ((st = ws.fft_work.reserve(fork ? 2 * work_b : work_b)) != SSBH_OK)
        return st;
    // Parity words: the regions of q_range, out_cap_bits / 64 + 3 n_sub words.
    if ((st = ws.fft_qbuf.reserve(((q.out_cap_bits >> 6) + 3ull * q.n_sub + 4) *
                                  sizeof(uint64_t))) != SSBH_OK)
        return st;
    FftArgs a{};
    uint64_t *plan = ws.plan.as<uint64_t>();
    a.sub = q.sub; a.len = q.len; a.woff = q.woff;
    a.mlen = plan; a.ooff = plan + q.n_sub;
    a.seed = q.seed; a.seed_bits = q.seed_bits;
    a.mcap = q.m_cap; a.ns = q.n_sub;
    a.L = L; a.n2 = (uint32_t)(L / kN1);
    a.nr = (uint32_t)row_length(L);
    const int levels = fft_levels(L);
    a.work = ws.fft_work.as<double2>();
    a.spec = ws.fft_spec.as<double2>();
    a.tw64 = tab->tw64.as<double2>();
    a.twr = tab->twr.as<double2>();
    for (int d = 0; d <= levels - 2; ++d) {
        a.wlo[d] = tab->lo[d].as<double2>();
        a.whi[d] = tab->hi[d].as<double2>();
    }
    a.tlo = a.wlo[0];
    a.thi = a.whi[0];
    a.rlo = a.wlo[levels - 2];
    a.rhi = a.whi[levels - 2];
    // Middle passes, forward (levels 1, 2) and inverse (2, 1).
    auto mids = [&](bool inv, uint32_t np, hipStream_t sm) {
        for (int i = 0; i < levels - 2; ++i) {
            const int d = inv ? levels - 2 - i : 1 + i;
            a.lvl = d;
            const uint64_t C = (L >> (6 * d)) >> 6;
            const dim3 g((uint32_t)(C / kN1), 1u << (6 * d), np);
            if (inv)
                hipLaunchKernelGGL(k_fft_mid<true>, g, dim3(kThreads), 0, sm, a);
            else
                hipLaunchKernelGGL(k_fft_mid<false>, g, dim3(kThreads), 0, sm, a);
        }
    };
    a.out = q.out;
    a.qbuf = ws.fft_qbuf.as<uint64_t>();
    a.status = q.status;
    a.stride = q.stride;
    const uint32_t tiles = a.n2 / kN1;
    a.per = per;
    // Seed spectrum: once for a shared seed (with a seed stride every
    // transform carries its own seed and is squared instead).
    auto spectrum = [&](uint64_t seed_off) {
        a.pair0 = 0;
        a.seed_off = seed_off;
        TimedLaunch timed(ws.timer, "k_fft_spectrum", stream);
        hipLaunchKernelGGL((k_fft_cols<true, false>), dim3(tiles, 1),
                           dim3(kThreads), 0, stream, a);
        mids(false, 1, stream);
        rows(a, 1, true, stream);
    };
    if (!joint) spectrum(0);
    char *work0 = ws.fft_work.as<char>();
    if (fork) {
        // The second stream starts after everything queued so far (the plan,
        // the output fill, the spectrum).
        SSBH_CHECK_HIP(hipEventRecord(ctx->fft_ev[0], stream));
        SSBH_CHECK_HIP(hipStreamWaitEvent(ctx->fft_side, ctx->fft_ev[0], 0));
    }
    uint64_t ci = 0;
    for (uint64_t p0 = 0; p0 < pairs; p0 += cp, ++ci) {
        const uint32_t np = (uint32_t)std::min<uint64_t>(cp, pairs - p0);
        const bool odd = fork && (ci & 1);
        hipStream_t sc = odd ? ctx->fft_side : stream;
        a.pair0 = (uint32_t)p0;
        a.work = reinterpret_cast<double2 *>(odd ? work0 + work_b : work0);
        if (narrow)
            launch_timed(&ws, "k_fft_cols", k_fft_cols<false, false, true, float2>,
                         dim3(tiles, np), dim3(kThreads), sc, a);
        else if (joint)
            launch_timed(&ws, "k_fft_cols", k_fft_cols<false, false, true>,
                         dim3(tiles, np), dim3(kThreads), sc, a);
        else if (per == 4)
            launch_timed(&ws, "k_fft_cols", k_fft_cols<false, true>, dim3(tiles, np),
                         dim3(kThreads), sc, a);
        else
            launch_timed(&ws, "k_fft_cols", k_fft_cols<false, false>, dim3(tiles, np),
                         dim3(kThreads), sc, a);
        if (levels > 2) {
            TimedLaunch timed(ws.timer, "k_fft_mid", sc);
            mids(false, np, sc);
        }
        rows(a, np, false, sc, &ws, joint, narrow);
        if (levels > 2) {
            TimedLaunch timed(ws.timer, "k_fft_mid", sc);
            mids(true, np, sc);
        }
        if (narrow)
            launch_timed(&ws, "k_fft_out", k_fft_out<false, true, float2>,
                         dim3(tiles, np), dim3(kThreads), sc, a);
        else if (joint)
            launch_timed(&ws, "k_fft_out", k_fft_out<false, true>, dim3(tiles, np),
                         dim3(kThreads), sc, a);
        else if (per == 4)
            launch_timed(&ws, "k_fft_out", k_fft_out<true>, dim3(tiles, np),
                         dim3(kThreads), sc, a);
        else
            launch_timed(&ws, "k_fft_out", k_fft_out<false>, dim3(tiles, np),
                         dim3(kThreads), sc, a);
    }
    if (fork) {
        // The emit pass (and the caller's later work) after both streams.
        SSBH_CHECK_HIP(hipEventRecord(ctx->fft_ev[1], ctx->fft_side));
        SSBH_CHECK_HIP(hipStreamWaitEvent(stream, ctx->fft_ev[1], 0));
    }
    {
        // Every sub-block's rows from the parity words, 2048 output words per
        // workgroup (a sub-block spans at most m_cap / 64 + 2 of them).
        const uint64_t wmax = (q.m_cap >> 6) + 2;
        launch_timed(&ws, "k_fft_emit", k_fft_emit,
                     dim3(q.n_sub, (uint32_t)((wmax + 2047) / 2048)), dim3(256),
                     stream, a);
    }
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

}  // namespace ssbh
