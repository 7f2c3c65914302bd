// Fused path for small permutation-split jobs in a graph pipeline: the whole
// step (Sec. III.B: division, hash of every sub-block, concatenation) in two
// kernels instead of seven, for sub-blocks of equal length L = n / N_S whose
// outputs start on 64-bit boundaries (m % 64 == 0).  All sizes are fixed on
// the host, so the plan, the tile list and the output fill of the general
// path are not needed:
//   k_small_gather  B[k] = A[pi[k]] into the sub-block buffer (64 bits per
//                   wavefront step, ballot), n_j and W_j, and one error flag
//                   per workgroup (an entry of pi outside [0, n)).
//   k_small_hash    workgroup (row tile, sub-block): the sub-block's bits and
//                   the seed window of the tile's rows staged in LDS, the
//                   bit-sliced AND-XOR over column words (a lane owns R rows
//                   32 apart, which share one sliding ring of seed windows),
//                   the column ranges of the 16 waves XOR-reduced in LDS, one
//                   plain store per output word.  Reads the gather's error
//                   flags first: on an error nothing is written to the
//                   output and the status is set.
// The result is the general path's bit for bit (tests/test_gpu_graph_tune.py).
#include <stdio.h>

#include <algorithm>

#include "ssbh_internal.hpp"

namespace ssbh {
namespace {

constexpr int kGatherU = 4;      // words per wavefront in the gather
constexpr int kR = 8;            // rows per lane (32 apart)
constexpr int kWaves = 16;       // column ranges per workgroup (a wave each)
constexpr int kRowsPerTile = 64 * kR;
static_assert(kR == 8, "the column loop unpacks two uint4 of x words");

struct SmallArgs {
    const uint64_t *in;
    uint64_t n;
    const uint32_t *perm;
    uint32_t ns;
    uint64_t L, wl;               // sub-block length, words per sub-block
    uint64_t m, mcap, stride;
    const uint32_t *seed32;
    int64_t seed_w32;             // readable 32-bit seed words
    uint64_t *sub;
    uint64_t *len, *woff, *out_total;
    uint32_t *out32;
    int32_t *flags;               // one per gather workgroup
    uint32_t nflags;
    int32_t *status;
};

__global__ __launch_bounds__(256) void k_small_gather(SmallArgs a) {
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t total = (uint64_t)a.ns * a.wl;
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    uint32_t p[kGatherU];
    bool ok[kGatherU];
    // All of this wavefront's pi entries first, then the input words, so
    // that the loads are in flight together.
#pragma unroll
    for (int u = 0; u < kGatherU; ++u) {
        const uint64_t w = wave * kGatherU + u;
        ok[u] = false;
        p[u] = 0;
        if (w < total) {
            const uint64_t j = w / a.wl, c = (w - j * a.wl) * 64 + lane;
            if (c < a.L) {
                p[u] = a.perm[j * a.L + c];
                ok[u] = true;
            }
        }
    }
    bool bad = false;
    uint64_t word[kGatherU];
#pragma unroll
    for (int u = 0; u < kGatherU; ++u) {
        word[u] = 0;
        if (ok[u]) {
            if (p[u] < a.n) word[u] = a.in[p[u] >> 6];
            else bad = true;
        }
    }
#pragma unroll
    for (int u = 0; u < kGatherU; ++u) {
        const uint64_t w = wave * kGatherU + u;
        const bool bit = ok[u] && p[u] < a.n && ((word[u] >> (p[u] & 63)) & 1ull);
        const uint64_t b = ballot64(bit);
        if (lane == 0 && w < total) a.sub[w] = b;
    }
    if (bad) atomicOr(&bad_s, 1);
    if (blockIdx.x == 0) {
        for (uint32_t j = threadIdx.x; j < a.ns; j += blockDim.x) {
            a.len[j] = a.L;
            a.woff[j] = (uint64_t)j * a.wl;
        }
        if (threadIdx.x == 0) *a.out_total = (uint64_t)a.ns * a.m;
    }
    __syncthreads();
    if (threadIdx.x == 0) a.flags[blockIdx.x] = bad_s ? (int32_t)SSBH_E_INVAL : 0;
}

// Column words per wave (a multiple of kR, so that the loop has no tail) and
// the staged seed words of a tile (see k_small_hash).
__host__ __device__ constexpr uint32_t col_words_per_wave(uint32_t xw) {
    return ((xw + kWaves - 1) / kWaves + kR - 1) / kR * kR;
}
__host__ __device__ constexpr uint32_t window_words(uint32_t xpad) {
    return xpad + (kRowsPerTile + 32 * kR + 160) / 32 + 2;
}

// acc ^= w & x: v_bitop3_b32 with truth table 0x6a = S2 ^ (S0 & S1) (the
// table is indexed by S0 S1 S2 as bits 2, 1, 0).
__device__ __forceinline__ uint32_t and_xor(uint32_t acc, uint32_t w, uint32_t x) {
    return __builtin_amdgcn_bitop3_b32(w, x, acc, 0x6a);
}

__global__ __launch_bounds__(64 * kWaves) void k_small_hash(SmallArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ int err_s;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) err_s = 0;
    __syncthreads();
    for (uint32_t k = t; k < a.nflags; k += blockDim.x)
        if (a.flags[k]) atomicOr(&err_s, 1);
    __syncthreads();
    if (err_s) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) *a.status = SSBH_E_INVAL;
        return;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) *a.status = 0;
    const uint64_t j = blockIdx.y;
    const uint64_t r0 = (uint64_t)blockIdx.x * kRowsPerTile;
    const uint64_t r1 = min<uint64_t>(r0 + kRowsPerTile, a.m);   // rows [r0, r1)
    const uint32_t xw = (uint32_t)((a.L + 31) / 32);             // column words
    const uint32_t cpw = col_words_per_wave(xw);                 // multiple of kR
    const uint32_t xpad = cpw * kWaves;                          // zero past xw
    const uint32_t nwin = window_words(xpad);
    uint32_t *xs = lds;                                          // [xpad]
    uint32_t *win = lds + xpad;                                  // [nwin]
    // Lanes read seed indices base + 32 c + M - 1 - r + [0, 64) for rows r in
    // [r0, r0 + kRowsPerTile) (rows past m too; their results are dropped)
    // and column words c in [-kR, xpad): the staged 32-bit words start at
    // ws0 <= (base + M - r0 - kRowsPerTile - 32 kR - 32) / 32 and cover
    // them all (window_words), so the loop reads LDS without bounds checks.
    const int64_t base = (int64_t)(j * a.stride);
    const int64_t lo_bit = base + (int64_t)a.mcap - (int64_t)r0 - kRowsPerTile -
                           32 * kR - 32;
    const int64_t ws0 = lo_bit >> 5;                             // floor
    const uint32_t *x32 = reinterpret_cast<const uint32_t *>(a.sub + j * a.wl);
    for (uint32_t k = t; k < xpad; k += blockDim.x) {
        uint32_t v = 0u;
        if (k < xw) {
            v = x32[k];
            const uint64_t c0 = (uint64_t)k * 32;
            if (c0 + 32 > a.L) v &= (1u << (a.L - c0)) - 1u;   // bits past n_j
        }
        xs[k] = v;
    }
    for (uint32_t k = t; k < nwin; k += blockDim.x) {
        const int64_t q = ws0 + k;
        win[k] = (q >= 0 && q < a.seed_w32) ? a.seed32[q] : 0u;
    }
    __syncthreads();

    // Lane rows: rb + 32 i, i < kR, rb = r0 + (lane & 31) + 32 kR (lane >> 5).
    const uint64_t rb = r0 + (uint64_t)(lane & 31) + 32ull * kR * (uint64_t)(lane >> 5);
    // Row r at column word c reads the 32 seed bits from index
    // base + 32 c + M - 1 - r, i.e. bit 32 c + e0 of the staged words with
    // e0 = base + M - 1 - rb - 32 ws0 (>= kRowsPerTile); row rb + 32 i reads
    // bit 32 (c - i) + e0: row rb's window at column word c - i.
    const int64_t e0 = base + (int64_t)a.mcap - 1 - (int64_t)rb - 32 * ws0;
    const uint32_t sh = (uint32_t)(e0 & 31);
    const uint32_t *wp0 = win + (e0 >> 5);     // low word of column 0's window
    const uint32_t cw0 = wv * cpw, cw1 = cw0 + cpw;
    uint32_t acc[kR], slot[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) acc[i] = 0u;
    // slot[(c - cw0) mod kR] holds row rb's window at column word c for the
    // last kR column words; start with c = cw0 - kR .. cw0 - 1.
    uint32_t lo = wp0[(int)cw0 - kR];
#pragma unroll
    for (int k = 0; k < kR; ++k) {
        const uint32_t hi = wp0[(int)cw0 - kR + k + 1];
        slot[k] = __builtin_amdgcn_alignbit(hi, lo, sh);
        lo = hi;
    }
    for (uint32_t cw = cw0; cw < cw1; cw += kR) {
        const uint32_t *wp = wp0 + cw + 1;
        const uint4 xa = *reinterpret_cast<const uint4 *>(xs + cw);
        const uint4 xb = *reinterpret_cast<const uint4 *>(xs + cw + 4);
        const uint32_t xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            const uint32_t hi = wp[u];
            slot[u] = __builtin_amdgcn_alignbit(hi, lo, sh);
            lo = hi;
#pragma unroll
            for (int i = 0; i < kR; ++i)
                acc[i] = and_xor(acc[i], slot[(u - i + kR) % kR], xv[u]);
        }
    }
    // Parity words: for each i, lanes 0..31 hold rows r0 + 32 i + l and lanes
    // 32..63 rows r0 + 32 kR + 32 i + (l - 32).
    uint32_t *red = win + nwin;              // [kWaves][kR][2]
    __syncthreads();                         // window reads done
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const uint64_t b = ballot64(__popc(acc[i]) & 1u);
        if (lane == 0) {
            red[(wv * kR + i) * 2] = (uint32_t)b;
            red[(wv * kR + i) * 2 + 1] = (uint32_t)(b >> 32);
        }
    }
    __syncthreads();
    if (t < 2 * kR) {
        const int i = t >> 1, half = t & 1;
        uint32_t v = 0;
        for (int w2 = 0; w2 < kWaves; ++w2) v ^= red[(w2 * kR + i) * 2 + half];
        const uint64_t row = r0 + 32ull * kR * half + 32ull * i;
        if (row < r1) a.out32[(j * a.m + row) >> 5] = v;
    }
}

}  // namespace

bool small_path_ok(const ssbh_pipeline_desc &d) {
    if (!d.d_in || d.mode != SSBH_SAMPLE_PERMUTE || d.d_keep || !d.d_assign)
        return false;
    if (d.kernel != SSBH_K_AUTO && d.kernel != SSBH_K_VALU) return false;
    if (d.n_sub == 0 || d.n_bits == 0 || d.n_bits % d.n_sub) return false;
    const uint64_t L = d.n_bits / d.n_sub;
    if (L > 65536) return false;
    uint64_t m;
    if (d.out_rule == SSBH_OUT_FIXED) m = d.out_a;
    else if (d.out_rule == SSBH_OUT_RATIO && d.out_b) m = L * d.out_a / d.out_b;
    else return false;
    if (m == 0 || m % 64 || m > d.m_cap || d.m_cap >= (1ull << 32)) return false;
    if (d.l_ub && L > d.l_ub) return false;            // every call aborts
    const uint64_t wl = (L + 63) / 64;
    if (d.sub_capacity_words < (uint64_t)d.n_sub * wl) return false;
    if (d.out_capacity_bits < (uint64_t)d.n_sub * m) return false;
    // Every sub-block's seed window inside the seed.
    const long double last = (long double)(d.n_sub - 1) * d.seed_stride +
                             (long double)L + (long double)d.m_cap - 1.0L;
    if (!d.d_seed || last > (long double)d.seed_bits) return false;
    // Enough workgroups to be worth it, few enough to stay small.
    const uint64_t tiles = (m + kRowsPerTile - 1) / kRowsPerTile * d.n_sub;
    return tiles <= 65535 && (uint64_t)d.n_sub * wl <= (1ull << 16);
}

size_t small_scratch(const ssbh_pipeline_desc &d) {
    const uint64_t L = d.n_bits / d.n_sub, wl = (L + 63) / 64;
    const uint64_t words = (uint64_t)d.n_sub * wl;
    const uint64_t blocks = (words + 4 * kGatherU - 1) / (4 * kGatherU);
    return (size_t)blocks * sizeof(int32_t) + 64;
}

ssbh_status launch_small_fused(ssbh_ctx *ctx, Workspace &ws,
                               const ssbh_pipeline_desc &d,
                               hipStream_t stream) {
    (void)ctx;
    SmallArgs a{};
    a.in = d.d_in; a.n = d.n_bits; a.perm = d.d_assign; a.ns = d.n_sub;
    a.L = d.n_bits / d.n_sub; a.wl = (a.L + 63) / 64;
    a.m = d.out_rule == SSBH_OUT_FIXED ? d.out_a : a.L * d.out_a / d.out_b;
    a.mcap = d.m_cap; a.stride = d.seed_stride;
    a.seed32 = reinterpret_cast<const uint32_t *>(d.d_seed);
    a.seed_w32 = (int64_t)(2 * ((d.seed_bits + 63) / 64));
    a.sub = d.d_sub; a.len = d.d_len; a.woff = d.d_word_off;
    a.out_total = d.d_out_total_bits;
    a.out32 = reinterpret_cast<uint32_t *>(d.d_out);
    a.status = d.d_status;
    const uint64_t words = (uint64_t)a.ns * a.wl;
    const uint32_t gblocks = (uint32_t)((words + 4 * kGatherU - 1) / (4 * kGatherU));
    ssbh_status st = ws.counters.reserve(small_scratch(d));
    if (st != SSBH_OK) return st;
    a.flags = ws.counters.as<int32_t>();
    a.nflags = gblocks;
    hipLaunchKernelGGL(k_small_gather, dim3(gblocks), dim3(256), 0, stream, a);
    const uint32_t xpad = col_words_per_wave((uint32_t)((a.L + 31) / 32)) * kWaves;
    const size_t lds = ((size_t)xpad + window_words(xpad) + 2 * kWaves * kR) *
                       sizeof(uint32_t);
    if ((st = ensure_dynamic_lds((const void *)k_small_hash, lds)) != SSBH_OK)
        return st;
    const dim3 grid((uint32_t)((a.m + kRowsPerTile - 1) / kRowsPerTile), a.ns);
    hipLaunchKernelGGL(k_small_hash, grid, dim3(64 * kWaves), lds, stream, a);
    SSBH_CHECK_HIP(hipGetLastError());
    snprintf(ws.last_schedule, sizeof ws.last_schedule, "small:%d:%d", kR, kWaves);
    return SSBH_OK;
}

}  // namespace ssbh
