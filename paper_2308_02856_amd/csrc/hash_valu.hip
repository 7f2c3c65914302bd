// Per-sub-block Toeplitz hashing and concatenation (Sec. I; Sec. III.B
// steps 3-4) with the vector ALUs of gfx950.
//
//   K_j[r] = XOR_{c<n_j} ( s[j*S + c - r + M - 1] AND x_j[c] )
//
// Bit-sliced form.  Take 32-bit column words x_j[w].  For a row r the seed
// bits that meet column word w form the 32-bit seed word starting at bit
// e_r + 32w with e_r = j*S + M - 1 - r.  Rows 32 apart use the same seed
// words shifted by one word, so a lane that owns rows r, r+32, ..., r+32(R-1)
// needs, at column word w, the words SW(w), SW(w-1), ..., SW(w-R+1) of ONE
// bit alignment (its own e_r mod 32).  The lane keeps them in a register ring
// and per column word does: one LDS read (next raw seed word), one
// v_alignbit_b32 (the new SW), and R v_bitop3_b32 (acc ^= SW & x), i.e. close
// to one VALU op per 32 AND-XOR bit-products.  The parity of every
// accumulator is its popcount mod 2; a wavefront ballot packs 32 rows into an
// output word.
//
// Tiles: (sub-block, ROWS rows, a column range).  A persistent grid claims
// tiles from a device-built list with one atomic counter, so uneven sub-block
// sizes run in one launch and the host never reads the sizes.  For every
// column chunk the workgroup stages the seed window (diagonal-constant, shared
// by all its rows) and the column words into LDS.  Partial parities of tiles
// that split the columns of a sub-block are merged with atomic XOR into the
// zeroed output, which also concatenates at arbitrary bit offsets; XOR is
// order independent, so every schedule gives the same bits.
#include <algorithm>

#include <stdio.h>

#include "ssbh_internal.hpp"

namespace ssbh {

struct Tile {
    uint32_t j;      // sub-block
    uint32_t row0;   // first row
    uint32_t cw0;    // first 32-bit column word
    uint32_t cw1;    // end column word (exclusive)
};

namespace {

struct PlanArgs {
    const uint64_t *len;
    const uint64_t *woff;
    uint32_t ns;
    uint32_t rule;
    uint64_t ra, rb;
    const uint64_t *out_len;
    uint64_t seed_bits, stride, mcap, sub_cap, out_cap;
    uint32_t rows;
    uint32_t tile_cols;   // 0 = whole sub-block
    uint64_t tile_cap;
    uint64_t *mlen, *ooff, *toff;
    uint64_t *counters;   // [0] tiles, [1] claim counter (low 32 bits)
    uint64_t *out_total;
    int32_t *status;
};

__device__ __forceinline__ uint64_t out_len_of(const PlanArgs &a, uint32_t j,
                                               uint64_t n) {
    if (a.rule == SSBH_OUT_FIXED) return a.ra;
    if (a.rule == SSBH_OUT_RATIO) return n * a.ra / a.rb;
    return a.out_len[j];
}

__device__ __forceinline__ uint64_t tiles_of(uint64_t n, uint64_t m,
                                             uint32_t rows, uint32_t tcols) {
    if (!n || !m) return 0;
    const uint64_t nw = (n + 31) / 32;
    const uint64_t ct = tcols ? (nw + tcols - 1) / tcols : 1;
    return ((m + rows - 1) / rows) * ct;
}

// Exclusive block scan of two u64 values (1024 threads); returns the block
// totals through *t1, *t2.
__device__ void block_scan2(uint64_t v1, uint64_t v2, uint64_t &e1,
                            uint64_t &e2, uint64_t &t1, uint64_t &t2) {
    __shared__ uint64_t s1[16], s2[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    uint64_t i1 = v1, i2 = v2;
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t a = __shfl_up(i1, d, 64), b = __shfl_up(i2, d, 64);
        if (lane >= d) { i1 += a; i2 += b; }
    }
    if (lane == 63) { s1[w] = i1; s2[w] = i2; }
    __syncthreads();
    uint64_t b1 = 0, b2 = 0, a1 = 0, a2 = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < w) { b1 += s1[k]; b2 += s2[k]; }
        a1 += s1[k]; a2 += s2[k];
    }
    e1 = b1 + i1 - v1;
    e2 = b2 + i2 - v2;
    t1 = a1;
    t2 = a2;
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_plan(PlanArgs a) {
    __shared__ int bad_s;
    if (*a.status) return;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    uint64_t carry_m = 0, carry_t = 0;
    for (uint32_t base = 0; base < a.ns; base += blockDim.x) {
        const uint32_t j = base + threadIdx.x;
        uint64_t m = 0, t = 0;
        if (j < a.ns) {
            const uint64_t n = a.len[j], W = a.woff[j];
            m = out_len_of(a, j, n);
            bool bad = m > a.mcap;
            const uint64_t words = (n + 63) / 64;
            bad |= W > a.sub_cap || words > a.sub_cap - W;
            if (n && m) {
                const uint64_t s0 = (uint64_t)j * a.stride;  // host-checked
                bad |= n > a.seed_bits || a.mcap > a.seed_bits ||
                       s0 > a.seed_bits - n - a.mcap + 1 ||
                       n + a.mcap - 1 > a.seed_bits;
            }
            t = tiles_of(n, m, a.rows, a.tile_cols);
            if (bad) atomicOr(&bad_s, 1);
        }
        uint64_t em, et, tm, tt;
        block_scan2(m, t, em, et, tm, tt);
        if (j < a.ns) {
            a.mlen[j] = m;
            a.ooff[j] = carry_m + em;
            a.toff[j] = carry_t + et;
        }
        carry_m += tm;
        carry_t += tt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (bad_s || carry_m > a.out_cap || carry_t > a.tile_cap) {
            *a.status = SSBH_E_INVAL;
        } else {
            a.counters[0] = carry_t;
            a.counters[1] = 0;
            *a.out_total = carry_m;
        }
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint64_t *p, uint64_t words,
                                                    const int32_t *status) {
    if (*status) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
         k < words; k += stride)
        p[k] = 0ull;
}

__global__ __launch_bounds__(256) void k_expand(PlanArgs a, Tile *tiles) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= a.ns) return;
    const uint64_t n = a.len[j], m = a.mlen[j];
    const uint64_t nt = tiles_of(n, m, a.rows, a.tile_cols);
    if (!nt) return;
    const uint64_t nw = (n + 31) / 32;
    const uint32_t tc = a.tile_cols ? a.tile_cols : (uint32_t)nw;
    const uint64_t ct = (nw + tc - 1) / tc;
    Tile *dst = tiles + a.toff[j];
    for (uint64_t k = lane; k < nt; k += 64) {
        const uint64_t rt = k / ct, c = k - rt * ct;
        Tile t;
        t.j = j;
        t.row0 = (uint32_t)(rt * a.rows);
        t.cw0 = (uint32_t)(c * tc);
        t.cw1 = (uint32_t)min<uint64_t>((c + 1) * tc, nw);
        dst[k] = t;
    }
}

struct ValuArgs {
    const uint32_t *sub32;
    const uint64_t *len, *woff, *mlen, *ooff;
    const uint32_t *seed32;
    int64_t seed_w32;     // 32-bit words readable in the seed buffer
    uint64_t stride, mcap;
    const Tile *tiles;
    const uint64_t *counters;
    uint32_t *claim;
    uint32_t *out32;
    uint32_t chunk;       // column words per LDS chunk (multiple of R)
    const int32_t *status;
};

template <int R>
__device__ __forceinline__ void block_of_steps(uint32_t (&acc)[R],
                                               uint32_t (&sw)[R], uint32_t &raw,
                                               const uint32_t *wq,
                                               const uint4 *xq, uint32_t sh) {
    // wq points at the LDS word of SW(first step) + 1; xq at its x words.
#pragma unroll
    for (int u4 = 0; u4 < R / 4; ++u4) {
        const uint4 x4 = xq[u4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int u = u4 * 4 + v;
            const uint32_t x = v == 0 ? x4.x : v == 1 ? x4.y : v == 2 ? x4.z : x4.w;
            const uint32_t nxt = wq[u];
            sw[u] = __builtin_amdgcn_alignbit(nxt, raw, sh);
            raw = nxt;
#pragma unroll
            for (int i = 0; i < R; ++i)
                acc[i] = __builtin_amdgcn_bitop3_b32(sw[(u - i + R) % R], x,
                                                     acc[i], 0x6a);
        }
    }
}

// Same step sequence with the column words already in scalar registers.
template <int R>
__device__ __forceinline__ void block_of_steps_s(uint32_t (&acc)[R],
                                                 uint32_t (&sw)[R],
                                                 uint32_t &raw,
                                                 const uint32_t *wq,
                                                 const uint32_t (&xs)[R],
                                                 uint32_t sh) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const uint32_t nxt = wq[u];
        sw[u] = __builtin_amdgcn_alignbit(nxt, raw, sh);
        raw = nxt;
#pragma unroll
        for (int i = 0; i < R; ++i)
            acc[i] = __builtin_amdgcn_bitop3_b32(sw[(u - i + R) % R], xs[u],
                                                 acc[i], 0x6a);
    }
}

typedef const __attribute__((address_space(4))) uint32_t *const_u32p;
typedef uint32_t u32x8a __attribute__((ext_vector_type(8), aligned(8)));
typedef const __attribute__((address_space(4))) u32x8a *const_u32x8p;

// R column words starting at an even word index (sub-blocks start on 64-bit
// words and blocks on multiples of R words), as wide scalar loads.
template <int R>
__device__ __forceinline__ void load_x_fast(uint32_t (&xs)[R], const_u32p Xc,
                                            uint32_t cw) {
#pragma unroll
    for (int q = 0; q < R / 8; ++q) {
        const u32x8a v = *(const_u32x8p)(Xc + cw + 8 * q);
#pragma unroll
        for (int u = 0; u < 8; ++u) xs[8 * q + u] = v[u];
    }
}

// Column words [cw, cw + R) of a sub-block, through the scalar cache.
// `fast` blocks lie before the end of the tile and before a partial last
// word; the others mask words past the tile and the bits past n.
template <int R>
__device__ __forceinline__ void load_x_block(uint32_t (&xs)[R], const_u32p Xc,
                                             uint32_t cw, bool fast,
                                             uint32_t ck1, uint32_t nw,
                                             uint32_t tailmask) {
    if (fast) {
#pragma unroll
        for (int u = 0; u < R; ++u) xs[u] = Xc[cw + u];
    } else {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            uint32_t x = (cw + u < ck1) ? Xc[cw + u] : 0u;
            if (cw + u == nw - 1) x &= tailmask;
            xs[u] = x;
        }
    }
}

template <int R, int WAVES, bool XS>
__global__ __launch_bounds__(64 * WAVES) void k_toeplitz_valu(ValuArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t tile_s;
    constexpr int ROWS = WAVES * 64 * R;
    if (*a.status) return;
    const uint32_t ntiles = (uint32_t)a.counters[0];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, b = lane & 31;
    uint32_t *xw = lds;                               // x words of the chunk
    uint32_t *win = lds + a.chunk + R;                // seed window

    for (;;) {
        if (threadIdx.x == 0) tile_s = atomicAdd(a.claim, 1u);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(tile_s);
        if (t >= ntiles) break;
        const Tile tl = a.tiles[t];
        const uint32_t j = tl.j;
        const uint64_t n = a.len[j], m = a.mlen[j];
        const uint64_t O = a.ooff[j];
        const uint32_t *X = a.sub32 + 2 * a.woff[j];
        const uint32_t nw = (uint32_t)((n + 31) / 32);
        const uint32_t tailmask = (n & 31) ? ((1u << (n & 31)) - 1u) : ~0u;
        // Seed index of (row row0, column 0).
        const int64_t cbase = (int64_t)(j * a.stride) + (int64_t)a.mcap - 1 -
                              (int64_t)tl.row0;
        const int64_t rowbase = (int64_t)tl.row0 + (int64_t)wave * 64 * R;
        const bool active = rowbase < (int64_t)m;
        // This lane's seed bit of (its row i = 0, column 0).
        const int64_t E = cbase - (int64_t)wave * 64 * R - 32 * h * R - b;
        const uint32_t sh = (uint32_t)(E & 31);

        uint32_t acc[R];
        uint32_t sw[R];
#pragma unroll
        for (int i = 0; i < R; ++i) { acc[i] = 0u; sw[i] = 0u; }
        uint32_t raw = 0u;

        for (uint32_t ck0 = tl.cw0; ck0 < tl.cw1; ck0 += a.chunk) {
            const uint32_t ck1 = min(ck0 + a.chunk, tl.cw1);
            const uint32_t nblk = (ck1 - ck0 + R - 1) / R;
            const uint32_t ckend = ck0 + nblk * R;
            const bool first = ck0 == tl.cw0;
            const int64_t pmin = first ? (int64_t)ck0 - (R - 1) : (int64_t)ck0;
            const int64_t lo = cbase - ROWS + 32 * R - 31 + 32 * pmin;
            const int64_t lo_w = lo >> 5;     // floor
            const int64_t hi = cbase + 32 * ((int64_t)ckend - 1) + 31;
            const int nwin = (int)(((hi - (lo_w << 5)) >> 5) + 2);
            for (int k = threadIdx.x; k < nwin; k += 64 * WAVES) {
                const int64_t g = lo_w + k;
                win[k] = (g >= 0 && g < a.seed_w32) ? a.seed32[g] : 0u;
            }
            if constexpr (!XS) {
                for (uint32_t k = threadIdx.x; k < ckend - ck0;
                     k += 64 * WAVES) {
                    const uint32_t cw = ck0 + k;
                    uint32_t x = cw < ck1 ? X[cw] : 0u;
                    if (cw == nw - 1) x &= tailmask;
                    xw[k] = x;
                }
            }
            __syncthreads();
            if (active) {
                // q(p) = qb + p indexes the low LDS word of SW(p).
                const int qb = (int)((E >> 5) - lo_w);
                if (first) {
#pragma unroll
                    for (int u = 1; u < R; ++u) {
                        const int p = (int)ck0 - R + u;
                        sw[u] = __builtin_amdgcn_alignbit(win[qb + p + 1],
                                                          win[qb + p], sh);
                    }
                }
                raw = win[qb + (int)ck0];
                if constexpr (XS) {
                    const const_u32p Xc = (const_u32p)X;
                    const uint32_t fast_end =
                        (ck1 < nw || tailmask == ~0u) ? ck1 : nw - 1;
                    uint32_t k = 0;
                    for (; k < nblk && ck0 + (k + 1) * R <= fast_end; ++k) {
                        const uint32_t cw = ck0 + k * R;
                        uint32_t xs[R];
                        load_x_fast<R>(xs, Xc, cw);
                        block_of_steps_s<R>(acc, sw, raw, win + qb + cw + 1,
                                            xs, sh);
                    }
                    for (; k < nblk; ++k) {
                        const uint32_t cw = ck0 + k * R;
                        uint32_t xs[R];
                        load_x_block<R>(xs, Xc, cw, false, ck1, nw, tailmask);
                        block_of_steps_s<R>(acc, sw, raw, win + qb + cw + 1,
                                            xs, sh);
                    }
                } else {
                    for (uint32_t k = 0; k < nblk; ++k) {
                        const uint32_t cw = ck0 + k * R;
                        block_of_steps<R>(
                            acc, sw, raw, win + qb + cw + 1,
                            reinterpret_cast<const uint4 *>(xw + k * R), sh);
                    }
                }
            }
            __syncthreads();
        }

        if (active) {
            // Parity of each accumulator; lane k < 2R then owns the 32 rows
            // starting at rowbase + 32k.
            uint32_t mine = 0u;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const uint64_t bal = ballot64(__builtin_popcount(acc[i]) & 1);
                if (lane == i) mine = (uint32_t)bal;
                if (lane == R + i) mine = (uint32_t)(bal >> 32);
            }
            if (lane < 2 * R) {
                const int64_t rs = rowbase + 32 * lane;
                const int64_t nvalid = (int64_t)m - rs;
                if (nvalid > 0) {
                    if (nvalid < 32) mine &= (1u << nvalid) - 1u;
                    if (mine) {
                        const uint64_t pos = O + (uint64_t)rs;
                        const uint64_t q = pos >> 5;
                        const uint32_t s = (uint32_t)(pos & 31);
                        atomicXor(a.out32 + q, mine << s);
                        if (s && (mine >> (32 - s)))
                            atomicXor(a.out32 + q + 1, mine >> (32 - s));
                    }
                }
            }
        }
    }
}

template <int R, int WAVES, bool XS>
ssbh_status run_valu(ssbh_ctx *ctx, const ValuArgs &va, hipStream_t stream) {
    const size_t lds = ((size_t)va.chunk + R +
                        (size_t)WAVES * 64 * R / 32 + va.chunk + 4 * R + 8) * 4;
    auto kern = k_toeplitz_valu<R, WAVES, XS>;
    ssbh_status st = ensure_dynamic_lds((const void *)kern, lds);
    if (st != SSBH_OK) return st;
    int per_cu = 0;
    SSBH_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, (const void *)kern, 64 * WAVES, lds));
    if (per_cu < 1) per_cu = 1;
    const uint32_t grid = (uint32_t)(ctx->num_cus * per_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WAVES), lds, stream, va);
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

}  // namespace

// Host-side bound on the tile count (sizes the tile list before the device
// knows the sub-block lengths): sum_j ceil(m_j/ROWS) ceil(w_j/C) <=
// M*sumw/(ROWS*C) + N_S*M/ROWS + sumw/C + N_S with sumw <= 2*sub_cap words.
static uint64_t tile_bound(uint64_t ns, uint64_t mcap, uint64_t sub_cap,
                           uint64_t rows, uint64_t tc_for_bound) {
    const long double sumw = 2.0L * (long double)sub_cap + (long double)ns;
    const long double C = (long double)tc_for_bound;
    long double v = (long double)mcap * sumw / ((long double)rows * C) +
                    (long double)ns * ((long double)mcap / rows + 1.0L) +
                    sumw / C + (long double)ns + 16.0L;
    if (v > 1e15L) v = 1e15L;
    return (uint64_t)v;
}

ssbh_status plan_and_fill(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                          uint32_t rows, uint32_t tile_cols,
                          hipStream_t stream, Tile **tiles_out,
                          bool want_tiles = true) {
    const uint64_t ns = q.n_sub;
    // tile_cols = 0 means one column range per sub-block; the bound then
    // uses the longest possible sub-block.
    const uint64_t tc_b = tile_cols ? tile_cols : (2 * q.sub_cap + 1);
    const uint64_t bound =
        want_tiles ? tile_bound(ns, q.m_cap, q.sub_cap, rows, tc_b) : 1;
    if (!want_tiles) rows = 1u << 31;   // tile counts are not used
    if (bound > (1ull << 28)) {
        set_error("tile list too large (%llu tiles); use a smaller m_cap or "
                  "sub_capacity_words", (unsigned long long)bound);
        return SSBH_E_UNSUPPORTED;
    }
    ssbh_status st;
    if ((st = ws.plan.reserve((size_t)ns * 3 * 8 + 64)) != SSBH_OK) return st;
    if ((st = ws.tiles.reserve(want_tiles ? (size_t)bound * sizeof(Tile) + 64
                                          : 64)) != SSBH_OK)
        return st;
    if ((st = ws.counters.reserve(64)) != SSBH_OK) return st;
    PlanArgs pa{};
    pa.len = q.len; pa.woff = q.woff; pa.ns = q.n_sub; pa.rule = q.out_rule;
    pa.ra = q.out_a; pa.rb = q.out_b ? q.out_b : 1; pa.out_len = q.out_len;
    pa.seed_bits = q.seed_bits; pa.stride = q.stride; pa.mcap = q.m_cap;
    pa.sub_cap = q.sub_cap; pa.out_cap = q.out_cap_bits;
    pa.rows = rows; pa.tile_cols = tile_cols;
    pa.tile_cap = want_tiles ? bound : ~0ull;
    uint64_t *plan = ws.plan.as<uint64_t>();
    pa.mlen = plan; pa.ooff = plan + ns; pa.toff = plan + 2 * ns;
    pa.counters = ws.counters.as<uint64_t>();
    pa.out_total = q.out_total; pa.status = q.status;
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, stream, pa);
    const uint64_t ow = (q.out_cap_bits + 63) / 64;
    if (ow) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((ow + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, stream,
                           q.out, ow, q.status);
    }
    if (ns && want_tiles) {
        hipLaunchKernelGGL(k_expand, dim3((uint32_t)((ns + 3) / 4)), dim3(256),
                           0, stream, pa, ws.tiles.as<Tile>());
    }
    SSBH_CHECK_HIP(hipGetLastError());
    *tiles_out = ws.tiles.as<Tile>();
    return SSBH_OK;
}

ScratchSizes hash_scratch(const ssbh_ctx *ctx, const HashRequest &q) {
    ScratchSizes z;
    z.plan = (size_t)q.n_sub * 3 * 8 + 64;
    z.counters = 64;
    if (q.kernel == SSBH_K_MFMA_I8 || q.kernel == SSBH_K_MFMA_F4) {
        z.tiles = 64;
        return z;
    }
    const ValuSchedule s = choose_valu(ctx, q);
    const uint64_t tc_b = s.tile_cols ? s.tile_cols : (2 * q.sub_cap + 1);
    z.tiles = (size_t)tile_bound(q.n_sub, q.m_cap, q.sub_cap, s.rows(), tc_b) *
                  sizeof(Tile) + 64;
    return z;
}

// Lengths, offsets, checks and the zeroed output, without a tile list.
ssbh_status plan_only(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                      hipStream_t stream) {
    Tile *unused = nullptr;
    return plan_and_fill(ctx, ws, q, 1, 0, stream, &unused, false);
}

ssbh_status launch_hash_valu(ssbh_ctx *ctx, Workspace &ws,
                             const HashRequest &q, const ValuSchedule &s,
                             hipStream_t stream) {
    Tile *tiles = nullptr;
    ssbh_status st = plan_and_fill(ctx, ws, q, (uint32_t)s.rows(),
                                   s.tile_cols, stream, &tiles);
    if (st != SSBH_OK) return st;
    snprintf(ws.last_schedule, sizeof ws.last_schedule, "valu:%d:%d:%u:%u",
             s.r, s.waves, s.chunk_cols, s.tile_cols);
    if (!q.n_sub) return SSBH_OK;
    ValuArgs va{};
    va.sub32 = reinterpret_cast<const uint32_t *>(q.sub);
    uint64_t *plan = ws.plan.as<uint64_t>();
    va.len = q.len; va.woff = q.woff; va.mlen = plan; va.ooff = plan + q.n_sub;
    va.seed32 = reinterpret_cast<const uint32_t *>(q.seed);
    va.seed_w32 = (int64_t)(2 * ((q.seed_bits + 63) / 64));
    va.stride = q.stride; va.mcap = q.m_cap;
    va.tiles = tiles;
    va.counters = ws.counters.as<uint64_t>();
    va.claim = reinterpret_cast<uint32_t *>(ws.counters.as<uint64_t>() + 1);
    va.out32 = reinterpret_cast<uint32_t *>(q.out);
    va.status = q.status;
    uint32_t chunk = s.chunk_cols ? s.chunk_cols : 4096;
    chunk = (chunk + s.r - 1) / s.r * s.r;
    va.chunk = chunk;
    TimedLaunch timed(ws.timer, "k_toeplitz_valu", stream);
#define SSBH_VALU_CASE(RR, WW)                                                \
    if (s.r == RR && s.waves == WW)                                           \
        return s.scalar_x ? run_valu<RR, WW, true>(ctx, va, stream)           \
                          : run_valu<RR, WW, false>(ctx, va, stream);
    SSBH_VALU_CASE(8, 2)
    SSBH_VALU_CASE(8, 4)
    SSBH_VALU_CASE(8, 8)
    SSBH_VALU_CASE(16, 2)
    SSBH_VALU_CASE(16, 4)
    SSBH_VALU_CASE(16, 8)
    SSBH_VALU_CASE(32, 2)
    SSBH_VALU_CASE(32, 4)
    SSBH_VALU_CASE(32, 8)
#undef SSBH_VALU_CASE
    set_error("unsupported VALU schedule R=%d waves=%d", s.r, s.waves);
    return SSBH_E_UNSUPPORTED;
}

}  // namespace ssbh
