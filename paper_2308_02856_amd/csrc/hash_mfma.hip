// Shared-seed contraction on the int8 matrix cores of gfx950.
//
// With one seed shared by all sub-blocks (stride S = 0), every T_j is the
// top-left corner of one M x n_max Toeplitz matrix T[r][c] = s[c - r + M - 1]
// (Sec. I), so hashing a group of sub-blocks is one dense product
//     K = (T . [x_j0 ... x_j0+B-1]) mod 2
// over 0/1 values.  v_mfma_i32_32x32x32_i8 multiplies 0/1 bytes and sums in
// int32; only the low bit of each sum is kept (int32 wrap-around keeps the
// parity exact for any length).  Columns past n_j are zero and rows past m_j
// are dropped, so uneven sizes share one launch.
//
// Work split: a workgroup owns BM rows x BN sub-blocks and a range of K
// chunks (split-K; partial parities merge by XOR, which is exact).  Block
// indices are remapped so that the row tiles and K splits of one sub-block
// group run on one XCD (blocks are dispatched to the 8 XCDs round-robin), so
// the group's column words are fetched into one L2 only.  The epilogue
// assembles each sub-block's BM output bits in LDS and stores whole 32-bit
// words; only the two end words of a segment (shared with the neighbouring
// row tile or sub-block) and split-K partials go through atomic XOR.
//
// Operands are built in registers from bit-packed data; T never exists in
// memory.  A-operand lane l (row i = l%32, k = 16*(l/32) + byte) needs 16
// consecutive seed bits; rows 32 apart at columns 32 apart need the same bits,
// so a wave that owns MT row tiles makes ONE new A operand per K step and
// rotates the others (diagonal constancy).  B-operand lane l (sub-block
// l%32) takes 16 data bits of its sub-block.  Bits become 0/1 bytes with one
// multiply per nibble: (nib * 0x204081) & 0x01010101.
#include <algorithm>
#include <cmath>

#include <stdio.h>

#include "ssbh_internal.hpp"

namespace ssbh {

ssbh_status plan_only(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                      hipStream_t stream);

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kKC = 2048;          // columns staged per chunk
constexpr int kKCW = kKC / 32;     // 32-bit words per sub-block per chunk

struct MfmaArgs {
    const uint32_t *sub32;
    const uint64_t *len, *woff, *mlen, *ooff;
    const uint32_t *seed32;
    int64_t seed_w32;
    uint64_t mcap;
    uint32_t ns;
    uint32_t m_tiles;
    uint32_t ksplit;         // K splits per tile (1 = the tile owns all K)
    uint32_t *out32;
    const int32_t *status;
};

// Bits base .. base+15 of b -> 16 bytes of 0/1 (byte t = bit base+t).
__device__ __forceinline__ v4i expand16(uint32_t b, uint32_t base = 0) {
    v4i r;
    r.x = (int)((__builtin_amdgcn_ubfe(b, base, 4) * 0x204081u) & 0x01010101u);
    r.y = (int)((__builtin_amdgcn_ubfe(b, base + 4, 4) * 0x204081u) & 0x01010101u);
    r.z = (int)((__builtin_amdgcn_ubfe(b, base + 8, 4) * 0x204081u) & 0x01010101u);
    r.w = (int)((__builtin_amdgcn_ubfe(b, base + 12, 4) * 0x204081u) & 0x01010101u);
    return r;
}

// Workgroup tile: BM = 32*MT*WM rows x BN = 32*NT sub-blocks; every wave
// owns MT row tiles and all NT sub-block tiles.
template <int MT, int NT, int WM>
struct MfmaTile {
    static constexpr int BM = 32 * MT * WM;
    static constexpr int BN = 32 * NT;
    static constexpr int NTH = 64 * WM;
    static constexpr int XS = kKCW + 1;                 // padded row stride
    static constexpr int WINW = (BM + kKC) / 32 + MT + 6;
    static constexpr int PFX = BN * kKCW / NTH;         // words per thread
    static constexpr int PFW = (WINW + NTH - 1) / NTH;  // window words/thread
    static constexpr int OBW = BM / 32 + 1;             // epilogue words/col
};

// Block b runs logical tile t: XCD x = b mod 8 takes the x-th contiguous
// range of logical tiles (a bijection for any grid size).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t g) {
    const uint32_t per = g >> 3, rem = g & 7u, x = b & 7u;
    const uint32_t start = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return start + (b >> 3);
}

template <int MT, int NT, int WM, int OCC>
__global__ __launch_bounds__(64 * WM) __attribute__((amdgpu_waves_per_eu(OCC)))
void k_toeplitz_mfma(MfmaArgs a) {
    using TT = MfmaTile<MT, NT, WM>;
    constexpr int BM = TT::BM, BN = TT::BN, NTH = TT::NTH, XS = TT::XS;
    constexpr int WINW = TT::WINW, PFX = TT::PFX, PFW = TT::PFW;
    constexpr int OBW = TT::OBW;
    static_assert(BN * kKCW % NTH == 0, "staging must divide evenly");
    static_assert(OBW <= XS, "epilogue image must fit the staging area");
    __shared__ uint32_t xs[BN * XS];
    __shared__ uint32_t win[WINW];
    __shared__ uint64_t woff_s[BN], mlen_s[BN], ooff_s[BN];
    __shared__ uint32_t nw_s[BN], tail_s[BN];
    __shared__ uint64_t nmax_s, mmax_s;
    if (*a.status) return;

    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t mt = t % a.m_tiles;
    const uint32_t rest = t / a.m_tiles;
    const uint32_t ks = rest % a.ksplit;
    const uint32_t grp = rest / a.ksplit;
    const int64_t R0 = (int64_t)mt * BM;
    const uint32_t J0 = grp * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, li = lane & 31;

    if (threadIdx.x == 0) { nmax_s = 0; mmax_s = 0; }
    __syncthreads();
    for (int jl = threadIdx.x; jl < BN; jl += NTH) {
        const uint32_t j = J0 + jl;
        uint64_t n = 0, m = 0, wo = 0, oo = 0;
        if (j < a.ns) {
            n = a.len[j]; m = a.mlen[j]; wo = a.woff[j]; oo = a.ooff[j];
        }
        woff_s[jl] = wo;
        mlen_s[jl] = m;
        ooff_s[jl] = oo;
        nw_s[jl] = (uint32_t)((n + 31) / 32);
        tail_s[jl] = (n & 31) ? ((1u << (n & 31)) - 1u) : ~0u;
        if (n) atomicMax((unsigned long long *)&nmax_s, (unsigned long long)n);
        if (m) atomicMax((unsigned long long *)&mmax_s, (unsigned long long)m);
    }
    __syncthreads();
    const uint64_t nmax = nmax_s, mmax = mmax_s;
    if (nmax == 0 || (uint64_t)R0 >= mmax) return;   // uniform
    const uint32_t nwords = (uint32_t)((nmax + 31) / 32);
    // This split's column words: whole chunks [c_lo, c_hi).
    const uint32_t nchunks = (nwords + kKCW - 1) / kKCW;
    const uint32_t c_lo = (uint32_t)((uint64_t)ks * nchunks / a.ksplit);
    const uint32_t c_hi = (uint32_t)((uint64_t)(ks + 1) * nchunks / a.ksplit);
    if (c_lo >= c_hi) return;                          // uniform
    const uint32_t cw_begin = c_lo * kKCW;
    const uint32_t cw_end = min(c_hi * (uint32_t)kKCW, nwords);
    const int64_t R0w = R0 + (int64_t)wave * 32 * MT;   // wave's first row

    // Register prefetch of one chunk: column words and seed window.
    uint32_t pfx[PFX], pfw[PFW];
    auto window_lo = [&](uint32_t cw0) -> int64_t {
        // Lowest seed bit of the chunk: column 32*cw0, row R0+BM-1; the first
        // chunk of the split also needs MT-1 earlier A operands.
        const int64_t lo = 32 * (int64_t)cw0 - (R0 + BM - 1) + (int64_t)a.mcap -
                           1 - (cw0 == cw_begin ? 32 * (MT - 1) : 0);
        return lo >> 5;
    };
    auto prefetch = [&](uint32_t cw0) {
#pragma unroll
        for (int i = 0; i < PFX; ++i) {
            const int t = threadIdx.x + i * NTH;
            const int jl = t / kKCW, w = t - jl * kKCW;
            const uint32_t cw = cw0 + w;
            uint32_t x = 0u;
            if (cw < nw_s[jl]) {
                x = a.sub32[2 * woff_s[jl] + cw];
                if (cw == nw_s[jl] - 1) x &= tail_s[jl];
            }
            pfx[i] = x;
        }
        const int64_t lo_w = window_lo(cw0);
#pragma unroll
        for (int i = 0; i < PFW; ++i) {
            const int t = threadIdx.x + i * NTH;
            const int64_t g = lo_w + t;
            pfw[i] = (t < WINW && g >= 0 && g < a.seed_w32) ? a.seed32[g] : 0u;
        }
    };

    v16i acc[MT][NT];
#pragma unroll
    for (int p = 0; p < MT; ++p)
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[p][q][r] = 0;
    // Ring of tile-0 A operands: slot (s mod MT) holds step s; tile p at
    // step s uses step s - p.
    v4i ring[MT];

    prefetch(cw_begin);
    for (uint32_t cw0 = cw_begin; cw0 < cw_end; cw0 += kKCW) {
#pragma unroll
        for (int i = 0; i < PFX; ++i) {
            const int t = threadIdx.x + i * NTH;
            const int jl = t / kKCW, w = t - jl * kKCW;
            xs[jl * XS + w] = pfx[i];
        }
#pragma unroll
        for (int i = 0; i < PFW; ++i) {
            const int t = threadIdx.x + i * NTH;
            if (t < WINW) win[t] = pfw[i];
        }
        const int64_t lo_w = window_lo(cw0);
        __syncthreads();
        if (cw0 + kKCW < cw_end) prefetch(cw0 + kKCW);

        // This lane's seed bit for (its row at tile 0, column 32*cw0 + 16h).
        const int64_t e = 32 * (int64_t)cw0 + 16 * h - (R0w + li) +
                          (int64_t)a.mcap - 1 - (lo_w << 5);
        const int qa = (int)(e >> 5);
        const uint32_t sha = (uint32_t)(e & 31);
        if (cw0 == cw_begin) {
            // Steps -1 .. -(MT-1) of tile 0 (slots MT-1 .. 1).
#pragma unroll
            for (int d = 1; d < MT; ++d) {
                const int qq = qa - d;
                ring[MT - d] = expand16(
                    __builtin_amdgcn_alignbit(win[qq + 1], win[qq], sha));
            }
        }
        // Steps of this chunk, rounded up to a multiple of MT (only the last
        // chunk of a sub-block group can be short; its staged column words
        // past the sub-blocks are zero).
        const uint32_t steps =
            (min((uint32_t)kKCW, cw_end - cw0) + MT - 1) / MT * MT;
        // Software pipeline: the operands of step s+1 are built while the
        // matrix cores run step s.
        v4i a_next, b_next[NT];
        const uint32_t hb = 16u * (uint32_t)h;
        auto build = [&](uint32_t s, v4i &an, v4i (&bn)[NT]) {
            const int qq = qa + (int)s;
            an = expand16(__builtin_amdgcn_alignbit(win[qq + 1], win[qq], sha));
#pragma unroll
            for (int q = 0; q < NT; ++q)
                bn[q] = expand16(xs[(32 * q + li) * XS + s], hb);
        };
        build(0, a_next, b_next);
        for (uint32_t s0 = 0; s0 < steps; s0 += MT) {
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                const uint32_t s = s0 + u;
                ring[u] = a_next;
                v4i bcur[NT];
#pragma unroll
                for (int q = 0; q < NT; ++q) bcur[q] = b_next[q];
                // Step s+1 <= kKCW stays inside the padded LDS arrays; its
                // operands are unused after the last step.
                build(s + 1, a_next, b_next);
#pragma unroll
                for (int p = 0; p < MT; ++p)
#pragma unroll
                    for (int q = 0; q < NT; ++q)
                        acc[p][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                            ring[(u - p + MT) % MT], bcur[q], acc[p][q], 0, 0, 0);
                // Interleave: LDS reads first, then one matrix op per three
                // vector ops.
                __builtin_amdgcn_sched_group_barrier(0x100, 1 + NT, 0);
#pragma unroll
                for (int k = 0; k < MT * NT; ++k) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
                }
            }
        }
        __syncthreads();
    }

    // Parity.  Lane l holds rows 8(r/4) + 4h + (r%4) of column l%32; the
    // partner lane l^32 holds the other 16 rows.  Each 32-row word goes to
    // the LDS image ob[sub-block][row word] (rows past m_j cleared).
    uint32_t *ob = xs;
#pragma unroll
    for (int p = 0; p < MT; ++p) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            uint32_t mine = 0u;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                mine |= ((uint32_t)acc[p][q][r] & 1u)
                        << (8 * (r / 4) + 4 * h + (r % 4));
            const uint32_t word = mine | (uint32_t)__shfl_xor((int)mine, 32, 64);
            const int jl = 32 * q + li;
            const int64_t nvalid = (int64_t)mlen_s[jl] - (R0w + 32 * p);
            uint32_t v = nvalid > 0 ? word : 0u;
            if (nvalid > 0 && nvalid < 32) v &= (1u << nvalid) - 1u;
            if (h == 0) ob[jl * OBW + wave * MT + p] = v;
        }
    }
    for (int jl = threadIdx.x; jl < BN; jl += NTH) ob[jl * OBW + OBW - 1] = 0u;
    __syncthreads();
    // Output words: sub-block j's rows R0 .. R0+nb-1 land at bits P .. P+nb-1
    // with P = O_j + R0.  Words wholly inside that range belong to this
    // workgroup alone (when it owns all of K) and are stored; the others are
    // merged with atomic XOR into the zeroed output.
    const bool owner = a.ksplit == 1;
    for (int idx = threadIdx.x; idx < BN * OBW; idx += NTH) {
        const int jl = idx / OBW, k = idx - jl * OBW;
        const uint64_t m = mlen_s[jl];
        if (m <= (uint64_t)R0) continue;
        const uint64_t nb = min(m - (uint64_t)R0, (uint64_t)BM);
        const uint64_t P = ooff_s[jl] + (uint64_t)R0;
        const uint32_t sh = (uint32_t)(P & 31);
        const uint64_t wq0 = P >> 5;
        if ((uint64_t)k > ((P + nb - 1) >> 5) - wq0) continue;
        const uint32_t *row = ob + jl * OBW;
        uint32_t val = row[k];
        if (sh) val = (val << sh) | (k ? row[k - 1] >> (32 - sh) : 0u);
        const uint64_t wstart = 32 * (wq0 + (uint64_t)k);
        if (owner && wstart >= P && wstart + 32 <= P + nb)
            a.out32[wq0 + k] = val;
        else if (val)
            atomicXor(a.out32 + wq0 + k, val);
    }
}

// fp4 variant (v_mfma_scale_f32_32x32x64_f8f6f4, e2m1 operands, unit
// scales): 0 and 1 are exact e2m1 values (codes 0 and 2) and the fp32 sums
// of 0/1 products stay exact integers below 2^24, so the low bit is the
// parity for sub-blocks of fewer than 2^24 bits (checked on the host).  One
// matrix op covers 64 columns: lane l (row or sub-block l%32) supplies the
// 32 columns 32*(l/32) .. +31 of the step as nibbles of four registers.
// Rows 32 apart at columns 32 apart share seed bits, so the A operand of
// tile p at step s is the 32-bit seed window W(2s + h - p); a ring of MT
// windows indexed by 2s - p (uniform across lanes) gets two new entries per
// step, W(2s + h) and W(2s - 1 + h).
// Bits become codes once per workgroup, when a chunk is staged: each 32-bit
// word of the sub-blocks and of the seed window is stored in LDS as the four
// registers of its nibble codes (byte d -> register d).  A wave then reads a
// B operand as one 16-byte LDS load, and a seed window that starts at bit b
// as the five code registers from b / 8 on, joined by four funnel shifts of
// 4 (b mod 8) bits; no wave expands bits in its step loop.
__device__ __forceinline__ uint32_t spread8(uint32_t b) {   // bit i -> code 2
    uint32_t t = b & 0xFFu;
    t = (t | (t << 12)) & 0x000F000Fu;
    t = (t | (t << 6)) & 0x03030303u;
    t = (t | (t << 3)) & 0x11111111u;
    return t << 1;
}
__device__ __forceinline__ v4i expand32_f4(uint32_t b) {
    v4i r;
    r.x = (int)spread8(b);
    r.y = (int)spread8(b >> 8);
    r.z = (int)spread8(b >> 16);
    r.w = (int)spread8(b >> 24);
    return r;
}

template <int MT, int NT, int WM, int OCC>
__global__ __launch_bounds__(64 * WM) __attribute__((amdgpu_waves_per_eu(OCC)))
void k_toeplitz_mfma_f4(MfmaArgs a) {
    static_assert(MT % 2 == 0, "the window ring needs an even MT");
    using TT = MfmaTile<MT, NT, WM>;
    constexpr int BM = TT::BM, BN = TT::BN, NTH = TT::NTH, XS = TT::XS;
    constexpr int WINW = TT::WINW, PFX = TT::PFX, PFW = TT::PFW;
    constexpr int OBW = TT::OBW;
    constexpr int U = MT / 2;                 // steps per ring turn
    // Code registers per sub-block row: 4 per word, padded by 4 so that the
    // 16-byte loads of 16 consecutive lanes (rows) cover all banks.
    constexpr int XS4 = 4 * kKCW + 4;
    (void)XS;
    static_assert(BN * kKCW % NTH == 0, "staging must divide evenly");
    static_assert(OBW <= XS4, "epilogue image must fit the staging area");
    __shared__ __align__(16) uint32_t xs4[BN * XS4];
    __shared__ __align__(16) uint32_t winx[4 * WINW];
    __shared__ uint64_t woff_s[BN], mlen_s[BN], ooff_s[BN];
    __shared__ uint32_t nw_s[BN], tail_s[BN];
    __shared__ uint64_t nmax_s, mmax_s;
    if (*a.status) return;

    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t mt = t % a.m_tiles;
    const uint32_t rest = t / a.m_tiles;
    const uint32_t ks = rest % a.ksplit;
    const uint32_t grp = rest / a.ksplit;
    const int64_t R0 = (int64_t)mt * BM;
    const uint32_t J0 = grp * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, li = lane & 31;

    if (threadIdx.x == 0) { nmax_s = 0; mmax_s = 0; }
    __syncthreads();
    for (int jl = threadIdx.x; jl < BN; jl += NTH) {
        const uint32_t j = J0 + jl;
        uint64_t n = 0, m = 0, wo = 0, oo = 0;
        if (j < a.ns) {
            n = a.len[j]; m = a.mlen[j]; wo = a.woff[j]; oo = a.ooff[j];
        }
        woff_s[jl] = wo;
        mlen_s[jl] = m;
        ooff_s[jl] = oo;
        nw_s[jl] = (uint32_t)((n + 31) / 32);
        tail_s[jl] = (n & 31) ? ((1u << (n & 31)) - 1u) : ~0u;
        if (n) atomicMax((unsigned long long *)&nmax_s, (unsigned long long)n);
        if (m) atomicMax((unsigned long long *)&mmax_s, (unsigned long long)m);
    }
    __syncthreads();
    const uint64_t nmax = nmax_s, mmax = mmax_s;
    if (nmax == 0 || (uint64_t)R0 >= mmax) return;   // uniform
    const uint32_t nwords = (uint32_t)((nmax + 31) / 32);
    const uint32_t nchunks = (nwords + kKCW - 1) / kKCW;
    const uint32_t c_lo = (uint32_t)((uint64_t)ks * nchunks / a.ksplit);
    const uint32_t c_hi = (uint32_t)((uint64_t)(ks + 1) * nchunks / a.ksplit);
    if (c_lo >= c_hi) return;                          // uniform
    const uint32_t cw_begin = c_lo * kKCW;
    const uint32_t cw_end = min(c_hi * (uint32_t)kKCW, nwords);
    const int64_t R0w = R0 + (int64_t)wave * 32 * MT;

    uint32_t pfx[PFX], pfw[PFW];
    auto window_lo = [&](uint32_t cw0) -> int64_t {
        const int64_t lo = 32 * (int64_t)cw0 - (R0 + BM - 1) + (int64_t)a.mcap -
                           1 - (cw0 == cw_begin ? 32 * (MT - 1) : 0);
        return lo >> 5;
    };
    auto prefetch = [&](uint32_t cw0) {
#pragma unroll
        for (int i = 0; i < PFX; ++i) {
            const int t = threadIdx.x + i * NTH;
            const int jl = t / kKCW, w = t - jl * kKCW;
            const uint32_t cw = cw0 + w;
            uint32_t x = 0u;
            if (cw < nw_s[jl]) {
                x = a.sub32[2 * woff_s[jl] + cw];
                if (cw == nw_s[jl] - 1) x &= tail_s[jl];
            }
            pfx[i] = x;
        }
        const int64_t lo_w = window_lo(cw0);
#pragma unroll
        for (int i = 0; i < PFW; ++i) {
            const int t = threadIdx.x + i * NTH;
            const int64_t g = lo_w + t;
            pfw[i] = (t < WINW && g >= 0 && g < a.seed_w32) ? a.seed32[g] : 0u;
        }
    };

    v16f acc[MT][NT];
#pragma unroll
    for (int p = 0; p < MT; ++p)
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[p][q][r] = 0.0f;
    v4i ring[MT];

    prefetch(cw_begin);
    for (uint32_t cw0 = cw_begin; cw0 < cw_end; cw0 += kKCW) {
#pragma unroll
        for (int i = 0; i < PFX; ++i) {
            const int t = threadIdx.x + i * NTH;
            const int jl = t / kKCW, w = t - jl * kKCW;
            *reinterpret_cast<v4i *>(&xs4[jl * XS4 + 4 * w]) = expand32_f4(pfx[i]);
        }
#pragma unroll
        for (int i = 0; i < PFW; ++i) {
            const int t = threadIdx.x + i * NTH;
            if (t < WINW) *reinterpret_cast<v4i *>(&winx[4 * t]) = expand32_f4(pfw[i]);
        }
        const int64_t lo_w = window_lo(cw0);
        __syncthreads();
        if (cw0 + kKCW < cw_end) prefetch(cw0 + kKCW);

        // Seed window W(t) for this lane's row at tile 0: bits at column
        // 32 cw0 + 32 t of the chunk, that is bits 32 (qa + t) + sha .. +31
        // of the staged window: code registers from 4 (qa + t) + sha / 8 on,
        // shifted by 4 (sha mod 8) bits.
        const int64_t e = 32 * (int64_t)cw0 - (R0w + li) + (int64_t)a.mcap - 1 -
                          (lo_w << 5);
        const int qa = (int)(e >> 5);
        const uint32_t sha = (uint32_t)(e & 31);
        const int cq = (int)(sha >> 3);
        const uint32_t sh4 = 4u * (sha & 7u);
        const uint32_t words = min((uint32_t)kKCW, cw_end - cw0);
        const uint32_t steps = ((words + 1) / 2 + U - 1) / U * U;
        // The LDS words of one step's operands: the five code registers of
        // each new seed window (W(2s + h), W(2s - 1 + h)) and the B codes.
        uint32_t rw[2][5];
        v4i rb[NT];
        auto load = [&](uint32_t s) {
            // Step s' <= steps - 1 keeps every LDS read inside its row; the
            // operands loaded for the step after the last are never used.
            const uint32_t sc = min(s, steps - 1);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t *c = winx + 4 * (qa + 2 * (int)sc - k + h) + cq;
#pragma unroll
                for (int d = 0; d < 5; ++d) rw[k][d] = c[d];
            }
#pragma unroll
            for (int q = 0; q < NT; ++q)
                rb[q] = *reinterpret_cast<const v4i *>(
                    &xs4[(32 * q + li) * XS4 + 4 * (2 * sc + h)]);
        };
        // W(t) from its five code registers: four funnel shifts.
        auto window = [&](const uint32_t (&c)[5]) {
            v4i r;
            r.x = (int)__builtin_amdgcn_alignbit(c[1], c[0], sh4);
            r.y = (int)__builtin_amdgcn_alignbit(c[2], c[1], sh4);
            r.z = (int)__builtin_amdgcn_alignbit(c[3], c[2], sh4);
            r.w = (int)__builtin_amdgcn_alignbit(c[4], c[3], sh4);
            return r;
        };
        if (cw0 == cw_begin) {
            // Slots -2 .. -(MT-1): W(h - p) for tiles p = 2 .. MT-1 at step 0.
#pragma unroll
            for (int p = 2; p < MT; ++p) {
                uint32_t c[5];
                const uint32_t *src = winx + 4 * (qa + h - p) + cq;
#pragma unroll
                for (int d = 0; d < 5; ++d) c[d] = src[d];
                ring[MT - p] = window(c);
            }
        }
        load(0);
        v4i a0_next = window(rw[0]), a1_next = window(rw[1]), b_next[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) b_next[q] = rb[q];
        auto mfma_tiles = [&](int u, int p0, int p1, const v4i (&bcur)[NT]) {
#pragma unroll
            for (int p = p0; p < p1; ++p) {
                const v4i ar = ring[(2 * u - p + 2 * MT) % MT];
                v8i A8 = {ar.x, ar.y, ar.z, ar.w, 0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    v8i B8 = {bcur[q].x, bcur[q].y, bcur[q].z, bcur[q].w,
                              0, 0, 0, 0};
                    acc[p][q] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        A8, B8, acc[p][q], 4, 4, 0, 127, 0, 127);
                }
            }
        };
        for (uint32_t s0 = 0; s0 < steps; s0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t s = s0 + u;
                ring[(2 * u) % MT] = a0_next;
                ring[(2 * u - 1 + MT) % MT] = a1_next;
                v4i bcur[NT];
#pragma unroll
                for (int q = 0; q < NT; ++q) bcur[q] = b_next[q];
                // The next step's LDS loads go out before this step's first
                // matrix ops and are shifted into operands halfway through,
                // so their latency hides behind the matrix cores.
                load(s + 1);
                __builtin_amdgcn_sched_barrier(0);
                mfma_tiles(u, 0, MT / 2, bcur);
                __builtin_amdgcn_sched_barrier(0);
                a0_next = window(rw[0]);
                a1_next = window(rw[1]);
#pragma unroll
                for (int q = 0; q < NT; ++q) b_next[q] = rb[q];
                mfma_tiles(u, MT / 2, MT, bcur);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();
    }

    uint32_t *ob = xs4;
#pragma unroll
    for (int p = 0; p < MT; ++p) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            uint32_t mine = 0u;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                mine |= ((uint32_t)(int)acc[p][q][r] & 1u)
                        << (8 * (r / 4) + 4 * h + (r % 4));
            const uint32_t word = mine | (uint32_t)__shfl_xor((int)mine, 32, 64);
            const int jl = 32 * q + li;
            const int64_t nvalid = (int64_t)mlen_s[jl] - (R0w + 32 * p);
            uint32_t v = nvalid > 0 ? word : 0u;
            if (nvalid > 0 && nvalid < 32) v &= (1u << nvalid) - 1u;
            if (h == 0) ob[jl * OBW + wave * MT + p] = v;
        }
    }
    for (int jl = threadIdx.x; jl < BN; jl += NTH) ob[jl * OBW + OBW - 1] = 0u;
    __syncthreads();
    const bool owner = a.ksplit == 1;
    for (int idx = threadIdx.x; idx < BN * OBW; idx += NTH) {
        const int jl = idx / OBW, k = idx - jl * OBW;
        const uint64_t m = mlen_s[jl];
        if (m <= (uint64_t)R0) continue;
        const uint64_t nb = min(m - (uint64_t)R0, (uint64_t)BM);
        const uint64_t P = ooff_s[jl] + (uint64_t)R0;
        const uint32_t sh = (uint32_t)(P & 31);
        const uint64_t wq0 = P >> 5;
        if ((uint64_t)k > ((P + nb - 1) >> 5) - wq0) continue;
        const uint32_t *row = ob + jl * OBW;
        uint32_t val = row[k];
        if (sh) val = (val << sh) | (k ? row[k - 1] >> (32 - sh) : 0u);
        const uint64_t wstart = 32 * (wq0 + (uint64_t)k);
        if (owner && wstart >= P && wstart + 32 <= P + nb)
            a.out32[wq0 + k] = val;
        else if (val)
            atomicXor(a.out32 + wq0 + k, val);
    }
}

// K splits per tile: enough tiles in flight to fill every CU in whole
// rounds (a short last round idles most of the chip), at least 8 K chunks
// per split.
uint32_t choose_ksplit(uint64_t tiles, uint64_t slots, uint64_t nchunks) {
    uint32_t best = 1;
    double best_eff = 0.0;
    for (uint32_t k = 1; k <= 4; ++k) {
        if (k > 1 && nchunks < 8ull * k) break;
        const double r = (double)(tiles * k) / (double)slots;
        const double eff = r / std::ceil(r) * (1.0 - 0.015 * (k - 1));
        if (eff > best_eff + 1e-9) { best_eff = eff; best = k; }
    }
    return best;
}

template <int MT, int NT, int WM, int OCC, bool F4>
ssbh_status run_mfma(ssbh_ctx *ctx, const MfmaArgs &ma, uint32_t ksplit,
                     uint64_t ncap, hipStream_t stream) {
    using TT = MfmaTile<MT, NT, WM>;
    MfmaArgs m = ma;
    m.m_tiles = (uint32_t)((ma.mcap + TT::BM - 1) / TT::BM);
    const uint64_t groups = (ma.ns + TT::BN - 1) / TT::BN;
    const uint64_t tiles = (uint64_t)m.m_tiles * groups;
    if (tiles == 0) return SSBH_OK;
    const uint64_t nchunks = (ncap + 32ull * kKCW - 1) / (32ull * kKCW);
    m.ksplit = ksplit ? ksplit
                      : choose_ksplit(tiles, (uint64_t)ctx->num_cus * OCC,
                                      nchunks);
    const uint64_t grid = tiles * m.ksplit;
    if (grid >= (1ull << 31)) {
        set_error("MFMA grid too large");
        return SSBH_E_UNSUPPORTED;
    }
    if constexpr (F4) {
        if constexpr (MT % 2 == 0)
            hipLaunchKernelGGL((k_toeplitz_mfma_f4<MT, NT, WM, OCC>),
                               dim3((uint32_t)grid), dim3(64 * WM), 0, stream, m);
    } else {
        hipLaunchKernelGGL((k_toeplitz_mfma<MT, NT, WM, OCC>), dim3((uint32_t)grid),
                           dim3(64 * WM), 0, stream, m);
    }
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

}  // namespace

ssbh_status launch_hash_mfma(ssbh_ctx *ctx, Workspace &ws,
                             const HashRequest &q, const MfmaSchedule &s,
                             hipStream_t stream) {
    if (q.stride != 0) {
        set_error("the MFMA kernel needs a shared seed (seed_stride = 0)");
        return SSBH_E_INVAL;
    }
    ssbh_status st = plan_only(ctx, ws, q, stream);
    if (st != SSBH_OK) return st;
    const bool f4 = q.kernel == SSBH_K_MFMA_F4;
    snprintf(ws.last_schedule, sizeof ws.last_schedule, "%s:%d:%d:%d:%d",
             f4 ? "mfma4" : "mfma", s.mt, s.nt, s.wm, s.ksplit);
    if (!q.n_sub) return st;
    MfmaArgs ma{};
    uint64_t *plan = ws.plan.as<uint64_t>();
    ma.sub32 = reinterpret_cast<const uint32_t *>(q.sub);
    ma.len = q.len; ma.woff = q.woff; ma.mlen = plan; ma.ooff = plan + q.n_sub;
    ma.seed32 = reinterpret_cast<const uint32_t *>(q.seed);
    ma.seed_w32 = (int64_t)(2 * ((q.seed_bits + 63) / 64));
    ma.mcap = q.m_cap;
    ma.ns = q.n_sub;
    ma.out32 = reinterpret_cast<uint32_t *>(q.out);
    ma.status = q.status;
    if (s.ksplit < 0 || s.ksplit > 64) {
        set_error("ksplit must be 0 (automatic) .. 64");
        return SSBH_E_INVAL;
    }
    // Mean sub-block length from the buffer capacity: the split count only
    // needs an estimate of the K chunks per tile.
    const uint64_t ncap = 64ull * q.sub_cap / q.n_sub + 64;
    if (f4 && (s.mt % 2 != 0)) {
        set_error("the fp4 matrix kernel needs an even MT");
        return SSBH_E_UNSUPPORTED;
    }
    TimedLaunch timed(ws.timer, f4 ? "k_toeplitz_mfma_f4" : "k_toeplitz_mfma",
                      stream);
#define SSBH_MFMA_CASE(A, B, C, O)                                            \
    if (s.mt == A && s.nt == B && s.wm == C)                                  \
        return f4 ? run_mfma<A, B, C, O, true>(ctx, ma, (uint32_t)s.ksplit,  \
                                               ncap, stream)                  \
                  : run_mfma<A, B, C, O, false>(ctx, ma, (uint32_t)s.ksplit, \
                                                ncap, stream);
    SSBH_MFMA_CASE(8, 2, 4, 1)
    SSBH_MFMA_CASE(4, 4, 4, 1)
    SSBH_MFMA_CASE(4, 2, 4, 2)
    SSBH_MFMA_CASE(4, 2, 8, 2)
    SSBH_MFMA_CASE(8, 1, 4, 1)
#undef SSBH_MFMA_CASE
    set_error("unsupported MFMA schedule");
    return SSBH_E_UNSUPPORTED;
}

}  // namespace ssbh
