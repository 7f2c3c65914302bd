// Sampling (Sec. III.B step 1) and the abort rule (Sec. III.B step 2,
// Sec. III.D) on gfx950.
//
// i.i.d. / explicit modes: the input is cut into segments of seg_bits bits.
//   k_hist_q   (default) one workgroup per segment: V_i for every bit
//              (recomputed from the counter-based generator, never stored),
//              LDS histograms per quarter -> counts[seg][j] and the quarter
//              counts; also clears the sub-block buffer.
//   k_hist     one wavefront per segment, counts[seg][j] only (fallback).
//   k_scan_*   column scans of counts over segments -> offs[seg][j] (where the
//              segment's run of sub-block j starts), n_j, W_j, max n_j, abort.
//   k_scatter_wg (default), k_scatter_tab, k_scatter: V_i again; a stable
//              rank of each bit among equal V_i; the bits are ORed into an
//              LDS image of the segment sorted by sub-block (stable), then
//              every run is copied to its place in sub-block j: whole 64-bit
//              words by plain stores, the two partial end words by atomic OR
//              (they are shared with the neighbouring segments' runs).  OR
//              into a zeroed buffer is order independent, so the result is
//              bit-identical for every schedule.
// Sifting (Sec. III.B step 2): with keep flags, V_i is still drawn for every
// round (the draws do not depend on the flags) but only rounds with keep_i = 1
// are counted and placed, which equals sifting every sub-block after the
// division.
// permutation mode: the gather B[k] = A[pi[k]] (gather.hip).
#include <algorithm>

#include "ssbh_internal.hpp"

namespace ssbh {
namespace {

constexpr uint32_t kSegChunk = 64;   // segments per partial-sum chunk
constexpr uint64_t kWgMaxSeg = 65024;  // workgroup scatter: 16-bit positions

struct SampleArgs {
    const uint64_t *in;
    uint64_t n;
    uint32_t ns;
    uint32_t vbits;          // ceil(log2(ns))
    uint32_t vshift;         // 32 - log2(ns) when ns is a power of two >= 2
    uint64_t key;
    const uint32_t *assign;  // explicit mode
    const uint64_t *keep;    // sifting flags (nullptr = keep every round)
    uint64_t seg_bits;       // multiple of 64
    uint32_t nseg;
    uint32_t nchunk;
    uint32_t *counts;        // [nseg][ns]
    uint16_t *qcnt;          // [nseg][3][ns] counts of quarters 0..2
    uint32_t *offs;          // [nseg][ns]
    uint32_t *part;          // [nchunk][ns]
    uint64_t *sub;
    uint64_t sub_cap;
    uint64_t *len;
    uint64_t *woff;
    uint64_t l_ub;
    int32_t *status;
};

template <bool EXPLICIT>
__device__ __forceinline__ uint32_t sample_v(const SampleArgs &a, uint64_t i) {
    if constexpr (EXPLICIT) {
        return a.assign[i];
    } else {
        const uint64_t r = splitmix64_at(a.key, i >> 1);
        const uint32_t u = (i & 1ull) ? (uint32_t)(r >> 32) : (uint32_t)r;
        return __umulhi(u, a.ns);   // floor(u * ns / 2^32)
    }
}

// V = floor(u * ns / 2^32); a shift when ns is a power of two (POW2).
template <bool POW2>
__device__ __forceinline__ uint32_t v_of(const SampleArgs &a, uint32_t u) {
    if constexpr (POW2) return u >> a.vshift;
    else return __umulhi(u, a.ns);
}

__global__ void k_init_status(int32_t *status) { *status = 0; }

// keep_i (1 without flags).  i >> 6 is the same word for all lanes of a step.
__device__ __forceinline__ bool kept(const SampleArgs &a, uint64_t i) {
    return !a.keep || ((a.keep[i >> 6] >> (i & 63)) & 1ull);
}

template <bool EXPLICIT>
__global__ __launch_bounds__(256) void k_hist(SampleArgs a) {
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    // Clear the sub-block buffer (the scatter ORs partial words into it).
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
         k < a.sub_cap; k += stride)
        a.sub[k] = 0ull;

    const uint32_t seg = blockIdx.x * wpb + w;
    if (seg >= a.nseg) return;      // per-wave exit, no block barriers below
    uint32_t *hist = lds + (size_t)w * a.ns;
    for (uint32_t j = lane; j < a.ns; j += 64) hist[j] = 0u;
    __builtin_amdgcn_wave_barrier();
    const uint64_t i0 = (uint64_t)seg * a.seg_bits;
    const uint64_t i1 = min(i0 + a.seg_bits, a.n);
    bool bad = false;
    for (uint64_t i = i0 + lane; i < i1; i += 64) {
        const uint32_t v = sample_v<EXPLICIT>(a, i);
        if (v >= a.ns) bad = true;
        else if (kept(a, i)) atomicAdd(&hist[v], 1u);
    }
    if (bad) atomicExch(a.status, (int32_t)SSBH_E_INVAL);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): LDS atomics done
    uint32_t *dst = a.counts + (uint64_t)seg * a.ns;
    for (uint32_t j = lane; j < a.ns; j += 64) dst[j] = hist[j];
}

// Histogram for the workgroup scatter: one workgroup of four wavefronts per
// segment, wavefront w counting quarter w of it.  Writes the segment totals
// counts[seg][j] and the counts of quarters 0..2, qcnt[seg][w][j] (uint16: a
// quarter has fewer than 2^16 rounds), which place each quarter's run inside
// the segment's run.  Counting does not depend on the order of the rounds,
// so lane l takes rounds 2l and 2l + 1 of every 128-round block from the low
// and high halves of one SplitMix64 output.
template <bool EXPLICIT, bool POW2>
__global__ __launch_bounds__(256) void k_hist_q(SampleArgs a) {
    extern __shared__ uint32_t lds[];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t ns = a.ns;
    // Clear the sub-block buffer (the scatter ORs partial words into it).
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + t; k < a.sub_cap;
         k += stride)
        a.sub[k] = 0ull;
    const uint32_t seg = blockIdx.x;
    if (seg >= a.nseg) return;      // whole workgroup
    uint32_t *hist = lds;           // [4][ns]
    for (uint32_t k = t; k < 4 * ns; k += 256) hist[k] = 0u;
    __syncthreads();
    const uint32_t sb = (uint32_t)a.seg_bits;
    const uint32_t i0 = seg * sb;
    const uint32_t i1 = min(i0 + sb, (uint32_t)a.n);   // n <= 2^32 - 2^20
    const uint32_t qlen = sb / 4;                       // multiple of 128
    const uint32_t qa = i0 + (uint32_t)w * qlen;
    const uint32_t qb = min(qa + qlen, i1);
    const uint32_t nw_in = (uint32_t)((a.n + 63) / 64);
    const uint32_t lane2 = 2u * (uint32_t)lane, sh = lane2 & 63u;
    uint32_t *h = hist + (uint32_t)w * ns;
    bool bad = false;
    // SplitMix64 counter of output (base / 2 + lane): advances by 64 outputs
    // per block of 128 rounds.
    uint64_t z = a.key + ((uint64_t)((qa >> 1) + (uint32_t)lane) + 1ull) * kSplitMixGamma;
    for (uint32_t base = qa; base < qb; base += 128, z += 64ull * kSplitMixGamma) {
        const uint32_t iA = base + lane2, iB = iA + 1;
        uint32_t vA, vB;
        if constexpr (EXPLICIT) {
            vA = iA < qb ? a.assign[iA] : 0u;
            vB = iB < qb ? a.assign[iB] : 0u;
        } else {
            const uint64_t r = splitmix64_mix(z);
            vA = v_of<POW2>(a, (uint32_t)r);
            vB = v_of<POW2>(a, (uint32_t)(r >> 32));
        }
        uint32_t kb = 3u;
        if (a.keep)
            kb = (uint32_t)(a.keep[min((base >> 6) + (uint32_t)(lane >> 5), nw_in - 1)] >> sh);
        bool okA = iA < qb && (kb & 1u), okB = iB < qb && (kb & 2u);
        if constexpr (EXPLICIT) {
            // Out-of-range V is an error even on a dropped (unkept) round.
            bad = bad || (iA < qb && vA >= ns) || (iB < qb && vB >= ns);
            okA = okA && vA < ns;
            okB = okB && vB < ns;
        }
        if (okA) atomicAdd(&h[vA], 1u);
        if (okB) atomicAdd(&h[vB], 1u);
    }
    if (bad) atomicExch(a.status, (int32_t)SSBH_E_INVAL);
    __syncthreads();
    uint32_t *dst = a.counts + (uint64_t)seg * ns;
    uint16_t *q = a.qcnt + (uint64_t)seg * 3 * ns;
    for (uint32_t j = t; j < ns; j += 256) {
        const uint32_t c0 = hist[j], c1 = hist[ns + j], c2 = hist[2 * ns + j];
        dst[j] = c0 + c1 + c2 + hist[3 * ns + j];
        q[j] = (uint16_t)c0;
        q[ns + j] = (uint16_t)c1;
        q[2 * ns + j] = (uint16_t)c2;
    }
}

// part[c][j] = sum of counts[seg][j] over the segments of chunk c.
__global__ __launch_bounds__(64) void k_scan_part(SampleArgs a) {
    const uint32_t j = blockIdx.x * 64 + threadIdx.x;
    const uint32_t c = blockIdx.y;
    if (j >= a.ns) return;
    const uint32_t s0 = c * kSegChunk, s1 = min(s0 + kSegChunk, a.nseg);
    uint32_t sum = 0;
    // Unrolled so that a thread's loads are in flight together.
#pragma unroll 16
    for (uint32_t s = s0; s < s1; ++s) sum += a.counts[(uint64_t)s * a.ns + j];
    a.part[(uint64_t)c * a.ns + j] = sum;
}

// Exclusive scan of part over chunks; n_j.
__global__ __launch_bounds__(64) void k_scan_mid(SampleArgs a) {
    const uint32_t j = blockIdx.x * 64 + threadIdx.x;
    if (j >= a.ns) return;
    uint64_t run = 0;
    // 16 loads before their stores, so that they are in flight together
    // (the stores could otherwise alias later loads).
    for (uint32_t c0 = 0; c0 < a.nchunk; c0 += 16) {
        uint32_t t[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            t[k] = c0 + k < a.nchunk ? a.part[(uint64_t)(c0 + k) * a.ns + j] : 0u;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (c0 + k < a.nchunk) {
                a.part[(uint64_t)(c0 + k) * a.ns + j] = (uint32_t)run;
                run += t[k];
            }
    }
    a.len[j] = run;
}

// offs[seg][j]: where segment seg's run of sub-block j starts in sub-block j.
__global__ __launch_bounds__(64) void k_scan_offs(SampleArgs a) {
    const uint32_t j = blockIdx.x * 64 + threadIdx.x;
    const uint32_t c = blockIdx.y;
    if (j >= a.ns) return;
    const uint32_t s0 = c * kSegChunk, s1 = min(s0 + kSegChunk, a.nseg);
    uint32_t run = a.part[(uint64_t)c * a.ns + j];
    // 16 loads before their stores, as in k_scan_mid.
    for (uint32_t b0 = s0; b0 < s1; b0 += 16) {
        uint32_t cnt[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            cnt[k] = b0 + k < s1 ? a.counts[(uint64_t)(b0 + k) * a.ns + j] : 0u;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (b0 + k < s1) {
                a.offs[(uint64_t)(b0 + k) * a.ns + j] = run;
                run += cnt[k];
            }
    }
}

// Word offsets W_j, the capacity check and the abort rule (one block).
__global__ __launch_bounds__(1024) void k_scan_words(SampleArgs a) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry_s;
    __shared__ uint64_t maxlen_s;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    if (threadIdx.x == 0) { carry_s = 0; maxlen_s = 0; }
    __syncthreads();
    for (uint32_t base = 0; base < a.ns; base += blockDim.x) {
        const uint32_t j = base + threadIdx.x;
        const uint64_t nj = j < a.ns ? a.len[j] : 0ull;
        const uint64_t v = (nj + 63) / 64;
        uint64_t incl = v;
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t t = __shfl_up(incl, d, 64);
            if (lane >= d) incl += t;
        }
        if (lane == 63) wsum[w] = incl;
        if (nj) atomicMax((unsigned long long *)&maxlen_s,
                          (unsigned long long)nj);
        __syncthreads();
        uint64_t before = 0;
        for (int k = 0; k < w; ++k) before += wsum[k];
        const uint64_t carry = carry_s;
        if (j < a.ns) a.woff[j] = carry + before + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t tot = 0;
            for (int k = 0; k < nw; ++k) tot += wsum[k];
            carry_s = carry + tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (*a.status == 0) {
            if (carry_s > a.sub_cap) *a.status = SSBH_E_INVAL;
            else if (a.l_ub && maxlen_s > a.l_ub)
                *a.status = SSBH_E_ABORT_OVERSIZE;
        }
    }
}

// 64 bits of the LDS segment image starting at bit p.
__device__ __forceinline__ uint64_t stage_bits64(const uint32_t *stage,
                                                 uint32_t p) {
    const uint32_t w = p >> 5, s = p & 31;
    const uint64_t lo = (uint64_t)stage[w] | ((uint64_t)stage[w + 1] << 32);
    if (s == 0) return lo;
    return (lo >> s) | ((uint64_t)stage[w + 2] << (64 - s));
}

// Input words for a run of 64 consecutive 64-bit steps: lane l holds word
// w0 + l (0 past the end); step k of the run reads it with two readlanes.
__device__ __forceinline__ uint64_t load_word_group(const uint64_t *in,
                                                    uint64_t w0, uint64_t nw,
                                                    int lane) {
    const uint64_t w = w0 + (uint64_t)lane;
    return w < nw ? in[w] : 0ull;
}

__device__ __forceinline__ uint64_t word_of_step(uint64_t group, uint32_t k) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)group, (int)k);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(group >> 32), (int)k);
    return ((uint64_t)hi << 32) | lo;
}

// Copy every run of the segment image to its sub-block.  After the scatter
// loop cursor[j] is the end of run j, so run j starts at cursor[j-1].  Whole
// 64-bit destination words are stored; the partial end words are ORed (they
// are shared with the neighbouring segments' runs of the same sub-block).
__device__ __forceinline__ void flush_runs(const SampleArgs &a, uint32_t seg,
                                           const uint32_t *cursor,
                                           const uint32_t *stage, int lane) {
    const uint32_t *off = a.offs + (uint64_t)seg * a.ns;
    for (uint32_t j = lane; j < a.ns; j += 64) {
        const uint32_t end = cursor[j];
        const uint32_t start = j ? cursor[j - 1] : 0u;
        const uint32_t c = end - start;
        if (!c) continue;
        const uint64_t dst = 64ull * a.woff[j] + off[j];
        const uint64_t d0 = dst >> 6, d1 = (dst + c - 1) >> 6;
        for (uint64_t d = d0; d <= d1; ++d) {
            const uint64_t lo = max(dst, d * 64), hi = min(dst + c, d * 64 + 64);
            const uint32_t nb = (uint32_t)(hi - lo);
            uint64_t bits = stage_bits64(stage, start + (uint32_t)(lo - dst));
            if (nb < 64) bits &= (1ull << nb) - 1ull;
            bits <<= (lo - d * 64);
            if (nb == 64) a.sub[d] = bits;
            else if (bits) atomicOr((unsigned long long *)&a.sub[d],
                                    (unsigned long long)bits);
        }
    }
}

template <bool EXPLICIT>
__global__ __launch_bounds__(64) void k_scatter(SampleArgs a) {
    extern __shared__ uint32_t lds[];
    if (*a.status) return;
    uint32_t *cursor = lds;
    uint32_t *stage = lds + a.ns;
    const uint32_t seg = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t nsw = (uint32_t)(a.seg_bits / 32) + 4;
    const uint32_t *cnt = a.counts + (uint64_t)seg * a.ns;

    // Local exclusive prefix of this segment's counts: where each
    // sub-block's run starts in the segment image.
    const uint32_t per = (a.ns + 63) / 64;
    const uint32_t j0 = min(lane * per, a.ns), j1 = min(j0 + per, a.ns);
    uint32_t s = 0;
    for (uint32_t j = j0; j < j1; ++j) s += cnt[j];
    uint32_t incl = s;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    uint32_t run = incl - s;
    for (uint32_t j = j0; j < j1; ++j) { cursor[j] = run; run += cnt[j]; }
    for (uint32_t k = lane; k < nsw; k += 64) stage[k] = 0u;
    __builtin_amdgcn_wave_barrier();

    const uint64_t i0 = (uint64_t)seg * a.seg_bits;
    const uint64_t i1 = min(i0 + a.seg_bits, a.n);
    const uint64_t nw_in = (a.n + 63) / 64;
    uint64_t grp = load_word_group(a.in, i0 >> 6, nw_in, lane);
    uint64_t grp_next = load_word_group(a.in, (i0 >> 6) + 64, nw_in, lane);
    for (uint64_t base = i0; base < i1; base += 64) {
        const uint64_t i = base + lane;
        const bool valid = i < i1 && kept(a, i);
        const uint32_t k = (uint32_t)((base - i0) >> 6) & 63u;
        if (k == 0 && base != i0) {
            grp = grp_next;
            grp_next = load_word_group(a.in, (base >> 6) + 64, nw_in, lane);
        }
        const uint32_t v = valid ? sample_v<EXPLICIT>(a, i) : 0u;
        const uint64_t word = word_of_step(grp, k);
        const uint32_t bit = valid ? (uint32_t)((word >> lane) & 1ull) : 0u;
        // Lanes holding the same V_i: intersect the ballots of every bit.
        uint64_t m = ballot64(valid);
        for (uint32_t b = 0; b < a.vbits; ++b) {
            const bool t = (v >> b) & 1u;
            const uint64_t bal = ballot64(t);
            m &= t ? bal : ~bal;
        }
        if (valid) {
            const uint32_t basepos = cursor[v];
            const uint32_t pos = basepos + rank_below(m);
            if (63 - __clzll((long long)m) == lane)
                cursor[v] = basepos + (uint32_t)__popcll(m);
            if (bit) atomicOr(&stage[pos >> 5], 1u << (pos & 31));
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();

    flush_runs(a, seg, cursor, stage, lane);
}

// The same scatter with an LDS match table instead of the ballot rounds:
// every lane ORs its lane bit into mask[V_i]; reading mask[V_i] back gives
// the lanes of this step that share V_i (LDS instructions of one wavefront
// execute in order, so the read sees every OR of the instruction before it).
// The highest lane of each group advances the cursor and clears the entry.
template <bool EXPLICIT>
__global__ __launch_bounds__(64) void k_scatter_tab(SampleArgs a) {
    extern __shared__ __align__(8) uint32_t lds[];
    if (*a.status) return;
    uint64_t *mask = reinterpret_cast<uint64_t *>(lds);
    uint32_t *cursor = lds + 2 * a.ns;
    uint32_t *stage = cursor + a.ns;
    const uint32_t seg = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t nsw = (uint32_t)(a.seg_bits / 32) + 4;
    const uint32_t *cnt = a.counts + (uint64_t)seg * a.ns;

    const uint32_t per = (a.ns + 63) / 64;
    const uint32_t j0 = min(lane * per, a.ns), j1 = min(j0 + per, a.ns);
    uint32_t s = 0;
    for (uint32_t j = j0; j < j1; ++j) s += cnt[j];
    uint32_t incl = s;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    uint32_t run = incl - s;
    for (uint32_t j = j0; j < j1; ++j) {
        cursor[j] = run;
        run += cnt[j];
        mask[j] = 0ull;
    }
    for (uint32_t k = lane; k < nsw; k += 64) stage[k] = 0u;
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();

    const uint64_t i0 = (uint64_t)seg * a.seg_bits;
    const uint64_t i1 = min(i0 + a.seg_bits, a.n);
    const uint64_t me = 1ull << lane;
    const uint64_t nw_in = (a.n + 63) / 64;
    uint64_t grp = load_word_group(a.in, i0 >> 6, nw_in, lane);
    uint64_t grp_next = load_word_group(a.in, (i0 >> 6) + 64, nw_in, lane);
    uint32_t v_next = (i0 + lane < i1) ? sample_v<EXPLICIT>(a, i0 + lane) : 0u;
    for (uint64_t base = i0; base < i1; base += 64) {
        const uint64_t i = base + lane;
        const bool valid = i < i1 && kept(a, i);
        const uint32_t v = v_next;
        const uint32_t k = (uint32_t)((base - i0) >> 6) & 63u;
        if (k == 0 && base != i0) {
            grp = grp_next;
            grp_next = load_word_group(a.in, (base >> 6) + 64, nw_in, lane);
        }
        const uint64_t word = word_of_step(grp, k);
        if (valid) atomicOr((unsigned long long *)&mask[v], (unsigned long long)me);
        // Next step's draw overlaps the LDS round trip.
        const uint64_t in = i + 64;
        v_next = (in < i1) ? sample_v<EXPLICIT>(a, in) : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            const uint64_t m = mask[v];
            const uint32_t basepos = cursor[v];
            const uint32_t pos = basepos + rank_below(m);
            if (63 - __clzll((long long)m) == lane) {
                cursor[v] = basepos + (uint32_t)__popcll(m);
                mask[v] = 0ull;
            }
            if ((word >> lane) & 1ull) atomicOr(&stage[pos >> 5], 1u << (pos & 31));
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    flush_runs(a, seg, cursor, stage, lane);
}

// Copy every run of the segment image to its sub-block (as flush_runs, with
// `nt` threads): ends[j] is the end of run j, run j starts at ends[j-1].
template <typename C>
__device__ __forceinline__ void flush_runs_t(const SampleArgs &a, uint32_t seg,
                                             const C *ends,
                                             const uint32_t *stage, int t,
                                             int nt) {
    const uint32_t *off = a.offs + (uint64_t)seg * a.ns;
    for (uint32_t j = t; j < a.ns; j += nt) {
        const uint32_t end = ends[j];
        const uint32_t start = j ? ends[j - 1] : 0u;
        const uint32_t c = end - start;
        if (!c) continue;
        const uint64_t dst = 64ull * a.woff[j] + off[j];
        const uint64_t d0 = dst >> 6, d1 = (dst + c - 1) >> 6;
        for (uint64_t d = d0; d <= d1; ++d) {
            const uint64_t lo = max(dst, d * 64), hi = min(dst + c, d * 64 + 64);
            const uint32_t nb = (uint32_t)(hi - lo);
            uint64_t bits = stage_bits64(stage, start + (uint32_t)(lo - dst));
            if (nb < 64) bits &= (1ull << nb) - 1ull;
            bits <<= (lo - d * 64);
            if (nb == 64) a.sub[d] = bits;
            else if (bits) atomicOr((unsigned long long *)&a.sub[d],
                                    (unsigned long long)bits);
        }
    }
}

// popcount(m & lanes below this one) + acc.
__device__ __forceinline__ uint32_t rank_below(uint64_t m, uint32_t acc) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
}

// m & ~(bal ^ e) on both halves, one v_bitop3 each (truth table 0x90):
// keeps the lanes whose bit equals this lane's bit (e = 0 or ~0, bal = the
// ballot of that bit).
__device__ __forceinline__ uint64_t narrow(uint64_t m, uint64_t bal, uint32_t e) {
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)m, (uint32_t)bal, e, 0x90);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(m >> 32),
                                                    (uint32_t)(bal >> 32), e, 0x90);
    return ((uint64_t)hi << 32) | lo;
}

// Scatter with one workgroup of 4 wavefronts per segment (at most 65024
// rounds, so positions fit 16-bit cursors); wavefront w takes the w-th
// quarter of the segment.
//   1. the segment totals and quarter counts of k_hist_q give each
//      wavefront's first position of every run in the LDS image of the
//      segment (sorted by sub-block, stable: quarter w comes after quarters
//      < w);
//   2. the wavefront walks its quarter in blocks of 128 rounds, lane l
//      holding rounds 2l ("even") and 2l + 1 ("odd") from the low and high
//      halves of one SplitMix64 output.  A 256-slot match table per
//      wavefront (slot V mod 256 holds the mask of even lanes and the mask of
//      odd lanes that ORed their bit there), narrowed by ballots on the HB
//      bits of V above 8, gives for each of the lane's two values the even
//      and the odd lanes holding it; the rank of a round among equal values
//      of the block counts the even and odd rounds before it.  Each value's
//      cursor is read once per block and advanced by the lane holding its
//      last round; the bits are ORed into the image;
//   3. all runs are copied out as in flush_runs.
// Round indices fit 32 bits (n <= 2^32 - 2^20, so index + segment does too).
// LDS: 4 match tables (16 KiB) and a zero slot, 4 cursor tables (4 n_sub
// uint16), the image (n_sub = 2048: 40,944 bytes with the scan words, so
// four workgroups share a CU's 160 KiB).
template <bool EXPLICIT, int HB, bool POW2>
__global__ __launch_bounds__(256) void k_scatter_wg(SampleArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t wsum[4];
    if (*a.status) return;
    const uint32_t ns = a.ns;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint64_t *tab = reinterpret_cast<uint64_t *>(lds);              // [4][256][2]
    const uint64_t *zero2 = tab + 4 * 256 * 2;        // one zero slot, never ORed
    uint16_t *cur = reinterpret_cast<uint16_t *>(tab + 4 * 256 * 2 + 2);  // [4][ns]
    uint32_t *stage = reinterpret_cast<uint32_t *>(cur + 4 * ns);
    const uint32_t seg = blockIdx.x;
    const uint32_t nsw = (uint32_t)(a.seg_bits / 32) + 4;
    for (uint32_t k = t; k < 4 * 256 * 2 + 2; k += 256) tab[k] = 0ull;
    for (uint32_t k = t; k < nsw; k += 256) stage[k] = 0u;

    const uint32_t n32 = (uint32_t)a.n;
    const uint32_t sb = (uint32_t)a.seg_bits;
    const uint32_t i0 = seg * sb;
    const uint32_t i1 = min(i0 + sb, n32);
    const uint32_t qlen = sb / 4;                       // multiple of 128
    const uint32_t qa = i0 + (uint32_t)w * qlen;
    const uint32_t qb = min(qa + qlen, i1);

    // 1. Run starts: exclusive scan over sub-blocks of the segment totals
    //    (from the histogram), then each quarter's offset inside its run from
    //    the counts of the quarters before it.
    {
        const uint32_t *cnt = a.counts + (uint64_t)seg * ns;
        const uint16_t *q = a.qcnt + (uint64_t)seg * 3 * ns;
        const uint32_t per = (ns + 255) / 256;
        const uint32_t v0 = min((uint32_t)t * per, ns), v1 = min(v0 + per, ns);
        uint32_t sum = 0;
        for (uint32_t v = v0; v < v1; ++v) sum += cnt[v];
        uint32_t incl = sum;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t x = __shfl_up(incl, d, 64);
            if (lane >= d) incl += x;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (int k = 0; k < w; ++k) run += wsum[k];
        for (uint32_t v = v0; v < v1; ++v) {
            const uint32_t c0 = q[v], c1 = q[ns + v], c2 = q[2 * ns + v];
            cur[v] = (uint16_t)run;
            cur[ns + v] = (uint16_t)(run + c0);
            cur[2 * ns + v] = (uint16_t)(run + c0 + c1);
            cur[3 * ns + v] = (uint16_t)(run + c0 + c1 + c2);
            run += cnt[v];
        }
    }
    __syncthreads();

    // 2. Stable placement, 128 rounds per step.
    uint64_t *mt = tab + (uint32_t)w * 512;             // [slot][even, odd]
    uint16_t *mc = cur + (uint32_t)w * ns;
    const uint64_t me = 1ull << lane;
    const uint32_t nw_in = (n32 + 63) / 64;
    const uint32_t lane2 = 2u * (uint32_t)lane;
    const uint32_t sh = lane2 & 63u;
    // Input and flag words of the next block are loaded one block ahead.
    const uint32_t wl = (uint32_t)(lane >> 5);
    uint64_t wd_next = 0ull, kw_next = ~0ull;
    if (qa < qb) {
        const uint32_t wi = min((qa >> 6) + wl, nw_in - 1);
        wd_next = a.in[wi];
        if (a.keep) kw_next = a.keep[wi];
    }
    // SplitMix64 counter of output (base / 2 + lane), 64 outputs per block.
    uint64_t z = a.key + ((uint64_t)((qa >> 1) + (uint32_t)lane) + 1ull) * kSplitMixGamma;
    for (uint32_t base = qa; base < qb; base += 128, z += 64ull * kSplitMixGamma) {
        const uint64_t wd = wd_next, kw = kw_next;
        if (base + 128 < qb) {
            const uint32_t wi = min(((base + 128) >> 6) + wl, nw_in - 1);
            wd_next = a.in[wi];
            if (a.keep) kw_next = a.keep[wi];
        }
        const uint32_t iE = base + lane2, iO = iE + 1;
        uint32_t vE, vO;
        if constexpr (EXPLICIT) {
            vE = iE < qb ? a.assign[iE] : 0u;
            vO = iO < qb ? a.assign[iO] : 0u;
        } else {
            const uint64_t r = splitmix64_mix(z);
            vE = v_of<POW2>(a, (uint32_t)r);
            vO = v_of<POW2>(a, (uint32_t)(r >> 32));
        }
        bool okE = iE < qb, okO = iO < qb;
        if constexpr (EXPLICIT) {
            okE = okE && vE < ns;
            okO = okO && vO < ns;
        }
        const uint32_t kb = (uint32_t)(kw >> sh);      // all ones without flags
        okE = okE && (kb & 1u);
        okO = okO && (kb & 2u);
        const uint32_t sE = vE & 255u, sO = vO & 255u;
        if (okE) atomicOr((unsigned long long *)&mt[2 * sE], (unsigned long long)me);
        if (okO) atomicOr((unsigned long long *)&mt[2 * sO + 1], (unsigned long long)me);
        __builtin_amdgcn_wave_barrier();
        // A round that is not placed reads the zero slot: all its masks are 0.
        const ulonglong2 pE = *reinterpret_cast<const ulonglong2 *>(okE ? &mt[2 * sE] : zero2);
        const ulonglong2 pO = *reinterpret_cast<const ulonglong2 *>(okO ? &mt[2 * sO] : zero2);
        uint64_t mEE = pE.x, mEO = pE.y, mOE = pO.x, mOO = pO.y;
#pragma unroll
        for (int b = 0; b < HB; ++b) {
            const uint32_t eE = (uint32_t)__builtin_amdgcn_sbfe((int)vE, 8 + b, 1);
            const uint32_t eO = (uint32_t)__builtin_amdgcn_sbfe((int)vO, 8 + b, 1);
            const uint64_t balE = ballot64(eE != 0u), balO = ballot64(eO != 0u);
            mEE = narrow(mEE, balE, eE);
            mEO = narrow(mEO, balO, eE);
            mOE = narrow(mOE, balE, eO);
            mOO = narrow(mOO, balO, eO);
        }
        const uint32_t cE = mc[okE ? vE : 0u];
        const uint32_t cO = mc[okO ? vO : 0u];
        __builtin_amdgcn_wave_barrier();
        // Even round: rank among equal values = even and odd lanes below.
        const uint32_t rEE = rank_below(mEE, 0u), rEO = rank_below(mEO, 0u);
        const uint32_t tEE = (uint32_t)__popcll(mEE), tEO = (uint32_t)__popcll(mEO);
        // Odd round: even lanes up to and including this one, odd lanes below.
        const uint32_t rOE = rank_below(mOE, (okE && vE == vO) ? 1u : 0u);
        const uint32_t rOO = rank_below(mOO, 0u);
        const uint32_t tOE = (uint32_t)__popcll(mOE), tOO = (uint32_t)__popcll(mOO);
        if (okE) {
            const uint32_t pos = cE + rEE + rEO;
            if (rEE + 1u == tEE) {                      // last even lane of V
                mt[2 * sE] = 0ull;
                if (rEO == tEO) mc[vE] = (uint16_t)(cE + tEE + tEO);
            }
            if ((wd >> sh) & 1ull) atomicOr(&stage[pos >> 5], 1u << (pos & 31));
        }
        if (okO) {
            const uint32_t pos = cO + rOE + rOO;
            if (rOO + 1u == tOO) {                      // last odd lane of V
                mt[2 * sO + 1] = 0ull;
                if (rOE == tOE) mc[vO] = (uint16_t)(cO + tOE + tOO);
            }
            if ((wd >> sh) & 2ull) atomicOr(&stage[pos >> 5], 1u << (pos & 31));
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __syncthreads();

    // 3. Runs out; the last quarter's cursors are the run ends.
    flush_runs_t(a, seg, cur + 3 * ns, stage, t, 256);
}

__global__ void k_perm_meta(uint32_t ns, uint64_t L, uint64_t wl,
                            uint64_t l_ub, uint64_t *len, uint64_t *woff,
                            int32_t *status) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < ns) { len[j] = L; woff[j] = (uint64_t)j * wl; }
    if (j == 0 && l_ub && L > l_ub) atomicCAS(status, 0, SSBH_E_ABORT_OVERSIZE);
}

__global__ void k_seed(uint64_t key, uint64_t *seed, uint64_t bits) {
    const uint64_t nw = (bits + 63) / 64;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nw;
         t += stride) {
        uint64_t v = splitmix64_at(key, t);
        if (t == nw - 1 && (bits & 63)) v &= (1ull << (bits & 63)) - 1ull;
        seed[t] = v;
    }
}

uint32_t ceil_log2(uint32_t x) {
    uint32_t b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

}  // namespace

// Segment length: about 32 rounds per sub-block, 2^14 .. 2^18 - 512 rounds
// (a quarter stays below 2^16 rounds), a multiple of 512; at most 65024 for
// n_sub <= 4096, so that the workgroup scatter (16-bit positions, LDS for up
// to 4096 sub-blocks) takes it: above 2032 sub-blocks that is fewer than 32
// rounds per sub-block, which costs shorter runs but runs 3-5 times faster
// than the one-wavefront scatters.
static uint64_t segment_bits(uint32_t ns) {
    uint64_t seg = 32ull * ns;
    seg = std::max<uint64_t>(seg, 1ull << 14);
    seg = std::min<uint64_t>(seg, (1ull << 18) - 512);
    seg = (seg + 511) / 512 * 512;
    if (seg > kWgMaxSeg && ns <= 4096) seg = kWgMaxSeg;
    return seg;
}

template <bool EX, bool P2>
void launch_scatter_wg_t(int hb, const SampleArgs &a, size_t lds,
                         hipStream_t stream) {
    const dim3 g(a.nseg), b(256);
    switch (hb) {
    case 0: hipLaunchKernelGGL((k_scatter_wg<EX, 0, P2>), g, b, lds, stream, a); break;
    case 1: hipLaunchKernelGGL((k_scatter_wg<EX, 1, P2>), g, b, lds, stream, a); break;
    case 2: hipLaunchKernelGGL((k_scatter_wg<EX, 2, P2>), g, b, lds, stream, a); break;
    case 3: hipLaunchKernelGGL((k_scatter_wg<EX, 3, P2>), g, b, lds, stream, a); break;
    default: hipLaunchKernelGGL((k_scatter_wg<EX, 4, P2>), g, b, lds, stream, a); break;
    }
}

// The workgroup scatter for ceil(log2 n_sub) - 8 = hb high bits (n_sub <=
// 4096 on this path, so hb <= 4); V by a shift when n_sub is a power of two.
void launch_scatter_wg(bool ex, int hb, const SampleArgs &a, size_t lds,
                       hipStream_t stream) {
    if (ex) launch_scatter_wg_t<true, false>(hb, a, lds, stream);
    else if (a.vshift) launch_scatter_wg_t<false, true>(hb, a, lds, stream);
    else launch_scatter_wg_t<false, false>(hb, a, lds, stream);
}

ScratchSizes sample_scratch(uint64_t n, uint32_t ns, uint32_t mode) {
    ScratchSizes z;
    if (mode == SSBH_SAMPLE_PERMUTE || ns == 0) return z;
    const uint64_t seg = segment_bits(ns);
    const uint64_t nseg = (n + seg - 1) / seg;
    const uint64_t nchunk = (nseg + kSegChunk - 1) / kSegChunk;
    // counts [nseg][ns] uint32, then the quarter counts [nseg][3][ns] uint16.
    z.offs = (size_t)std::max<uint64_t>(nseg, 1) * ns * 4;
    z.counts = z.offs + (size_t)std::max<uint64_t>(nseg, 1) * ns * 6;
    z.part = (size_t)std::max<uint64_t>(nchunk, 1) * ns * 4;
    return z;
}

ssbh_status launch_seed(uint64_t key, uint64_t *d_seed, uint64_t seed_bits,
                        hipStream_t stream) {
    const uint64_t nw = (seed_bits + 63) / 64;
    if (!nw) return SSBH_OK;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((nw + 255) / 256, 4096);
    hipLaunchKernelGGL(k_seed, dim3(blocks), dim3(256), 0, stream, key, d_seed,
                       seed_bits);
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

ssbh_status launch_sample(ssbh_ctx *ctx, Workspace &ws, const uint64_t *d_in,
                          const uint64_t *d_keep, uint64_t n, uint32_t ns,
                          uint32_t mode, uint64_t key,
                          const uint32_t *d_assign, uint64_t l_ub,
                          uint64_t *d_sub, uint64_t sub_cap, uint64_t *d_len,
                          uint64_t *d_woff, int32_t *d_status,
                          hipStream_t stream) {
    if (ns == 0) SSBH_INVAL("n_sub must be >= 1");
    if (!d_sub || !d_len || !d_woff || !d_status)
        SSBH_INVAL("d_sub, d_len, d_word_off and d_status must be non-null");
    if (n && !d_in) SSBH_INVAL("d_in is null");
    if (n > SSBH_MAX_SAMPLE_BITS) {
        set_error("n_bits must be at most %llu", (unsigned long long)SSBH_MAX_SAMPLE_BITS);
        return SSBH_E_UNSUPPORTED;
    }
    (void)hipGetLastError();   // clear errors left by earlier calls
    hipLaunchKernelGGL(k_init_status, dim3(1), dim3(1), 0, stream, d_status);
    SSBH_CHECK_HIP(hipGetLastError());

    if (mode == SSBH_SAMPLE_PERMUTE) {
        if (d_keep) SSBH_INVAL("sifting flags need i.i.d. or explicit V");
        if (n % ns) SSBH_INVAL("n_sub (%u) must divide n_bits (%llu)", ns,
                               (unsigned long long)n);
        const uint64_t L = n / ns, wl = (L + 63) / 64;
        if (sub_cap < (uint64_t)ns * wl)
            SSBH_INVAL("sub_capacity_words %llu < %llu",
                       (unsigned long long)sub_cap,
                       (unsigned long long)((uint64_t)ns * wl));
        // The keyed path may keep the gather's bucketing, unless this call
        // aborts (the bucket pass then does nothing).
        const bool keyed = !d_assign && n && !(l_ub && L > l_ub);
        if (!d_assign && n) {
            // The keyed permutation of sample_key, built in the workspace
            // unless it already holds that of (sample_key, n): it depends on
            // nothing else.
            ssbh_status st = ws.perm_pi.reserve((size_t)n * sizeof(uint32_t));
            if (st != SSBH_OK) return st;
            if (ws.perm_ptr != ws.perm_pi.ptr || ws.perm_key != key ||
                ws.perm_n != n) {
                ws.perm_ptr = nullptr;
                st = launch_permutation(ctx, ws.perm_tmp, key, n,
                                        ws.perm_pi.as<uint32_t>(), stream);
                if (st != SSBH_OK) return st;
                ws.perm_ptr = ws.perm_pi.ptr;
                ws.perm_key = key;
                ws.perm_n = n;
            }
            d_assign = ws.perm_pi.as<uint32_t>();
        }
        hipLaunchKernelGGL(k_perm_meta, dim3((ns + 255) / 256), dim3(256), 0,
                           stream, ns, L, wl, l_ub, d_len, d_woff, d_status);
        SSBH_CHECK_HIP(hipGetLastError());
        return launch_perm_gather(ctx, ws, d_in, n, d_assign, ns, L, wl, d_sub,
                                  d_status, stream, keyed, key);
    }
    if (mode != SSBH_SAMPLE_IID && mode != SSBH_SAMPLE_EXPLICIT)
        SSBH_INVAL("unknown sampling mode %u", mode);
    if (mode == SSBH_SAMPLE_EXPLICIT && n && !d_assign)
        SSBH_INVAL("explicit mode needs d_assign");
    if (ns > SSBH_MAX_SUB_LDS) {
        set_error("n_sub %u exceeds %u for this sampling mode", ns,
                  SSBH_MAX_SUB_LDS);
        return SSBH_E_UNSUPPORTED;
    }
    const uint64_t need = (n + 63) / 64 + ns;
    if (sub_cap < need)
        SSBH_INVAL("sub_capacity_words %llu < ceil(n_bits/64)+n_sub = %llu",
                   (unsigned long long)sub_cap, (unsigned long long)need);

    SampleArgs a{};
    a.in = d_in; a.n = n; a.ns = ns; a.vbits = ceil_log2(ns); a.key = key;
    a.vshift = (ns >= 2 && (ns & (ns - 1)) == 0) ? 32 - a.vbits : 0;
    a.assign = d_assign; a.keep = d_keep; a.sub = d_sub; a.sub_cap = sub_cap; a.len = d_len;
    a.woff = d_woff; a.l_ub = l_ub; a.status = d_status;
    const uint64_t seg = segment_bits(ns);
    a.seg_bits = seg;
    a.nseg = (uint32_t)((n + seg - 1) / seg);
    a.nchunk = (a.nseg + kSegChunk - 1) / kSegChunk;
    const ScratchSizes sz = sample_scratch(n, ns, mode);
    ssbh_status st;
    if ((st = ws.counts.reserve(sz.counts)) != SSBH_OK) return st;
    if ((st = ws.offs.reserve(sz.offs)) != SSBH_OK) return st;
    if ((st = ws.part.reserve(sz.part)) != SSBH_OK) return st;
    a.counts = ws.counts.as<uint32_t>();
    a.qcnt = reinterpret_cast<uint16_t *>(a.counts + (size_t)std::max<uint32_t>(a.nseg, 1) * ns);
    a.offs = ws.offs.as<uint32_t>();
    a.part = ws.part.as<uint32_t>();

    const bool ex = mode == SSBH_SAMPLE_EXPLICIT;
    // Histogram: wavefronts per block limited by LDS (4 B per sub-block).
    int wpb = (int)std::min<uint64_t>(4, std::max<uint64_t>(1, (32768u) / ns));
    const uint32_t hist_blocks = std::max<uint32_t>(
        1, std::max<uint32_t>((a.nseg + wpb - 1) / wpb,
                         (uint32_t)std::min<uint64_t>((sub_cap + 255) / 256, 2048)));
    const size_t hist_lds = (size_t)wpb * ns * 4;
    const size_t scat_lds = (size_t)ns * 4 + ((size_t)(seg / 32) + 4) * 4;
    const size_t tab_lds = scat_lds + (size_t)ns * 8;
    const bool use_tab = tab_lds <= 48 * 1024;
    const size_t wg_lds = ((size_t)4 * 256 * 2 + 2) * 8 + (size_t)4 * ns * 2 +
                          ((size_t)(seg / 32) + 4) * 4;
    const bool use_wg = ns >= 2 && ns <= 4096 && seg <= kWgMaxSeg &&
                        wg_lds <= 64 * 1024 && ctx->forced_scatter != 1;
    {
        const void *kh = ex ? (const void *)k_hist<true> : (const void *)k_hist<false>;
        const void *ksc = ex ? (const void *)k_scatter<true>
                             : (const void *)k_scatter<false>;
        if ((st = ensure_dynamic_lds(kh, hist_lds)) != SSBH_OK) return st;
        const void *kt = ex ? (const void *)k_scatter_tab<true>
                            : (const void *)k_scatter_tab<false>;
        if (use_wg) {
            // at most 64 KiB: no opt-in needed
        } else if (use_tab) {
            if ((st = ensure_dynamic_lds(kt, tab_lds)) != SSBH_OK) return st;
        } else if ((st = ensure_dynamic_lds(ksc, scat_lds)) != SSBH_OK) {
            return st;
        }
    }
    if (use_wg) {
        // One workgroup per segment (extra workgroups only clear the buffer).
        const uint32_t blocks = std::max<uint32_t>(
            std::max<uint32_t>(a.nseg, 1),
            (uint32_t)std::min<uint64_t>((sub_cap + 255) / 256, 2048));
        const size_t q_lds = (size_t)4 * ns * 4;
        TimedLaunch timed(ws.timer, "k_hist", stream);
        if (ex)
            hipLaunchKernelGGL((k_hist_q<true, false>), dim3(blocks), dim3(256),
                               q_lds, stream, a);
        else if (a.vshift)
            hipLaunchKernelGGL((k_hist_q<false, true>), dim3(blocks), dim3(256),
                               q_lds, stream, a);
        else
            hipLaunchKernelGGL((k_hist_q<false, false>), dim3(blocks), dim3(256),
                               q_lds, stream, a);
    } else {
        TimedLaunch timed(ws.timer, "k_hist", stream);
        if (ex)
            hipLaunchKernelGGL(k_hist<true>, dim3(hist_blocks), dim3(64 * wpb),
                               hist_lds, stream, a);
        else
            hipLaunchKernelGGL(k_hist<false>, dim3(hist_blocks), dim3(64 * wpb),
                               hist_lds, stream, a);
    }
    const uint32_t jb = (ns + 63) / 64;
    if (a.nseg) {
        hipLaunchKernelGGL(k_scan_part, dim3(jb, a.nchunk), dim3(64), 0,
                           stream, a);
    }
    hipLaunchKernelGGL(k_scan_mid, dim3(jb), dim3(64), 0, stream, a);
    if (a.nseg) {
        hipLaunchKernelGGL(k_scan_offs, dim3(jb, a.nchunk), dim3(64), 0,
                           stream, a);
    }
    hipLaunchKernelGGL(k_scan_words, dim3(1), dim3(1024), 0, stream, a);
    if (a.nseg) {
        TimedLaunch timed(ws.timer, "k_scatter", stream);
        if (use_wg)
            launch_scatter_wg(ex, a.vbits > 8 ? a.vbits - 8 : 0, a, wg_lds, stream);
        else if (use_tab && ex)
            hipLaunchKernelGGL(k_scatter_tab<true>, dim3(a.nseg), dim3(64),
                               tab_lds, stream, a);
        else if (use_tab)
            hipLaunchKernelGGL(k_scatter_tab<false>, dim3(a.nseg), dim3(64),
                               tab_lds, stream, a);
        else if (ex)
            hipLaunchKernelGGL(k_scatter<true>, dim3(a.nseg), dim3(64),
                               scat_lds, stream, a);
        else
            hipLaunchKernelGGL(k_scatter<false>, dim3(a.nseg), dim3(64),
                               scat_lds, stream, a);
    }
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

}  // namespace ssbh
