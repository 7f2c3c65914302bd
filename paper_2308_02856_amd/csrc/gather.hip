// Permutation sampling (Sec. III.B step 1 with a permutation: sub-block j
// takes B[jL, (j+1)L), B[k] = A[pi[k]]): the gather of the n input bits.
//
// A direct gather reads one input word per output bit at a random place: past
// the caches' reach (A is n / 8 bytes) every bit costs a cache-line transfer.
// For large n the gather is done in three streaming passes instead, over
// chunks of 2^18 output positions (in output-word order) and source windows
// of 2^20 input bits (one window fills 128 KiB of LDS):
//   k_pg_bucket  chunk g: reads pi[k], appends the window offset p mod 2^20
//                to cell (g, p >> 20) of a fixed capacity and stores k's
//                cell slot (window * cap + rank, rank from an LDS counter);
//   k_pg_window  window b: its input bits in LDS; every cell (g, b) becomes a
//                string of looked-up bits, one ballot per 64 entries;
//   k_pg_merge   chunk g: its cells' bits (one contiguous region) in LDS;
//                B[k] = bit at k's slot, one ballot per output word.
// The cell capacity is twice the expected occupancy plus 64; a permutation
// that overfills a cell (far outside the binomial spread of a random one)
// sets a flag, the window and merge passes then do nothing and the direct
// gather, which runs after them only when the flag is set, writes the output.
// The bucket pass depends on pi alone: for the context's keyed permutation
// its result (and flag) is kept for later calls with the same key and split.
#include <algorithm>

#include "ssbh_internal.hpp"

namespace ssbh {
namespace {

constexpr uint32_t kPgWinBits = 20;                 // source window: 2^20 bits
constexpr uint32_t kPgChunkWords = 4096;            // 2^18 output bits per chunk
constexpr uint64_t kPgMinBits = 1ull << 26;         // smaller inputs gather directly

struct PgArgs {
    const uint64_t *in;
    uint64_t n;
    const uint32_t *perm;
    uint32_t ns;
    uint64_t L, wl;          // sub-block bits, words per sub-block
    uint64_t *sub;
    uint32_t nb;             // windows
    uint32_t ng;             // chunks
    uint32_t cap;            // cell capacity (multiple of 64)
    uint32_t *items;         // [ng][nb][cap] window offsets
    uint32_t *slots;         // [n] cell slot of output bit k
    uint32_t *cnt;           // [nb][ng] cell occupancy (clamped to cap)
    uint64_t *bits;          // [ng][nb][cap / 64] looked-up bits
    uint32_t *flag;          // 1 = some cell overflowed
    int32_t *status;
};

__global__ void k_pg_init(uint32_t *flag) { *flag = 0u; }

// A wavefront-uniform 64-bit value, marked as such so that addresses built
// from it stay in scalar registers (one vector offset serves every load).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Output word w of the sub-block buffer holds bits k = j L + 64 ww + lane
// for 64 ww + lane < L (w = j wl + ww).  A wavefront walks words at a fixed
// stride, so (j, ww) advance without a division; all of it is the same for
// the whole wavefront and runs on the scalar unit.
template <bool ALIGNED>
struct WordPos {
    uint64_t kw0, cw0;       // k of the word's bit 0, and 64 ww
    __device__ __forceinline__ void start(uint64_t w, uint64_t wl, uint64_t L) {
        if constexpr (ALIGNED) {
            kw0 = w * 64;
            cw0 = 0;
        } else {
            const uint64_t j = w / wl, ww = w - j * wl;
            cw0 = ww * 64;
            kw0 = j * L + cw0;
        }
    }
    // Advance by step words (a sub-block is 64 wl buffer bits, L of them
    // real; with ALIGNED, L = 64 wl and buffer bit = k).
    __device__ __forceinline__ void advance(uint64_t step, uint64_t wl, uint64_t L) {
        kw0 += 64 * step;
        if constexpr (!ALIGNED) {
            cw0 += 64 * step;
            while (cw0 >= 64 * wl) { cw0 -= 64 * wl; kw0 -= 64 * wl - L; }
        }
    }
    __device__ __forceinline__ uint64_t k0() const { return kw0; }
    // Real bits of the word: lanes below L - 64 ww.
    __device__ __forceinline__ bool real(int lane, uint64_t L) const {
        if constexpr (ALIGNED) return true;
        else return cw0 + (uint64_t)lane < L;
    }
};

// Bucket pass: one workgroup per chunk, in sub-chunks of kPgSubWords output
// words (2^14 bits).  Per sub-chunk: each thread's 16 entries of pi, counts
// per window (LDS atomics), a scan of the counts, the entries placed in LDS
// sorted by window (atomics on a copy of the run starts; k's slot is set
// then), and one coalesced copy of the stage into the cells.  The stage
// holds pi itself: window = p >> 20, offset = p mod 2^20, and an entry's
// rank in its cell is the cell's fill before the sub-chunk plus its place
// in the window's run.  cc[b] is cell b's fill so far.
constexpr uint32_t kPgSubWords = 256;
constexpr uint32_t kPgPer = kPgSubWords / 16;   // words per wavefront

template <bool ALIGNED>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_pg_bucket(PgArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ int live_s;
    __shared__ uint32_t part[16];
    const uint32_t nb4 = (a.nb + 3u) & ~3u;
    uint32_t *cl = lds;                       // [nb] sub-chunk counts
    uint32_t *lc = cl + nb4;                  // [nb] placement cursors
    uint32_t *db = lc + nb4;                  // [nb] slot = db + stage index
    uint16_t *cc = reinterpret_cast<uint16_t *>(db + nb4);  // cell fill
    uint32_t *stage = reinterpret_cast<uint32_t *>(cc + nb4);  // pi values
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const uint32_t g = blockIdx.x;
    for (uint32_t b = t; b < a.nb; b += 1024) { cl[b] = 0u; cc[b] = 0u; }
    // Other workgroups may set the status meanwhile: one read per workgroup
    // keeps the barriers below uniform.
    if (t == 0) live_s = *a.status == 0;
    __syncthreads();
    const uint64_t total = (uint64_t)a.ns * a.wl;
    const uint64_t w0 = (uint64_t)g * kPgChunkWords;
    const uint64_t w1 = min(w0 + kPgChunkWords, total);
    uint32_t *cell = a.items + (uint64_t)g * a.nb * a.cap;
    bool bad = false, over = false;
    const bool live = live_s != 0;
    WordPos<ALIGNED> pos;
    pos.start(w0 + (uint64_t)wv, a.wl, a.L);
    for (uint64_t s0 = w0; live && s0 < w1; s0 += kPgSubWords) {
        // 1. pi of words s0 + 16 i + wv, one word per wavefront and step;
        //    counts per window.
        // The entries stay in the stage in load order (thread t's entry i
        // at 1024 i + t) until step 3 sorts them in place.
        uint32_t okm = 0;                     // bit i: entry i is a real bit
        const WordPos<ALIGNED> first = pos;   // walked again for the slots
        for (int h = 0; h < (int)kPgPer; h += 8) {   // 8 loads in flight
            uint32_t pv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = h + u;
                const uint64_t w = s0 + 16u * i + (uint64_t)wv;
                const bool ok = w < w1 && pos.real(lane, a.L);
                okm |= ok ? 1u << i : 0u;
                pv[u] = ok ? (a.perm + uniform64(pos.k0()))[lane] : 0xffffffffu;
                pos.advance(16, a.wl, a.L);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                stage[1024u * (h + u) + t] = pv[u];
                if ((okm >> (h + u)) & 1u) {
                    if (pv[u] < a.n) atomicAdd(&cl[pv[u] >> kPgWinBits], 1u);
                    else bad = true;
                }
            }
        }
        __syncthreads();
        // 2. run starts: exclusive scan of cl over the windows.
        uint32_t tot;
        {
            uint32_t x = 0;
            for (uint32_t b = (uint32_t)t * 4u; b < min((uint32_t)t * 4u + 4u, a.nb); ++b)
                x += cl[b];
            uint32_t incl = x;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            if (lane == 63) part[wv] = incl;
            __syncthreads();
            uint32_t run = incl - x;
            for (int v = 0; v < wv; ++v) run += part[v];
            tot = 0;
            for (int v = 0; v < 16; ++v) tot += part[v];
            // A window's run at stage [run, run + cl) becomes cell ranks
            // [cc, cc + cl): slot = b cap + cc + (x - run), below nb cap.  A
            // run that would pass the capacity marks the chunk overflowed
            // (the direct gather then writes the output); its db puts every
            // slot at nb cap or above, so nothing of it is stored.
            for (uint32_t b = (uint32_t)t * 4u; b < min((uint32_t)t * 4u + 4u, a.nb); ++b) {
                const uint32_t c = cl[b], f = cc[b];
                lc[b] = run;
                if (f + c <= a.cap) {
                    db[b] = b * a.cap + f - run;       // mod 2^32; + x >= run
                } else {
                    db[b] = a.nb * a.cap - run;
                    over = true;
                }
                run += c;
            }
        }
        __syncthreads();
        // 3. entries sorted by window in place (all read before any is
        //    moved); the slots of k.
        {
            uint32_t pv[kPgPer];
#pragma unroll
            for (int i = 0; i < (int)kPgPer; ++i) pv[i] = stage[1024u * i + t];
            __syncthreads();
            WordPos<ALIGNED> again = first;
#pragma unroll
            for (int i = 0; i < (int)kPgPer; ++i) {
                const uint64_t k0 = again.k0();
                again.advance(16, a.wl, a.L);
                if (!((okm >> i) & 1u)) continue;
                uint32_t slot = 0;
                if (pv[i] < a.n) {
                    const uint32_t b = pv[i] >> kPgWinBits;
                    const uint32_t x = atomicAdd(&lc[b], 1u);
                    stage[x] = pv[i];
                    const uint32_t d = db[b] + x;
                    slot = d < a.nb * a.cap ? d : 0u;
                }
                (a.slots + uniform64(k0))[lane] = slot;
            }
        }
        __syncthreads();
        // 4. the stage into the cells (a window's run is contiguous in
        //    both); 5. cell fills.
        for (uint32_t x = (uint32_t)t; x < tot; x += 1024) {
            const uint32_t p = stage[x];
            const uint32_t d = db[p >> kPgWinBits] + x;
            if (d < a.nb * a.cap) cell[d] = p & ((1u << kPgWinBits) - 1u);
        }
        __syncthreads();
        for (uint32_t b = t; b < a.nb; b += 1024) {
            cc[b] = (uint16_t)min<uint32_t>(cc[b] + cl[b], 0xffffu);
            cl[b] = 0u;
        }
        __syncthreads();
    }
    if (bad) atomicExch(a.status, (int32_t)SSBH_E_INVAL);
    if (over) atomicOr(a.flag, 1u);
    for (uint32_t b = t; b < a.nb; b += 1024)
        a.cnt[(uint64_t)b * a.ng + g] = min(cc[b], a.cap);
}

// Window pass: one workgroup per window; each wavefront takes cells in turn.
__global__ __launch_bounds__(1024) void k_pg_window(PgArgs a) {
    extern __shared__ uint64_t win[];                 // 2^20 bits
    if (*a.status || *a.flag) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const uint32_t b = blockIdx.x;
    const uint64_t nw_in = (a.n + 63) / 64;
    const uint64_t wbase = (uint64_t)b << (kPgWinBits - 6);
    constexpr uint32_t kWinWords = 1u << (kPgWinBits - 6);
    for (uint32_t i = t; i < kWinWords; i += 1024)
        win[i] = wbase + i < nw_in ? a.in[wbase + i] : 0ull;
    __syncthreads();
    const uint32_t *cw = a.cnt + (uint64_t)b * a.ng;
    // Two cells per wavefront at a time: the first 512 entries of both are
    // loaded before either is looked up.
    for (uint32_t g = wv; g < a.ng; g += 32) {
        const uint32_t gB = g + 16;
        const uint32_t cA = cw[g], cB = gB < a.ng ? cw[gB] : 0u;
        const uint64_t cellA = ((uint64_t)g * a.nb + b) * a.cap;
        const uint64_t cellB = ((uint64_t)gB * a.nb + b) * a.cap;
        uint32_t oA[8], oB[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t q = 64u * u + (uint32_t)lane;
            oA[u] = q < cA ? a.items[cellA + q] : 0xffffffffu;
            oB[u] = q < cB ? a.items[cellB + q] : 0xffffffffu;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t cc_ = h ? cB : cA;
            const uint64_t cell = h ? cellB : cellA;
            uint64_t *out = a.bits + cell / 64;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t o = h ? oB[u] : oA[u];
                if (64u * u >= cc_) break;
                const bool bit = o != 0xffffffffu && ((win[o >> 6] >> (o & 63)) & 1ull);
                const uint64_t word = ballot64(bit);
                if (lane == 0) out[u] = word;
            }
            for (uint32_t q0 = 512; q0 < cc_; q0 += 64) {
                const uint32_t q = q0 + (uint32_t)lane;
                const uint32_t o = q < cc_ ? a.items[cell + q] : 0xffffffffu;
                const bool bit = o != 0xffffffffu && ((win[o >> 6] >> (o & 63)) & 1ull);
                const uint64_t word = ballot64(bit);
                if (lane == 0) out[q0 / 64] = word;
            }
        }
    }
}

// Merge pass: one workgroup per chunk; each wavefront loads the slots of
// eight output words before looking them up.
template <bool ALIGNED>
__global__ __launch_bounds__(1024) void k_pg_merge(PgArgs a) {
    extern __shared__ uint64_t cells[];               // nb * cap bits
    if (*a.status || *a.flag) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const uint32_t g = blockIdx.x;
    const uint32_t nwords = a.nb * (a.cap / 64);
    const uint64_t *src = a.bits + (uint64_t)g * nwords;
    for (uint32_t i = t; i < nwords; i += 1024) cells[i] = src[i];
    __syncthreads();
    const uint64_t total = (uint64_t)a.ns * a.wl;
    const uint64_t w0 = (uint64_t)g * kPgChunkWords;
    const uint64_t w1 = min(w0 + kPgChunkWords, total);
    WordPos<ALIGNED> pos;
    pos.start(w0 + 8u * (uint64_t)wv, a.wl, a.L);
    for (uint64_t wq = w0 + 8u * (uint64_t)wv; wq < w1; wq += 128) {
        uint32_t sv[8];
        bool okv[8];
        WordPos<ALIGNED> pu = pos;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t w = wq + u;
            okv[u] = w < w1 && pu.real(lane, a.L);
            sv[u] = okv[u] ? (a.slots + uniform64(pu.k0()))[lane] : 0u;
            pu.advance(1, a.wl, a.L);
        }
        pos.advance(128, a.wl, a.L);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (wq + u >= w1) break;
            const bool bit = okv[u] && ((cells[sv[u] >> 6] >> (sv[u] & 63)) & 1ull);
            const uint64_t word = ballot64(bit);
            if (lane == 0) a.sub[wq + u] = word;
        }
    }
}

// Direct gather: one wavefront per 64 output bits.  With only_if, it runs
// only when *only_if is nonzero (the streaming passes gave up).
__global__ __launch_bounds__(256) void k_perm_gather(
        const uint64_t *in, uint64_t n, const uint32_t *perm, uint32_t ns,
        uint64_t L, uint64_t wl, uint64_t *sub, const uint32_t *only_if,
        int32_t *status) {
    if (*status) return;
    if (only_if && *only_if == 0u) return;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) +
                          (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nwave = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t total = (uint64_t)ns * wl;
    bool bad = false;
    for (uint64_t w = wave; w < total; w += nwave) {
        const uint32_t j = (uint32_t)w / (uint32_t)wl;   // fewer than 2^26 words
        const uint64_t c0 = (w - (uint64_t)j * wl) * 64;
        const uint64_t k0 = (uint64_t)j * L + c0;
        const uint64_t c = c0 + (uint64_t)lane;
        bool bit = false;
        if (c < L) {
            const uint32_t p = perm[k0 + lane];
            if (p < n) bit = (in[p >> 6] >> (p & 63)) & 1ull;
            else bad = true;
        }
        const uint64_t word = ballot64(bit);
        if (lane == 0) sub[w] = word;
    }
    if (bad) atomicExch(status, (int32_t)SSBH_E_INVAL);
}

struct PgLayout {
    uint32_t nb = 0, ng = 0, cap = 0;
    size_t items_off = 0, slots_off = 0, cnt_off = 0, bits_off = 0,
           flag_off = 0, bytes = 0;
};

PgLayout pg_layout(uint64_t n, uint32_t ns, uint64_t wl) {
    PgLayout p;
    p.nb = (uint32_t)((n + (1ull << kPgWinBits) - 1) >> kPgWinBits);
    const uint64_t total = (uint64_t)ns * wl;
    p.ng = (uint32_t)((total + kPgChunkWords - 1) / kPgChunkWords);
    const uint64_t mean = ((uint64_t)kPgChunkWords * 64 + p.nb - 1) / p.nb;
    p.cap = (uint32_t)((2 * mean + 64 + 63) / 64 * 64);
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t off = 0;
    p.items_off = off; off += r256((size_t)p.ng * p.nb * p.cap * 4);
    p.slots_off = off; off += r256((size_t)n * 4);
    p.cnt_off = off;   off += r256((size_t)p.nb * p.ng * 4);
    p.bits_off = off;  off += r256((size_t)p.ng * p.nb * p.cap / 8);
    p.flag_off = off;  off += 256;
    p.bytes = off;
    return p;
}

}  // namespace

ssbh_status launch_perm_gather(ssbh_ctx *ctx, Workspace &ws,
                               const uint64_t *d_in, uint64_t n,
                               const uint32_t *d_perm, uint32_t ns, uint64_t L,
                               uint64_t wl, uint64_t *d_sub, int32_t *d_status,
                               hipStream_t stream, bool keyed, uint64_t key) {
    const uint64_t total = (uint64_t)ns * wl;
    if (!total) return SSBH_OK;
    const uint32_t *only_if = nullptr;
    bool streamed = false;
    if (n >= kPgMinBits && ctx->forced_scatter != 1) {
        const PgLayout P = pg_layout(n, ns, wl);
        const size_t merge_lds = (size_t)P.nb * P.cap / 8;
        if (merge_lds <= 144 * 1024 && ws.pg.reserve(P.bytes) == SSBH_OK) {
            uint8_t *base = ws.pg.as<uint8_t>();
            PgArgs a{};
            a.in = d_in; a.n = n; a.perm = d_perm; a.ns = ns; a.L = L; a.wl = wl;
            a.sub = d_sub; a.nb = P.nb; a.ng = P.ng; a.cap = P.cap;
            a.items = reinterpret_cast<uint32_t *>(base + P.items_off);
            a.slots = reinterpret_cast<uint32_t *>(base + P.slots_off);
            a.cnt = reinterpret_cast<uint32_t *>(base + P.cnt_off);
            a.bits = reinterpret_cast<uint64_t *>(base + P.bits_off);
            a.flag = reinterpret_cast<uint32_t *>(base + P.flag_off);
            a.status = d_status;
            ssbh_status st;
            const size_t win_lds = (size_t)8 << (kPgWinBits - 6);
            const size_t bucket_lds =
                (size_t)14 * ((P.nb + 3) & ~3u) + (size_t)kPgSubWords * 64 * 4;
            const bool aligned = L == 64 * wl;
            const void *kb = aligned ? (const void *)k_pg_bucket<true>
                                     : (const void *)k_pg_bucket<false>;
            const void *km = aligned ? (const void *)k_pg_merge<true>
                                     : (const void *)k_pg_merge<false>;
            if ((st = ensure_dynamic_lds(kb, bucket_lds)) != SSBH_OK)
                return st;
            if ((st = ensure_dynamic_lds((const void *)k_pg_window, win_lds)) != SSBH_OK)
                return st;
            if ((st = ensure_dynamic_lds(km, merge_lds)) != SSBH_OK)
                return st;
            // The cells, slots and overflow flag depend on pi alone: for the
            // context's keyed permutation they stay valid while the key, the
            // split and the scratch buffer do (the caller's own pi may
            // change between calls, so it is always bucketed again).
            const bool reuse = keyed && ws.pg_ptr == ws.pg.ptr &&
                               ws.pg_key == key && ws.pg_n == n && ws.pg_ns == ns;
            if (!reuse) {
                ws.pg_ptr = nullptr;
                hipLaunchKernelGGL(k_pg_init, dim3(1), dim3(1), 0, stream, a.flag);
                TimedLaunch timed(ws.timer, "k_pg_bucket", stream);
                if (aligned)
                    hipLaunchKernelGGL(k_pg_bucket<true>, dim3(P.ng), dim3(1024),
                                       bucket_lds, stream, a);
                else
                    hipLaunchKernelGGL(k_pg_bucket<false>, dim3(P.ng), dim3(1024),
                                       bucket_lds, stream, a);
                if (keyed) {
                    ws.pg_ptr = ws.pg.ptr;
                    ws.pg_key = key;
                    ws.pg_n = n;
                    ws.pg_ns = ns;
                }
            }
            {
                TimedLaunch timed(ws.timer, "k_pg_window", stream);
                hipLaunchKernelGGL(k_pg_window, dim3(P.nb), dim3(1024), win_lds,
                                   stream, a);
            }
            {
                TimedLaunch timed(ws.timer, "k_pg_merge", stream);
                if (aligned)
                    hipLaunchKernelGGL(k_pg_merge<true>, dim3(P.ng), dim3(1024),
                                       merge_lds, stream, a);
                else
                    hipLaunchKernelGGL(k_pg_merge<false>, dim3(P.ng), dim3(1024),
                                       merge_lds, stream, a);
            }
            only_if = a.flag;
            streamed = true;
        } else {
            (void)hipGetLastError();
            clear_error();
        }
    }
    // The direct gather: the whole job, or only when a cell overflowed.
    const uint64_t waves = std::min<uint64_t>(total, (uint64_t)ctx->num_cus * 32);
    {
        TimedLaunch timed(streamed ? nullptr : ws.timer, "k_perm_gather", stream);
        hipLaunchKernelGGL(k_perm_gather, dim3((uint32_t)((waves + 3) / 4)),
                           dim3(256), 0, stream, d_in, n, d_perm, ns, L, wl,
                           d_sub, only_if, d_status);
    }
    SSBH_CHECK_HIP(hipGetLastError());
    return SSBH_OK;
}

}  // namespace ssbh
