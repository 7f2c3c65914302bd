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

// Output word w of the sub-block buffer holds bits k = j L + 64 ww + lane
// for 64 ww + lane < L (w = j wl + ww).  A wavefront walks words at a fixed
// stride, so (j, ww) advance without a division; all of it is the same for
// the whole wavefront and runs on the scalar unit.
struct WordPos {
    uint64_t j, ww;
    __device__ __forceinline__ void start(uint64_t w, uint64_t wl) {
        j = w / wl;
        ww = w - j * wl;
    }
    __device__ __forceinline__ void advance(uint64_t step, uint64_t wl) {
        ww += step;
        while (ww >= wl) { ww -= wl; ++j; }
    }
    __device__ __forceinline__ uint64_t k0(uint64_t L) const { return j * L + ww * 64; }
    __device__ __forceinline__ uint64_t c0() const { return ww * 64; }
};

// Bucket pass: one workgroup per chunk, in sub-chunks of kPgSubWords output
// words (2^13 bits).  Per sub-chunk: each thread's 8 entries of pi, ranks
// from LDS counters, a scan of the counts, the window offsets sorted by
// window in LDS with their cell slots beside them, then one coalesced copy
// of the stage into the cells.  cc[b] is cell b's fill so far.
constexpr uint32_t kPgSubWords = 128;
constexpr uint32_t kPgPer = kPgSubWords / 16;   // words per wavefront

__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_pg_bucket(PgArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ int live_s;
    const uint32_t nb4 = (a.nb + 3u) & ~3u;
    uint32_t *cl = lds;                       // [nb] sub-chunk counts
    uint32_t *lb = cl + nb4;                  // [nb] sub-chunk run starts
    uint32_t *cc = lb + nb4;                  // [nb] cell fill
    uint32_t *part = cc + nb4;                // [16] wave sums of the scan
    uint32_t *stage = part + 16;              // [kPgSubWords * 64] offsets
    uint32_t *sslot = stage + kPgSubWords * 64;  // their slots in the chunk
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
    WordPos pos;
    pos.start(w0 + (uint64_t)wv, a.wl);
    for (uint64_t s0 = w0; live && s0 < w1; s0 += kPgSubWords) {
        // 1. pi of words s0 + 16 i + wv, one word per wavefront and step.
        uint32_t pv[kPgPer], rv[kPgPer];
        uint64_t k0v[kPgPer];
        uint32_t okm = 0;                     // bit i: entry i is a real bit
#pragma unroll
        for (int i = 0; i < (int)kPgPer; ++i) {
            const uint64_t w = s0 + 16u * i + (uint64_t)wv;
            k0v[i] = pos.k0(a.L);
            const bool ok = w < w1 && pos.c0() + (uint64_t)lane < a.L;
            okm |= ok ? 1u << i : 0u;
            pv[i] = ok ? a.perm[k0v[i] + lane] : 0xffffffffu;
            pos.advance(16, a.wl);
        }
        // 2. ranks within the sub-chunk (any order: the slot records it).
#pragma unroll
        for (int i = 0; i < (int)kPgPer; ++i) {
            rv[i] = 0u;
            if ((okm >> i) & 1u) {
                if (pv[i] < a.n) rv[i] = atomicAdd(&cl[pv[i] >> kPgWinBits], 1u);
                else bad = true;
            }
        }
        __syncthreads();
        // 3. run starts: exclusive scan of cl over the windows.
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
            for (uint32_t b = (uint32_t)t * 4u; b < min((uint32_t)t * 4u + 4u, a.nb); ++b) {
                lb[b] = run;
                run += cl[b];
            }
        }
        __syncthreads();
        // 4. offsets sorted by window, each with its slot (window * cap +
        //    rank in the cell; ~0 past the capacity); the slots of k.
#pragma unroll
        for (int i = 0; i < (int)kPgPer; ++i) {
            if (!((okm >> i) & 1u)) continue;
            uint32_t slot = 0;
            if (pv[i] < a.n) {
                const uint32_t b = pv[i] >> kPgWinBits;
                const uint32_t x = lb[b] + rv[i];
                const uint32_t r = cc[b] + rv[i];
                slot = r < a.cap ? b * a.cap + r : 0u;
                stage[x] = pv[i] & ((1u << kPgWinBits) - 1u);
                sslot[x] = r < a.cap ? b * a.cap + r : 0xffffffffu;
            }
            a.slots[k0v[i] + lane] = slot;
        }
        __syncthreads();
        // 5. the stage into the cells (runs of a window are contiguous in
        //    both); 6. cell fills.
        for (uint32_t x = (uint32_t)t; x < tot; x += 1024) {
            const uint32_t d = sslot[x];
            if (d != 0xffffffffu) cell[d] = stage[x];
            else over = true;
        }
        for (uint32_t b = t; b < a.nb; b += 1024) {
            cc[b] += cl[b];
            cl[b] = 0u;
        }
        __syncthreads();
    }
    if (bad) atomicExch(a.status, (int32_t)SSBH_E_INVAL);
    if (over) atomicOr(a.flag, 1u);
    for (uint32_t b = t; b < a.nb; b += 1024)
        a.cnt[(uint64_t)b * a.ng + g] = min(cc[b], a.cap);
}

// Window pass: one workgroup per window; each wavefront takes cells in turn
// and loads up to 8 x 64 of a cell's entries before looking them up.
__global__ __launch_bounds__(1024) void k_pg_window(PgArgs a) {
    extern __shared__ uint64_t win[];                 // 2^20 bits
    if (*a.status || *a.flag) return;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t b = blockIdx.x;
    const uint64_t nw_in = (a.n + 63) / 64;
    const uint64_t wbase = (uint64_t)b << (kPgWinBits - 6);
    constexpr uint32_t kWinWords = 1u << (kPgWinBits - 6);
    for (uint32_t i = t; i < kWinWords; i += 1024)
        win[i] = wbase + i < nw_in ? a.in[wbase + i] : 0ull;
    __syncthreads();
    const uint32_t *cw = a.cnt + (uint64_t)b * a.ng;
    for (uint32_t g = wv; g < a.ng; g += 16) {
        const uint32_t ccount = cw[g];
        const uint64_t cell = ((uint64_t)g * a.nb + b) * a.cap;
        const uint32_t *it = a.items + cell;
        uint64_t *out = a.bits + cell / 64;
        for (uint32_t q0 = 0; q0 < ccount; q0 += 512) {
            uint32_t o[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t q = q0 + 64u * u + (uint32_t)lane;
                o[u] = q < ccount ? it[q] : 0xffffffffu;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t q = q0 + 64u * u;
                if (q >= ccount) break;
                const bool bit = o[u] != 0xffffffffu &&
                                 ((win[o[u] >> 6] >> (o[u] & 63)) & 1ull);
                const uint64_t word = ballot64(bit);
                if (lane == 0) out[q / 64] = word;
            }
        }
    }
}

// Merge pass: one workgroup per chunk; each wavefront loads the slots of
// four output words before looking them up.
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
    WordPos pos;
    pos.start(w0 + 4u * (uint64_t)wv, a.wl);
    for (uint64_t wq = w0 + 4u * (uint64_t)wv; wq < w1; wq += 64) {
        uint32_t sv[4];
        bool okv[4];
        WordPos pu = pos;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t w = wq + u;
            okv[u] = w < w1 && pu.c0() + (uint64_t)lane < a.L;
            sv[u] = okv[u] ? a.slots[pu.k0(a.L) + lane] : 0u;
            pu.advance(1, a.wl);
        }
        pos.advance(64, a.wl);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
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
                               hipStream_t stream) {
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
                ((size_t)3 * ((P.nb + 3) & ~3u) + 16 + 2 * kPgSubWords * 64) * 4;
            if ((st = ensure_dynamic_lds((const void *)k_pg_bucket, bucket_lds)) != SSBH_OK)
                return st;
            if ((st = ensure_dynamic_lds((const void *)k_pg_window, win_lds)) != SSBH_OK)
                return st;
            if ((st = ensure_dynamic_lds((const void *)k_pg_merge, merge_lds)) != SSBH_OK)
                return st;
            hipLaunchKernelGGL(k_pg_init, dim3(1), dim3(1), 0, stream, a.flag);
            {
                TimedLaunch timed(ws.timer, "k_pg_bucket", stream);
                hipLaunchKernelGGL(k_pg_bucket, dim3(P.ng), dim3(1024),
                                   bucket_lds, stream, a);
            }
            {
                TimedLaunch timed(ws.timer, "k_pg_window", stream);
                hipLaunchKernelGGL(k_pg_window, dim3(P.nb), dim3(1024), win_lds,
                                   stream, a);
            }
            {
                TimedLaunch timed(ws.timer, "k_pg_merge", stream);
                hipLaunchKernelGGL(k_pg_merge, dim3(P.ng), dim3(1024), merge_lds,
                                   stream, a);
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
