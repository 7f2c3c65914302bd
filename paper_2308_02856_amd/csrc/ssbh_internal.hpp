// Internal declarations of the ssbh library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/ssbh.h"

namespace ssbh {

// ------------------------------------------------------------- errors ---

void set_error(const char *fmt, ...);
void clear_error();

#define SSBH_CHECK_HIP(expr)                                                  \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess) {                                               \
            ::ssbh::set_error("%s failed: %s (%s:%d)", #expr,                 \
                              hipGetErrorString(e_), __FILE__, __LINE__);     \
            return SSBH_E_DEVICE;                                             \
        }                                                                     \
    } while (0)

#define SSBH_INVAL(...)                                                       \
    do {                                                                      \
        ::ssbh::set_error(__VA_ARGS__);                                       \
        return SSBH_E_INVAL;                                                  \
    } while (0)

// ------------------------------------------------------ device scratch ---

// A growable device buffer owned by a context.  Growing frees the old
// allocation (hipFree waits for the device), so pointers handed to kernels
// stay valid for the work already enqueued.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool external = false;   // memory lent by the serving arena: never grown
    ssbh_status reserve(size_t need);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Scratch used by one sample / hash pipeline.
// Optional per-kernel timing with HIP events on the launch stream (off by
// default; never used on a captured stream).
struct KernelTimer {
    struct Rec { const char *name; hipEvent_t start, stop; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    int begin(const char *name, hipStream_t stream);
    void end(int idx, hipStream_t stream);
    // Events for a launch that records them itself (hipExtLaunchKernelGGL:
    // the kernel's own start and end, without the dispatch around it).
    void begin_ext(const char *name, hipEvent_t *start, hipEvent_t *stop);
    std::string report();          // waits, aggregates, clears
    ~KernelTimer();
private:
    hipEvent_t take();             // from the pool, else a new event
};

struct TimedLaunch {
    KernelTimer *t;
    hipStream_t s;
    int idx;
    TimedLaunch(KernelTimer *timer, const char *name, hipStream_t stream)
        : t(timer), s(stream), idx(timer ? timer->begin(name, stream) : -1) {}
    ~TimedLaunch() { if (t) t->end(idx, s); }
};

struct Workspace {
    DevBuf counts;     // sampling: per-segment bucket counts  [segs][n_sub]
    DevBuf offs;       // sampling: per-segment bucket offsets [segs][n_sub]
    DevBuf part;       // sampling: per-chunk partial sums
    DevBuf plan;       // hashing: m_j, O_j, tile offsets (3 * n_sub u64)
    DevBuf tiles;      // hashing: tile list
    DevBuf counters;   // hashing: tile count, claim counter
    DevBuf fft_spec;   // FFT hash: seed spectrum (L complex doubles)
    DevBuf fft_work;   // FFT hash: transforms of a chunk of sub-block pairs
    DevBuf fft_qbuf;   // FFT hash: parity words in transform order
    DevBuf perm_tmp;   // keyed permutation: counts, groups, chain links
    DevBuf perm_pi;    // keyed permutation built for permutation sampling
    // perm_pi holds the keyed permutation of (perm_key, perm_n) while
    // perm_ptr == perm_pi.ptr (a grown buffer starts empty).
    uint64_t perm_key = 0, perm_n = 0;
    const void *perm_ptr = nullptr;
    DevBuf pg;         // permutation gather: cells, slots, looked-up bits
    // pg holds the bucketing of the keyed permutation (pg_key, pg_n) split
    // into pg_ns sub-blocks while pg_ptr == pg.ptr.
    uint64_t pg_key = 0, pg_n = 0;
    uint32_t pg_ns = 0;
    const void *pg_ptr = nullptr;
    char last_schedule[48] = "";   // kernel and schedule of the last hash
    KernelTimer *timer = nullptr;  // per-kernel event timing (optional)
    void release();
};

// A VALU hash schedule: rows per lane R, waves per workgroup, column words
// per tile, column words per LDS chunk.
struct ValuSchedule {
    int r = 16;
    int waves = 4;
    uint32_t tile_cols = 0;   // 0 = whole sub-block
    uint32_t chunk_cols = 4096;
    bool scalar_x = false;    // column words through the scalar cache
    int rows() const { return r * 64 * waves; }
};

struct MfmaSchedule {
    int mt = 8;      // 32-row tiles per wave
    int nt = 2;      // 32-sub-block tiles per wave (all waves share them)
    int wm = 4;      // waves per workgroup, along rows
    int ksplit = 0;  // K splits per tile (0 = fill the chip in whole rounds)
};

// FFT hash schedule: sub-block pairs transformed per chunk (0 = default).
struct FftSchedule {
    uint32_t chunk_pairs = 0;
    // Chunks alternate between the caller's stream and a second stream of
    // the context (two work buffers), so that one chunk's passes run while
    // the other's kernel boundaries drain.  Only for calls on the context's
    // own workspace; off under graph capture, with per-kernel timing and for
    // serving jobs (their own streams overlap).
    bool overlap = true;
    // Transform data between passes: 0 = library choice (complex floats
    // where fft_narrow allows), 64 = complex doubles, 32 = complex floats.
    int storage = 0;
};
constexpr uint64_t kMaxFftLength = 1ull << 31;   // transform length limit

struct ServeState;   // serving scheduler (serve.hip)

}  // namespace ssbh

struct ssbh_ctx {
    int device = 0;
    int num_cus = 0;
    size_t lds_per_block = 0;
    uint64_t hbm_budget = 0;
    std::mutex mu;                 // guards the default workspace
    ssbh::Workspace ws;            // scratch of the synchronous entry points
    std::vector<std::pair<std::string, std::string>> tune_cache;
    ssbh::ServeState *serve = nullptr;
    int forced_valu_r = 0;         // tests / autotuner: force a schedule
    int forced_valu_waves = 0;
    uint32_t forced_tile_cols = 0;
    uint32_t forced_chunk_cols = 0;
    int forced_scalar_x = -1;      // -1 = library choice
    int forced_mfma[4] = {0, 0, 0, 0};
    uint32_t forced_fft_chunk = 0;
    int forced_fft_pack = 0;       // 0 = library choice, 1 / 2 sub-blocks per part
    int forced_fft_storage = 0;    // 0 = library choice, 64 / 32 bits per real
    int forced_scatter = 0;        // 0 = library choice, 1 = one wave per segment
    hipStream_t fft_side = nullptr;   // second stream of the FFT hash chunks
    hipEvent_t fft_ev[2] = {nullptr, nullptr};   // fork and join
};

namespace ssbh {

// Schedule of an explicit matrix-core request: the one forced with
// ssbh_set_mfma_schedule, else two waves per SIMD, where one wave's operand
// work runs beside the other's matrix ops: (4,2,4) for int8 (36.5 against
// 38.0 ms at (8,2,4) on 8192 sub-blocks of 2^17 bits) and (4,2,8) for fp4,
// whose eight waves share one staging of the codes (20.3 against 22.4 ms at
// (4,2,4) and 23.0 at (8,2,4)).
inline MfmaSchedule explicit_mfma_schedule(const ssbh_ctx *ctx, bool fp4) {
    MfmaSchedule ms;
    ms.mt = 4;
    ms.nt = 2;
    ms.wm = fp4 ? 8 : 4;
    if (ctx->forced_mfma[0]) {
        ms.mt = ctx->forced_mfma[0];
        ms.nt = ctx->forced_mfma[1];
        ms.wm = ctx->forced_mfma[2];
    }
    ms.ksplit = ctx->forced_mfma[3];
    return ms;
}

// Kernel-launch layers (one per source file).
ssbh_status launch_sample(ssbh_ctx *ctx, Workspace &ws, const uint64_t *d_in,
                          const uint64_t *d_keep, uint64_t n_bits,
                          uint32_t n_sub, uint32_t mode,
                          uint64_t key, const uint32_t *d_assign,
                          uint64_t l_ub, uint64_t *d_sub, uint64_t sub_cap,
                          uint64_t *d_len, uint64_t *d_woff, int32_t *d_status,
                          hipStream_t stream);

struct HashRequest {
    const uint64_t *sub;
    uint64_t sub_cap;
    const uint64_t *len;
    const uint64_t *woff;
    uint32_t n_sub;
    uint32_t out_rule;
    uint64_t out_a, out_b;
    const uint64_t *out_len;
    const uint64_t *seed;
    uint64_t seed_bits;
    uint64_t stride;
    uint64_t m_cap;
    uint32_t kernel;
    uint64_t *out;
    uint64_t out_cap_bits;
    uint64_t *out_total;
    int32_t *status;
};

ssbh_status launch_hash(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                        hipStream_t stream);
ssbh_status check_hash_request(const HashRequest &q);

ssbh_status launch_hash_valu(ssbh_ctx *ctx, Workspace &ws,
                             const HashRequest &q, const ValuSchedule &s,
                             hipStream_t stream);

ssbh_status launch_hash_mfma(ssbh_ctx *ctx, Workspace &ws,
                             const HashRequest &q, const MfmaSchedule &s,
                             hipStream_t stream);
ssbh_status launch_hash_fft(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                            const FftSchedule &s, hipStream_t stream);
uint64_t fft_length(uint64_t seed_bits);
bool fft_can_pack(const HashRequest &q, uint64_t L);
uint32_t fft_chunk_of_bytes(uint64_t L, uint64_t mib, uint64_t point_bytes);
bool fft_narrow(const HashRequest &q, uint64_t L, int storage);
uint64_t fft_point_bytes(const HashRequest &q, uint64_t L, int storage);
int fft_per_transform(const ssbh_ctx *ctx, const HashRequest &q, uint64_t L);

ssbh_status launch_seed(uint64_t key, uint64_t *d_seed, uint64_t seed_bits,
                        hipStream_t stream);

// Keyed Durstenfeld permutation of 0..n-1 into d_perm (permute.hip);
// `scratch` grows to permutation_scratch(n) bytes.
ssbh_status launch_permutation(ssbh_ctx *ctx, DevBuf &scratch, uint64_t key,
                               uint64_t n, uint32_t *d_perm,
                               hipStream_t stream);
size_t permutation_scratch(uint64_t n);

// Permutation sampling's gather B[k] = A[pi[k]] (gather.hip).
// keyed: d_perm is the workspace's keyed permutation of `key`, so that the
// gather's bucketing may be kept for the next call with the same key.
ssbh_status launch_perm_gather(ssbh_ctx *ctx, Workspace &ws,
                               const uint64_t *d_in, uint64_t n,
                               const uint32_t *d_perm, uint32_t ns, uint64_t L,
                               uint64_t wl, uint64_t *d_sub, int32_t *d_status,
                               hipStream_t stream, bool keyed, uint64_t key);

// Fused two-kernel path of a graph pipeline for small permutation-split jobs
// with equal sub-blocks and 64-bit aligned outputs (small.hip).
bool small_path_ok(const ssbh_pipeline_desc &d);
ssbh_status launch_small_fused(ssbh_ctx *ctx, Workspace &ws,
                               const ssbh_pipeline_desc &d, hipStream_t stream);

// Scratch each launch layer will reserve for the given request (bytes per
// Workspace buffer), so callers can lend pre-sized memory.
struct ScratchSizes {
    size_t counts = 0, offs = 0, part = 0, plan = 0, tiles = 0, counters = 0;
    size_t total() const {
        return counts + offs + part + plan + tiles + counters;
    }
};
ScratchSizes sample_scratch(uint64_t n_bits, uint32_t n_sub, uint32_t mode);
ScratchSizes hash_scratch(const ssbh_ctx *ctx, const HashRequest &q);
ValuSchedule choose_valu(const ssbh_ctx *ctx, const HashRequest &q);
bool fft_pays(const HashRequest &q);
std::string tune_bucket(const HashRequest &q);

// Allow `kernel` to take `bytes` of dynamic LDS (needed above 64 KiB).
ssbh_status ensure_dynamic_lds(const void *kernel, size_t bytes);

// --------------------------------------------------------- device code ---

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output t of the stream
// seeded with `key` is mix(key + (t + 1) * golden_gamma).
constexpr uint64_t kSplitMixGamma = 0x9E3779B97F4A7C15ull;
// The output function of SplitMix64 applied to the counter value z.
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t key, uint64_t t) {
    return splitmix64_mix(key + (t + 1ull) * kSplitMixGamma);
}

__device__ __forceinline__ uint64_t ballot64(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `m` strictly below the calling lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace ssbh
