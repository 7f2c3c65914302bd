// C-ABI entry points of the ssbh library: context, errors, argument checks
// and kernel selection.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "ssbh_internal.hpp"

namespace ssbh {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

ssbh_status DevBuf::reserve(size_t need) {
    if (need <= bytes) return SSBH_OK;
    if (external) {
        set_error("scratch lent by the serving arena is too small (%zu < %zu)",
                  bytes, need);
        return SSBH_E_NOMEM;
    }
    size_t grow = std::max(need, bytes + bytes / 2);
    grow = (grow + 255) & ~(size_t)255;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        if (e != hipSuccess) {
            set_error("hipFree failed: %s", hipGetErrorString(e));
            return SSBH_E_DEVICE;
        }
    }
    hipError_t e = hipMalloc(&ptr, grow);
    if (e != hipSuccess) {
        ptr = nullptr;
        set_error("hipMalloc(%zu) failed: %s", grow, hipGetErrorString(e));
        return SSBH_E_NOMEM;
    }
    bytes = grow;
    return SSBH_OK;
}

ssbh_status ensure_dynamic_lds(const void *kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return SSBH_OK;
    static std::mutex mu;
    static std::vector<std::pair<const void *, size_t>> done;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &d : done)
        if (d.first == kernel && d.second >= bytes) return SSBH_OK;
    hipError_t e = hipFuncSetAttribute(
        kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("kernel needs %zu bytes of LDS: %s", bytes,
                  hipGetErrorString(e));
        return SSBH_E_UNSUPPORTED;
    }
    done.emplace_back(kernel, bytes);
    return SSBH_OK;
}

void DevBuf::release() {
    if (ptr && !external) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

hipEvent_t KernelTimer::take() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) { e = pool.back(); pool.pop_back(); }
    else if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    return e;
}

int KernelTimer::begin(const char *name, hipStream_t stream) {
    Rec r{name, take(), take()};
    if (r.start) (void)hipEventRecord(r.start, stream);
    recs.push_back(r);
    return (int)recs.size() - 1;
}

void KernelTimer::begin_ext(const char *name, hipEvent_t *start, hipEvent_t *stop) {
    Rec r{name, take(), take()};
    recs.push_back(r);
    *start = r.start;
    *stop = r.stop;
}

void KernelTimer::end(int idx, hipStream_t stream) {
    if (idx >= 0 && recs[idx].stop) (void)hipEventRecord(recs[idx].stop, stream);
}

std::string KernelTimer::report() {
    std::vector<std::pair<std::string, std::pair<long, double>>> agg;
    for (Rec &r : recs) {
        float ms = 0.f;
        if (r.start && r.stop && hipEventSynchronize(r.stop) == hipSuccess &&
            hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            bool found = false;
            for (auto &a : agg)
                if (a.first == r.name) {
                    a.second.first += 1;
                    a.second.second += ms;
                    found = true;
                }
            if (!found) agg.push_back({r.name, {1, (double)ms}});
        }
        if (r.start) pool.push_back(r.start);
        if (r.stop) pool.push_back(r.stop);
    }
    recs.clear();
    std::string out;
    char line[160];
    for (auto &a : agg) {
        snprintf(line, sizeof line, "%s %ld %.6f\n", a.first.c_str(),
                 a.second.first, a.second.second);
        out += line;
    }
    return out;
}

KernelTimer::~KernelTimer() {
    for (Rec &r : recs) {
        if (r.start) (void)hipEventDestroy(r.start);
        if (r.stop) (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

void Workspace::release() {
    counts.release();
    offs.release();
    part.release();
    plan.release();
    tiles.release();
    counters.release();
    fft_spec.release();
    fft_work.release();
    fft_qbuf.release();
    perm_tmp.release();
    perm_pi.release();
    perm_ptr = nullptr;
    pg.release();
    pg_ptr = nullptr;
    delete timer;
    timer = nullptr;
}

// Default VALU schedule: 16 rows per lane, 4 wavefronts (4096 rows per
// tile); columns are split only when the row tiles alone cannot fill the
// device several times over.
ValuSchedule choose_valu(const ssbh_ctx *ctx, const HashRequest &q) {
    ValuSchedule s;
    if (ctx->forced_valu_r) s.r = ctx->forced_valu_r;
    if (ctx->forced_valu_waves) s.waves = ctx->forced_valu_waves;
    const double rows = (double)s.rows();
    const double row_tiles = (double)q.n_sub * std::ceil((double)q.m_cap / rows);
    const double target = 16.0 * ctx->num_cus;
    if (ctx->forced_tile_cols) {
        s.tile_cols = ctx->forced_tile_cols;
    } else if (row_tiles < target && q.n_sub) {
        const double mean_words = 2.0 * (double)q.sub_cap / q.n_sub;
        const double splits = std::ceil(target / std::max(row_tiles, 1.0));
        double tc = std::ceil(mean_words / splits / 32.0) * 32.0;
        tc = std::max(tc, 256.0);
        if (tc < mean_words) s.tile_cols = (uint32_t)std::min(tc, 4.0e9);
    }
    s.chunk_cols = ctx->forced_chunk_cols ? ctx->forced_chunk_cols : 4096;
    if (ctx->forced_scalar_x >= 0) s.scalar_x = ctx->forced_scalar_x != 0;
    return s;
}

// Shape bucket of a hash request (used by the autotuner's table).
std::string tune_bucket(const HashRequest &q) {
    auto lg = [](double v) { return v <= 1 ? 0 : (int)std::floor(std::log2(v)); };
    const double mean_words = q.n_sub ? 2.0 * (double)q.sub_cap / q.n_sub : 0;
    char b[96];
    snprintf(b, sizeof b, "%s/ns%d/m%d/w%d", q.stride ? "indep" : "shared",
             lg(q.n_sub), lg((double)q.m_cap), lg(mean_words));
    return b;
}

// Untuned choice between the FFT and the quadratic kernels.  Per sub-block
// the quadratic kernels take about 7e-16 s per bit-product (n * m of them);
// the FFT takes a share (1/2, or 1/4 when four sub-blocks ride in a
// transform; all of it with independent seeds, where a transform carries one
// sub-block and its seed) of a forward and inverse transform, about
// 7e-13 s per point-level (L log2 L of them), both measured on MI355X at the
// batched length: break-even near n * m = 1000 L log2 L per transform.  The
// FFT is taken when n * m >= 1024 L log2 L / (sub-blocks per transform), n
// estimated from the seed length (n_max + m_cap - 1 bits, or the stride).
bool fft_pays(const HashRequest &q) {
    const uint64_t span = q.stride ? q.stride : q.seed_bits;
    const uint64_t L = fft_length(span);
    if (L > kMaxFftLength || span + 1 <= q.m_cap) return false;
    const double n = (double)(span + 1 - q.m_cap);
    const double m = (double)q.m_cap;
    // Sub-blocks per transform: one with a stride or a single sub-block
    // (the joint transform), else four or two.
    const double per = (q.stride || q.n_sub == 1) ? 1.0 : fft_can_pack(q, L) ? 4.0 : 2.0;
    return n * m >= 1024.0 / per * (double)L * std::log2((double)L);
}

ssbh_status launch_hash(ssbh_ctx *ctx, Workspace &ws, const HashRequest &q,
                        hipStream_t stream) {
    (void)hipGetLastError();   // clear errors left by earlier calls
    if (q.kernel == SSBH_K_AUTO) {
        HashRequest r = q;
        std::string choice;
        {
            const std::string key = tune_bucket(q);
            for (auto &kv : ctx->tune_cache)
                if (kv.first == key) choice = kv.second;
        }
        if (!choice.empty()) {
            int a = 0, b = 0, c = 0, k = 0;
            unsigned d = 0, e = 0;
            if (sscanf(choice.c_str(), "mfma:%d:%d:%d:%d", &a, &b, &c, &k) == 4 &&
                q.stride == 0) {
                MfmaSchedule ms;
                ms.mt = a; ms.nt = b; ms.wm = c; ms.ksplit = k;
                r.kernel = SSBH_K_MFMA_I8;
                return launch_hash_mfma(ctx, ws, r, ms, stream);
            }
            if (sscanf(choice.c_str(), "fft:%u", &d) == 1) {
                FftSchedule fs;
                fs.chunk_pairs = d;
                fs.storage = ctx->forced_fft_storage;
                r.kernel = SSBH_K_FFT;
                return launch_hash_fft(ctx, ws, r, fs, stream);
            }
            if (sscanf(choice.c_str(), "valu:%d:%d:%u:%u", &a, &b, &d, &e) == 4) {
                ValuSchedule vs = choose_valu(ctx, q);
                vs.r = a; vs.waves = b; vs.chunk_cols = d; vs.tile_cols = e;
                r.kernel = SSBH_K_VALU;
                return launch_hash_valu(ctx, ws, r, vs, stream);
            }
        }
        if (!ctx->forced_valu_r && fft_pays(q)) {
            r.kernel = SSBH_K_FFT;
            return launch_hash(ctx, ws, r, stream);
        }
        if (q.stride == 0 && q.n_sub >= 64 && !ctx->forced_valu_r) {
            r.kernel = SSBH_K_MFMA_I8;
            return launch_hash(ctx, ws, r, stream);
        }
        r.kernel = SSBH_K_VALU;
        return launch_hash_valu(ctx, ws, r, choose_valu(ctx, r), stream);
    }
    if (q.kernel == SSBH_K_MFMA_I8 || q.kernel == SSBH_K_MFMA_F4) {
        const MfmaSchedule ms =
            explicit_mfma_schedule(ctx, q.kernel == SSBH_K_MFMA_F4);
        return launch_hash_mfma(ctx, ws, q, ms, stream);
    }
    if (q.kernel == SSBH_K_FFT) {
        FftSchedule fs;
        fs.chunk_pairs = ctx->forced_fft_chunk;
        fs.storage = ctx->forced_fft_storage;
        return launch_hash_fft(ctx, ws, q, fs, stream);
    }
    if (q.kernel != SSBH_K_VALU) SSBH_INVAL("unknown kernel %u", q.kernel);
    return launch_hash_valu(ctx, ws, q, choose_valu(ctx, q), stream);
}

// Host-visible argument checks of ssbh_hash_batch (and of its variant
// without allocation).
ssbh_status check_hash_request(const HashRequest &q) {
    if (!q.len || !q.woff || !q.status || !q.out_total)
        SSBH_INVAL("d_len, d_word_off, d_out_total_bits and d_status must be "
                   "non-null");
    if (q.n_sub && !q.sub) SSBH_INVAL("d_sub is null");
    if (q.out_cap_bits && !q.out) SSBH_INVAL("d_out is null");
    if (q.out_rule == SSBH_OUT_RATIO) {
        if (q.out_b == 0) SSBH_INVAL("out_b must be > 0");
        if (q.out_a >= (1ull << 24) || q.out_b >= (1ull << 24))
            SSBH_INVAL("ratio terms must be below 2^24");
    } else if (q.out_rule == SSBH_OUT_EXPLICIT) {
        if (q.n_sub && !q.out_len) SSBH_INVAL("explicit lengths need d_out_len");
    } else if (q.out_rule != SSBH_OUT_FIXED) {
        SSBH_INVAL("unknown out_rule %u", q.out_rule);
    }
    if (q.m_cap == 0 && q.out_rule == SSBH_OUT_FIXED && q.out_a > 0)
        SSBH_INVAL("m_cap must be >= out_a");
    if (q.m_cap >= (1ull << 32)) {
        set_error("m_cap must be below 2^32");
        return SSBH_E_UNSUPPORTED;
    }
    if (q.sub_cap >= (1ull << 36)) {
        set_error("sub_capacity_words must be below 2^36");
        return SSBH_E_UNSUPPORTED;
    }
    if (q.n_sub > 1 && q.stride) {
        const long double last = (long double)(q.n_sub - 1) * q.stride;
        if (last > (long double)q.seed_bits)
            SSBH_INVAL("seed too short for %u sub-blocks at stride %llu",
                       q.n_sub, (unsigned long long)q.stride);
    }
    if (q.seed_bits && !q.seed) SSBH_INVAL("d_seed is null");
    if ((q.kernel == SSBH_K_MFMA_I8 || q.kernel == SSBH_K_MFMA_F4) && q.stride != 0)
        SSBH_INVAL("the MFMA kernels need a shared seed (seed_stride = 0)");
    if (q.kernel == SSBH_K_MFMA_F4 && q.seed_bits + 1 > (1ull << 24) + q.m_cap) {
        set_error("the fp4 matrix kernel needs seed_bits + 1 - m_cap <= 2^24 "
                  "(exact fp32 sums)");
        return SSBH_E_UNSUPPORTED;
    }
    if (q.kernel == SSBH_K_FFT &&
        fft_length(q.stride ? q.stride : q.seed_bits) > kMaxFftLength) {
        set_error("the FFT hash supports seeds (or seed strides) of at most "
                  "%llu bits", (unsigned long long)kMaxFftLength);
        return SSBH_E_UNSUPPORTED;
    }
    if (q.kernel > SSBH_K_MFMA_F4) SSBH_INVAL("unknown kernel %u", q.kernel);
    return SSBH_OK;
}

}  // namespace ssbh

using namespace ssbh;

extern "C" {

const char *ssbh_last_error(void) { return g_err; }

ssbh_status ssbh_create(int device, uint64_t hbm_budget_bytes, ssbh_ctx **out) {
    clear_error();
    if (!out) SSBH_INVAL("out is null");
    *out = nullptr;
    int count = 0;
    SSBH_CHECK_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        SSBH_INVAL("device %d out of range (%d devices)", device, count);
    SSBH_CHECK_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    SSBH_CHECK_HIP(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("device %d is %s; this library is built for gfx950 only",
                  device, prop.gcnArchName);
        return SSBH_E_UNSUPPORTED;
    }
    ssbh_ctx *c = new ssbh_ctx();
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    if (!hbm_budget_bytes) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess)
            hbm_budget_bytes = (uint64_t)(fr * 0.8);
    }
    c->hbm_budget = hbm_budget_bytes;
    *out = c;
    return SSBH_OK;
}

void ssbh_serve_shutdown(ssbh_ctx *ctx);   // serve.hip

void ssbh_destroy(ssbh_ctx *ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    ssbh_serve_shutdown(ctx);
    hipDeviceSynchronize();
    ctx->ws.release();
    if (ctx->fft_side) hipStreamDestroy(ctx->fft_side);
    for (hipEvent_t e : ctx->fft_ev)
        if (e) hipEventDestroy(e);
    delete ctx;
}

int ssbh_num_cus(const ssbh_ctx *ctx) { return ctx ? ctx->num_cus : 0; }

ssbh_status ssbh_sample(ssbh_ctx *ctx, const uint64_t *d_in, uint64_t n_bits,
                        uint32_t n_sub, uint32_t mode, uint64_t sample_key,
                        const uint32_t *d_assign, uint64_t l_ub,
                        uint64_t *d_sub, uint64_t sub_capacity_words,
                        uint64_t *d_len, uint64_t *d_word_off,
                        int32_t *d_status, void *stream) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    return launch_sample(ctx, ctx->ws, d_in, nullptr, n_bits, n_sub, mode,
                         sample_key, d_assign, l_ub, d_sub, sub_capacity_words,
                         d_len, d_word_off, d_status, (hipStream_t)stream);
}

ssbh_status ssbh_sample_sifted(ssbh_ctx *ctx, const uint64_t *d_in,
                               const uint64_t *d_keep, uint64_t n_bits,
                               uint32_t n_sub, uint32_t mode,
                               uint64_t sample_key, const uint32_t *d_assign,
                               uint64_t l_ub, uint64_t *d_sub,
                               uint64_t sub_capacity_words, uint64_t *d_len,
                               uint64_t *d_word_off, int32_t *d_status,
                               void *stream) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (n_bits && !d_keep) SSBH_INVAL("d_keep is null");
    if (mode == SSBH_SAMPLE_PERMUTE)
        SSBH_INVAL("sifting flags need i.i.d. or explicit V");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    return launch_sample(ctx, ctx->ws, d_in, d_keep, n_bits, n_sub, mode,
                         sample_key, d_assign, l_ub, d_sub, sub_capacity_words,
                         d_len, d_word_off, d_status, (hipStream_t)stream);
}

ssbh_status ssbh_hash_batch(ssbh_ctx *ctx, const uint64_t *d_sub,
                            uint64_t sub_capacity_words,
                            const uint64_t *d_len, const uint64_t *d_word_off,
                            uint32_t n_sub, uint32_t out_rule, uint64_t out_a,
                            uint64_t out_b, const uint64_t *d_out_len,
                            const uint64_t *d_seed, uint64_t seed_bits,
                            uint64_t seed_stride, uint64_t m_cap,
                            uint32_t kernel, uint64_t *d_out,
                            uint64_t out_capacity_bits,
                            uint64_t *d_out_total_bits, int32_t *d_status,
                            void *stream) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    HashRequest q{d_sub, sub_capacity_words, d_len, d_word_off, n_sub,
                  out_rule, out_a, out_b, d_out_len, d_seed, seed_bits,
                  seed_stride, m_cap, kernel, d_out, out_capacity_bits,
                  d_out_total_bits, d_status};
    ssbh_status st = check_hash_request(q);
    if (st != SSBH_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    return launch_hash(ctx, ctx->ws, q, (hipStream_t)stream);
}

ssbh_status ssbh_permutation(ssbh_ctx *ctx, uint64_t key, uint64_t n,
                             uint32_t *d_perm, void *stream) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    return launch_permutation(ctx, ctx->ws.perm_tmp, key, n, d_perm,
                              (hipStream_t)stream);
}

ssbh_status ssbh_seed_from_key(ssbh_ctx *ctx, uint64_t seed_key,
                               uint64_t *d_seed, uint64_t seed_bits,
                               void *stream) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (seed_bits && !d_seed) SSBH_INVAL("d_seed is null");
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    return launch_seed(seed_key, d_seed, seed_bits, (hipStream_t)stream);
}

// Force the VALU schedule (0 = library choice).
ssbh_status ssbh_set_schedule(ssbh_ctx *ctx, int r, int waves,
                              uint32_t tile_cols, uint32_t chunk_cols) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (r && r != 8 && r != 16 && r != 32) SSBH_INVAL("r must be 8, 16 or 32");
    if (waves && waves != 2 && waves != 4 && waves != 8)
        SSBH_INVAL("waves must be 2, 4 or 8");
    if (chunk_cols && (chunk_cols % 32 || chunk_cols > 16384))
        SSBH_INVAL("chunk_cols must be a multiple of 32 and at most 16384");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_valu_r = r;
    ctx->forced_valu_waves = waves;
    ctx->forced_tile_cols = tile_cols;
    ctx->forced_chunk_cols = chunk_cols;
    return SSBH_OK;
}

ssbh_status ssbh_set_timing(ssbh_ctx *ctx, int on) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    if (on && !ctx->ws.timer) ctx->ws.timer = new KernelTimer();
    if (!on && ctx->ws.timer) {
        (void)hipDeviceSynchronize();
        delete ctx->ws.timer;
        ctx->ws.timer = nullptr;
    }
    return SSBH_OK;
}

ssbh_status ssbh_timing_report(ssbh_ctx *ctx, char *buf, uint64_t len) {
    clear_error();
    if (!ctx || !buf || !len) SSBH_INVAL("ctx and buf must be non-null");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    const std::string t = ctx->ws.timer ? ctx->ws.timer->report() : std::string();
    strncpy(buf, t.c_str(), len - 1);
    buf[len - 1] = 0;
    return SSBH_OK;
}

ssbh_status ssbh_set_sample_path(ssbh_ctx *ctx, int path) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (path < 0 || path > 1) SSBH_INVAL("path must be 0 or 1");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_scatter = path;
    return SSBH_OK;
}

ssbh_status ssbh_set_fft_schedule(ssbh_ctx *ctx, uint32_t chunk_pairs) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_fft_chunk = chunk_pairs;
    return SSBH_OK;
}

ssbh_status ssbh_set_fft_packing(ssbh_ctx *ctx, int per_part) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (per_part < 0 || per_part > 2) SSBH_INVAL("per_part must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_fft_pack = per_part;
    return SSBH_OK;
}

ssbh_status ssbh_set_fft_storage(ssbh_ctx *ctx, int bits) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (bits != 0 && bits != 32 && bits != 64) SSBH_INVAL("bits must be 0, 32 or 64");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_fft_storage = bits;
    return SSBH_OK;
}

ssbh_status ssbh_set_mfma_schedule(ssbh_ctx *ctx, int mt, int nt, int wm,
                                   int ksplit) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (ksplit < 0 || ksplit > 64) SSBH_INVAL("ksplit must be 0 .. 64");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_mfma[0] = mt;
    ctx->forced_mfma[1] = nt;
    ctx->forced_mfma[2] = wm;
    ctx->forced_mfma[3] = ksplit;
    return SSBH_OK;
}

// Column words through LDS (0), the scalar cache (1) or library choice (-1).
ssbh_status ssbh_set_column_path(ssbh_ctx *ctx, int scalar_x) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (scalar_x < -1 || scalar_x > 1) SSBH_INVAL("scalar_x must be -1, 0 or 1");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_scalar_x = scalar_x;
    return SSBH_OK;
}

}  // extern "C"
