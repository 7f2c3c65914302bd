// Autotuner for the hash kernels: times candidate kernels and schedules on
// the caller's real arguments and records the fastest per shape bucket.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include <algorithm>

#include "ssbh_internal.hpp"

namespace ssbh {

namespace {

struct Candidate {
    std::string name;
    bool mfma;
    bool fft = false;
    ValuSchedule v;
    MfmaSchedule m;
    FftSchedule f;
};

std::vector<Candidate> candidates(const ssbh_ctx *ctx, const HashRequest &q) {
    std::vector<Candidate> c;
    const ValuSchedule base = choose_valu(ctx, q);
    const int vs[][3] = {{16, 4, 4096}, {32, 2, 2048}, {32, 4, 2048},
                         {16, 8, 2048}, {16, 2, 1024}};
    for (auto &x : vs) {
        Candidate k;
        k.mfma = false;
        k.v = base;
        k.v.r = x[0];
        k.v.waves = x[1];
        k.v.chunk_cols = (uint32_t)x[2];
        // Keep the column split of the default schedule, scaled to the rows.
        HashRequest r = q;
        ssbh_ctx tmp;
        tmp.num_cus = ctx->num_cus;
        tmp.forced_valu_r = x[0];
        tmp.forced_valu_waves = x[1];
        k.v.tile_cols = choose_valu(&tmp, r).tile_cols;
        char b[64];
        snprintf(b, sizeof b, "valu:%d:%d:%u:%u", k.v.r, k.v.waves,
                 k.v.chunk_cols, k.v.tile_cols);
        k.name = b;
        c.push_back(k);
    }
    const uint64_t span = q.stride ? q.stride : q.seed_bits;
    if (fft_length(span) <= kMaxFftLength) {
        // Chunks of 64 .. 256 MiB of transforms (two are in flight at once:
        // below, around and above the last-level cache), as transform counts
        // at this length.
        const uint64_t L = fft_length(span);
        std::vector<uint32_t> cps;
        for (uint64_t mib : {64ull, 96ull, 128ull, 160ull, 192ull, 256ull}) {
            const uint32_t cp = fft_chunk_of_bytes(
                L, mib, fft_point_bytes(q, L, ctx->forced_fft_storage));
            if (std::find(cps.begin(), cps.end(), cp) == cps.end()) cps.push_back(cp);
        }
        for (uint32_t cp : cps) {
            Candidate k;
            k.mfma = false;
            k.fft = true;
            k.f.chunk_pairs = cp;
            k.f.storage = ctx->forced_fft_storage;
            char b[64];
            snprintf(b, sizeof b, "fft:%u", cp);
            k.name = b;
            c.push_back(k);
        }
    }
    if (q.stride == 0) {
        // ksplit 0 = the launcher's whole-rounds choice.
        const int ms[][4] = {{8, 2, 4, 0}, {8, 2, 4, 1}, {4, 2, 4, 0},
                             {8, 1, 4, 0}, {4, 4, 4, 0}};
        for (auto &x : ms) {
            Candidate k;
            k.mfma = true;
            k.m.mt = x[0];
            k.m.nt = x[1];
            k.m.wm = x[2];
            k.m.ksplit = x[3];
            char b[64];
            snprintf(b, sizeof b, "mfma:%d:%d:%d:%d", x[0], x[1], x[2], x[3]);
            k.name = b;
            c.push_back(k);
        }
    }
    return c;
}

}  // namespace
}  // namespace ssbh

using namespace ssbh;

extern "C" {

ssbh_status ssbh_tune(ssbh_ctx *ctx, const uint64_t *d_sub,
                      uint64_t sub_capacity_words, const uint64_t *d_len,
                      const uint64_t *d_word_off, uint32_t n_sub,
                      uint32_t out_rule, uint64_t out_a, uint64_t out_b,
                      const uint64_t *d_out_len, const uint64_t *d_seed,
                      uint64_t seed_bits, uint64_t seed_stride, uint64_t m_cap,
                      uint64_t *d_out, uint64_t out_capacity_bits,
                      uint64_t *d_out_total_bits, int32_t *d_status,
                      uint32_t reps, char *report, uint64_t report_len,
                      void *stream) {
    clear_error();
    if (!ctx || !d_status || !d_len || !d_word_off || !d_out_total_bits)
        SSBH_INVAL("ctx, d_len, d_word_off, d_out_total_bits, d_status "
                   "must be non-null");
    if (!n_sub) SSBH_INVAL("n_sub must be >= 1");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int32_t h_status = 0;
    SSBH_CHECK_HIP(hipMemcpyAsync(&h_status, d_status, 4, hipMemcpyDeviceToHost, st));
    SSBH_CHECK_HIP(hipStreamSynchronize(st));
    if (h_status) SSBH_INVAL("d_status is nonzero (%d) before tuning", h_status);
    HashRequest q{d_sub, sub_capacity_words, d_len, d_word_off, n_sub,
                  out_rule, out_a, out_b, d_out_len, d_seed, seed_bits,
                  seed_stride, m_cap, SSBH_K_AUTO, d_out, out_capacity_bits,
                  d_out_total_bits, d_status};
    hipEvent_t e0, e1;
    SSBH_CHECK_HIP(hipEventCreate(&e0));
    SSBH_CHECK_HIP(hipEventCreate(&e1));
    std::string best;
    float best_ms = 1e30f;
    std::string table;
    if (!reps) reps = 2;
    for (const Candidate &c : candidates(ctx, q)) {
        std::vector<float> times;
        ssbh_status rc = SSBH_OK;
        for (uint32_t k = 0; k <= reps && rc == SSBH_OK; ++k) {
            (void)hipEventRecord(e0, st);
            HashRequest r = q;
            r.kernel = c.fft ? SSBH_K_FFT : c.mfma ? SSBH_K_MFMA_I8 : SSBH_K_VALU;
            rc = c.fft ? launch_hash_fft(ctx, ctx->ws, r, c.f, st)
                 : c.mfma ? launch_hash_mfma(ctx, ctx->ws, r, c.m, st)
                          : launch_hash_valu(ctx, ctx->ws, r, c.v, st);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (k) times.push_back(ms);   // the first run warms up
        }
        SSBH_CHECK_HIP(hipMemcpyAsync(&h_status, d_status, 4,
                                      hipMemcpyDeviceToHost, st));
        SSBH_CHECK_HIP(hipStreamSynchronize(st));
        char line[128];
        if (rc != SSBH_OK || h_status) {
            snprintf(line, sizeof line, "%-24s failed (%d/%d)\n", c.name.c_str(),
                     (int)rc, h_status);
            if (h_status) {
                table += line;
                break;              // a device-side argument error: stop
            }
        } else {
            // The median of the timed runs: one slow run (another process,
            // a clock change) does not decide the choice.
            std::sort(times.begin(), times.end());
            const size_t h = times.size() / 2;
            const float ms = times.size() % 2 ? times[h]
                                               : 0.5f * (times[h - 1] + times[h]);
            snprintf(line, sizeof line, "%-24s %10.3f ms\n", c.name.c_str(), ms);
            if (ms < best_ms) { best_ms = ms; best = c.name; }
        }
        table += line;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (report && report_len) {
        strncpy(report, table.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    if (best.empty()) {
        set_error("no candidate succeeded:\n%s", table.c_str());
        return h_status ? (ssbh_status)h_status : SSBH_E_DEVICE;
    }
    const std::string key = tune_bucket(q);
    bool found = false;
    for (auto &kv : ctx->tune_cache)
        if (kv.first == key) { kv.second = best; found = true; }
    if (!found) ctx->tune_cache.emplace_back(key, best);
    return SSBH_OK;
}

ssbh_status ssbh_tune_table(ssbh_ctx *ctx, char *buf, uint64_t len) {
    clear_error();
    if (!ctx || !buf || !len) SSBH_INVAL("ctx and buf must be non-null");
    std::string t;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : ctx->tune_cache) t += kv.first + "=" + kv.second + "\n";
    }
    strncpy(buf, t.c_str(), len - 1);
    buf[len - 1] = 0;
    return SSBH_OK;
}

ssbh_status ssbh_last_schedule(ssbh_ctx *ctx, char *buf, uint64_t len) {
    clear_error();
    if (!ctx || !buf || !len) SSBH_INVAL("ctx and buf must be non-null");
    std::lock_guard<std::mutex> lk(ctx->mu);
    strncpy(buf, ctx->ws.last_schedule, len - 1);
    buf[len - 1] = 0;
    return SSBH_OK;
}

}  // extern "C"
