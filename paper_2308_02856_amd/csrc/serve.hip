// Serving: continuous batching of extraction jobs under an HBM budget.
//
// ssbh_submit queues a job and returns at once.  A scheduler thread owned by
// the context admits queued jobs in FIFO order whenever a stream slot is idle
// and the job's whole device footprint (input copy, sub-blocks, seed, output,
// sampling and hashing scratch) fits in the budget arena, enqueues the job's
// pipeline on that slot's stream (seed from key -> sampling with the abort
// rule -> per-sub-block hash + concatenation -> result copies), and reaps
// finished jobs by polling their completion events, returning their memory to
// the arena so the next queued jobs can start while others are still on the
// GPU.  Jobs on different slots overlap on the device.  Every job is a pure
// function of its parameters, so its output is the same alone or in a mix.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "ssbh_internal.hpp"

namespace ssbh {

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator over one device allocation (offsets kept in a map of
// free ranges, coalesced on release).
class Arena {
  public:
    ssbh_status init(size_t bytes) {
        bytes = round256(bytes);
        hipError_t e = hipMalloc(&base_, bytes);
        if (e != hipSuccess) {
            base_ = nullptr;
            set_error("serving arena of %zu bytes: %s", bytes,
                      hipGetErrorString(e));
            return SSBH_E_NOMEM;
        }
        size_ = bytes;
        free_[0] = bytes;
        return SSBH_OK;
    }
    void destroy() {
        if (base_) hipFree(base_);
        base_ = nullptr;
        free_.clear();
    }
    bool ready() const { return base_ != nullptr; }
    size_t size() const { return size_; }
    uint8_t *alloc(size_t bytes) {
        bytes = round256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rem = it->second - bytes;
            free_.erase(it);
            if (rem) free_[off + bytes] = rem;
            return base_ + off;
        }
        return nullptr;
    }
    void release(uint8_t *p, size_t bytes) {
        bytes = round256(bytes);
        size_t off = (size_t)(p - base_);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    uint8_t *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
};

struct JobPlan {
    uint64_t n = 0, l_ub = 0, n_cap = 0, m_cap = 0, stride = 0;
    uint64_t seed_bits = 0, out_words = 0, sub_cap = 0;
    ScratchSizes samp, hash;
    // Hash kernel and schedule, fixed at submission (the footprint depends
    // on them): the FFT hash (one transform per sub-block with its own seed)
    // when it pays, else the bit-sliced VALU kernel.
    bool fft = false;
    ValuSchedule valu;
    FftSchedule fsched;
    size_t fft_work_b = 0, fft_qbuf_b = 0;
    size_t in_b = 0, sub_b = 0, len_b = 0, seed_b = 0, out_b = 0, misc_b = 256;
    size_t total = 0;
};

enum { kPending = 0, kRunning = 1, kDone = 2 };

struct Job {
    uint64_t id = 0;
    ssbh_job spec{};
    JobPlan plan;
    int state = kPending;
    int slot = -1;
    uint8_t *mem = nullptr;
    int32_t status = 0;
    uint64_t out_bits = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct SlotResult {
    int32_t status;
    int32_t pad;
    uint64_t total;
};

struct ServeState {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int> free_slots;
    std::vector<uint64_t> slot_job;
    SlotResult *pinned = nullptr;
    Arena arena;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1, running = 0, finished = 0;
};

static constexpr int kSlots = 6;
static constexpr uint64_t kServeFftChunkMiB = 48;

uint64_t job_out_words(const ssbh_job &j) {
    uint64_t cap;
    if (j.out_rule == SSBH_OUT_RATIO)
        cap = (uint64_t)((unsigned __int128)j.n_bits * j.out_a / j.out_b);
    else
        cap = (uint64_t)j.n_sub * j.out_a;
    return (cap + 64 + 63) / 64;
}

static ssbh_status plan_job(const ssbh_ctx *ctx, const ssbh_job &j,
                            JobPlan &p) {
    if (j.n_sub == 0 || j.n_sub > SSBH_MAX_SUB_LDS)
        SSBH_INVAL("n_sub must be in [1, %u]", SSBH_MAX_SUB_LDS);
    if (j.n_bits > SSBH_MAX_SAMPLE_BITS)
        SSBH_INVAL("n_bits must be at most %llu", (unsigned long long)SSBH_MAX_SAMPLE_BITS);
    if (j.n_bits && !j.in) SSBH_INVAL("job input is null");
    if (!j.out) SSBH_INVAL("job output is null");
    if (j.out_rule == SSBH_OUT_RATIO) {
        if (!j.out_b || j.out_a >= (1ull << 24) || j.out_b >= (1ull << 24))
            SSBH_INVAL("ratio terms must be in [1, 2^24)");
    } else if (j.out_rule != SSBH_OUT_FIXED) {
        SSBH_INVAL("serving jobs use SSBH_OUT_FIXED or SSBH_OUT_RATIO");
    }
    p.n = j.n_bits;
    const double mean = (double)j.n_bits / j.n_sub;
    p.l_ub = j.l_ub ? j.l_ub
                    : (uint64_t)std::ceil(mean + 8.0 * std::sqrt(mean)) + 64;
    p.n_cap = std::min<uint64_t>(p.l_ub, j.n_bits);
    p.m_cap = j.out_rule == SSBH_OUT_RATIO ? p.n_cap * j.out_a / j.out_b
                                           : j.out_a;
    if (p.m_cap >= (1ull << 32)) SSBH_INVAL("output length too large");
    p.stride = p.n_cap + (p.m_cap ? p.m_cap - 1 : 0);
    p.seed_bits = (uint64_t)j.n_sub * p.stride;
    p.out_words = job_out_words(j);
    p.sub_cap = (j.n_bits + 63) / 64 + j.n_sub;
    p.samp = sample_scratch(j.n_bits, j.n_sub, SSBH_SAMPLE_IID);
    HashRequest q{};
    q.n_sub = j.n_sub;
    q.sub_cap = p.sub_cap;
    q.m_cap = p.m_cap;
    q.stride = p.stride;
    q.seed_bits = p.seed_bits;
    q.out_cap_bits = p.out_words * 64;
    p.fft = fft_pays(q);
    if (p.fft) {
        // Transforms of at most kServeFftChunkMiB per chunk: a job's share of
        // the budget stays modest, so several jobs fit at once.
        const uint64_t L = fft_length(p.stride);
        // Library choice of the transform storage, fixed here with the
        // footprint.
        const uint64_t pb = fft_point_bytes(q, L, 0);
        p.fsched.chunk_pairs = fft_chunk_of_bytes(L, kServeFftChunkMiB, pb);
        p.fsched.overlap = false;
        p.fsched.storage = pb == 8 ? 32 : 64;
        const uint64_t cp = std::min<uint64_t>(p.fsched.chunk_pairs, j.n_sub);
        p.fft_work_b = (size_t)cp * L * pb;
        p.fft_qbuf_b = (size_t)(q.out_cap_bits / 64 + 3ull * j.n_sub + 4) * 8;
        q.kernel = SSBH_K_FFT;
    } else {
        q.kernel = SSBH_K_VALU;
        p.valu = choose_valu(ctx, q);
    }
    p.hash = hash_scratch(ctx, q);
    p.in_b = j.in_on_device ? 0 : round256((j.n_bits + 63) / 64 * 8);
    p.sub_b = round256(p.sub_cap * 8);
    p.len_b = round256((size_t)j.n_sub * 8);
    p.seed_b = round256((p.seed_bits + 63) / 64 * 8);
    p.out_b = j.out_on_device ? 0 : round256(p.out_words * 8);
    p.total = p.in_b + p.sub_b + 2 * p.len_b + p.seed_b + p.out_b + p.misc_b +
              round256(p.samp.counts) + round256(p.samp.offs) +
              round256(p.samp.part) + round256(p.hash.plan) +
              round256(p.hash.tiles) + round256(p.hash.counters) +
              round256(p.fft_work_b) + round256(p.fft_qbuf_b);
    return SSBH_OK;
}

// Carve the job's memory and enqueue its pipeline on its slot's stream.
static ssbh_status enqueue_job(ssbh_ctx *ctx, ServeState &S, Job &job) {
    const JobPlan &p = job.plan;
    const ssbh_job &j = job.spec;
    hipStream_t st = S.streams[job.slot];
    uint8_t *cur = job.mem;
    auto take = [&](size_t b) { uint8_t *r = cur; cur += round256(b); return r; };
    const uint64_t *d_in = j.in;
    if (!j.in_on_device) d_in = reinterpret_cast<const uint64_t *>(take(p.in_b));
    uint64_t *d_sub = reinterpret_cast<uint64_t *>(take(p.sub_b));
    uint64_t *d_len = reinterpret_cast<uint64_t *>(take(p.len_b));
    uint64_t *d_woff = reinterpret_cast<uint64_t *>(take(p.len_b));
    uint64_t *d_seed = reinterpret_cast<uint64_t *>(take(p.seed_b));
    uint64_t *d_out = j.out;
    if (!j.out_on_device) d_out = reinterpret_cast<uint64_t *>(take(p.out_b));
    uint8_t *misc = take(p.misc_b);
    int32_t *d_status = reinterpret_cast<int32_t *>(misc);
    uint64_t *d_total = reinterpret_cast<uint64_t *>(misc + 64);
    Workspace ws;
    auto lend = [&](DevBuf &b, size_t bytes) {
        b.ptr = take(bytes);
        b.bytes = round256(bytes);
        b.external = true;
    };
    lend(ws.counts, p.samp.counts);
    lend(ws.offs, p.samp.offs);
    lend(ws.part, p.samp.part);
    lend(ws.plan, p.hash.plan);
    lend(ws.tiles, p.hash.tiles);
    lend(ws.counters, p.hash.counters);
    if (p.fft) {
        lend(ws.fft_work, p.fft_work_b);
        lend(ws.fft_qbuf, p.fft_qbuf_b);
    }

    if (!j.in_on_device && p.n) {
        SSBH_CHECK_HIP(hipMemcpyAsync((void *)d_in, j.in, (p.n + 63) / 64 * 8,
                                      hipMemcpyHostToDevice, st));
    }
    ssbh_status rc = launch_seed(j.seed_key, d_seed, p.seed_bits, st);
    if (rc != SSBH_OK) return rc;
    rc = launch_sample(ctx, ws, d_in, nullptr, p.n, j.n_sub, SSBH_SAMPLE_IID,
                       j.sample_key, nullptr, p.l_ub, d_sub, p.sub_cap, d_len,
                       d_woff, d_status, st);
    if (rc != SSBH_OK) return rc;
    HashRequest q{d_sub, p.sub_cap, d_len, d_woff, j.n_sub, j.out_rule,
                  j.out_a, j.out_b, nullptr, d_seed, p.seed_bits, p.stride,
                  p.m_cap, p.fft ? SSBH_K_FFT : SSBH_K_VALU, d_out,
                  p.out_words * 64, d_total, d_status};
    (void)hipGetLastError();   // clear errors left by earlier calls
    rc = p.fft ? launch_hash_fft(ctx, ws, q, p.fsched, st)
               : launch_hash_valu(ctx, ws, q, p.valu, st);
    if (rc != SSBH_OK) return rc;
    if (!j.out_on_device) {
        SSBH_CHECK_HIP(hipMemcpyAsync(j.out, d_out, p.out_words * 8,
                                      hipMemcpyDeviceToHost, st));
    }
    SSBH_CHECK_HIP(hipMemcpyAsync(&S.pinned[job.slot].status, d_status, 4,
                                  hipMemcpyDeviceToHost, st));
    SSBH_CHECK_HIP(hipMemcpyAsync(&S.pinned[job.slot].total, d_total, 8,
                                  hipMemcpyDeviceToHost, st));
    SSBH_CHECK_HIP(hipEventRecord(S.events[job.slot], st));
    return SSBH_OK;
}

static void finish_job(ServeState &S, Job &job, int32_t status) {
    if (job.mem) S.arena.release(job.mem, job.plan.total);
    job.mem = nullptr;
    if (job.slot >= 0) {
        S.free_slots.push_back(job.slot);
        S.slot_job[job.slot] = 0;
        S.running--;
    }
    job.slot = -1;
    job.status = status;
    job.state = kDone;
    job.t_done = now_s();
    S.finished++;
}

static void scheduler(ssbh_ctx *ctx) {
    ServeState &S = *ctx->serve;
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(S.mu);
    for (;;) {
        // Reap finished jobs.
        for (int s = 0; s < (int)S.streams.size(); ++s) {
            const uint64_t id = S.slot_job[s];
            if (!id) continue;
            if (hipEventQuery(S.events[s]) != hipSuccess) continue;
            Job &job = *S.jobs[id];
            job.out_bits = S.pinned[s].total;
            finish_job(S, job, S.pinned[s].status);
        }
        // Admit queued jobs (FIFO) while a slot and memory are free.
        while (!S.stop && !S.pending.empty() && !S.free_slots.empty()) {
            Job &job = *S.jobs[S.pending.front()];
            uint8_t *mem = S.arena.alloc(job.plan.total);
            if (!mem) break;
            S.pending.pop_front();
            job.mem = mem;
            job.slot = S.free_slots.back();
            S.free_slots.pop_back();
            S.slot_job[job.slot] = job.id;
            S.running++;
            job.state = kRunning;
            job.t_admit = now_s();
            S.pinned[job.slot].status = 0;
            S.pinned[job.slot].total = 0;
            const ssbh_status rc = enqueue_job(ctx, S, job);
            if (rc != SSBH_OK) {
                (void)hipStreamSynchronize(S.streams[job.slot]);
                finish_job(S, job, rc);
            }
        }
        if (S.stop && S.running == 0) break;
        if (S.running == 0 && S.pending.empty()) {
            S.cv.wait_for(lk, std::chrono::milliseconds(50));
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

static ssbh_status serve_init(ssbh_ctx *ctx) {
    if (ctx->serve) return SSBH_OK;
    auto *S = new ServeState();
    ssbh_status rc = S->arena.init(ctx->hbm_budget);
    if (rc != SSBH_OK) {
        delete S;
        return rc;
    }
    S->streams.resize(kSlots);
    S->events.resize(kSlots);
    S->slot_job.assign(kSlots, 0);
    if (hipHostMalloc((void **)&S->pinned, sizeof(SlotResult) * kSlots,
                      hipHostMallocDefault) != hipSuccess) {
        S->arena.destroy();
        delete S;
        set_error("pinned result buffer allocation failed");
        return SSBH_E_NOMEM;
    }
    for (int s = 0; s < kSlots; ++s) {
        // Default priority streams only.
        if (hipStreamCreateWithFlags(&S->streams[s], hipStreamNonBlocking) !=
                hipSuccess ||
            hipEventCreateWithFlags(&S->events[s], hipEventDisableTiming) !=
                hipSuccess) {
            set_error("stream or event creation failed");
            return SSBH_E_DEVICE;
        }
        S->free_slots.push_back(kSlots - 1 - s);
    }
    ctx->serve = S;
    S->worker = std::thread(scheduler, ctx);
    return SSBH_OK;
}

}  // namespace ssbh

using namespace ssbh;

extern "C" {

uint64_t ssbh_job_out_words(const ssbh_job *job) {
    return job ? job_out_words(*job) : 0;
}

ssbh_status ssbh_submit(ssbh_ctx *ctx, const ssbh_job *job, uint64_t *job_id) {
    clear_error();
    if (!ctx || !job || !job_id) SSBH_INVAL("ctx, job and job_id must be non-null");
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    auto j = std::make_unique<Job>();
    j->spec = *job;
    ssbh_status rc;
    {
        // The plan reads the context's forced schedules: under its lock.
        std::lock_guard<std::mutex> g(ctx->mu);
        rc = plan_job(ctx, *job, j->plan);
        if (rc == SSBH_OK) rc = serve_init(ctx);
    }
    if (rc != SSBH_OK) return rc;
    ServeState &S = *ctx->serve;
    if (round256(j->plan.total) > S.arena.size()) {
        set_error("job needs %zu bytes of device memory, budget is %zu",
                  j->plan.total, S.arena.size());
        return SSBH_E_NOMEM;
    }
    j->t_submit = now_s();
    {
        std::lock_guard<std::mutex> g(S.mu);
        j->id = S.next_id++;
        *job_id = j->id;
        S.pending.push_back(j->id);
        S.jobs[j->id] = std::move(j);
    }
    S.cv.notify_one();
    return SSBH_OK;
}

ssbh_status ssbh_poll(ssbh_ctx *ctx, uint64_t job_id, ssbh_result *res) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (!ctx->serve) {
        set_error("unknown job %llu", (unsigned long long)job_id);
        return SSBH_E_UNKNOWN_JOB;
    }
    ServeState &S = *ctx->serve;
    std::lock_guard<std::mutex> g(S.mu);
    auto it = S.jobs.find(job_id);
    if (it == S.jobs.end()) {
        set_error("unknown job %llu", (unsigned long long)job_id);
        return SSBH_E_UNKNOWN_JOB;
    }
    Job &job = *it->second;
    if (job.state != kDone) return SSBH_PENDING;
    if (res) {
        res->status = job.status;
        res->out_bits = job.out_bits;
        res->device_bytes = job.plan.total;
        res->t_submit = job.t_submit;
        res->t_admit = job.t_admit;
        res->t_done = job.t_done;
    }
    const ssbh_status st = (ssbh_status)job.status;
    S.jobs.erase(it);
    return st;
}

ssbh_status ssbh_serve_counts(ssbh_ctx *ctx, uint64_t *pending,
                              uint64_t *running, uint64_t *finished) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    uint64_t p = 0, r = 0, f = 0;
    if (ctx->serve) {
        std::lock_guard<std::mutex> g(ctx->serve->mu);
        p = ctx->serve->pending.size();
        r = ctx->serve->running;
        f = ctx->serve->finished;
    }
    if (pending) *pending = p;
    if (running) *running = r;
    if (finished) *finished = f;
    return SSBH_OK;
}

void ssbh_serve_shutdown(ssbh_ctx *ctx) {
    if (!ctx || !ctx->serve) return;
    ServeState *S = ctx->serve;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        S->pending.clear();          // queued jobs are dropped
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();   // waits for running jobs
    for (auto &st : S->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto &e : S->events) (void)hipEventDestroy(e);
    if (S->pinned) (void)hipHostFree(S->pinned);
    S->arena.destroy();
    delete S;
    ctx->serve = nullptr;
}

}  // extern "C"
