// ssbh_hash_batch without any allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The hashing plan (m_j, O_j, tile offsets), the VALU tile list and the
// claim counters live in one fixed device array, `scratch`, instead of the
// context's growable workspace.  Each GPU holds its own copy of the array
// until the process ends; its device address is looked up once per device
// with hipGetSymbolAddress and only that address is handed to kernels.  The
// kernels of the path initialise every word they read (the plan kernel writes
// the counters and the tile list), so nothing depends on what an earlier call
// left in the array.  Calls that overlap on one GPU share the array and race.
#include <mutex>
#include <vector>

#include "ssbh_internal.hpp"

namespace ssbh {
namespace {

constexpr size_t kScratchBytes = SSBH_NOALLOC_SCRATCH_BYTES;
constexpr size_t kCounterBytes = 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<std::pair<int, void *>> g_addr;   // (device, address of scratch)

// Device address of `scratch` on the current device (looked up once).
ssbh_status scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &d : g_addr)
        if (d.first == device) { *out = d.second; return SSBH_OK; }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error("hipGetSymbolAddress(scratch) failed on device %d: %s",
                  device, hipGetErrorString(e));
        return SSBH_E_DEVICE;
    }
    g_addr.emplace_back(device, p);
    *out = p;
    return SSBH_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace ssbh

using namespace ssbh;

extern "C" ssbh_status ssbh_hash_batch_noalloc(
        ssbh_ctx *ctx, const uint64_t *d_sub, uint64_t sub_capacity_words,
        const uint64_t *d_len, const uint64_t *d_word_off, uint32_t n_sub,
        uint32_t out_rule, uint64_t out_a, uint64_t out_b,
        const uint64_t *d_out_len, const uint64_t *d_seed, uint64_t seed_bits,
        uint64_t seed_stride, uint64_t m_cap, uint32_t kernel, uint64_t *d_out,
        uint64_t out_capacity_bits, uint64_t *d_out_total_bits,
        int32_t *d_status, void *stream) {
    clear_error();
    if (!ctx) SSBH_INVAL("ctx is null");
    if (kernel == SSBH_K_FFT) {
        set_error("the FFT hash needs transform buffers; it has no variant "
                  "without allocation");
        return SSBH_E_UNSUPPORTED;
    }
    HashRequest q{d_sub, sub_capacity_words, d_len, d_word_off, n_sub,
                  out_rule, out_a, out_b, d_out_len, d_seed, seed_bits,
                  seed_stride, m_cap, kernel, d_out, out_capacity_bits,
                  d_out_total_bits, d_status};
    ssbh_status st = check_hash_request(q);
    if (st != SSBH_OK) return st;
    if (q.kernel == SSBH_K_AUTO)   // the choice ssbh_hash_batch makes without the FFT
        q.kernel = (q.stride == 0 && q.n_sub >= 64) ? SSBH_K_MFMA_I8 : SSBH_K_VALU;

    // Scratch layout: plan, counters, tile list.
    const ScratchSizes need = hash_scratch(ctx, q);
    const size_t plan_b = align256(need.plan);
    const size_t tiles_b = align256(need.tiles);
    if (plan_b + kCounterBytes + tiles_b > kScratchBytes) {
        set_error("this request needs %zu bytes of hashing scratch; the fixed "
                  "array holds %zu (SSBH_NOALLOC_SCRATCH_BYTES)",
                  plan_b + kCounterBytes + tiles_b, kScratchBytes);
        return SSBH_E_UNSUPPORTED;
    }
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    void *base = nullptr;
    if ((st = scratch_address(ctx->device, &base)) != SSBH_OK) return st;
    unsigned char *b = static_cast<unsigned char *>(base);
    Workspace ws;   // borrowed memory only: reserve() never allocates
    ws.plan.ptr = b;
    ws.plan.bytes = plan_b;
    ws.plan.external = true;
    ws.counters.ptr = b + plan_b;
    ws.counters.bytes = kCounterBytes;
    ws.counters.external = true;
    ws.tiles.ptr = b + plan_b + kCounterBytes;
    ws.tiles.bytes = kScratchBytes - plan_b - kCounterBytes;
    ws.tiles.external = true;
    (void)hipGetLastError();
    if (q.kernel == SSBH_K_VALU)
        return launch_hash_valu(ctx, ws, q, choose_valu(ctx, q),
                                (hipStream_t)stream);
    const MfmaSchedule ms =
        explicit_mfma_schedule(ctx, q.kernel == SSBH_K_MFMA_F4);
    return launch_hash_mfma(ctx, ws, q, ms, (hipStream_t)stream);
}
