// The hot path captured into a HIP graph: one launch replays the sampling
// kernels, the plan, the output fill and the hash kernel on fixed buffers.
// Every kernel of the path clears what it needs with its own stores (no
// hipMemsetAsync nodes), so replays are self-contained.
#include <new>

#include "ssbh_internal.hpp"

struct ssbh_pipeline {
    ssbh_ctx *ctx = nullptr;
    ssbh_pipeline_desc d{};
    ssbh::Workspace ws;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace ssbh {

static ssbh_status enqueue_pipeline(ssbh_pipeline *p, hipStream_t st) {
    const ssbh_pipeline_desc &d = p->d;
    ssbh_status rc;
    if (small_path_ok(d) && !p->ctx->forced_valu_r)
        return launch_small_fused(p->ctx, p->ws, d, st);
    if (d.d_in) {
        rc = launch_sample(p->ctx, p->ws, d.d_in, d.d_keep, d.n_bits, d.n_sub,
                           d.mode,
                           d.sample_key, d.d_assign, d.l_ub, d.d_sub,
                           d.sub_capacity_words, d.d_len, d.d_word_off,
                           d.d_status, st);
        if (rc != SSBH_OK) return rc;
    }
    HashRequest q{d.d_sub, d.sub_capacity_words, d.d_len, d.d_word_off,
                  d.n_sub, d.out_rule, d.out_a, d.out_b, d.d_out_len,
                  d.d_seed, d.seed_bits, d.seed_stride, d.m_cap, d.kernel,
                  d.d_out, d.out_capacity_bits, d.d_out_total_bits,
                  d.d_status};
    return launch_hash(p->ctx, p->ws, q, st);
}

}  // namespace ssbh

using namespace ssbh;

extern "C" {

void ssbh_pipeline_destroy(ssbh_pipeline *p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    p->ws.release();
    delete p;
}

ssbh_status ssbh_pipeline_create(ssbh_ctx *ctx, const ssbh_pipeline_desc *desc,
                                 ssbh_pipeline **out) {
    clear_error();
    if (!ctx || !desc || !out) SSBH_INVAL("ctx, desc and out must be non-null");
    *out = nullptr;
    if (!desc->d_status || !desc->d_len || !desc->d_word_off ||
        !desc->d_out_total_bits)
        SSBH_INVAL("d_status, d_len, d_word_off and d_out_total_bits must "
                   "be non-null");
    SSBH_CHECK_HIP(hipSetDevice(ctx->device));
    auto *p = new (std::nothrow) ssbh_pipeline();
    if (!p) return SSBH_E_NOMEM;
    p->ctx = ctx;
    p->d = *desc;
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        set_error("stream creation failed");
        return SSBH_E_DEVICE;
    }
    // Eager run: sizes the scratch, sets kernel attributes, validates.
    ssbh_status rc = enqueue_pipeline(p, p->stream);
    if (rc == SSBH_OK && hipStreamSynchronize(p->stream) != hipSuccess) {
        set_error("eager pipeline run failed");
        rc = SSBH_E_DEVICE;
    }
    if (rc == SSBH_OK) {
        if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) !=
            hipSuccess) {
            set_error("hipStreamBeginCapture failed");
            rc = SSBH_E_DEVICE;
        } else {
            rc = enqueue_pipeline(p, p->stream);
            const hipError_t e = hipStreamEndCapture(p->stream, &p->graph);
            if (rc == SSBH_OK && e != hipSuccess) {
                set_error("hipStreamEndCapture: %s", hipGetErrorString(e));
                rc = SSBH_E_DEVICE;
            }
        }
    }
    if (rc == SSBH_OK &&
        hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("hipGraphInstantiate failed");
        rc = SSBH_E_DEVICE;
    }
    if (rc != SSBH_OK) {
        ssbh_pipeline_destroy(p);
        return rc;
    }
    *out = p;
    return SSBH_OK;
}

ssbh_status ssbh_pipeline_launch(ssbh_pipeline *p, void *stream) {
    clear_error();
    if (!p || !p->exec) SSBH_INVAL("pipeline is null");
    SSBH_CHECK_HIP(hipSetDevice(p->ctx->device));
    SSBH_CHECK_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return SSBH_OK;
}

}  // extern "C"
