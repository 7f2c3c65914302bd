// Serving scheduler (continuous batching) - placeholder until implemented.
#include "ssbh_internal.hpp"

extern "C" void ssbh_serve_shutdown(ssbh_ctx *ctx) { (void)ctx; }
