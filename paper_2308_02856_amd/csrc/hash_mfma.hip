// Shared-seed contraction on int8 matrix cores - placeholder.
#include "ssbh_internal.hpp"

namespace ssbh {
ssbh_status launch_hash_mfma(ssbh_ctx *, Workspace &, const HashRequest &,
                             const MfmaSchedule &, hipStream_t) {
    set_error("MFMA kernel not built");
    return SSBH_E_UNSUPPORTED;
}
}  // namespace ssbh
