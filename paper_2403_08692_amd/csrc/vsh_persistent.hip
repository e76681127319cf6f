// vsh_persistent.hip -- persistent-wave form of the shower (placeholder until
// the persistent kernel lands).
#include "vsh_internal.hpp"

namespace vsh {

vsh_status generate_persistent(vsh_ctx* ctx, const vsh_request*, vsh_result**) {
  set_error(ctx, "persistent form not available");
  return VSH_E_INVALID;
}

uint64_t persistent_workspace_bytes(const vsh_request*) { return 0; }

vsh_status persistent_into(vsh_ctx* ctx, const vsh_request*, hipStream_t, void*, double*, double*,
                           int32_t*, uint64_t*) {
  set_error(ctx, "persistent form not available");
  return VSH_E_INVALID;
}

}  // namespace vsh
