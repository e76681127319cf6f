// vsh_serve.hip -- serving loop (placeholder until continuous batching lands).
#include "vsh_internal.hpp"

namespace vsh {
void serve_shutdown(vsh_ctx*) {}
}  // namespace vsh

extern "C" {
vsh_status vsh_submit(vsh_ctx* ctx, const vsh_request*, uint64_t*) {
  vsh::set_error(ctx, "serving not available");
  return VSH_E_INVALID;
}
vsh_status vsh_poll(vsh_ctx*, uint64_t, int*) { return VSH_E_NOTFOUND; }
vsh_status vsh_wait(vsh_ctx*, uint64_t, vsh_result**) { return VSH_E_NOTFOUND; }
vsh_status vsh_cancel(vsh_ctx*, uint64_t) { return VSH_E_NOTFOUND; }
}
