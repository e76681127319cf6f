// vsh_noalloc.hip -- vsh_generate_into_static: the plain-form launch sequence
// of vsh_generate_into with its workspace in a device array the library
// owns, for callers that cannot allocate device memory (code under graph
// capture, serving loops that must not call hipMalloc, harnesses that forbid
// it).  The caller still passes the histogram and summary buffers.
//
// The array is a file-scope __device__ variable: the code object's loader
// gives every device that runs the library its own copy, held until the
// process ends.  In host code the variable's name is only a host-side
// stand-in for it, so its device address is looked up once per device
// (static_scratch_init, from vsh_create with that device current) and kept;
// kernels are only ever handed that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/vsh.h"
#include "vsh_internal.hpp"

namespace vsh {

static_assert(VSH_STATIC_SCRATCH_BYTES % 256 == 0, "the static workspace is a whole number of 256-byte granules");

static __device__ __align__(256) unsigned char scratch[VSH_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

vsh_status static_scratch_init(vsh_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) {
    set_error(ctx, "device %d: the static workspace table holds devices 0..%d", ctx->device, kMaxDevices - 1);
    return VSH_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  void*& slot = g_scratch_ptr[ctx->device];
  if (!slot) {
    void* p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error(ctx, "hipGetSymbolAddress of the static workspace: %s", hipGetErrorString(err));
      return VSH_E_DEVICE;
    }
    slot = p;
  }
  ctx->static_scratch = slot;
  return VSH_OK;
}

}  // namespace vsh

using namespace vsh;

extern "C" vsh_status vsh_generate_into_static(vsh_ctx* ctx, const vsh_request* req, void* stream, double* dev_hist,
                                               double* dev_sum_d, int32_t* dev_sum_i, uint64_t* dev_hash) {
  if (!ctx) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  vsh_status rc = validate_request(ctx, req, true);
  if (rc) return rc;
  if (!dev_hist) {
    set_error(ctx, "dev_hist is required");
    return VSH_E_INVALID;
  }
  if (req->flags & (VSH_RECORDS | VSH_FORM_PERSISTENT)) {
    set_error(ctx, "vsh_generate_into_static runs the plain form and returns summaries and histograms only");
    return VSH_E_INVALID;
  }
  if (!(req->flags & VSH_INPUTS_ON_DEVICE) && (req->ecm_per_event || req->tcut_per_event)) {
    set_error(ctx, "per-event arrays of vsh_generate_into_static must be device pointers (VSH_INPUTS_ON_DEVICE)");
    return VSH_E_INVALID;
  }
  const uint64_t need = vsh_workspace_size(req);
  if (need > VSH_STATIC_SCRATCH_BYTES) {
    set_error(ctx, "request needs %llu bytes of workspace; the static workspace holds %llu (split the request "
              "by event ids, or use vsh_generate_into)", (unsigned long long)need,
              (unsigned long long)VSH_STATIC_SCRATCH_BYTES);
    return VSH_E_NOMEM;
  }
  (void)hipSetDevice(ctx->device);
  if (!ctx->static_scratch) {  // not found at vsh_create: look it up now, on this device
    rc = static_scratch_init(ctx);
    if (rc) return rc;
  }
  return plain_into(ctx, req, (hipStream_t)stream, ctx->static_scratch, dev_hist, dev_sum_d, dev_sum_i, dev_hash,
                    false);
}
