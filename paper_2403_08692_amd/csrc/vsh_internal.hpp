// vsh_internal.hpp -- host-side internals shared by the C-ABI translation
// units: the context, the device arena, the plain-form layout and results.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstddef>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/vsh.h"
#include "vsh_kernels.hpp"

namespace vsh {
// a request's quark masses (d, u, s massless) and whether any is above zero
inline QuarkMasses request_masses(const vsh_request& r) { return QuarkMasses{0.0, 0.0, 0.0, r.mass_c, r.mass_b}; }
inline uint32_t request_massive(const vsh_request& r) { return r.mass_c > 0.0 || r.mass_b > 0.0 ? 1u : 0u; }
}  // namespace vsh
#include "vsh_persistent.hpp"

namespace vsh {

constexpr uint32_t kMaxCap = 1024;
constexpr double kMinTcut = 0.01;  // GeV^2; the one-loop Landau pole is at 0.0077 GeV^2

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct Arena {
  void* ptr = nullptr;
  uint64_t size = 0;
  vsh_status reserve(vsh_ctx* ctx, uint64_t bytes);
  void release();
};

// Pinned host memory for the copies back of vsh_generate (grown on demand).
struct HostStage {
  void* ptr = nullptr;
  uint64_t size = 0;
  vsh_status reserve(vsh_ctx* ctx, uint64_t bytes);
  void release();
};

struct PlainLayout {
  Records rec;
  uint64_t* cache;  // end cache of the flattened kernel, [event][cap] entries of kCacheWords words
  Scratch sc;
  Summary sum;
  double *ecm, *tcut, *hist;
  char* end;
};

// launch parameters picked by the autotuner (defaults until it has run)
struct Tuned {
  uint32_t plain_block = 64;
  uint32_t plain_waves = 3;       // register budget of the plain lane kernel: resident waves per SIMD
  uint32_t plain_mapping = 1;     // plain form: 0 lane per event, 1 flattened trials
  uint32_t pers_block = 256;
  uint32_t pers_waves_per_cu = 16;
  uint32_t refill_period = 1;      // veto cycles between compaction / refill passes
  uint32_t refill_threshold = 16;  // idle lanes needed before a wave refills
  uint32_t mapping = 1;           // persistent mapping: 0 lane per event, 1 flattened trials
};

struct ServeState;

}  // namespace vsh

struct vsh_ctx {
  int device = 0;
  int n_cu = 0;
  uint64_t budget = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t idle_ev[4] = {nullptr, nullptr, nullptr, nullptr};  // graph event nodes when not timing
  vsh::BatchGraph graph;
  vsh::Arena arena, arena2;
  vsh::HostStage stage;
  vsh::Tuned tuned;
  float tuned_ms = 0.0f;  // shower-kernel time of the autotuner's choice on its sample
  std::string tuner_cache_path;  // file of earlier tunings (empty: none)
  std::mutex mu;
  std::string error;
  vsh::ServeState* serve = nullptr;  // owned; torn down by serve_shutdown
  void* static_scratch = nullptr;    // device address of the static workspace on this device
  // stage timing of vsh_generate_into: 4 events per call
  bool timing = false;
  uint32_t timing_calls = 0;
  std::vector<hipEvent_t> timing_ev;
};

namespace vsh {

struct ResultBox {
  vsh_result pub;
  std::vector<double> hist, lo, hi, sum_d;
  std::vector<int32_t> sum_i;
  std::vector<uint64_t> hash, rec_offsets;
  std::vector<double> rec_p;
  std::vector<int8_t> rec_pid;
  std::vector<uint16_t> rec_col, rec_acol;
};

void set_error(vsh_ctx* ctx, const char* fmt, ...);
vsh_status hip_fail(vsh_ctx* ctx, hipError_t err, const char* what);
vsh_status validate_request(vsh_ctx* ctx, const vsh_request* req, bool need_energy);
ResultBox* new_result(uint64_t n_events, bool summary);
void finish_result(ResultBox* b);
void tally_chunk(ResultBox* b, const int32_t* si, const double* sd, uint64_t stride, uint64_t count);
void tally_fields(ResultBox* b, const int32_t* si0, uint64_t stride, const double* w, uint64_t count);
vsh_status copy_back_chunk(vsh_ctx* ctx, hipStream_t st, const double* dev_hist, const Summary& dev_sum,
                           uint64_t stride, uint64_t count, bool all_fields, ResultBox* box, uint64_t first_idx,
                           const int32_t** n_host);
uint64_t plain_layout_bytes(uint64_t stride, uint32_t cap, bool massive);
PlainLayout carve_plain(void* base, uint64_t stride, uint32_t cap, bool massive);

vsh_status gather_records(vsh_ctx* ctx, const Records& r, const int32_t* n_dev, const int32_t* n_host,
                          uint64_t count, ResultBox* box);

vsh_status generate_plain(vsh_ctx* ctx, const vsh_request* req, const uint64_t* offsets, const double* p,
                          const int8_t* pid, const uint16_t* col, const uint16_t* acol, vsh_result** out);

// persistent form (vsh_persistent.hip)
uint32_t persistent_lanes(const vsh_ctx* ctx);
uint64_t batch_bytes(uint64_t n, uint32_t cap, bool massive);
BatchLayout carve_batch(void* base, uint64_t n, uint32_t cap, bool massive);
vsh_status run_batch(vsh_ctx* ctx, const vsh_request* req, uint64_t first_idx, uint64_t n, hipStream_t st,
                     void* base, const double* ecm_dev, const double* tcut_dev, double* hist, bool use_graph,
                     BatchLayout* out_layout);
vsh_status generate_persistent(vsh_ctx* ctx, const vsh_request* req, vsh_result** out);
uint64_t persistent_workspace_bytes(const vsh_request* req);
hipEvent_t* timing_slot(vsh_ctx* ctx);
vsh_status persistent_into(vsh_ctx* ctx, const vsh_request* req, hipStream_t st, void* ws,
                           double* dev_hist, double* dev_sum_d, int32_t* dev_sum_i,
                           uint64_t* dev_hash);

vsh_status plain_into(vsh_ctx* ctx, const vsh_request* req, hipStream_t st, void* ws, double* dev_hist,
                      double* dev_sum_d, int32_t* dev_sum_i, uint64_t* dev_hash, bool timed);

// the library-owned workspace of vsh_generate_into_static (vsh_noalloc.hip):
// its device address on the current device, looked up once per device
vsh_status static_scratch_init(vsh_ctx* ctx);

// serving (vsh_serve.hip)
void serve_shutdown(vsh_ctx* ctx);

}  // namespace vsh
