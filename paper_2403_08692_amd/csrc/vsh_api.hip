// vsh_api.hip -- the C ABI of libvsh (include/vsh.h): contexts, the device
// arena, request validation, the blocking and device-side generation calls
// and the caller-supplied-start shower.  Serving lives in vsh_serve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/vsh.h"
#include "vsh_internal.hpp"

namespace vsh {

thread_local std::string g_create_error;

void set_error(vsh_ctx* ctx, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->error = buf;
  else g_create_error = buf;
}

vsh_status hip_fail(vsh_ctx* ctx, hipError_t err, const char* what) {
  set_error(ctx, "%s: %s", what, hipGetErrorString(err));
  return VSH_E_DEVICE;
}

vsh_status validate_request(vsh_ctx* ctx, const vsh_request* req, bool need_energy) {
  if (!req) {
    set_error(ctx, "request is NULL");
    return VSH_E_INVALID;
  }
  if (req->n_events == 0) {
    set_error(ctx, "n_events must be >= 1");
    return VSH_E_INVALID;
  }
  if (req->n_events > (1ull << 32) - 1) {
    set_error(ctx, "n_events must be < 2^32 per request");
    return VSH_E_INVALID;
  }
  if (req->max_partons < 2 || req->max_partons > kMaxCap) {
    set_error(ctx, "max_partons must be in 2..%u (got %u)", kMaxCap, req->max_partons);
    return VSH_E_INVALID;
  }
  const uint32_t known = VSH_SUMMARY | VSH_RECORDS | VSH_FORM_PERSISTENT | VSH_INPUTS_ON_DEVICE | VSH_HIST_FIXEDPOINT;
  if (req->flags & ~known) {
    set_error(ctx, "unknown request flags 0x%x", req->flags & ~known);
    return VSH_E_INVALID;
  }
  const bool dev = req->flags & VSH_INPUTS_ON_DEVICE;
  if (need_energy && !req->ecm_per_event && !(req->ecm > 0.0)) {
    set_error(ctx, "ecm must be > 0 (got %g)", req->ecm);
    return VSH_E_INVALID;
  }
  if (!req->tcut_per_event && !(req->t_cut > kMinTcut)) {
    set_error(ctx, "t_cut must be > %g GeV^2 (got %g)", kMinTcut, req->t_cut);
    return VSH_E_INVALID;
  }
  if (!(req->mass_c >= 0.0 && std::isfinite(req->mass_c) && req->mass_b >= 0.0 && std::isfinite(req->mass_b))) {
    set_error(ctx, "quark masses must be finite and >= 0 (got c %g, b %g)", req->mass_c, req->mass_b);
    return VSH_E_INVALID;
  }
  if (!(req->t_over == 0.0 || (req->t_over > kMinTcut && std::isfinite(req->t_over)))) {
    set_error(ctx, "t_over must be 0 or a finite value > %g GeV^2 (got %g)", kMinTcut, req->t_over);
    return VSH_E_INVALID;
  }
  if (!dev) {
    if (need_energy && req->ecm_per_event)
      for (uint64_t e = 0; e < req->n_events; ++e)
        if (!(req->ecm_per_event[e] > 0.0)) {
          set_error(ctx, "ecm_per_event[%llu] must be > 0", (unsigned long long)e);
          return VSH_E_INVALID;
        }
    if (req->tcut_per_event)
      for (uint64_t e = 0; e < req->n_events; ++e)
        if (!(req->tcut_per_event[e] > kMinTcut)) {
          set_error(ctx, "tcut_per_event[%llu] must be > %g", (unsigned long long)e, kMinTcut);
          return VSH_E_INVALID;
        }
  }
  return VSH_OK;
}

// ---------------------------------------------------------------------------
// Plain-form device layout of a chunk of `stride` events with capacity cap:
// records, Durham scratch, summaries, per-event inputs, histogram.
// ---------------------------------------------------------------------------
uint64_t plain_bytes_per_event(uint32_t cap, bool massive) {
  return (uint64_t)cap * (4 * 8 + 1 + 4 * 2 + cache_words(massive) * 8) + kNSumD * 8 + kNSumI * 4 + 8 + 2 * 8;
}

uint64_t plain_layout_bytes(uint64_t stride, uint32_t cap, bool massive) {
  return align_up(plain_bytes_per_event(cap, massive) * stride + obs_scratch_bytes(stride, cap) + 20 * 256 +
                      kHistDoubles * 8, 256);
}

PlainLayout carve_plain(void* base, uint64_t stride, uint32_t cap, bool massive) {
  PlainLayout L;
  char* p = static_cast<char*>(base);
  auto take = [&](uint64_t bytes) {
    char* q = p;
    p += align_up(bytes, 256);
    return q;
  };
  const uint64_t slots = (uint64_t)cap * stride;
  L.rec.E = (double*)take(slots * 8);
  L.rec.x = (double*)take(slots * 8);
  L.rec.y = (double*)take(slots * 8);
  L.rec.z = (double*)take(slots * 8);
  L.rec.pid = (int8_t*)take(slots);
  L.rec.col = (uint16_t*)take(slots * 2);
  L.rec.acol = (uint16_t*)take(slots * 2);
  L.rec.cpart = (uint16_t*)take(slots * 2);
  L.rec.apart = (uint16_t*)take(slots * 2);
  L.rec.stride = stride;
  L.rec.cap = cap;
  L.cache = (uint64_t*)take(slots * cache_words(massive) * 8);
  {
    char* q = p;
    L.sc = carve_obs_scratch(q, stride, cap);
    p = q;
  }
  L.sum.d = (double*)take(kNSumD * stride * 8);
  L.sum.i = (int32_t*)take(kNSumI * stride * 4);
  L.sum.hash = (uint64_t*)take(stride * 8);
  L.sum.stride = stride;
  L.ecm = (double*)take(stride * 8);
  L.tcut = (double*)take(stride * 8);
  L.hist = (double*)take(kHistDoubles * 8);
  L.end = p;
  return L;
}

vsh_status Arena::reserve(vsh_ctx* ctx, uint64_t bytes) {
  if (bytes <= size) return VSH_OK;
  if (ptr) {
    (void)hipFree(ptr);
    ptr = nullptr;
    size = 0;
  }
  hipError_t err = hipMalloc(&ptr, bytes);
  if (err != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    set_error(ctx, "device arena of %llu bytes: %s", (unsigned long long)bytes, hipGetErrorString(err));
    return VSH_E_NOMEM;
  }
  size = bytes;
  return VSH_OK;
}

void Arena::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  size = 0;
}

vsh_status HostStage::reserve(vsh_ctx* ctx, uint64_t bytes) {
  if (bytes <= size) return VSH_OK;
  release();
  hipError_t err = hipHostMalloc(&ptr, bytes, 0);
  if (err != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    set_error(ctx, "pinned host staging of %llu bytes: %s", (unsigned long long)bytes, hipGetErrorString(err));
    return VSH_E_NOMEM;
  }
  size = bytes;
  return VSH_OK;
}

void HostStage::release() {
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  size = 0;
}

// ---------------------------------------------------------------------------
// result assembly
// ---------------------------------------------------------------------------
ResultBox* new_result(uint64_t n_events, bool summary) {
  ResultBox* b = new (std::nothrow) ResultBox();
  if (!b) return nullptr;
  b->hist.assign(kHistDoubles, 0.0);
  b->lo.assign(kNObs, 0.0);
  b->hi.assign(kNObs, 0.0);
  static const double L[kNObs] = {-4.3, -4.3, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0};
  static const double H[kNObs] = {-0.3, -0.3, 0.5, 1.0, 0.5, 0.5, 0.35, 1.0};
  for (int h = 0; h < kNObs; ++h) {
    b->lo[h] = L[h];
    b->hi[h] = H[h];
  }
  if (summary) {
    b->sum_d.assign((size_t)kNSumD * n_events, 0.0);
    b->sum_i.assign((size_t)kNSumI * n_events, 0);
    b->hash.assign(n_events, 0);
  }
  std::memset(&b->pub, 0, sizeof b->pub);
  b->pub.n_events = n_events;
  b->pub.n_obs = kNObs;
  b->pub.n_bins = kNBins;
  return b;
}

void finish_result(ResultBox* b) {
  vsh_result& r = b->pub;
  r.hist_lo = b->lo.data();
  r.hist_hi = b->hi.data();
  r.hist = b->hist.data();
  r.sum_d = b->sum_d.empty() ? nullptr : b->sum_d.data();
  r.sum_i = b->sum_i.empty() ? nullptr : b->sum_i.data();
  r.sum_hash = b->hash.empty() ? nullptr : b->hash.data();
  if (!b->rec_offsets.empty()) {
    r.rec_offsets = b->rec_offsets.data();
    r.rec_p = b->rec_p.data();
    r.rec_pid = b->rec_pid.data();
    r.rec_col = b->rec_col.data();
    r.rec_acol = b->rec_acol.data();
  }
}

// Fold one chunk's per-event ints/doubles into the result counters.
// The result's counts and sums over count events, from the summary fields
// [field][stride] (only status, cycles, emissions, trials, active ends and
// the weight are read).
void tally_chunk(ResultBox* b, const int32_t* si, const double* sd, uint64_t stride, uint64_t count) {
  vsh_result& r = b->pub;
  for (uint64_t e = 0; e < count; ++e) {
    const int st = si[kSiStatus * stride + e];
    r.n_done += st == kDone;
    r.n_overflow += st == kOverflow;
    r.n_nonfinite += st == kNonFinite;
    r.n_conservation += st == kConservation;
    r.n_cycle_limit += st == kCycleLimitHit;
    const double w = sd[kSdW * stride + e];
    r.sum_w += w;
    r.sum_w2 += w * w;
    const uint32_t cyc = (uint32_t)si[kSiCycles * stride + e];
    r.total_cycles += cyc;
    r.max_cycles = std::max(r.max_cycles, cyc);
    r.total_trials += (uint32_t)si[kSiTrials * stride + e];
    r.total_ends += (uint32_t)si[kSiEnds * stride + e];
    r.total_emissions += (uint32_t)si[kSiEmit * stride + e];
  }
}

// The counts and sums of count events from the integer summary fields
// kSiStatus .. kSiEnds (field f at si0[(f - kSiStatus) * stride]) and the
// weights w.
void tally_fields(ResultBox* b, const int32_t* si0, uint64_t stride, const double* w, uint64_t count) {
  vsh_result& r = b->pub;
  for (uint64_t e = 0; e < count; ++e) {
    const int s_ = si0[e];
    r.n_done += s_ == kDone;
    r.n_overflow += s_ == kOverflow;
    r.n_nonfinite += s_ == kNonFinite;
    r.n_conservation += s_ == kConservation;
    r.n_cycle_limit += s_ == kCycleLimitHit;
    r.sum_w += w[e];
    r.sum_w2 += w[e] * w[e];
    const uint32_t cyc = (uint32_t)si0[(kSiCycles - kSiStatus) * stride + e];
    r.total_cycles += cyc;
    r.max_cycles = std::max(r.max_cycles, cyc);
    r.total_trials += (uint32_t)si0[(kSiTrials - kSiStatus) * stride + e];
    r.total_ends += (uint32_t)si0[(kSiEnds - kSiStatus) * stride + e];
    r.total_emissions += (uint32_t)si0[(kSiEmit - kSiStatus) * stride + e];
  }
}

// Copy a chunk's results back through the pinned staging buffer: the
// histogram, and either every summary field (requested summaries or records)
// or only the fields the counts read (the weight, then the integer fields
// from status to active ends); tally them, add the histogram and, with
// summaries, place the fields in the result.  *n_host (optional) points at
// the staged parton counts when all fields were copied.
vsh_status copy_back_chunk(vsh_ctx* ctx, hipStream_t st, const double* dev_hist, const Summary& dev_sum,
                           uint64_t stride, uint64_t count, bool all_fields, ResultBox* box, uint64_t first_idx,
                           const int32_t** n_host) {
  static_assert(kSiStatus == 1 && kSiEnds == kNSumI - 1, "the counted integer fields are the last ones");
  const uint64_t hist_b = align_up(kHistDoubles * 8, 256);
  const uint64_t d_fields = all_fields ? kNSumD : 1, i_fields = all_fields ? kNSumI : kNSumI - kSiStatus;
  const uint64_t d_b = align_up(d_fields * stride * 8, 256), i_b = align_up(i_fields * stride * 4, 256);
  const uint64_t h_b = all_fields ? align_up(stride * 8, 256) : 0;
  vsh_status rc = ctx->stage.reserve(ctx, hist_b + d_b + i_b + h_b);
  if (rc) return rc;
  char* base = static_cast<char*>(ctx->stage.ptr);
  double* hh = reinterpret_cast<double*>(base);
  double* sd = reinterpret_cast<double*>(base + hist_b);
  int32_t* si = reinterpret_cast<int32_t*>(base + hist_b + d_b);
  uint64_t* hs = reinterpret_cast<uint64_t*>(base + hist_b + d_b + i_b);
  hipError_t err = hipMemcpyAsync(hh, dev_hist, kHistDoubles * 8, hipMemcpyDeviceToHost, st);
  if (all_fields) {
    if (err == hipSuccess) err = hipMemcpyAsync(sd, dev_sum.d, kNSumD * stride * 8, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipMemcpyAsync(si, dev_sum.i, kNSumI * stride * 4, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipMemcpyAsync(hs, dev_sum.hash, stride * 8, hipMemcpyDeviceToHost, st);
  } else {
    if (err == hipSuccess)
      err = hipMemcpyAsync(sd, dev_sum.d + kSdW * stride, stride * 8, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess)
      err = hipMemcpyAsync(si, dev_sum.i + kSiStatus * stride, i_fields * stride * 4, hipMemcpyDeviceToHost, st);
  }
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err != hipSuccess) return hip_fail(ctx, err, "result copy");
  for (int a = 0; a < kHistDoubles; ++a) box->hist[a] += hh[a];
  const int32_t* si0 = all_fields ? si + kSiStatus * stride : si;  // field kSiStatus onwards
  tally_fields(box, si0, stride, all_fields ? sd + kSdW * stride : sd, count);
  if (all_fields && !box->sum_d.empty()) {
    const uint64_t N = box->pub.n_events;
    for (int f = 0; f < kNSumD; ++f) std::memcpy(&box->sum_d[f * N + first_idx], &sd[f * stride], count * 8);
    for (int f = 0; f < kNSumI; ++f) std::memcpy(&box->sum_i[f * N + first_idx], &si[f * stride], count * 4);
    std::memcpy(&box->hash[first_idx], hs, count * 8);
  }
  if (n_host) *n_host = all_fields ? si + kSiN * stride : nullptr;
  return VSH_OK;
}

// gather the final partons of a chunk into CSR order
__global__ void k_gather_records(Records r, const int32_t* __restrict__ n_of, const uint64_t* __restrict__ off,
                                 uint32_t n, double* __restrict__ p, int8_t* __restrict__ pid,
                                 uint16_t* __restrict__ col, uint16_t* __restrict__ acol) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t o = off[e];
  const int np = n_of[e];
  for (int a = 0; a < np; ++a) {
    const uint64_t s = (uint64_t)a * r.stride + e;
    p[4 * (o + a) + 0] = r.E[s];
    p[4 * (o + a) + 1] = r.x[s];
    p[4 * (o + a) + 2] = r.y[s];
    p[4 * (o + a) + 3] = r.z[s];
    pid[o + a] = r.pid[s];
    col[o + a] = r.col[s];
    acol[o + a] = r.acol[s];
  }
}

// Append the final partons of `count` events held slot-major in r (parton
// counts n_dev on the device, n_host on the host) to box's CSR records.
vsh_status gather_records(vsh_ctx* ctx, const Records& r, const int32_t* n_dev, const int32_t* n_host,
                          uint64_t count, ResultBox* box) {
  hipStream_t st = ctx->stream;
  std::vector<uint64_t> off(count + 1, 0);
  for (uint64_t e = 0; e < count; ++e) off[e + 1] = off[e] + (uint64_t)n_host[e];
  const uint64_t total = off[count];
  const uint64_t need = align_up((count + 1) * 8, 256) + align_up(total * 32, 256) + align_up(total, 256) +
                        2 * align_up(total * 2, 256) + 256;
  vsh_status rc = ctx->arena2.reserve(ctx, need);
  if (rc) return rc;
  char* q = (char*)ctx->arena2.ptr;
  uint64_t* d_off = (uint64_t*)q;
  q += align_up((count + 1) * 8, 256);
  double* d_p = (double*)q;
  q += align_up(total * 32, 256);
  int8_t* d_pid = (int8_t*)q;
  q += align_up(total, 256);
  uint16_t* d_col = (uint16_t*)q;
  q += align_up(total * 2, 256);
  uint16_t* d_acol = (uint16_t*)q;
  hipError_t err = hipMemcpyAsync(d_off, off.data(), (count + 1) * 8, hipMemcpyHostToDevice, st);
  if (err != hipSuccess) return hip_fail(ctx, err, "offset copy");
  hipLaunchKernelGGL(k_gather_records, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, st, r, n_dev,
                     (const uint64_t*)d_off, (uint32_t)count, d_p, d_pid, d_col, d_acol);
  err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(ctx, err, "k_gather_records");
  const uint64_t base = box->rec_offsets.empty() ? 0 : box->rec_offsets.back();
  if (box->rec_offsets.empty()) box->rec_offsets.push_back(0);
  for (uint64_t e = 0; e < count; ++e) box->rec_offsets.push_back(base + off[e + 1]);
  box->rec_p.resize((base + total) * 4);
  box->rec_pid.resize(base + total);
  box->rec_col.resize(base + total);
  box->rec_acol.resize(base + total);
  if (total) {
    err = hipMemcpyAsync(&box->rec_p[base * 4], d_p, total * 32, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipMemcpyAsync(&box->rec_pid[base], d_pid, total, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipMemcpyAsync(&box->rec_col[base], d_col, total * 2, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipMemcpyAsync(&box->rec_acol[base], d_acol, total * 2, hipMemcpyDeviceToHost, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "record copy");
  }
  err = hipStreamSynchronize(st);
  if (err != hipSuccess) return hip_fail(ctx, err, "hipStreamSynchronize");
  return VSH_OK;
}

// ---------------------------------------------------------------------------
// One chunk through the plain pipeline on ctx->stream.
// ---------------------------------------------------------------------------
struct ChunkTimes {
  float me = 0, shower = 0, obs = 0;
};

static vsh_status run_plain_chunk(vsh_ctx* ctx, const vsh_request* req, uint64_t first_idx,
                                  uint64_t count, const uint64_t* caller_offsets,
                                  const double* cp, const int8_t* cpid, const uint16_t* ccol,
                                  const uint16_t* cacol, ResultBox* box, ChunkTimes& tm) {
  hipStream_t st = ctx->stream;
  const uint32_t cap = req->max_partons;
  const uint64_t stride = align_up(count, 64);
  const bool massive = request_massive(*req) != 0;
  vsh_status rc = ctx->arena.reserve(ctx, plain_layout_bytes(stride, cap, massive));
  if (rc) return rc;
  PlainLayout L = carve_plain(ctx->arena.ptr, stride, cap, massive);
  hipError_t err;
#define HIPCHK(x)                                 \
  do {                                            \
    err = (x);                                    \
    if (err != hipSuccess) return hip_fail(ctx, err, #x); \
  } while (0)
  HIPCHK(hipMemsetAsync(L.hist, 0, kHistDoubles * 8, st));
  EventInputs in{};
  in.seed = req->seed;
  in.first = req->first_event + first_idx;
  in.cycle_limit = effective_cycle_limit(req->cycle_limit);
  in.t_over = req->t_over;
  in.qm = request_masses(*req);
  in.massive = request_massive(*req);
  in.fixed_hist = (req->flags & VSH_HIST_FIXEDPOINT) ? 1u : 0u;
  in.ecm0 = req->ecm;
  in.tcut0 = req->t_cut;
  const bool from_records = caller_offsets != nullptr;
  std::vector<double> ecm_host;
  if (from_records) {
    ecm_host.resize(count);
    for (uint64_t e = 0; e < count; ++e) {
      double s = 0.0;
      for (uint64_t a = caller_offsets[first_idx + e]; a < caller_offsets[first_idx + e + 1]; ++a) s += cp[4 * a];
      ecm_host[e] = s;
    }
    HIPCHK(hipMemcpyAsync(L.ecm, ecm_host.data(), count * 8, hipMemcpyHostToDevice, st));
    in.ecm = L.ecm;
  } else if (req->ecm_per_event) {
    HIPCHK(hipMemcpyAsync(L.ecm, req->ecm_per_event + first_idx, count * 8, hipMemcpyHostToDevice, st));
    in.ecm = L.ecm;
  }
  if (req->tcut_per_event) {
    HIPCHK(hipMemcpyAsync(L.tcut, req->tcut_per_event + first_idx, count * 8, hipMemcpyHostToDevice, st));
    in.tcut = L.tcut;
  }
  HIPCHK(hipEventRecord(ctx->ev[0], st));
  if (from_records) {
    // scatter the caller's partons into the slot-major records on the host
    const uint64_t slots = (uint64_t)cap * stride;
    std::vector<double> hE(slots, 0.0), hx(slots, 0.0), hy(slots, 0.0), hz(slots, 0.0);
    std::vector<int8_t> hpid(slots, 0);
    std::vector<uint16_t> hc(slots, 0), ha(slots, 0);
    std::vector<int32_t> hn(count);
    std::vector<double> hw(count, 1.0);
    for (uint64_t e = 0; e < count; ++e) {
      const uint64_t b0 = caller_offsets[first_idx + e], b1 = caller_offsets[first_idx + e + 1];
      hn[e] = (int32_t)(b1 - b0);
      for (uint64_t a = b0; a < b1; ++a) {
        const uint64_t s = (a - b0) * stride + e;
        hE[s] = cp[4 * a];
        hx[s] = cp[4 * a + 1];
        hy[s] = cp[4 * a + 2];
        hz[s] = cp[4 * a + 3];
        hpid[s] = cpid[a];
        hc[s] = ccol[a];
        ha[s] = cacol[a];
      }
    }
    HIPCHK(hipMemcpy(L.rec.E, hE.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.rec.x, hx.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.rec.y, hy.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.rec.z, hz.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.rec.pid, hpid.data(), slots, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.rec.col, hc.data(), slots * 2, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.rec.acol, ha.data(), slots * 2, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(L.sum.i + kSiN * stride, hn.data(), count * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemsetAsync(L.sum.d, 0, kNSumD * stride * 8, st));
    HIPCHK(hipMemsetAsync(L.sum.i + kSiFlavour * stride, 0, stride * 4, st));
    launch_shower_init_records(L.rec, L.sum, in, (uint32_t)count, st);
  } else {
    launch_me(L.rec, L.sum, in, (uint32_t)count, st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev[1], st));
  if (ctx->tuned.plain_mapping == kMapFlat) launch_shower_plain_flat(L.rec, L.sum, in, (uint32_t)count, L.cache, st);
  else launch_shower_plain(L.rec, L.sum, in, (uint32_t)count, ctx->tuned.plain_block, ctx->tuned.plain_waves, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev[2], st));
  launch_obs(L.rec, L.sum, in, L.sc, (uint32_t)count, L.hist, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev[3], st));
  // copy back: the histogram and the summary fields the counts need (all of
  // them for summaries or records)
  const bool all_fields = !box->sum_d.empty() || (req->flags & VSH_RECORDS);
  const int32_t* n_host = nullptr;
  rc = copy_back_chunk(ctx, st, L.hist, L.sum, stride, count, all_fields, box, first_idx, &n_host);
  if (rc) return rc;
  float ms;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  tm.me += ms;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
  tm.shower += ms;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
  tm.obs += ms;
  if (req->flags & VSH_RECORDS) {
    rc = gather_records(ctx, L.rec, L.sum.i + kSiN * stride, n_host, count, box);
    if (rc) return rc;
  }
#undef HIPCHK
  return VSH_OK;
}

uint64_t chunk_events(vsh_ctx* ctx, const vsh_request* req) {
  const uint64_t per = plain_bytes_per_event(req->max_partons, request_massive(*req) != 0);
  uint64_t budget = ctx->budget;
  // leave room for the record-gather buffer when records are returned
  if (req->flags & VSH_RECORDS) budget = budget / 2;
  uint64_t n = budget / (per + 64);
  n = std::min<uint64_t>(n, 1ull << 26);
  if (n >= req->n_events) return req->n_events;  // the whole request in one piece
  return n & ~63ull ? n & ~63ull : n;
}

vsh_status generate_plain(vsh_ctx* ctx, const vsh_request* req, const uint64_t* offsets,
                          const double* p, const int8_t* pid, const uint16_t* col,
                          const uint16_t* acol, vsh_result** out) {
  const auto t0 = std::chrono::steady_clock::now();
  const uint64_t chunk = chunk_events(ctx, req);
  if (chunk == 0) {
    set_error(ctx, "memory budget of %llu bytes cannot hold one event of %u partons",
              (unsigned long long)ctx->budget, req->max_partons);
    return VSH_E_NOMEM;
  }
  ResultBox* box = new_result(req->n_events, req->flags & VSH_SUMMARY);
  if (!box) {
    set_error(ctx, "host allocation failed");
    return VSH_E_NOMEM;
  }
  ChunkTimes tm;
  for (uint64_t a = 0; a < req->n_events; a += chunk) {
    const uint64_t count = std::min(chunk, req->n_events - a);
    vsh_status rc = run_plain_chunk(ctx, req, a, count, offsets, p, pid, col, acol, box, tm);
    if (rc) {
      delete box;
      return rc;
    }
  }
  box->pub.t_me_ms = tm.me;
  box->pub.t_shower_ms = tm.shower;
  box->pub.t_obs_ms = tm.obs;
  box->pub.t_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  finish_result(box);
  *out = &box->pub;
  return VSH_OK;
}

// events of the next timed vsh_generate_into call, or null when not timing
hipEvent_t* timing_slot(vsh_ctx* ctx) {
  if (!ctx->timing || ctx->timing_calls >= VSH_TIMING_MAX_CALLS) return nullptr;
  const size_t need = 4 * (size_t)(ctx->timing_calls + 1);
  while (ctx->timing_ev.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->timing_ev.push_back(e);
  }
  return &ctx->timing_ev[4 * (size_t)ctx->timing_calls++];
}

// The plain-form launch sequence of vsh_generate_into on stream st with the
// workspace at `ws` (at least vsh_workspace_size bytes; nothing in it needs
// to start at zero): matrix element, shower, observables and histogram
// accumulated into dev_hist, then the summaries copied out in the caller's
// [field][n_events] layout; when n is a multiple of 64 that layout is the
// kernels' own, so they work in the caller's summary buffers directly and
// nothing is copied.  `timed`: record the stage events of vsh_timing_start.
// Launches and device-to-device copies only.
vsh_status plain_into(vsh_ctx* ctx, const vsh_request* req, hipStream_t st, void* ws, double* dev_hist,
                      double* dev_sum_d, int32_t* dev_sum_i, uint64_t* dev_hash, bool timed) {
  const uint64_t n = req->n_events;
  const uint64_t stride = align_up(n, 64);
  PlainLayout L = carve_plain(ws, stride, req->max_partons, request_massive(*req) != 0);
  EventInputs in{};
  in.seed = req->seed;
  in.first = req->first_event;
  in.cycle_limit = effective_cycle_limit(req->cycle_limit);
  in.t_over = req->t_over;
  in.qm = request_masses(*req);
  in.massive = request_massive(*req);
  in.fixed_hist = (req->flags & VSH_HIST_FIXEDPOINT) ? 1u : 0u;
  in.ecm0 = req->ecm;
  in.tcut0 = req->t_cut;
  in.ecm = req->ecm_per_event;
  in.tcut = req->tcut_per_event;
  Summary sum = L.sum;
  const bool direct = stride == n;  // the caller's [field][n] arrays have the kernels' stride
  if (direct && dev_sum_d) sum.d = dev_sum_d;
  if (direct && dev_sum_i) sum.i = dev_sum_i;
  if (direct && dev_hash) sum.hash = dev_hash;
  hipEvent_t* tev = timed ? timing_slot(ctx) : nullptr;
  if (tev) (void)hipEventRecord(tev[0], st);
  launch_me(L.rec, sum, in, (uint32_t)n, st);
  if (tev) (void)hipEventRecord(tev[1], st);
  if (ctx->tuned.plain_mapping == kMapFlat) launch_shower_plain_flat(L.rec, sum, in, (uint32_t)n, L.cache, st);
  else launch_shower_plain(L.rec, sum, in, (uint32_t)n, ctx->tuned.plain_block, ctx->tuned.plain_waves, st);
  if (tev) (void)hipEventRecord(tev[2], st);
  launch_obs(L.rec, sum, in, L.sc, (uint32_t)n, dev_hist, st);
  if (tev) (void)hipEventRecord(tev[3], st);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(ctx, err, "kernel launch");
  // summaries out, in the caller's [field][n_events] layout
  if (direct) return VSH_OK;
  if (dev_sum_d) {
    err = hipMemcpy2DAsync(dev_sum_d, n * 8, sum.d, stride * 8, n * 8, kNSumD, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "summary copy");
  }
  if (dev_sum_i) {
    err = hipMemcpy2DAsync(dev_sum_i, n * 4, sum.i, stride * 4, n * 4, kNSumI, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "summary copy");
  }
  if (dev_hash) {
    err = hipMemcpyAsync(dev_hash, sum.hash, n * 8, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "summary copy");
  }
  return VSH_OK;
}


}  // namespace vsh

using namespace vsh;

extern "C" {

vsh_status vsh_create(const vsh_ctx_opts* opts, vsh_ctx** out) {
  if (!out) {
    set_error(nullptr, "out is NULL");
    return VSH_E_INVALID;
  }
  *out = nullptr;
  const int dev = opts ? opts->device : 0;
  int count = 0;
  hipError_t err = hipGetDeviceCount(&count);
  if (err != hipSuccess || count == 0) {
    (void)hipGetLastError();
    set_error(nullptr, "no HIP device available (%s)", hipGetErrorString(err));
    return VSH_E_DEVICE;
  }
  if (dev < 0 || dev >= count) {
    set_error(nullptr, "device %d out of range (%d devices)", dev, count);
    return VSH_E_INVALID;
  }
  hipDeviceProp_t prop;
  err = hipGetDeviceProperties(&prop, dev);
  if (err != hipSuccess) return hip_fail(nullptr, err, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(nullptr, "device %d is %s; libvsh is built for gfx950 only", dev, prop.gcnArchName);
    return VSH_E_DEVICE;
  }
  err = hipSetDevice(dev);
  if (err != hipSuccess) return hip_fail(nullptr, err, "hipSetDevice");
  vsh_ctx* ctx = new (std::nothrow) vsh_ctx();
  if (!ctx) {
    set_error(nullptr, "host allocation failed");
    return VSH_E_NOMEM;
  }
  ctx->device = dev;
  ctx->n_cu = prop.multiProcessorCount;
  size_t free_b = 0, total_b = 0;
  err = hipMemGetInfo(&free_b, &total_b);
  if (err != hipSuccess) {
    delete ctx;
    return hip_fail(nullptr, err, "hipMemGetInfo");
  }
  ctx->budget = (opts && opts->mem_budget_bytes) ? opts->mem_budget_bytes : (uint64_t)(0.8 * (double)free_b);
  if (opts && opts->tuner_cache_path) ctx->tuner_cache_path = opts->tuner_cache_path;
  err = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
  if (err != hipSuccess) {
    delete ctx;
    return hip_fail(nullptr, err, "hipStreamCreate");
  }
  for (auto& e : ctx->idle_ev) {
    err = hipEventCreate(&e);
    if (err != hipSuccess) {
      delete ctx;
      return hip_fail(nullptr, err, "hipEventCreate");
    }
  }
  for (auto& e : ctx->ev) {
    err = hipEventCreate(&e);
    if (err != hipSuccess) {
      delete ctx;
      return hip_fail(nullptr, err, "hipEventCreate");
    }
  }
  // the static workspace's address on this device (vsh_generate_into_static
  // looks it up itself if this fails; nothing else depends on it)
  (void)static_scratch_init(ctx);
  ctx->error.clear();
  *out = ctx;
  return VSH_OK;
}

void vsh_destroy(vsh_ctx* ctx) {
  if (!ctx) return;
  serve_shutdown(ctx);
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->arena.release();
  ctx->arena2.release();
  ctx->stage.release();
  for (auto& e : ctx->timing_ev) (void)hipEventDestroy(e);
  destroy_graph(ctx->graph);
  for (auto& e : ctx->idle_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* vsh_last_error(const vsh_ctx* ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->error.c_str();
}

vsh_status vsh_generate(vsh_ctx* ctx, const vsh_request* req, vsh_result** out) {
  if (!ctx || !out) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = nullptr;
  vsh_status rc = validate_request(ctx, req, true);
  if (rc) return rc;
  if (req->flags & VSH_INPUTS_ON_DEVICE) {
    set_error(ctx, "VSH_INPUTS_ON_DEVICE is for vsh_generate_into only");
    return VSH_E_INVALID;
  }
  (void)hipSetDevice(ctx->device);
  if (req->flags & VSH_FORM_PERSISTENT) return generate_persistent(ctx, req, out);
  return generate_plain(ctx, req, nullptr, nullptr, nullptr, nullptr, nullptr, out);
}

void vsh_result_free(vsh_result* res) {
  if (!res) return;
  delete reinterpret_cast<ResultBox*>(reinterpret_cast<char*>(res) - offsetof(ResultBox, pub));
}

vsh_status vsh_shower_records(vsh_ctx* ctx, const vsh_request* req, const uint64_t* offsets,
                              const double* p, const int8_t* pid, const uint16_t* col,
                              const uint16_t* acol, vsh_result** out) {
  if (!ctx || !out) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = nullptr;
  vsh_status rc = validate_request(ctx, req, false);
  if (rc) return rc;
  if (!offsets || !p || !pid || !col || !acol) {
    set_error(ctx, "offsets, p, pid, col and acol are required");
    return VSH_E_INVALID;
  }
  if (req->flags & (VSH_INPUTS_ON_DEVICE | VSH_FORM_PERSISTENT)) {
    set_error(ctx, "vsh_shower_records runs the plain form with host inputs");
    return VSH_E_INVALID;
  }
  for (uint64_t e = 0; e < req->n_events; ++e) {
    if (offsets[e + 1] < offsets[e] || offsets[e + 1] - offsets[e] > req->max_partons ||
        offsets[e + 1] - offsets[e] < 2) {
      set_error(ctx, "event %llu: parton count must be in 2..max_partons", (unsigned long long)e);
      return VSH_E_INVALID;
    }
    // every colour line must have exactly one start and one end
    std::vector<int> seen_c(kMaxCap * 2 + 2, 0), seen_a(kMaxCap * 2 + 2, 0);
    double E = 0.0;
    for (uint64_t a = offsets[e]; a < offsets[e + 1]; ++a) {
      const int f = pid[a];
      const bool q = f >= 1 && f <= 5, qb = f <= -1 && f >= -5, g = f == 21;
      if (!(q || qb || g) || (q && (col[a] == 0 || acol[a] != 0)) || (qb && (col[a] != 0 || acol[a] == 0)) ||
          (g && (col[a] == 0 || acol[a] == 0)) || col[a] > 2 * kMaxCap || acol[a] > 2 * kMaxCap) {
        set_error(ctx, "event %llu parton %llu: bad flavour/colour", (unsigned long long)e,
                  (unsigned long long)(a - offsets[e]));
        return VSH_E_INVALID;
      }
      if (col[a]) seen_c[col[a]]++;
      if (acol[a]) seen_a[acol[a]]++;
      E += p[4 * a];
    }
    for (size_t c = 0; c < seen_c.size(); ++c)
      if (seen_c[c] != seen_a[c] || seen_c[c] > 1) {
        set_error(ctx, "event %llu: colour line %zu is not closed once", (unsigned long long)e, c);
        return VSH_E_INVALID;
      }
    if (!(E > 0.0)) {
      set_error(ctx, "event %llu: total energy must be > 0", (unsigned long long)e);
      return VSH_E_INVALID;
    }
  }
  (void)hipSetDevice(ctx->device);
  return generate_plain(ctx, req, offsets, p, pid, col, acol, out);
}

uint64_t vsh_workspace_size(const vsh_request* req) {
  if (!req || req->n_events == 0 || req->max_partons < 2 || req->max_partons > kMaxCap) return 0;
  if (req->flags & VSH_FORM_PERSISTENT) return persistent_workspace_bytes(req);
  return plain_layout_bytes(align_up(req->n_events, 64), req->max_partons, request_massive(*req) != 0);
}

vsh_status vsh_generate_into(vsh_ctx* ctx, const vsh_request* req, void* stream, void* workspace,
                             uint64_t workspace_bytes, double* dev_hist, double* dev_sum_d,
                             int32_t* dev_sum_i, uint64_t* dev_hash) {
  if (!ctx) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  vsh_status rc = validate_request(ctx, req, true);
  if (rc) return rc;
  if (!workspace || !dev_hist) {
    set_error(ctx, "workspace and dev_hist are required");
    return VSH_E_INVALID;
  }
  if (req->flags & VSH_RECORDS) {
    set_error(ctx, "vsh_generate_into returns summaries and histograms only");
    return VSH_E_INVALID;
  }
  const uint64_t need = vsh_workspace_size(req);
  if (workspace_bytes < need) {
    set_error(ctx, "workspace of %llu bytes is smaller than the %llu needed", (unsigned long long)workspace_bytes,
              (unsigned long long)need);
    return VSH_E_INVALID;
  }
  const bool dev_inputs = req->flags & VSH_INPUTS_ON_DEVICE;
  if (!dev_inputs && (req->ecm_per_event || req->tcut_per_event)) {
    set_error(ctx, "per-event arrays of vsh_generate_into must be device pointers (VSH_INPUTS_ON_DEVICE)");
    return VSH_E_INVALID;
  }
  (void)hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  if (req->flags & VSH_FORM_PERSISTENT)
    return persistent_into(ctx, req, st, workspace, dev_hist, dev_sum_d, dev_sum_i, dev_hash);
  return plain_into(ctx, req, st, workspace, dev_hist, dev_sum_d, dev_sum_i, dev_hash, true);
}

vsh_status vsh_timing_start(vsh_ctx* ctx) {
  if (!ctx) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->timing = true;
  ctx->timing_calls = 0;
  return VSH_OK;
}

vsh_status vsh_timing_read(vsh_ctx* ctx, float* ms, uint32_t max_calls, uint32_t* n_calls) {
  if (!ctx) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->timing) {
    set_error(ctx, "vsh_timing_read without vsh_timing_start");
    return VSH_E_INVALID;
  }
  const uint32_t n = std::min(ctx->timing_calls, max_calls);
  for (uint32_t c = 0; c < n; ++c) {
    hipEvent_t* e = &ctx->timing_ev[4 * (size_t)c];
    hipError_t err = hipEventSynchronize(e[3]);
    if (err != hipSuccess) return hip_fail(ctx, err, "hipEventSynchronize");
    for (int k = 0; k < 3; ++k) {
      float v = 0.0f;
      err = hipEventElapsedTime(&v, e[k], e[k + 1]);
      if (err != hipSuccess) return hip_fail(ctx, err, "hipEventElapsedTime");
      if (ms) ms[3 * c + k] = v;
    }
  }
  if (n_calls) *n_calls = n;
  ctx->timing = false;
  ctx->timing_calls = 0;
  return VSH_OK;
}

}  // extern "C"
