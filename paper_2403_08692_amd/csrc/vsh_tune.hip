// vsh_tune.hip -- launch-parameter tuning of the two forms.
//
// The autotuner times candidate settings on a sample of the caller's
// workload with HIP events around the shower kernel, checks that every
// candidate produces the same per-event summaries as the first (the events
// do not depend on the launch shape), and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "vsh_internal.hpp"

namespace vsh {

static uint32_t clampu(uint32_t v, uint32_t lo, uint32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static uint32_t block_choice(uint32_t b) { return b <= 64 ? 64 : (b <= 128 ? 128 : 256); }

static vsh_tuning to_pub(const Tuned& t) {
  vsh_tuning p{};
  p.plain_block = t.plain_block;
  p.plain_waves = t.plain_waves;
  p.plain_mapping = t.plain_mapping;
  p.mapping = t.mapping;
  p.waves_per_cu = t.pers_waves_per_cu;
  p.block = t.pers_block;
  p.refill_threshold = t.refill_threshold;
  p.refill_period = t.refill_period;
  return p;
}

static Tuned from_pub(const vsh_tuning& p) {
  Tuned t;
  t.plain_block = block_choice(p.plain_block);
  t.plain_waves = clampu(p.plain_waves, 2, 4);
  t.plain_mapping = p.plain_mapping ? kMapFlat : kMapLane;
  t.mapping = p.mapping ? kMapFlat : kMapLane;
  t.pers_waves_per_cu = clampu(p.waves_per_cu, 1, 16);
  t.pers_block = block_choice(p.block);
  t.refill_threshold = clampu(p.refill_threshold, 1, 64);
  t.refill_period = clampu(p.refill_period, 1, 64);
  return t;
}

// Time the persistent kernel of one batch (sample events [0, m)) under the
// settings in ctx->tuned; return its milliseconds and the summaries.
static vsh_status time_persistent(vsh_ctx* ctx, const vsh_request* req, uint64_t m, const double* ecm_dev,
                                  const double* tcut_dev, void* base, double* hist, float* ms,
                                  std::vector<int32_t>* si, std::vector<uint64_t>* hs) {
  const bool was = ctx->timing;
  const uint32_t was_calls = ctx->timing_calls;
  ctx->timing = true;
  ctx->timing_calls = 0;
  BatchLayout L;
  vsh_status rc = run_batch(ctx, req, 0, m, ctx->stream, base, ecm_dev, tcut_dev, hist, false, &L);
  hipError_t err = hipSuccess;
  if (!rc) err = hipStreamSynchronize(ctx->stream);
  if (!rc && err == hipSuccess) err = hipEventElapsedTime(ms, ctx->timing_ev[1], ctx->timing_ev[2]);
  ctx->timing = was;
  ctx->timing_calls = was_calls;
  if (rc) return rc;
  if (err != hipSuccess) return hip_fail(ctx, err, "autotune timing");
  if (si) {
    si->resize((size_t)kNSumI * m);
    hs->resize(m);
    err = hipMemcpy(si->data(), L.buf.sum.i, si->size() * 4, hipMemcpyDeviceToHost);
    if (err == hipSuccess) err = hipMemcpy(hs->data(), L.buf.sum.hash, m * 8, hipMemcpyDeviceToHost);
    if (err != hipSuccess) return hip_fail(ctx, err, "autotune copy");
  }
  return VSH_OK;
}

static vsh_status autotune_persistent(vsh_ctx* ctx, const vsh_request* req) {
  const uint64_t m = std::min<uint64_t>(req->n_events, 1ull << 18);
  const uint32_t cap = req->max_partons;
  const Tuned keep = ctx->tuned;
  const bool massive = request_massive(*req) != 0;
  const uint64_t need = batch_bytes(m, cap, massive);
  vsh_status rc = ctx->arena.reserve(ctx, need);
  if (rc) return rc;
  void* base = ctx->arena.ptr;
  BatchLayout L = carve_batch(base, m, cap, massive);
  hipError_t err;
  const double* ecm_dev = nullptr;
  const double* tcut_dev = nullptr;
  // the per-event inputs live outside the batch layout of any candidate
  rc = ctx->arena2.reserve(ctx, 2 * m * 8 + 2 * kHistDoubles * 8 + 512);
  if (rc) return rc;
  double* in_buf = (double*)ctx->arena2.ptr;
  double* hist = in_buf + 2 * m;
  (void)L;
  if (req->ecm_per_event) {
    err = hipMemcpy(in_buf, req->ecm_per_event, m * 8, hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(ctx, err, "autotune input");
    ecm_dev = in_buf;
  }
  if (req->tcut_per_event) {
    err = hipMemcpy(in_buf + m, req->tcut_per_event, m * 8, hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(ctx, err, "autotune input");
    tcut_dev = in_buf + m;
  }
  std::vector<Tuned> cands;
  for (uint32_t mapping : {kMapFlat, kMapLane})
    for (uint32_t waves : {4u, 8u, 16u})
      for (uint32_t thr : {16u, 32u})
        for (uint32_t per : {1u, 4u}) {
          Tuned t = keep;
          t.mapping = mapping;
          t.pers_waves_per_cu = waves;
          t.pers_block = 256;
          t.refill_threshold = thr;
          t.refill_period = per;
          cands.push_back(t);
        }
  std::vector<int32_t> ref_si, si;
  std::vector<uint64_t> ref_hs, hs;
  float best_ms = 1e30f;
  Tuned best = keep;
  for (size_t c = 0; c < cands.size(); ++c) {
    ctx->tuned = cands[c];
    float ms1 = 0, ms2 = 0;
    rc = time_persistent(ctx, req, m, ecm_dev, tcut_dev, base, hist, &ms1, c == 0 ? &ref_si : &si,
                         c == 0 ? &ref_hs : &hs);
    if (!rc) rc = time_persistent(ctx, req, m, ecm_dev, tcut_dev, base, hist, &ms2, nullptr, nullptr);
    if (rc) {
      ctx->tuned = keep;
      return rc;
    }
    if (c > 0 && (si != ref_si || hs != ref_hs)) {
      ctx->tuned = keep;
      set_error(ctx, "autotune: candidate %zu changed the events (internal error)", c);
      return VSH_E_INTERNAL;
    }
    const float ms = std::min(ms1, ms2);
    if (ms < best_ms) {
      best_ms = ms;
      best = cands[c];
    }
  }
  ctx->tuned = best;
  ctx->tuned_ms = best_ms;
  destroy_graph(ctx->graph);
  return VSH_OK;
}

static vsh_status autotune_plain(vsh_ctx* ctx, const vsh_request* req) {
  vsh_request r = *req;
  r.n_events = std::min<uint64_t>(req->n_events, 1ull << 18);
  r.flags = VSH_SUMMARY;
  const Tuned keep = ctx->tuned;
  float best_ms = 1e30f;
  Tuned best = keep;
  std::vector<int32_t> ref;
  struct Cand {
    uint32_t block, waves, mapping;
  };
  std::vector<Cand> cands{{64, 2, kMapFlat}};
  for (uint32_t w : {2u, 3u, 4u})
    for (uint32_t b : {256u, 64u}) cands.push_back({b, w, kMapLane});
  for (const Cand& cd : cands) {
    const uint32_t b = cd.block, wv = cd.waves;
    ctx->tuned.plain_block = b;
    ctx->tuned.plain_waves = wv;
    ctx->tuned.plain_mapping = cd.mapping;
    float ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      vsh_result* out = nullptr;
      vsh_status rc = generate_plain(ctx, &r, nullptr, nullptr, nullptr, nullptr, nullptr, &out);
      if (rc) {
        ctx->tuned = keep;
        return rc;
      }
      ms = std::min<float>(ms, (float)out->t_shower_ms);
      std::vector<int32_t> si(out->sum_i, out->sum_i + (size_t)kNSumI * r.n_events);
      vsh_result_free(out);
      if (ref.empty()) ref = si;
      else if (si != ref) {
        ctx->tuned = keep;
        set_error(ctx, "autotune: plain block %u changed the events (internal error)", b);
        (void)wv;
        return VSH_E_INTERNAL;
      }
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = ctx->tuned;
    }
  }
  ctx->tuned = keep;
  ctx->tuned.plain_block = best.plain_block;
  ctx->tuned.plain_waves = best.plain_waves;
  ctx->tuned.plain_mapping = best.plain_mapping;
  return VSH_OK;
}

// ---------------------------------------------------------------------------
// Tuner cache: one line per tuned sample, "<key> <8 settings> <ms>", appended
// after each tuning; the last line with a matching key wins.  The key names
// everything the choice depends on: library version, device (architecture
// and compute units), form, record capacity, sample size and the sample's
// physics (sqrt(s), t_C or a hash of the per-event arrays, masses, t_over,
// cycle limit).
// ---------------------------------------------------------------------------
static uint64_t fnv_bytes(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
  return h;
}

static std::string cache_key(const vsh_ctx* ctx, const vsh_request* req) {
  const uint64_t m = std::min<uint64_t>(req->n_events, 1ull << 18);
  uint64_t h = 0xcbf29ce484222325ull;
  if (req->ecm_per_event) h = fnv_bytes(h, req->ecm_per_event, m * 8);
  if (req->tcut_per_event) h = fnv_bytes(h, req->tcut_per_event, m * 8);
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "vsh%d.%d|gfx950|cu=%d|form=%s|cap=%u|n=%" PRIu64 "|ecm=%.17g|tcut=%.17g|arrays=%016" PRIx64
                "|mc=%.17g|mb=%.17g|tover=%.17g|climit=%u",
                VSH_VERSION_MAJOR, VSH_VERSION_MINOR, ctx->n_cu,
                (req->flags & VSH_FORM_PERSISTENT) ? "persistent" : "plain", req->max_partons, m,
                req->ecm_per_event ? 0.0 : req->ecm, req->tcut_per_event ? 0.0 : req->t_cut,
                (req->ecm_per_event || req->tcut_per_event) ? h : (uint64_t)0, req->mass_c, req->mass_b, req->t_over,
                req->cycle_limit);
  return buf;
}

// The cached settings of `key`, if the file has them.
static bool cache_lookup(const std::string& path, const std::string& key, vsh_tuning* t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    vsh_tuning v{};
    float ms = 0.0f;
    if (!(is >> k) || k != key) continue;
    if (is >> v.plain_block >> v.plain_waves >> v.plain_mapping >> v.mapping >> v.waves_per_cu >> v.block >>
        v.refill_threshold >> v.refill_period >> ms) {
      *t = v;
      found = true;
    }
  }
  return found;
}

static void cache_store(const std::string& path, const std::string& key, const vsh_tuning& v, float ms) {
  char buf[256];
  std::snprintf(buf, sizeof buf, " %u %u %u %u %u %u %u %u %.6g\n", v.plain_block, v.plain_waves, v.plain_mapping,
                v.mapping, v.waves_per_cu, v.block, v.refill_threshold, v.refill_period, ms);
  const std::string line = key + buf;
  if (FILE* f = std::fopen(path.c_str(), "a")) {  // one write per line: concurrent appends stay whole lines
    (void)std::fwrite(line.data(), 1, line.size(), f);
    std::fclose(f);
  }
}

}  // namespace vsh

using namespace vsh;

extern "C" {

vsh_status vsh_get_tuning(vsh_ctx* ctx, vsh_tuning* out) {
  if (!ctx || !out) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = to_pub(ctx->tuned);
  return VSH_OK;
}

vsh_status vsh_set_tuning(vsh_ctx* ctx, const vsh_tuning* t) {
  if (!ctx || !t) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->tuned = from_pub(*t);
  destroy_graph(ctx->graph);
  return VSH_OK;
}

vsh_status vsh_autotune(vsh_ctx* ctx, const vsh_request* sample, vsh_tuning* chosen) {
  if (!ctx) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  vsh_status rc = validate_request(ctx, sample, true);
  if (rc) return rc;
  if (sample->flags & VSH_INPUTS_ON_DEVICE) {
    set_error(ctx, "vsh_autotune takes host inputs");
    return VSH_E_INVALID;
  }
  (void)hipSetDevice(ctx->device);
  const bool persistent = (sample->flags & VSH_FORM_PERSISTENT) != 0;
  const std::string key = ctx->tuner_cache_path.empty() ? std::string() : cache_key(ctx, sample);
  vsh_tuning cached{};
  if (!key.empty() && cache_lookup(ctx->tuner_cache_path, key, &cached)) {
    const Tuned t = from_pub(cached);
    if (persistent) {  // only the form that was tuned takes the cached settings
      ctx->tuned.mapping = t.mapping;
      ctx->tuned.pers_waves_per_cu = t.pers_waves_per_cu;
      ctx->tuned.pers_block = t.pers_block;
      ctx->tuned.refill_threshold = t.refill_threshold;
      ctx->tuned.refill_period = t.refill_period;
      destroy_graph(ctx->graph);
    } else {
      ctx->tuned.plain_block = t.plain_block;
      ctx->tuned.plain_waves = t.plain_waves;
      ctx->tuned.plain_mapping = t.plain_mapping;
    }
    if (chosen) {
      *chosen = to_pub(ctx->tuned);
      chosen->from_cache = 1;
    }
    return VSH_OK;
  }
  rc = persistent ? autotune_persistent(ctx, sample) : autotune_plain(ctx, sample);
  if (rc) return rc;
  if (!key.empty()) cache_store(ctx->tuner_cache_path, key, to_pub(ctx->tuned), persistent ? ctx->tuned_ms : 0.0f);
  if (chosen) {
    *chosen = to_pub(ctx->tuned);
    chosen->from_cache = 0;
  }
  return VSH_OK;
}

}  // extern "C"
