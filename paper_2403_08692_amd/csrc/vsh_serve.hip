// vsh_serve.hip -- serving: continuous batching of event-generation requests.
//
// vsh_submit copies a request and returns a ticket.  A serving thread per
// context
//   * admits queued requests in arrival order while their event-record
//     memory (every event's final record at its request's capacity, the
//     summaries and the histogram) fits a device pool; a request that does
//     not fit yet waits, one that can never fit is rejected at submission;
//   * launches bounded epochs of the persistent shower kernel whose work list
//     holds segments of every admitted request with events left, oldest
//     first, so requests that arrive while others run join the next epoch;
//     two epochs may be in flight on two streams, the second filling compute
//     units the first's tail frees;
//   * when all events of a request are finished, computes its observables and
//     histogram on a drain stream, copies the result to the host and completes
//     the ticket, returning its memory to the pool.
// Every event is a pure function of (request seed, event id), so a request's
// events are the same alone or in any mix; only the summation order of its
// FP64 histogram can differ.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vsh_internal.hpp"

namespace vsh {

using Clock = std::chrono::steady_clock;

// first-fit sub-allocator over one device region (256-byte granules)
struct Pool {
  char* base = nullptr;
  uint64_t size = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length

  bool pinned = false;  // host memory (hipHostMalloc) instead of device memory

  hipError_t init(uint64_t bytes, bool host = false) {
    size = align_up(bytes, 256);
    pinned = host;
    hipError_t err = host ? hipHostMalloc((void**)&base, size, 0) : hipMalloc(&base, size);
    if (err != hipSuccess) {
      base = nullptr;
      size = 0;
      return err;
    }
    free_.clear();
    free_[0] = size;
    return hipSuccess;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = align_up(bytes, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes;
        const uint64_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = align_up(bytes, 256);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  void destroy() {
    if (base) (void)(pinned ? hipHostFree(base) : hipFree(base));
    base = nullptr;
    size = 0;
    free_.clear();
  }
};

enum ReqState { kQueued, kAdmitted, kDraining, kFinished, kCancelledState, kFailed };

struct ServeReq {
  uint64_t ticket = 0;
  vsh_request req{};
  std::vector<double> ecm, tcut;
  Clock::time_point t_arrival;
  int state = kQueued;
  bool cancel = false;
  uint64_t pool_off = 0, pool_bytes = 0;
  ReqBuffers buf{};
  uint64_t scheduled = 0, finished = 0;
  int inflight = 0;
  hipEvent_t drained = nullptr;
  // the drain's copies land in pinned host memory (S.host): the histogram,
  // then every summary field (with VSH_SUMMARY) or only the weight and the
  // counted integer fields
  uint64_t host_off = 0, host_bytes = 0;
  char* own_host = nullptr;  // a staging of its own when the request outgrows the shared one
  double* h_hist = nullptr;
  double* h_sd = nullptr;
  int32_t* h_si = nullptr;
  uint64_t* h_hs = nullptr;
  ResultBox* box = nullptr;
  vsh_status fail_code = VSH_OK;  // set when the request failed (state kFailed once nothing is in flight)
  std::string fail_msg;
};

constexpr uint32_t kMaxEpochReqs = 512;

struct Epoch {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<std::pair<uint64_t, uint64_t>> parts;  // (ticket, events)
  ReqDev* reqs_host = nullptr;                       // pinned
  Segment* segs_host = nullptr;                      // pinned
  char* dev = nullptr;                               // descriptors, counter, slots
  uint64_t dev_bytes = 0;
};

struct ServeState {
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;  // admitted, in admission order
  std::unordered_map<uint64_t, std::unique_ptr<ServeReq>> reqs;
  Pool pool;
  Pool host;  // pinned host memory for the drains' copies
  std::deque<uint64_t> to_drain;  // finished requests waiting for pinned staging
  Epoch ep[2];
  hipStream_t drain = nullptr;
  hipStream_t admit_stream = nullptr;  // admissions' input copies and matrix elements
  hipEvent_t admitted = nullptr;       // recorded after each admission; epochs wait on it
  char* scratch = nullptr;
  uint64_t scratch_bytes = 0;
  uint32_t fail_epochs = 0;  // testing: epochs still to report a device error without launching
};

static uint64_t request_bytes(const vsh_request& r) { return request_out_bytes(r.n_events, r.max_partons, false); }

static void finish_request(ServeState& S, ServeReq& r, int state) {
  if (r.pool_bytes) {
    S.pool.release(r.pool_off, r.pool_bytes);
    r.pool_bytes = 0;
  }
  if (r.host_bytes) {
    S.host.release(r.host_off, r.host_bytes);
    r.host_bytes = 0;
  }
  if (r.own_host) {
    (void)hipHostFree(r.own_host);
    r.own_host = nullptr;
  }
  if (r.drained) {
    (void)hipEventDestroy(r.drained);
    r.drained = nullptr;
  }
  r.state = state;
  S.active.erase(std::remove(S.active.begin(), S.active.end(), r.ticket), S.active.end());
  S.done_cv.notify_all();
}

// Mark a request failed: no further events of it are scheduled, and it
// finishes (state kFailed) as soon as none of its events is in flight.
static void fail_request(ServeState& S, ServeReq& r, vsh_status code, const char* what, hipError_t err) {
  if (r.fail_code == VSH_OK) {
    r.fail_code = code;
    r.fail_msg = what;
    if (err != hipSuccess) r.fail_msg += std::string(": ") + hipGetErrorString(err);
  }
  r.cancel = true;
  if (r.inflight == 0 && r.state != kFinished && r.state != kCancelledState && r.state != kFailed)
    finish_request(S, r, kFailed);
}

static bool admit(vsh_ctx* ctx, ServeState& S) {
  bool progress = false;
  while (!S.pending.empty()) {
    ServeReq& r = *S.reqs[S.pending.front()];
    if (r.cancel) {
      S.pending.pop_front();
      finish_request(S, r, kCancelledState);
      progress = true;
      continue;
    }
    const uint64_t bytes = request_bytes(r.req);
    uint64_t off = 0;
    if (!S.pool.alloc(bytes, &off)) break;  // oldest first: wait for memory
    S.pending.pop_front();
    r.pool_off = off;
    r.pool_bytes = bytes;
    Carver c(S.pool.base + off);
    r.buf = carve_request(c, r.req.n_events, r.req.max_partons, false);
    const uint64_t n = r.req.n_events;
    hipError_t err = hipSuccess;
    if (!r.ecm.empty()) err = hipMemcpyAsync(r.buf.ecm, r.ecm.data(), n * 8, hipMemcpyHostToDevice, S.admit_stream);
    if (err == hipSuccess && !r.tcut.empty())
      err = hipMemcpyAsync(r.buf.tcut, r.tcut.data(), n * 8, hipMemcpyHostToDevice, S.admit_stream);
    launch_zero(r.buf.hist, kHistDoubles, S.admit_stream);
    EventInputs in{};
    in.ecm = r.ecm.empty() ? nullptr : r.buf.ecm;
    in.tcut = r.tcut.empty() ? nullptr : r.buf.tcut;
    in.ecm0 = r.req.ecm;
    in.tcut0 = r.req.t_cut;
    in.seed = r.req.seed;
    in.first = r.req.first_event;
    in.cycle_limit = effective_cycle_limit(r.req.cycle_limit);
    in.t_over = r.req.t_over;
    in.qm = request_masses(r.req);
    in.massive = request_massive(r.req);
    in.fixed_hist = (r.req.flags & VSH_HIST_FIXEDPOINT) ? 1u : 0u;
    launch_me(r.buf.out, r.buf.sum, in, (uint32_t)n, S.admit_stream);  // LO partons of every event
    const hipError_t lerr = hipGetLastError();
    if (err == hipSuccess) err = lerr;
    // every later epoch waits for this event: inputs and LO events are on
    // the device before an epoch reads them, with no host wait here
    if (err == hipSuccess) err = hipEventRecord(S.admitted, S.admit_stream);
    r.state = kAdmitted;
    S.active.push_back(r.ticket);
    if (err != hipSuccess) fail_request(S, r, VSH_E_DEVICE, "admission", err);
    progress = true;
  }
  (void)ctx;
  return progress;
}

static bool ensure_epoch_memory(vsh_ctx* ctx, Epoch& E, uint64_t lanes, uint32_t cap) {
  const uint64_t need = align_up(kMaxEpochReqs * sizeof(ReqDev), 256) +
                        align_up(kMaxEpochReqs * sizeof(Segment), 256) + 256 + slots_bytes(lanes, cap);
  if (need <= E.dev_bytes) return true;
  if (E.dev) (void)hipFree(E.dev);
  E.dev = nullptr;
  E.dev_bytes = 0;
  if (hipMalloc(&E.dev, need) != hipSuccess) {
    (void)hipGetLastError();
    E.dev = nullptr;
    return false;
  }
  E.dev_bytes = need;
  (void)ctx;
  return true;
}

static bool launch_epoch(vsh_ctx* ctx, ServeState& S) {
  Epoch* E = nullptr;
  for (auto& e : S.ep)
    if (!e.busy) {
      E = &e;
      break;
    }
  if (!E) return false;
  const Tuned tn = ctx->tuned;
  const uint64_t lanes = persistent_lanes(ctx);
  const uint64_t limit = std::max<uint64_t>(2 * lanes, 1 << 16);
  E->parts.clear();
  uint64_t total = 0;
  uint32_t nreq = 0, nseg = 0, cap = 2;
  bool massive = false;  // any request of the epoch with quark masses
  for (uint64_t t : S.active) {
    ServeReq& r = *S.reqs[t];
    if (r.cancel || r.state != kAdmitted || r.scheduled >= r.req.n_events) continue;
    if (nreq >= kMaxEpochReqs || total >= limit) break;
    const uint64_t take = std::min(r.req.n_events - r.scheduled, limit - total);
    ReqDev& d = E->reqs_host[nreq];
    d.out = r.buf.out;
    d.sum = r.buf.sum;
    d.ecm = r.ecm.empty() ? nullptr : r.buf.ecm;
    d.tcut = r.tcut.empty() ? nullptr : r.buf.tcut;
    d.ecm0 = r.req.ecm;
    d.tcut0 = r.req.t_cut;
    d.seed = r.req.seed;
    d.first = r.req.first_event;
    d.count = r.req.n_events;
    d.cycle_limit = effective_cycle_limit(r.req.cycle_limit);
    d.t_over = r.req.t_over;
    d.qm = request_masses(r.req);
    d.massive = request_massive(r.req);
    massive |= d.massive != 0;
    Segment& sg = E->segs_host[nseg];
    sg.req = nreq;
    sg.pad = 0;
    sg.lo = r.scheduled;
    sg.hi = r.scheduled + take;
    sg.start = total;
    r.scheduled += take;
    r.inflight += 1;
    total += take;
    cap = std::max(cap, r.req.max_partons);
    E->parts.emplace_back(t, take);
    ++nreq;
    ++nseg;
  }
  if (total == 0) return false;
  if (!ensure_epoch_memory(ctx, *E, lanes, cap)) {
    // give the events back; retry when memory frees up
    for (auto& p : E->parts) {
      ServeReq& r = *S.reqs[p.first];
      r.scheduled -= p.second;
      r.inflight -= 1;
    }
    E->parts.clear();
    return false;
  }
  Carver c(E->dev);
  ReqDev* rd = (ReqDev*)c.take(kMaxEpochReqs * sizeof(ReqDev));
  Segment* sd = (Segment*)c.take(kMaxEpochReqs * sizeof(Segment));
  unsigned long long* counter = (unsigned long long*)c.take(256);
  Records slots = carve_slots(c, lanes, cap);
  hipError_t err = hipStreamWaitEvent(E->stream, S.admitted, 0);
  if (err == hipSuccess) err = hipMemcpyAsync(rd, E->reqs_host, nreq * sizeof(ReqDev), hipMemcpyHostToDevice, E->stream);
  if (err == hipSuccess) err = hipMemcpyAsync(sd, E->segs_host, nseg * sizeof(Segment), hipMemcpyHostToDevice, E->stream);
  if (err == hipSuccess) err = hipMemsetAsync(counter, 0, 8, E->stream);
  PersistArgs A;
  A.slots = slots;
  A.reqs = rd;
  A.segs = sd;
  A.n_segs = nseg;
  A.threshold = tn.refill_threshold;
  A.pad = 0;
  A.cache = EndCache{nullptr, 0};
  A.total = total;
  A.next = counter;
  A.period = tn.refill_period;
  if (err == hipSuccess && S.fail_epochs > 0) {  // testing hook: report a device error, launch nothing
    --S.fail_epochs;
    err = hipErrorLaunchFailure;
  }
  if (err == hipSuccess) {
    launch_persistent(A, lanes, tn.pers_block, tn.mapping, false, massive, E->stream);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipEventRecord(E->done, E->stream);
  if (err != hipSuccess) {
    // nothing of this epoch runs: its requests fail (work already queued on
    // the stream finishes before the stream is used again)
    for (auto& p : E->parts) {
      ServeReq& r = *S.reqs[p.first];
      r.inflight -= 1;
      fail_request(S, r, VSH_E_DEVICE, "epoch launch", err);
    }
    E->parts.clear();
    return false;
  }
  E->busy = true;
  return true;
}

// Start computing a finished request's observables and copying its results
// back.  False (nothing started) while the pinned staging is full: the
// request waits in S.to_drain.
static bool start_drain(vsh_ctx* ctx, ServeState& S, ServeReq& r) {
  const uint64_t n = r.req.n_events;
  const uint32_t cap = r.req.max_partons;
  const bool all_fields = (r.req.flags & VSH_SUMMARY) != 0;
  static_assert(kSiStatus == 1 && kSiEnds == kNSumI - 1, "the counted integer fields are the last ones");
  const uint64_t i_fields = all_fields ? kNSumI : kNSumI - kSiStatus, d_fields = all_fields ? kNSumD : 1;
  const uint64_t hb = align_up(kHistDoubles * 8, 256), db = align_up(d_fields * n * 8, 256),
                 ib = align_up(i_fields * n * 4, 256), sb = all_fields ? align_up(n * 8, 256) : 0;
  const uint64_t need_host = hb + db + ib + sb;
  char* hbase = nullptr;
  if (need_host > S.host.size) {  // larger than the whole shared staging: one of its own
    if (hipHostMalloc((void**)&r.own_host, need_host, 0) != hipSuccess) {
      (void)hipGetLastError();
      r.own_host = nullptr;
      fail_request(S, r, VSH_E_NOMEM, "pinned staging of the results", hipSuccess);
      return true;
    }
    hbase = r.own_host;
  } else {
    uint64_t off = 0;
    if (!S.host.alloc(need_host, &off)) return false;
    r.host_off = off;
    r.host_bytes = need_host;
    hbase = S.host.base + off;
  }
  r.h_hist = reinterpret_cast<double*>(hbase);
  r.h_sd = reinterpret_cast<double*>(hbase + hb);
  r.h_si = reinterpret_cast<int32_t*>(hbase + hb + db);
  r.h_hs = all_fields ? reinterpret_cast<uint64_t*>(hbase + hb + db + ib) : nullptr;
  const uint64_t need = obs_scratch_bytes(n, cap);
  if (need > S.scratch_bytes) {
    (void)hipStreamSynchronize(S.drain);
    if (S.scratch) (void)hipFree(S.scratch);
    S.scratch = nullptr;
    S.scratch_bytes = 0;
    if (hipMalloc(&S.scratch, need) == hipSuccess) S.scratch_bytes = need;
    else (void)hipGetLastError();
  }
  if (!S.scratch) {  // cannot compute its observables: fail the request
    fail_request(S, r, VSH_E_NOMEM, "observables scratch", hipSuccess);
    return true;
  }
  Carver c(S.scratch);
  Scratch sc = carve_scratch(c, n, cap);
  EventInputs in{};
  in.ecm = r.ecm.empty() ? nullptr : r.buf.ecm;
  in.tcut = r.tcut.empty() ? nullptr : r.buf.tcut;
  in.ecm0 = r.req.ecm;
  in.tcut0 = r.req.t_cut;
  in.seed = r.req.seed;
  in.first = r.req.first_event;
  in.cycle_limit = effective_cycle_limit(r.req.cycle_limit);
  in.t_over = r.req.t_over;
  in.qm = request_masses(r.req);
  in.massive = request_massive(r.req);
  in.fixed_hist = (r.req.flags & VSH_HIST_FIXEDPOINT) ? 1u : 0u;
  launch_obs(r.buf.out, r.buf.sum, in, sc, (uint32_t)n, r.buf.hist, S.drain);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess)
    err = hipMemcpyAsync(r.h_hist, r.buf.hist, kHistDoubles * 8, hipMemcpyDeviceToHost, S.drain);
  if (all_fields) {
    if (err == hipSuccess) err = hipMemcpyAsync(r.h_sd, r.buf.sum.d, kNSumD * n * 8, hipMemcpyDeviceToHost, S.drain);
    if (err == hipSuccess) err = hipMemcpyAsync(r.h_si, r.buf.sum.i, kNSumI * n * 4, hipMemcpyDeviceToHost, S.drain);
    if (err == hipSuccess) err = hipMemcpyAsync(r.h_hs, r.buf.sum.hash, n * 8, hipMemcpyDeviceToHost, S.drain);
  } else {
    if (err == hipSuccess)
      err = hipMemcpyAsync(r.h_sd, r.buf.sum.d + kSdW * n, n * 8, hipMemcpyDeviceToHost, S.drain);
    if (err == hipSuccess)
      err = hipMemcpyAsync(r.h_si, r.buf.sum.i + kSiStatus * n, i_fields * n * 4, hipMemcpyDeviceToHost, S.drain);
  }
  if (err == hipSuccess) err = hipEventCreateWithFlags(&r.drained, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventRecord(r.drained, S.drain);
  if (err != hipSuccess) {
    fail_request(S, r, VSH_E_DEVICE, "observables launch", err);
    return true;
  }
  r.state = kDraining;
  (void)ctx;
  return true;
}

static bool retire_epochs(vsh_ctx* ctx, ServeState& S) {
  bool progress = false;
  for (auto& E : S.ep) {
    if (!E.busy) continue;
    const hipError_t q = hipEventQuery(E.done);
    if (q == hipErrorNotReady) continue;
    for (auto& p : E.parts) {
      auto it = S.reqs.find(p.first);
      if (it == S.reqs.end()) continue;
      ServeReq& r = *it->second;
      r.finished += p.second;
      r.inflight -= 1;
      if (q != hipSuccess) {
        fail_request(S, r, VSH_E_DEVICE, "epoch", q);
      } else if (r.cancel) {
        if (r.inflight == 0 && r.state == kAdmitted)
          finish_request(S, r, r.fail_code != VSH_OK ? kFailed : kCancelledState);
      } else if (r.finished == r.req.n_events) {
        if (!start_drain(ctx, S, r)) S.to_drain.push_back(r.ticket);
      }
    }
    E.parts.clear();
    E.busy = false;
    progress = true;
  }
  return progress;
}

static bool poll_drains(ServeState& S) {
  bool progress = false;
  std::vector<uint64_t> done;
  std::vector<std::pair<uint64_t, hipError_t>> failed;
  for (uint64_t t : S.active) {
    ServeReq& r = *S.reqs[t];
    if (r.state != kDraining) continue;
    const hipError_t q = hipEventQuery(r.drained);
    if (q == hipSuccess) done.push_back(t);
    else if (q != hipErrorNotReady) failed.emplace_back(t, q);
  }
  for (auto& f : failed) {
    fail_request(S, *S.reqs[f.first], VSH_E_DEVICE, "observables", f.second);
    progress = true;
  }
  for (uint64_t t : done) {
    ServeReq& r = *S.reqs[t];
    const uint64_t n = r.req.n_events;
    ResultBox* box = new_result(n, r.req.flags & VSH_SUMMARY);
    if (box) {
      box->hist.assign(r.h_hist, r.h_hist + kHistDoubles);
      const bool all_fields = r.h_hs != nullptr;
      tally_fields(box, all_fields ? r.h_si + kSiStatus * n : r.h_si, n, all_fields ? r.h_sd + kSdW * n : r.h_sd, n);
      if (!box->sum_d.empty()) {
        std::memcpy(box->sum_d.data(), r.h_sd, kNSumD * n * 8);
        std::memcpy(box->sum_i.data(), r.h_si, kNSumI * n * 4);
        std::memcpy(box->hash.data(), r.h_hs, n * 8);
      }
      box->pub.t_total_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.t_arrival).count();
      finish_result(box);
    }
    r.box = box;
    finish_request(S, r, kFinished);
    progress = true;
  }
  return progress;
}

// Start the drains that waited for pinned staging, oldest first.
static bool retry_drains(vsh_ctx* ctx, ServeState& S) {
  bool progress = false;
  while (!S.to_drain.empty()) {
    auto it = S.reqs.find(S.to_drain.front());
    if (it == S.reqs.end() || it->second->state != kAdmitted || it->second->cancel) {
      S.to_drain.pop_front();  // gone, cancelled or failed meanwhile
      progress = true;
      continue;
    }
    if (!start_drain(ctx, S, *it->second)) break;  // still full
    S.to_drain.pop_front();
    progress = true;
  }
  return progress;
}

static void serve_loop(vsh_ctx* ctx) {
  (void)hipSetDevice(ctx->device);
  ServeState& S = *ctx->serve;
  std::unique_lock<std::mutex> lk(S.mu);
  while (!S.stop) {
    bool progress = false;
    progress |= admit(ctx, S);
    progress |= retire_epochs(ctx, S);
    progress |= poll_drains(S);
    progress |= retry_drains(ctx, S);
    while (launch_epoch(ctx, S)) progress = true;
    if (!progress) S.cv.wait_for(lk, std::chrono::microseconds(100));
  }
}

static vsh_status serve_start(vsh_ctx* ctx) {
  if (ctx->serve) return VSH_OK;
  auto S = std::make_unique<ServeState>();
  const uint64_t pool_bytes = std::min<uint64_t>(ctx->budget / 2, 32ull << 30);
  hipError_t err = S->pool.init(pool_bytes);
  if (err != hipSuccess) return hip_fail(ctx, err, "serving pool");
  err = S->host.init(1ull << 30, true);
  if (err != hipSuccess) return hip_fail(ctx, err, "serving pinned staging");
  err = hipStreamCreateWithFlags(&S->drain, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&S->admit_stream, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&S->admitted, hipEventDisableTiming);
  if (err != hipSuccess) return hip_fail(ctx, err, "hipStreamCreate");
  for (auto& E : S->ep) {
    err = hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&E.done, hipEventDisableTiming);
    if (err == hipSuccess) err = hipHostMalloc((void**)&E.reqs_host, kMaxEpochReqs * sizeof(ReqDev), 0);
    if (err == hipSuccess) err = hipHostMalloc((void**)&E.segs_host, kMaxEpochReqs * sizeof(Segment), 0);
    if (err != hipSuccess) return hip_fail(ctx, err, "serving setup");
  }
  ctx->serve = S.release();
  ctx->serve->th = std::thread(serve_loop, ctx);
  return VSH_OK;
}

void serve_shutdown(vsh_ctx* ctx) {
  ServeState* S = ctx->serve;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  for (auto& E : S->ep) {
    if (E.stream) (void)hipStreamSynchronize(E.stream);
  }
  if (S->drain) (void)hipStreamSynchronize(S->drain);
  if (S->admit_stream) (void)hipStreamSynchronize(S->admit_stream);
  for (auto& kv : S->reqs) {
    ServeReq& r = *kv.second;
    if (r.drained) (void)hipEventDestroy(r.drained);
    if (r.own_host) (void)hipHostFree(r.own_host);
    if (r.box) vsh_result_free(&r.box->pub);
  }
  for (auto& E : S->ep) {
    if (E.dev) (void)hipFree(E.dev);
    if (E.reqs_host) (void)hipHostFree(E.reqs_host);
    if (E.segs_host) (void)hipHostFree(E.segs_host);
    if (E.done) (void)hipEventDestroy(E.done);
    if (E.stream) (void)hipStreamDestroy(E.stream);
  }
  if (S->scratch) (void)hipFree(S->scratch);
  if (S->drain) (void)hipStreamDestroy(S->drain);
  if (S->admitted) (void)hipEventDestroy(S->admitted);
  if (S->admit_stream) (void)hipStreamDestroy(S->admit_stream);
  S->pool.destroy();
  S->host.destroy();
  delete S;
  ctx->serve = nullptr;
}

}  // namespace vsh

using namespace vsh;

extern "C" {

vsh_status vsh_test_fail_epochs(vsh_ctx* ctx, uint32_t count) {
  if (!ctx) return VSH_E_INVALID;
  std::lock_guard<std::mutex> api(ctx->mu);
  (void)hipSetDevice(ctx->device);
  const vsh_status rc = serve_start(ctx);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ctx->serve->mu);
  ctx->serve->fail_epochs = count;
  return VSH_OK;
}

vsh_status vsh_submit(vsh_ctx* ctx, const vsh_request* req, uint64_t* ticket) {
  if (!ctx || !ticket) return VSH_E_INVALID;
  std::lock_guard<std::mutex> api(ctx->mu);
  vsh_status rc = validate_request(ctx, req, true);
  if (rc) return rc;
  if (req->flags & (VSH_RECORDS | VSH_INPUTS_ON_DEVICE)) {
    set_error(ctx, "served requests return summaries and histograms from host inputs");
    return VSH_E_INVALID;
  }
  (void)hipSetDevice(ctx->device);
  rc = serve_start(ctx);
  if (rc) return rc;
  ServeState& S = *ctx->serve;
  if (request_bytes(*req) > S.pool.size) {
    set_error(ctx, "request needs %llu bytes of event records; the serving pool holds %llu",
              (unsigned long long)request_bytes(*req), (unsigned long long)S.pool.size);
    return VSH_E_NOMEM;
  }
  auto r = std::make_unique<ServeReq>();
  r->req = *req;
  r->req.ecm_per_event = nullptr;
  r->req.tcut_per_event = nullptr;
  if (req->ecm_per_event) r->ecm.assign(req->ecm_per_event, req->ecm_per_event + req->n_events);
  if (req->tcut_per_event) r->tcut.assign(req->tcut_per_event, req->tcut_per_event + req->n_events);
  r->t_arrival = Clock::now();
  {
    std::lock_guard<std::mutex> lk(S.mu);
    r->ticket = S.next_ticket++;
    *ticket = r->ticket;
    S.pending.push_back(r->ticket);
    S.reqs.emplace(r->ticket, std::move(r));
  }
  S.cv.notify_all();
  return VSH_OK;
}

vsh_status vsh_poll(vsh_ctx* ctx, uint64_t ticket, int* done) {
  if (!ctx || !done) return VSH_E_INVALID;
  ServeState* S = ctx->serve;
  if (!S) return VSH_E_NOTFOUND;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error(ctx, "unknown ticket %llu", (unsigned long long)ticket);
    return VSH_E_NOTFOUND;
  }
  const int st = it->second->state;
  *done = (st == kFinished || st == kCancelledState || st == kFailed) ? 1 : 0;
  return VSH_OK;
}

vsh_status vsh_wait(vsh_ctx* ctx, uint64_t ticket, vsh_result** out) {
  if (!ctx || !out) return VSH_E_INVALID;
  *out = nullptr;
  ServeState* S = ctx->serve;
  if (!S) return VSH_E_NOTFOUND;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error(ctx, "unknown ticket %llu", (unsigned long long)ticket);
    return VSH_E_NOTFOUND;
  }
  ServeReq* r = it->second.get();
  S->done_cv.wait(lk, [&] { return r->state == kFinished || r->state == kCancelledState || r->state == kFailed; });
  vsh_status rc = VSH_OK;
  if (r->state == kFailed) {
    set_error(ctx, "ticket %llu failed: %s", (unsigned long long)ticket, r->fail_msg.c_str());
    rc = r->fail_code;
  } else if (r->state == kCancelledState) {
    set_error(ctx, "ticket %llu was cancelled", (unsigned long long)ticket);
    rc = VSH_E_CANCELLED;
  } else if (!r->box) {
    set_error(ctx, "host allocation failed for ticket %llu", (unsigned long long)ticket);
    rc = VSH_E_NOMEM;
  } else {
    *out = &r->box->pub;
    r->box = nullptr;
  }
  S->reqs.erase(it);
  return rc;
}

vsh_status vsh_cancel(vsh_ctx* ctx, uint64_t ticket) {
  if (!ctx) return VSH_E_INVALID;
  ServeState* S = ctx->serve;
  if (!S) return VSH_E_NOTFOUND;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
      set_error(ctx, "unknown ticket %llu", (unsigned long long)ticket);
      return VSH_E_NOTFOUND;
    }
    ServeReq& r = *it->second;
    if (r.state == kFinished || r.state == kCancelledState || r.state == kFailed) return VSH_OK;
    r.cancel = true;
    if (r.state == kAdmitted && r.inflight == 0) finish_request(*S, r, kCancelledState);
  }
  S->cv.notify_all();
  return VSH_OK;
}

}  // extern "C"
