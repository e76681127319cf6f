// vsh_serve.hip -- serving: continuous batching of event-generation requests.
//
// vsh_submit copies a request and returns a ticket.  A serving thread per
// context
//   * admits queued requests in arrival order while their event-record
//     memory (every event's final record at its request's capacity, the
//     summaries and the histogram) fits a device pool; a request that does
//     not fit yet waits, one that can never fit is rejected at submission;
//   * launches bounded epochs whose work list holds segments of every
//     admitted request with events left, oldest first, so requests that
//     arrive while others run join the next epoch.  Two epochs are in flight
//     on two streams, the second filling compute units the first's tail
//     frees.  An epoch's stream runs, in order: the matrix elements of the
//     requests it starts, the persistent shower kernel over its segments,
//     then, for every request whose last events it holds, the observables,
//     the histogram and one copy of the results into pinned host memory.
//     Where a request's events span both epochs, the stream waits on the
//     other epoch's event instead of on the host;
//   * when an epoch's last event completes, hands its finished requests
//     their results and returns their memory to the pool.
// Every event is a pure function of (request seed, event id), so a request's
// events are the same alone or in any mix; only the summation order of its
// FP64 histogram can differ (none with VSH_HIST_FIXEDPOINT).
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

enum ReqState { kQueued, kAdmitted, kFinished, kCancelledState, kFailed };

struct ServeReq {
  uint64_t ticket = 0;
  vsh_request req{};
  std::vector<double> ecm, tcut;
  Clock::time_point t_arrival, t_admit;
  uint32_t queue_ahead = 0;  // requests waiting for admission when it was submitted
  int state = kQueued;
  bool cancel = false;
  uint64_t pool_off = 0, pool_bytes = 0;
  ReqBuffers buf{};
  uint64_t scheduled = 0, finished = 0;
  int inflight = 0;       // epochs in flight that hold events of the request
  int me_slot = -1;       // epoch (slot, generation) whose stream computes its LO events
  uint64_t me_gen = 0;
  uint64_t seg_gen[2] = {0, 0};  // latest generation of each slot holding some of its events
  bool drained = false;   // its observables and copy have completed
  // the drain's one copy lands in pinned host memory (S.host): the
  // histogram, the integer fields and the weights, and with VSH_SUMMARY the
  // other doubles and the hash
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
  hipEvent_t me_done = nullptr;      // after the matrix elements of the requests it starts
  hipEvent_t shower_done = nullptr;  // after its shower kernel
  hipEvent_t done = nullptr;         // after its drains and copies
  bool busy = false;
  uint64_t gen = 0;                  // launch generation of this slot
  std::vector<std::pair<uint64_t, uint64_t>> parts;  // (ticket, events)
  std::vector<uint64_t> finishing;   // tickets whose observables and copy it runs
  ReqDev* reqs_host = nullptr;       // pinned
  Segment* segs_host = nullptr;      // pinned
  char* dev = nullptr;               // descriptors, counter, slots, end cache
  uint64_t dev_bytes = 0;
  char* scratch = nullptr;           // observables scratch of its drains
  uint64_t scratch_bytes = 0;
};

struct ServeState {
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t next_gen = 1;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;  // admitted, in admission order
  std::unordered_map<uint64_t, std::unique_ptr<ServeReq>> reqs;
  Pool pool;
  Pool host;  // pinned host memory for the drains' copies
  Epoch ep[2];
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

// Admission: a request whose event-record memory fits the pool (oldest
// first) gets its device buffers; its matrix elements run in the first
// epoch that schedules its events.
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
    r.t_admit = Clock::now();
    r.state = kAdmitted;
    S.active.push_back(r.ticket);
    progress = true;
  }
  (void)ctx;
  return progress;
}

// Device memory of an epoch: descriptors, work counter, the lanes' staging
// slots and, when it fits, their end cache (cache_words words per parton
// slot; without it the flattened kernel recomputes every end each cycle).
// Grown on demand; *cached tells whether the cache is there.
static bool ensure_epoch_memory(vsh_ctx* ctx, Epoch& E, uint64_t lanes, uint32_t cap, bool massive, bool* cached) {
  const uint64_t base = align_up(kMaxEpochReqs * sizeof(ReqDev), 256) + align_up(kMaxEpochReqs * sizeof(Segment), 256) +
                        256 + slots_bytes(lanes, cap);
  const uint64_t with_cache = base + align_up(lanes * cap * cache_words(massive) * 8, 256);
  *cached = true;
  if (with_cache <= E.dev_bytes) return true;
  if (E.dev) (void)hipFree(E.dev);
  E.dev = nullptr;
  E.dev_bytes = 0;
  for (const uint64_t need : {with_cache, base}) {
    if (hipMalloc(&E.dev, need) == hipSuccess) {
      E.dev_bytes = need;
      *cached = need == with_cache;
      return true;
    }
    (void)hipGetLastError();
    E.dev = nullptr;
  }
  (void)ctx;
  return false;
}

static EventInputs request_inputs(const ServeReq& r) {
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
  return in;
}

// Pinned host memory for a finishing request's results (the span of
// carve_request from the histogram to the weights, or to the hash with
// VSH_SUMMARY), from the shared staging or, when it is full or too small,
// an allocation of the request's own.
static hipError_t reserve_staging(ServeState& S, ServeReq& r, uint64_t* bytes) {
  static_assert(kSdW == 0, "the weight is the first double field");
  const uint64_t n = r.req.n_events;
  const char* dev0 = reinterpret_cast<const char*>(r.buf.hist);
  const uint64_t off_i = reinterpret_cast<const char*>(r.buf.sum.i) - dev0;
  const uint64_t off_d = reinterpret_cast<const char*>(r.buf.sum.d) - dev0;
  const uint64_t off_h = reinterpret_cast<const char*>(r.buf.sum.hash) - dev0;
  const bool all_fields = (r.req.flags & VSH_SUMMARY) != 0;
  *bytes = all_fields ? off_h + n * 8 : off_d + n * 8;
  char* hbase = nullptr;
  uint64_t off = 0;
  if (*bytes <= S.host.size && S.host.alloc(*bytes, &off)) {
    r.host_off = off;
    r.host_bytes = *bytes;
    hbase = S.host.base + off;
  } else {
    const hipError_t err = hipHostMalloc((void**)&r.own_host, *bytes, 0);
    if (err != hipSuccess) {
      (void)hipGetLastError();
      r.own_host = nullptr;
      return err;
    }
    hbase = r.own_host;
  }
  r.h_hist = reinterpret_cast<double*>(hbase);
  r.h_si = reinterpret_cast<int32_t*>(hbase + off_i);
  r.h_sd = reinterpret_cast<double*>(hbase + off_d);
  r.h_hs = all_fields ? reinterpret_cast<uint64_t*>(hbase + off_h) : nullptr;
  return hipSuccess;
}

static bool launch_epoch(vsh_ctx* ctx, ServeState& S) {
  int ei = -1;
  for (int k = 0; k < 2; ++k)
    if (!S.ep[k].busy) {
      ei = k;
      break;
    }
  if (ei < 0) return false;
  Epoch* E = &S.ep[ei];
  const Epoch& O = S.ep[1 - ei];
  const Tuned tn = ctx->tuned;
  const uint64_t lanes = persistent_lanes(ctx);
  const uint64_t limit = std::max<uint64_t>(2 * lanes, 1 << 16);
  E->parts.clear();
  E->finishing.clear();
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
    total += take;
    cap = std::max(cap, r.req.max_partons);
    E->parts.emplace_back(t, take);
    ++nreq;
    ++nseg;
  }
  if (total == 0) return false;
  bool cached = false;
  if (!ensure_epoch_memory(ctx, *E, lanes, cap, massive, &cached)) {
    E->parts.clear();  // nothing scheduled; retried when memory frees up
    return false;
  }
  // from here on the parts belong to this epoch
  E->gen = S.next_gen++;
  for (auto& p : E->parts) {
    ServeReq& r = *S.reqs[p.first];
    r.scheduled += p.second;
    r.inflight += 1;
    r.seg_gen[ei] = E->gen;
  }
  auto fail_all = [&](const char* what, hipError_t err) {
    // whatever was queued on the stream ends before its memory is reused
    (void)hipStreamSynchronize(E->stream);
    (void)hipGetLastError();
    for (auto& p : E->parts) {
      ServeReq& r = *S.reqs[p.first];
      r.inflight -= 1;
      fail_request(S, r, VSH_E_DEVICE, what, err);
    }
    E->parts.clear();
    E->finishing.clear();
    return false;
  };
  if (S.fail_epochs > 0) {  // testing hook: report a device error, launch nothing
    --S.fail_epochs;
    return fail_all("epoch launch", hipErrorLaunchFailure);
  }
  Carver c(E->dev);
  ReqDev* rd = (ReqDev*)c.take(kMaxEpochReqs * sizeof(ReqDev));
  Segment* sd = (Segment*)c.take(kMaxEpochReqs * sizeof(Segment));
  unsigned long long* counter = (unsigned long long*)c.take(256);
  Records slots = carve_slots(c, lanes, cap);
  const EndCache cache{cached ? (uint64_t*)c.take(lanes * cap * cache_words(massive) * 8) : nullptr, cap};
  hipError_t err = hipSuccess;
  // the LO events of the requests that start here; requests whose LO events
  // the other epoch computes make this stream wait for them
  bool wait_me = false;
  for (auto& p : E->parts) {
    const ServeReq& r = *S.reqs[p.first];
    wait_me |= r.me_slot == 1 - ei && O.busy && r.me_gen == O.gen;
  }
  if (wait_me) err = hipStreamWaitEvent(E->stream, O.me_done, 0);
  for (auto& p : E->parts) {
    ServeReq& r = *S.reqs[p.first];
    if (err != hipSuccess) break;
    if (r.me_slot >= 0) continue;
    const uint64_t n = r.req.n_events;
    if (!r.ecm.empty()) err = hipMemcpyAsync(r.buf.ecm, r.ecm.data(), n * 8, hipMemcpyHostToDevice, E->stream);
    if (err == hipSuccess && !r.tcut.empty())
      err = hipMemcpyAsync(r.buf.tcut, r.tcut.data(), n * 8, hipMemcpyHostToDevice, E->stream);
    if (err != hipSuccess) break;
    // LO partons of every event; the request's histogram cleared on the way
    launch_me(r.buf.out, r.buf.sum, request_inputs(r), (uint32_t)n, E->stream, r.buf.hist);
    r.me_slot = ei;
    r.me_gen = E->gen;
  }
  if (err == hipSuccess) err = hipGetLastError();
  if (err == hipSuccess) err = hipEventRecord(E->me_done, E->stream);
  // the shower
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
  A.cache = cache;
  A.total = total;
  A.next = counter;
  A.period = tn.refill_period;
  if (err == hipSuccess) {
    launch_persistent(A, lanes, tn.pers_block, tn.mapping, false, massive, E->stream);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipEventRecord(E->shower_done, E->stream);
  if (err != hipSuccess) return fail_all("epoch launch", err);
  // the requests whose last events are here: observables, histogram and one
  // copy of their results, after the other epoch's shower where it holds
  // some of their events
  bool wait_other = false;
  for (auto& p : E->parts) {
    ServeReq& r = *S.reqs[p.first];
    if (r.scheduled != r.req.n_events) continue;
    E->finishing.push_back(p.first);
    wait_other |= O.busy && r.seg_gen[1 - ei] == O.gen;
  }
  if (wait_other) err = hipStreamWaitEvent(E->stream, O.shower_done, 0);
  uint64_t scratch_need = 0;
  for (uint64_t t : E->finishing) {
    const ServeReq& r = *S.reqs[t];
    scratch_need = std::max(scratch_need, obs_scratch_bytes(r.req.n_events, r.req.max_partons));
  }
  if (err == hipSuccess && scratch_need > E->scratch_bytes) {
    if (E->scratch) (void)hipFree(E->scratch);  // this stream's earlier work has completed
    E->scratch = nullptr;
    E->scratch_bytes = 0;
    err = hipMalloc(&E->scratch, scratch_need);
    if (err == hipSuccess) E->scratch_bytes = scratch_need;
    else E->scratch = nullptr;
  }
  for (uint64_t t : E->finishing) {
    ServeReq& r = *S.reqs[t];
    if (err != hipSuccess) break;
    uint64_t bytes = 0;
    err = reserve_staging(S, r, &bytes);
    if (err != hipSuccess) break;
    Carver sc_c(E->scratch);
    const Scratch sc = carve_scratch(sc_c, r.req.n_events, r.req.max_partons);
    launch_obs(r.buf.out, r.buf.sum, request_inputs(r), sc, (uint32_t)r.req.n_events, r.buf.hist, E->stream);
    err = hipGetLastError();
    if (err == hipSuccess) err = hipMemcpyAsync(r.h_hist, r.buf.hist, bytes, hipMemcpyDeviceToHost, E->stream);
  }
  if (err == hipSuccess) err = hipEventRecord(E->done, E->stream);
  if (err != hipSuccess) return fail_all("observables launch", err);
  E->busy = true;
  return true;
}

// The result of a request whose events and drain have completed, from its
// pinned staging.
static void complete_request(ServeState& S, ServeReq& r) {
  const uint64_t n = r.req.n_events;
  ResultBox* box = new_result(n, r.req.flags & VSH_SUMMARY);
  if (box) {
    box->hist.assign(r.h_hist, r.h_hist + kHistDoubles);
    tally_fields(box, r.h_si + kSiStatus * n, n, r.h_sd + kSdW * n, n);
    if (!box->sum_d.empty()) {
      std::memcpy(box->sum_d.data(), r.h_sd, kNSumD * n * 8);
      std::memcpy(box->sum_i.data(), r.h_si, kNSumI * n * 4);
      std::memcpy(box->hash.data(), r.h_hs, n * 8);
    }
    box->pub.t_total_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.t_arrival).count();
    box->pub.t_queue_ms = std::chrono::duration<double, std::milli>(r.t_admit - r.t_arrival).count();
    box->pub.queue_ahead = r.queue_ahead;
    finish_result(box);
  }
  r.box = box;
  finish_request(S, r, kFinished);
}

static bool retire_epochs(vsh_ctx* ctx, ServeState& S) {
  bool progress = false;
  for (auto& E : S.ep) {
    if (!E.busy) continue;
    const hipError_t q = hipEventQuery(E.done);
    if (q == hipErrorNotReady) continue;
    for (uint64_t t : E.finishing) {
      auto it = S.reqs.find(t);
      if (it != S.reqs.end() && q == hipSuccess) it->second->drained = true;
    }
    for (auto& p : E.parts) {
      auto it = S.reqs.find(p.first);
      if (it == S.reqs.end()) continue;
      ServeReq& r = *it->second;
      r.finished += p.second;
      r.inflight -= 1;
      if (q != hipSuccess) fail_request(S, r, VSH_E_DEVICE, "epoch", q);
    }
    // requests with nothing in flight any more: done, cancelled or failed
    for (auto& p : E.parts) {
      auto it = S.reqs.find(p.first);
      if (it == S.reqs.end()) continue;
      ServeReq& r = *it->second;
      if (r.inflight != 0 || r.state != kAdmitted) continue;
      if (r.cancel) finish_request(S, r, r.fail_code != VSH_OK ? kFailed : kCancelledState);
      else if (r.drained) complete_request(S, r);
    }
    E.parts.clear();
    E.finishing.clear();
    E.busy = false;
    progress = true;
  }
  (void)ctx;
  return progress;
}

static void serve_loop(vsh_ctx* ctx) {
  (void)hipSetDevice(ctx->device);
  ServeState& S = *ctx->serve;
  std::unique_lock<std::mutex> lk(S.mu);
  while (!S.stop) {
    bool progress = false;
    progress |= retire_epochs(ctx, S);
    progress |= admit(ctx, S);
    while (launch_epoch(ctx, S)) progress = true;
    if (!progress) S.cv.wait_for(lk, std::chrono::microseconds(50));
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
  for (auto& E : S->ep) {
    err = hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&E.me_done, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&E.shower_done, hipEventDisableTiming);
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
  for (auto& kv : S->reqs) {
    ServeReq& r = *kv.second;
    if (r.own_host) (void)hipHostFree(r.own_host);
    if (r.box) vsh_result_free(&r.box->pub);
  }
  for (auto& E : S->ep) {
    if (E.dev) (void)hipFree(E.dev);
    if (E.scratch) (void)hipFree(E.scratch);
    if (E.reqs_host) (void)hipHostFree(E.reqs_host);
    if (E.segs_host) (void)hipHostFree(E.segs_host);
    for (hipEvent_t ev : {E.me_done, E.shower_done, E.done})
      if (ev) (void)hipEventDestroy(ev);
    if (E.stream) (void)hipStreamDestroy(E.stream);
  }
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
    r->queue_ahead = (uint32_t)S.pending.size();
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
