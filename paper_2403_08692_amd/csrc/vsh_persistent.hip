// vsh_persistent.hip -- the batched form: persistent waves that keep every
// lane busy with a fresh event until the work runs out.
//
// The paper's parallel veto algorithm (Sec. 2) runs one step for all events
// in lockstep and leaves finished events idle until the last one reaches the
// cutoff (Fig. 3; Fig. 7 shows the long tail).  Here each lane of a resident
// wave owns one event slot.  After every `period` veto cycles the wave takes a
// ballot of its idle lanes; if at least `threshold` are idle (or all are), one
// lane claims that many event indices from a global work counter with a
// single atomic, and the idle lanes take consecutive indices in lane order
// (prefix count of the ballot below the lane).  A lane whose event finishes
// copies the final partons and summary to the event's own output position.
// A wave exits when the counter is exhausted and none of its lanes is busy.
//
// The work space is a list of segments (request, event range), so events of
// several requests share one launch (serving); observables and histograms are
// computed afterwards per request by k_obs over its output records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <type_traits>
#include <vector>

#include "vsh_internal.hpp"
#include "vsh_observables.hpp"
#include "vsh_persistent.hpp"
#include "vsh_shower.hpp"

namespace vsh {

__device__ __forceinline__ uint32_t find_segment(const Segment* segs, uint32_t n, uint64_t w) {
  uint32_t lo = 0, hi = n;  // segs[k].start ascending; find last k with start <= w
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (segs[mid].start <= w) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Claim work for the idle lanes of this wave (see the file comment).  Returns
// true for a lane that took an event; sets req/ev and, once the counter is
// exhausted, drained.  Claims are whole multiples of kGranule events, so with
// kGranule = 16 every claim starts on a 16-event boundary and each 128-byte
// line of a record column (16 doubles of consecutive events) belongs to one
// wave: needed when the events evolve in place, where neighbouring events of
// one line would otherwise be written by waves on different XCDs.
template <uint32_t kGranule>
__device__ __forceinline__ bool refill(const PersistArgs& A, bool busy, uint32_t wave_lanes, uint32_t lane,
                                      uint32_t& since, bool& drained, uint32_t& req, uint64_t& ev) {
  const uint64_t idle = __ballot(!busy);
  const uint32_t n_idle = __popcll(idle);
  const uint32_t take = n_idle / kGranule * kGranule;
  if (drained || take == 0 || (n_idle != wave_lanes && (since < A.period || n_idle < A.threshold)))
    return false;
  since = 0;
  const uint32_t leader = __ffsll((unsigned long long)idle) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(A.next, (unsigned long long)take);
  base = __shfl(base, leader);
  if (base + take >= A.total) drained = true;
  if (busy) return false;
  const uint32_t rank = __popcll(idle & ((1ull << lane) - 1));
  const uint64_t w = base + rank;
  if (rank >= take || w >= A.total) return false;
  const uint32_t sg = find_segment(A.segs, A.n_segs, w);
  req = A.segs[sg].req;
  ev = A.segs[sg].lo + (w - A.segs[sg].start);
  return true;
}

// Start event ev of request R in working slot `slot`.  In place, the slots
// are R's own output records, where the matrix-element pass has already
// left the LO partons and their partner links.
template <bool kInPlace>
__device__ __forceinline__ void start_event(EvState& s, const PersistArgs& A, const ReqDev& R, uint64_t ev,
                                            uint64_t slot) {
  const double ecm = R.ecm ? R.ecm[ev] : R.ecm0;
  const double tcut = R.tcut ? R.tcut[ev] : R.tcut0;
  const Keyed key = make_keyed(R.seed, R.first + ev);
  if (kInPlace) lo_state(s, key, ecm, tcut, R.t_over, (int)R.out.cap);
  else start_from_record(s, R.out, ev, A.slots, slot, key, ecm, tcut, R.t_over, (int)R.out.cap);
}

// Record a finished event: its summary, and (unless in place) its partons
// copied from the working slot to the request's output.
template <bool kInPlace>
__device__ __forceinline__ void finish_event(const EvState& s, const PersistArgs& A, const ReqDev& R, uint64_t ev,
                                             uint64_t slot) {
  if (!kInPlace) {
    const Records& o = R.out;
    for (int a = 0; a < s.n; ++a) {
      const uint64_t from = (uint64_t)a * A.slots.stride + slot;
      const uint64_t to = (uint64_t)a * o.stride + ev;
      o.E[to] = A.slots.E[from];
      o.x[to] = A.slots.x[from];
      o.y[to] = A.slots.y[from];
      o.z[to] = A.slots.z[from];
      o.pid[to] = A.slots.pid[from];
      o.col[to] = A.slots.col[from];
      o.acol[to] = A.slots.acol[from];
    }
  }
  write_state(s, R.sum, ev);
}

template <bool kInPlace, bool kMassive = false>
__global__ void __launch_bounds__(256) k_shower_persistent(PersistArgs A) {
  const uint64_t L = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // this lane's working slot
  const uint32_t lane = __lane_id();
  const uint32_t wave_lanes = __popcll(__ballot(1));
  EvState s = {};
  s.status = kDone;
  bool busy = false;
  bool drained = false;
  uint32_t req = 0;
  uint64_t ev = 0;  // event index within its request
  uint64_t slot = L;
  uint32_t since = 0;
  while (true) {
    if (refill<(kInPlace ? 16u : 1u)>(A, busy, wave_lanes, lane, since, drained, req, ev)) {
      slot = kInPlace ? ev : L;
      start_event<kInPlace>(s, A, A.reqs[req], ev, slot);
      busy = true;
    }
    if (!__any(busy)) break;  // counter exhausted and nothing left in this wave
    if (busy) {
      if constexpr (kMassive) veto_cycle_massive(s, A.slots, slot, A.reqs[req].qm);
      else veto_cycle(s, A.slots, slot);
      if (s.status == kRunning && s.cycle >= A.reqs[req].cycle_limit) s.status = kCycleLimitHit;
      if (s.status != kRunning) {
        finish_event<kInPlace>(s, A, A.reqs[req], ev, slot);
        busy = false;
      }
    }
    ++since;
  }
}

// ---------------------------------------------------------------------------
// Flattened mapping.  Same refill as above, but each veto cycle's trials of a
// wave's 64 events are spread over its 64 lanes: the work items are the
// partons of all busy events, taken 64 per round; item (owner o, parton i)
// runs that parton's dipole ends.  A gluon item (two ends, three Philox
// blocks and two logs per end) costs about four quark items (one end, one
// block, one log), so gluon and quark partons get rounds of their own: first
// the gluons of every event (event-major), padded to a whole round, then the
// quarks.  Each event keeps a bit mask of its gluon slots in LDS, so item r of
// an owner is its r-th set (or clear) bit.  Within a round a segmented max
// over consecutive lanes of the same owner leaves the owner's round best on
// its last lane, which folds it into the owner's running best in LDS.  Both
// compare (larger ln t, then smaller packed (i, k, K)): the paper's loop
// order keeps the first of equal trials, and this rule picks that one in
// whatever order the items come.  Each owner then decides its own cycle.
// ---------------------------------------------------------------------------
// Launch-wide constants of the kernels whose events all belong to one
// request: each event's key is make_keyed(seed, first + its record column)
// and the cycle limit is one, so neither is kept per event in LDS (kOne),
// and, for four waves per SIMD (kFour, records of at most 128 partons), the
// item list (whose free tail holds the stale partons) is shorter (its
// overflow takes the offsets' path): 9.2 KB + 1 KB of masks, sixteen blocks
// per CU at 64 partons, fourteen at 128.  With
// 256-parton records the layout leaves room for one more block per CU.
struct OneRequest {
  uint64_t seed, first;
  uint32_t climit;
};
constexpr uint32_t kOneAboveCap = 64;  // massive plain kernel: the per-event layout up to here
constexpr uint32_t kFourMaxCap = 128;  // massless: four-wave builds up to here (LDS-bound above)

template <bool kOne_, bool kFour_ = false, bool kRegW_ = false>
struct FlatShared {
  static constexpr bool kOne = kOne_, kFour = kFour_, kRegW = kRegW_;
  double lt[64], tcut[64], ltc[64], cfac[64];
  uint32_t slot[64];  // record columns (a launch covers fewer than 2^32)
  uint32_t key[4][kOne ? 1 : 64];
  uint32_t cycle[64];
  uint32_t gstart[65], qstart[65];  // per-owner item offsets in the gluon and quark sections
  uint32_t sstart[65];              // per-owner offsets in the list of stale partons
  // the cycle's items, owner << 10 | parton: gluon items (a gluon twice,
  // once per dipole end, when rounds allow), then quark items, then the
  // stale partons in what the items leave free (two spare entries)
  uint16_t item[1024 + (kFour || kRegW ? 100 : 384) + 4];
  double best_v[64];
  uint32_t best_idx[64];  // packed (i, k, K) << 6 | the lane whose item made it
  double best_c[2][64];   // per owner: those of its running best
  uint32_t counts[64];  // the cycle's trials (low 16 bits) and active ends (high 16 bits) per owner
  uint32_t climit[kOne ? 1 : 64];  // each event's cycle limit
  double wsh[kRegW ? 1 : 64];  // each event's shower weight (weighted veto), unless held in a register
  union {
    double coef[2][64];     // massless: per item lane, its best end's 1/ca, 1/cb
    struct {
      double mc[64], mb[64];  // massive: each event's charm and bottom masses
    };
  };
};

// per-owner gluon masks, then per-owner stale masks (partons whose cached end
// coefficients must be recomputed), ceil(cap / 64) words each, in dynamic LDS
extern __shared__ uint64_t flat_gmask[];

__device__ __forceinline__ uint32_t mask_words(uint32_t cap) { return (cap + 63) / 64; }


__device__ __forceinline__ uint32_t owner_of(const uint32_t* start, uint32_t j) {
  uint32_t lo = 0, hi = 64;  // last o with start[o] <= j (owners with no items have start[o] == start[o+1])
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (start[mid] <= j) lo = mid;
    else hi = mid;
  }
  return lo;
}

// position of the r-th (from 0) set bit of x; x has more than r set bits
__device__ __forceinline__ uint32_t select64(uint64_t x, uint32_t r) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t w = 32; w >= 1; w >>= 1) {
    const uint32_t c = __popcll(x & ((1ull << w) - 1));
    if (r >= c) {
      r -= c;
      x >>= w;
      pos += w;
    }
  }
  return pos;
}

// slot of the r-th gluon (gluon = true) or r-th quark of an event's mask
__device__ __forceinline__ uint32_t select_slot(const uint64_t* m, uint32_t words, uint32_t r, bool gluon) {
  for (uint32_t w = 0; w < words; ++w) {
    const uint64_t x = gluon ? m[w] : ~m[w];
    const uint32_t c = __popcll(x);
    if (r < c) return 64 * w + select64(x, r);
    r -= c;
  }
  return 0;  // not reached for r below the owner's count
}

// The gluon mask of the event in column `slot`, from its partons' ids, and
// its stale mask with every parton set.
__device__ __forceinline__ void mask_init(uint64_t* m, uint64_t* st, uint32_t words, const Records& r,
                                          uint64_t slot, int n) {
  for (uint32_t w = 0; w < words; ++w) {
    m[w] = 0ull;
    const int lo = 64 * (int)w;
    st[w] = n >= lo + 64 ? ~0ull : (n > lo ? (1ull << (n - lo)) - 1ull : 0ull);
  }
  for (int a = 0; a < n; ++a)
    if (r.pid[(uint64_t)a * r.stride + slot] == kGluon) m[a >> 6] |= 1ull << (a & 63);
}

__device__ __forceinline__ void set_bit(uint64_t* m, int a) {
  if (a >= 0 && a != kNoPartner) m[a >> 6] |= 1ull << (a & 63);
}

// Trials of parton i of the event in column `slot`.  Each lane's event keeps,
// per parton, one cache entry of kCacheWords words at
// rec[((col * cap) + i) * kCacheWords]: its id and its spectators in
// ascending order (packed in word 0), then per end the trial coefficients
// (quark kernel or g -> g g, and g -> f fbar; 0 = no phase space; a quark
// end keeps the g -> f fbar form cfac T_R/2 (z+ - z-) too, from which the
// decision recovers the end's range and mass).  An entry
// changes only when an emission touches the parton or its partners, which
// marks it stale: then it is rebuilt from the records (the values a
// recomputation gives).  A fresh parton needs nothing but its entry.  Same
// trials, same order, same winner as parton_trials.
__device__ __forceinline__ uint64_t pack_meta(int pid, int k1, int k2) {
  return (uint64_t)(uint8_t)(int8_t)pid | ((uint64_t)(uint16_t)k1 << 8) | ((uint64_t)(uint16_t)k2 << 24);
}

// Rebuild the cache entry of parton i of the event in column `slot` from the
// records (the stale rounds of a cycle).
__device__ __forceinline__ void entry_build(double cfac, double tcut, const Records& r, uint64_t slot, int i,
                                            const EndCache& ec, uint64_t col) {
  uint64_t* ent = ec.rec + ((col * ec.cap) + (uint64_t)i) * kCacheWords;
  const uint64_t oi = (uint64_t)i * r.stride + slot;
  const int pid_i = r.pid[oi];
  int k1 = r.cpart[oi], k2 = r.apart[oi];
  if (k2 == k1) k2 = kNoPartner;
  if (k1 > k2) {
    const int t = k1;
    k1 = k2;
    k2 = t;
  }
  const P4 pi = r.load(i, slot);
  uint64_t w[kCacheWords];
  w[0] = pack_meta(pid_i, k1, k2);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int k = e == 0 ? k1 : k2;
    double ia = 0.0, ib = 0.0;  // 0: no end, or no phase space above the cutoff
    if (k != kNoPartner) {
      double q2, zm, zp, L;
      if (!end_coeffs(cfac, tcut, pid_i, pi, r.load(k, slot), q2, zm, zp, L, ia, ib)) ia = ib = 0.0;
    }
    w[1 + 2 * e] = (uint64_t)__double_as_longlong(ia);
    w[2 + 2 * e] = (uint64_t)__double_as_longlong(ib);
  }
#pragma unroll
  for (int q = 0; q < kCacheWords; ++q) ent[q] = w[q];
}

// The same for an event with quark masses: per end the four class
// coefficients of massive_end_coeffs.
__device__ __forceinline__ void entry_build_massive(double cfac, double tcut, const Records& r, uint64_t slot, int i,
                                                    const EndCache& ec, uint64_t col, const QuarkMasses& qm) {
  uint64_t* ent = ec.rec + ((col * ec.cap) + (uint64_t)i) * kMCacheWords;
  const uint64_t oi = (uint64_t)i * r.stride + slot;
  const int pid_i = r.pid[oi];
  int k1 = r.cpart[oi], k2 = r.apart[oi];
  if (k2 == k1) k2 = kNoPartner;
  if (k1 > k2) {
    const int t = k1;
    k1 = k2;
    k2 = t;
  }
  const P4 pi = r.load(i, slot);
  const TrialCtx c{Keyed{0u, 0u, 0u, 0u}, 0.0, tcut, 0.0, cfac, 0u};  // the ranges read t_C and cfac only
  uint64_t w[kMCacheWords];
  w[0] = pack_meta(pid_i, k1, k2);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int k = e == 0 ? k1 : k2;
    double cc[4] = {0.0, 0.0, 0.0, 0.0};
    if (k != kNoPartner) massive_end_coeffs(c, pid_i, r.pid[(uint64_t)k * r.stride + slot], pi, r.load(k, slot), qm, cc);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[1 + 4 * e + q] = (uint64_t)__double_as_longlong(cc[q]);
  }
#pragma unroll
  for (int q = 0; q < kMCacheWords; ++q) ent[q] = w[q];
}

// Trials of parton i of an event with quark masses from its fresh cache
// entry (the stale rounds rebuilt it): the draws and counts of
// parton_trials_massive; only the item's best (i, k, K) is kept.
__device__ __forceinline__ void parton_trials_mcached(const TrialCtx& c, uint64_t col, int i, const EndCache& ec,
                                                      double& best, uint32_t& widx, uint32_t& trials,
                                                      uint32_t& ends) {
  const uint64_t* ent = ec.rec + ((col * ec.cap) + (uint64_t)i) * kMCacheWords;
  uint64_t w[kMCacheWords];
#pragma unroll
  for (int q = 0; q < kMCacheWords; ++q) w[q] = ent[q];
  const int pid_i = (int)(int8_t)(uint8_t)(w[0] & 0xFFu);
  const int ks[2] = {(int)((w[0] >> 8) & 0xFFFFu), (int)((w[0] >> 24) & 0xFFFFu)};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (ks[e] == kNoPartner) continue;
    double cc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cc[q] = __longlong_as_double((long long)w[1 + 4 * e + q]);
    const int K = end_draws_massive(c, i, ks[e], pid_i, cc, best, trials, ends);
    if (K >= 0) widx = pack_trial(i, ks[e], K);
  }
}

// An item's end-cache entry, when loaded ahead of its round.
struct Ent5 {
  uint64_t w[kCacheWords];
};

// Trials of one item of a massless event: ends e_lo .. e_hi of parton i (a
// gluon's item takes one or both of its ends; a quark's both, the second
// empty as a quark has one colour partner), from the parton's fresh cache
// entry (cached; the stale rounds rebuilt it) or from the records.  The
// winning end's reciprocal coefficients come back in (wia, wib).
__device__ __forceinline__ void item_trials(const TrialCtx& c, const Records& r, uint64_t slot, int i, int e_lo,
                                            int e_hi, const EndCache& ec, uint64_t col, bool cached, bool pre,
                                            const Ent5& pw, double& best, uint32_t& widx, double& wia, double& wib,
                                            uint32_t& trials, uint32_t& ends) {
  uint64_t w[kCacheWords];
  int pid_i, k1, k2;
  P4 pi{0.0, 0.0, 0.0, 0.0};
  if (cached) {  // the entry as loaded ahead (pre), or from the cache now
    const uint64_t* ent = ec.rec + ((col * ec.cap) + (uint64_t)i) * kCacheWords;
#pragma unroll
    for (int q = 0; q < kCacheWords; ++q) w[q] = pre ? pw.w[q] : ent[q];
    pid_i = (int)(int8_t)(uint8_t)(w[0] & 0xFFu);
    k1 = (int)((w[0] >> 8) & 0xFFFFu);
    k2 = (int)((w[0] >> 24) & 0xFFFFu);
  } else {
    const uint64_t oi = (uint64_t)i * r.stride + slot;
    pid_i = r.pid[oi];
    k1 = r.cpart[oi];
    k2 = r.apart[oi];
    if (k2 == k1) k2 = kNoPartner;
    if (k1 > k2) {
      const int t = k1;
      k1 = k2;
      k2 = t;
    }
    pi = r.load(i, slot);
  }
  // the q-th end of the item is end e_lo + q: lanes of gluon items with
  // different ends and of quark items take their first end together
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = e_lo + q;
    const int k = e == 0 ? k1 : k2;
    if (e > e_hi || k == kNoPartner) continue;
    double ia, ib;
    if (cached) {
      ia = __longlong_as_double((long long)(e == 0 ? w[1] : w[3]));
      ib = __longlong_as_double((long long)(e == 0 ? w[2] : w[4]));
    } else {
      double q2, zm, zp, L;
      if (!end_coeffs(c.cfac, c.tcut, pid_i, pi, r.load(k, slot), q2, zm, zp, L, ia, ib)) ia = ib = 0.0;
    }
    if (ia == 0.0) continue;  // no phase space above the cutoff
    ends += 1;
    const int K = end_draws(c, i, k, pid_i, ia, ib, best, trials);
    if (K >= 0) {
      widx = pack_trial(i, k, K);
      wia = ia;
      wib = ib;
    }
  }
}

// Trials of parton i of an event with quark masses in column `slot`: the
// massive ends compute their ranges themselves each cycle (no end cache);
// only the item's best (i, k, K) is kept.
__device__ __forceinline__ void parton_trials_mflat(const TrialCtx& c, const Records& r, uint64_t slot, int i,
                                                    const QuarkMasses& qm, double& best, uint32_t& widx,
                                                    uint32_t& trials, uint32_t& ends) {
  MWinner W{Winner{0.0, 0.0, 0.0, 0.0, -1, 0, 0}, 0.0, 0.0, 0.0, 0.0, 1.0, false};
  parton_trials_massive(c, r, slot, i, qm, best, W, trials, ends);
  if (W.w.i >= 0) widx = pack_trial(W.w.i, W.w.k, W.w.K);
}

// Load the end-cache entry of the item at list position `at` into pw; false
// (nothing loaded) past the cycle's items or the list's end.
__device__ __forceinline__ bool prefetch_entry(const uint16_t* item, uint32_t at, uint32_t n_items, uint32_t n_list,
                                               const EndCache& ec, uint64_t wave_col, Ent5& pw) {
  if (at >= n_items || at >= n_list) return false;
  const uint32_t it = item[at];
  const uint64_t* ent = ec.rec + (((wave_col + (it >> 10)) * ec.cap) + (uint64_t)(it & 1023u)) * kCacheWords;
#pragma unroll
  for (int q = 0; q < kCacheWords; ++q) pw.w[q] = ent[q];
  return true;
}

// (v, idx) beats (w, jdx): larger ln t, or equal and earlier in loop order
__device__ __forceinline__ bool beats(double v, uint32_t idx, double w, uint32_t jdx) {
  return idx != kNoTrial && (jdx == kNoTrial || v > w || (v == w && idx < jdx));
}

// One veto cycle of every busy event of this wave whose last accepted
// emission has been built, the trials spread over the lanes; each owner lane
// then decides its own event's cycle.  An accepted emission stays pending
// (the event makes no trials meanwhile) until at least half of the busy
// events have one; then the wave builds them together (a quarter, three
// quarters and all of them measured slower on LEP, mixed and stress events).
// Deferring an emission changes nothing in the event: its random numbers are
// keyed by the event's own cycle.  The event of the calling lane sits in
// column `slot` of `slots`; its gluon mask at gm + lane * words.
constexpr uint32_t kEmitDiv = 2;

// kCached: the kernel has an end cache (ec); the cycle then starts with
// rounds that rebuild the entries of stale partons, so that every trial
// round reads fresh entries only.  Without it, each item computes its
// parton's coefficients itself.  kMassive: the events carry quark masses
// (qm, the calling lane's event's); no end cache, the owner recomputes its
// winner's range from the records.
// kAhead: the owner's trial constants (key, scales, cycle) are reloaded from
// LDS after the rounds, so their registers are free during them; for
// massless cached events each round then loads the end-cache entries of the
// next round's items while it reduces its winners.  The four-wave builds
// take it to fit 128 registers; at three waves the plain kernel takes it
// with quark masses only (for massless events it measured 1% slower there).
//
// kAheadCycles (massless cached events): a wave cycle may evaluate K = 2^m
// consecutive veto cycles of each event that makes trials.  A trial's scale
// is ln t + ln(R)/c, with c fixed until an emission changes the event, so
// between emissions the winner of a veto cycle (the largest ln(R)/c) does
// not depend on the scale it starts from; only the decision does.  The
// rounds therefore draw the trials of cycles c .. c+K-1 together (item j of
// cycle k at position j K + k of its section, keyed by that cycle), each
// (event, cycle) pair keeps its best ln(R)/c, then one lane per pair chains
// the scales in order (ln t of cycle k = that of cycle k-1 plus the pair's
// best, the same additions a cycle-by-cycle evaluation makes) and makes the
// pair's CheckCutoff, alpha_s and AcceptOrVeto with the pair's accept block.
// Each event then takes its pairs in order up to the first that ends the
// cycle sequence (cutoff, acceptance, cycle limit); later pairs are dropped
// and drawn again, keyed by the same cycles, after the emission.  K is the
// largest power of two with at most 64 pairs, at most kAheadMax cycles and
// at most kAheadRounds more rounds than one cycle's items take.
constexpr uint32_t kAheadLgMax = 3;  // kAheadMax = 8
constexpr uint32_t kAheadRounds = 3;
enum : uint32_t { kPairVeto = 0, kPairAccept = 1, kPairDone = 2, kPairLimit = 3 };

__device__ __forceinline__ uint32_t list_pos(uint32_t v, uint32_t vg, uint32_t n_g, uint32_t lg) {
  return v < vg ? v >> lg : n_g + ((v - vg) >> lg);
}

template <bool kCached, bool kMassive = false, bool kAhead = false, bool kAheadCycles = false, bool kOne = false,
          class SH>
__device__ __forceinline__ void flat_cycle(SH& sh, const OneRequest& one, uint64_t* gm, uint32_t words, EvState& s, bool busy,
                                           bool& pend, Pending& pd, const Records& slots, uint64_t slot,
                                           const EndCache& ec, uint64_t wave_col, uint32_t lane,
                                           const QuarkMasses& qm = QuarkMasses{0.0, 0.0, 0.0, 0.0, 0.0}) {
  const bool trial = busy && !pend;
  // this lane's event's shower weight: in LDS, or (kRegW) in the event state
  auto wsh = [&]() -> double& {
    if constexpr (SH::kRegW) return s.wsh;
    else return sh.wsh[lane];
  };
  // the key and cycle limit of the event in column o of this wave
  // (kOne: the seed's words come from LDS at each use, so that the
  // compiler does not hold Philox's round keys in registers for the kernel)
  auto key_of = [&](uint32_t o) -> Keyed {
    if constexpr (kOne) {
      const uint64_t ev = one.first + sh.slot[o];
      return Keyed{(uint32_t)ev, (uint32_t)(ev >> 32), sh.key[2][0], sh.key[3][0]};
    } else {
      return Keyed{sh.key[0][o], sh.key[1][o], sh.key[2][o], sh.key[3][o]};
    }
  };
  auto climit_of = [&](uint32_t o) -> uint32_t {
    if constexpr (kOne) return one.climit;
    else return sh.climit[o];
  };
  uint64_t* mym = gm + (uint64_t)lane * words;
  uint64_t* sm = gm + (uint64_t)64 * words;  // stale masks
  uint64_t* mys = sm + (uint64_t)lane * words;
  // --- publish the events that make trials, the item ranges of both
  // sections and of the stale partons (counts in 21-bit fields: at most 64
  // events of 1024 partons)
  constexpr uint64_t kF = (1ull << 21) - 1;
  // the cycle's accept block depends on the event and cycle only: drawn here,
  // where its arithmetic overlaps the waits of the publishing
  const U4 acc = trial ? accept_draw(s) : U4{0u, 0u, 0u, 0u};
  uint32_t ng = 0, ns = 0;
  if (trial)
    for (uint32_t w = 0; w < words; ++w) {
      const int lo = 64 * (int)w;
      const uint64_t live = s.n >= lo + 64 ? ~0ull : (s.n > lo ? (1ull << (s.n - lo)) - 1ull : 0ull);
      ng += __popcll(mym[w] & live);
      if (kCached) ns += __popcll(mys[w] & live);
    }
  const uint64_t mine = trial ? ((uint64_t)ng | ((uint64_t)((uint32_t)s.n - ng) << 21) | ((uint64_t)ns << 42)) : 0ull;
  const uint64_t incl = wave_inclusive_sum(mine);  // every lane of the wave takes part
  const uint64_t excl = incl - mine;
  const uint64_t tot = lane63(incl);
  const uint32_t n_g1 = (uint32_t)(tot & kF), n_q = (uint32_t)((tot >> 21) & kF), n_s = (uint32_t)(tot >> 42);
  // cycles evaluated ahead: K = 2^lg_ (1 without kAheadCycles); a trialing
  // event's rank is the number of trialing lanes below its own
  uint32_t lg_ = 0;
  const uint64_t tmask = kAheadCycles ? __ballot(trial) : 0ull;
  if (kAheadCycles) {
    const uint32_t n_tr = (uint32_t)__popcll(tmask), n1 = n_g1 + n_q, r1 = (n1 + 63) / 64;
    while (lg_ < kAheadLgMax && (n_tr << (lg_ + 1)) <= 64u && ((n1 << (lg_ + 1)) + 63) / 64 <= r1 + kAheadRounds)
      ++lg_;
  }
  const uint32_t lg = lg_, K = 1u << lg_;
  const bool ahead = kAheadCycles && lg_ > 0;  // one cycle at a time otherwise
  // A massless gluon's two dipole ends become two items (half the longest
  // lane's work in a round) whenever that takes no more rounds than one item
  // per gluon; otherwise, and with quark masses, one item per gluon.
  const uint32_t kge = !kMassive && (K * (2 * n_g1 + n_q) + 63) / 64 == (K * (n_g1 + n_q) + 63) / 64 ? 2u : 1u;
  const uint32_t n_g = kge * n_g1;
  const uint32_t vg = K * n_g, vt = vg + K * n_q;  // positions of the rounds: gluon items, then quark items
  sh.gstart[lane] = kge * (uint32_t)(excl & kF);
  sh.qstart[lane] = (uint32_t)((excl >> 21) & kF);
  sh.sstart[lane] = (uint32_t)(excl >> 42);
  if (lane == 63) {
    sh.gstart[64] = n_g;
    sh.qstart[64] = n_q;
    sh.sstart[64] = n_s;
  }
  // longest per-event run of items in either section: a round's segmented
  // max needs only the shuffle steps below it
  const uint32_t gmax = kge * wave_max((uint32_t)(mine & kF)), qmax = wave_max((uint32_t)((mine >> 21) & kF));
  // list length; a spare entry past its end takes the writes beyond it, so
  // the listing loops need no branch.  The stale partons follow the items.
  constexpr uint32_t kItems = sizeof(sh.item) / sizeof(sh.item[0]) - 2;
  const uint32_t sbase = n_g + n_q < kItems ? n_g + n_q : kItems;
  if (trial) {  // list this event's items (beyond the lists' lengths rounds search the offsets instead)
    uint32_t gpos = kge * (uint32_t)(excl & kF), qpos = n_g + (uint32_t)((excl >> 21) & kF),
             spos = (uint32_t)(excl >> 42);
    for (uint32_t w = 0; w < words; ++w) {
      const int lo = 64 * (int)w;
      const uint64_t live = s.n >= lo + 64 ? ~0ull : (s.n > lo ? (1ull << (s.n - lo)) - 1ull : 0ull);
      const uint32_t top = (lane << 10) | (uint32_t)lo;
      for (uint64_t x = mym[w] & live; x; x &= x - 1) {  // gluons, ascending
        const uint16_t item = (uint16_t)(top | (uint32_t)__builtin_ctzll(x));
        sh.item[gpos < kItems ? gpos : kItems] = item;
        sh.item[gpos + kge - 1 < kItems ? gpos + kge - 1 : kItems] = item;  // the second end's item
        gpos += kge;
      }
      for (uint64_t x = ~mym[w] & live; x; x &= x - 1) {  // quarks, ascending
        sh.item[qpos < kItems ? qpos : kItems] = (uint16_t)(top | (uint32_t)__builtin_ctzll(x));
        ++qpos;
      }
      if (kCached)
        for (uint64_t x = mys[w] & live; x; x &= x - 1) {  // stale partons
          sh.item[sbase + spos < kItems ? sbase + spos : kItems] = (uint16_t)(top | (uint32_t)__builtin_ctzll(x));
          ++spos;
        }
    }
  }
  sh.lt[lane] = s.lt;
  sh.tcut[lane] = s.tcut;
  sh.ltc[lane] = s.ltc;
  sh.cfac[lane] = s.cfac;
  sh.slot[lane] = (uint32_t)slot;
  if constexpr (!kOne) {
    sh.key[0][lane] = s.key.ev_lo;
    sh.key[1][lane] = s.key.ev_hi;
    sh.key[2][lane] = s.key.k0;
    sh.key[3][lane] = s.key.k1;
  } else if (lane == 0) {
    sh.key[2][0] = (uint32_t)one.seed;
    sh.key[3][0] = (uint32_t)(one.seed >> 32);
  }
  sh.cycle[lane] = s.cycle;
  sh.best_v[lane] = -INFINITY;
  sh.best_idx[lane] = kNoTrial;
  sh.counts[lane] = 0;
  if (kMassive) {
    sh.mc[lane] = qm.c;
    sh.mb[lane] = qm.b;
  }
  __syncthreads();
  // --- rebuild the cache entries of the stale partons, 64 per round
  if (kCached && n_s > 0) {
    for (uint32_t r0 = 0; r0 < n_s; r0 += 64) {
      const uint32_t at = r0 + lane;
      if (at < n_s) {
        uint32_t o, i;
        if (sbase + at < kItems) {
          const uint32_t it = sh.item[sbase + at];
          o = it >> 10;
          i = it & 1023u;
        } else {
          o = owner_of(sh.sstart, at);
          i = select_slot(sm + (uint64_t)o * words, words, at - sh.sstart[o], true);
        }
        if constexpr (kMassive)
          entry_build_massive(sh.cfac[o], sh.tcut[o], slots, sh.slot[o], (int)i, ec, wave_col + o,
                              QuarkMasses{0.0, 0.0, 0.0, sh.mc[o], sh.mb[o]});
        else
          entry_build(sh.cfac[o], sh.tcut[o], slots, sh.slot[o], (int)i, ec, wave_col + o);
      }
    }
    __threadfence_block();  // the rebuilt entries are stored before any trial round reads them
    __syncthreads();
    if (trial)
      for (uint32_t w = 0; w < words; ++w) mys[w] = 0ull;
  }
  // --- trials, 64 items per round: the gluon items, then the quark items
  // (a round may hold the end of one and the start of the other: its quark
  // lanes finish early, in time the round takes for its gluons anyway); with
  // cycles evaluated ahead, item j of a section takes its positions j K ..
  // j K + K - 1, one per cycle, so each (event, cycle) run strides by K
  const uint32_t run = gmax > qmax ? gmax : qmax;
  // the end-cache entry of the lane's item in the coming round is loaded
  // while the current round reduces its winners (an item past the list's
  // end loads its own)
  constexpr bool kPre = kAhead && kCached && !kMassive;
  Ent5 pw{{0ull, 0ull, 0ull, 0ull, 0ull}};
  bool pre = false;
  if (kPre) pre = prefetch_entry(sh.item, list_pos(lane, vg, n_g, lg), n_g + n_q, kItems, ec, wave_col, pw);
  // (the rounds' code compiled twice: one cycle at a time it takes no cycle
  // index and no pair rank)
  auto rounds = [&](auto kA) {
    constexpr bool A = decltype(kA)::value;
    const uint32_t lg = A ? lg_ : 0u, K = 1u << lg;
    for (uint32_t r0 = 0; r0 < vt; r0 += 64) {
      const uint32_t at = r0 + lane;  // position in the rounds
      const bool gsec = at < vg;
      const uint32_t* st = gsec ? sh.gstart : sh.qstart;
      const uint32_t vbase = gsec ? 0u : vg;  // first position of the section
      const uint32_t j = (at - vbase) >> lg;  // item index within the section
      const uint32_t k = (at - vbase) & (K - 1u);  // cycle ahead
      const bool active = at < vt;
      double v = -INFINITY;
      uint32_t idx = kNoTrial;
      uint32_t o = 63, first = 0, last = 0, pr = 63;
      if (active) {
        uint32_t i;
        const uint32_t lp = (gsec ? 0u : n_g) + j;  // list position
        if (lp < kItems) {
          const uint32_t it = sh.item[lp];
          o = it >> 10;
          i = it & 1023u;
        } else {
          o = owner_of(st, j);
          i = select_slot(gm + (uint64_t)o * words, words, gsec ? (j - st[o]) / kge : j - st[o], gsec);
        }
        // a gluon item's ends: both, or (two items per gluon) the parity of
        // its place in the owner's run
        const int e_lo = gsec && kge == 2 ? (int)((j - st[o]) & 1u) : 0, e_hi = gsec && kge == 2 ? e_lo : 1;
        first = vbase + (st[o] << lg) + k;  // position of the owner's first item of this cycle in the section
        last = (j + 1 == st[o + 1]) || lane + K > 63u;
        pr = A ? ((uint32_t)__popcll(tmask & ((1ull << o) - 1ull)) << lg) | k : o;
        // ahead: trials compared by ln(R)/c alone (the scale added at the decision)
        const TrialCtx c{key_of(o),
                         A ? 0.0 : sh.lt[o], sh.tcut[o], sh.ltc[o], sh.cfac[o], sh.cycle[o] + k};
        double best = A ? -INFINITY : c.ltc, wia = 0.0, wib = 0.0;
        uint32_t widx = kNoTrial;
        uint32_t nt = 0, ne = 0;
        if constexpr (kMassive && kCached)
          parton_trials_mcached(c, wave_col + o, (int)i, ec, best, widx, nt, ne);
        else if constexpr (kMassive)
          parton_trials_mflat(c, slots, sh.slot[o], (int)i, QuarkMasses{0.0, 0.0, 0.0, sh.mc[o], sh.mb[o]}, best,
                              widx, nt, ne);
        else
          item_trials(c, slots, sh.slot[o], (int)i, e_lo, e_hi, ec, wave_col + o, kCached, kPre && pre, pw, best, widx,
                      wia, wib, nt, ne);
        if (widx != kNoTrial) {
          v = best;
          idx = (widx << 6) | lane;  // same order as widx: items of one pair differ in i
          if constexpr (!kMassive) {
            sh.coef[0][lane] = wia;
            sh.coef[1][lane] = wib;
          }
        }
        atomicAdd(&sh.counts[pr], nt | (ne << 16));  // at most 12 x 1024 trials and 2048 ends per cycle
      }
      if (kPre) pre = prefetch_entry(sh.item, list_pos(r0 + 64 + lane, vg, n_g, lg), n_g + n_q, kItems, ec, wave_col, pw);
      for (uint32_t d = 1; (d << lg) < 64 && d < run; d <<= 1) {
        const uint32_t dd = d << lg;
        const double vn = __shfl_up(v, dd);
        const uint32_t in = __shfl_up(idx, dd);
        if (active && lane >= dd && at - dd >= first && beats(vn, in, v, idx)) {
          v = vn;
          idx = in;
        }
      }
      // fold each run's best into its pair's: gluon runs first, then quark
      // runs (one pair may end a run of each kind in the same round)
      if (active && last && gsec && beats(v, idx, sh.best_v[pr], sh.best_idx[pr])) {
        sh.best_v[pr] = v;
        sh.best_idx[pr] = idx;
        if constexpr (!kMassive) {
          sh.best_c[0][pr] = sh.coef[0][idx & 63u];
          sh.best_c[1][pr] = sh.coef[1][idx & 63u];
        }
      }
      if (active && last && !gsec && beats(v, idx, sh.best_v[pr], sh.best_idx[pr])) {
        sh.best_v[pr] = v;
        sh.best_idx[pr] = idx;
        if constexpr (!kMassive) {
          sh.best_c[0][pr] = sh.coef[0][idx & 63u];
          sh.best_c[1][pr] = sh.coef[1][idx & 63u];
        }
      }
      __syncthreads();
    }
  };
  if (ahead) rounds(std::true_type{});
  else rounds(std::false_type{});
  if (kAhead) {  // the event's trial constants, published to LDS above, come back from there
    s.key = key_of(lane);
    s.lt = sh.lt[lane];
    s.tcut = sh.tcut[lane];
    s.ltc = sh.ltc[lane];
    s.cfac = sh.cfac[lane];
    s.cycle = sh.cycle[lane];
  }
  // --- each owner that made trials decides its cycle
  if (ahead) {
    // one lane per (event, cycle) pair: the pair's scale, cutoff and veto;
    // its outcome goes into the low bits of its best_idx entry (the lane
    // of the winning item is not needed any more)
    const uint32_t n_pairs = (uint32_t)__popcll(tmask) << lg;
    const uint32_t o = lane < n_pairs ? select64(tmask, lane >> lg) : lane;  // the pair's event
    const double asmax = __shfl(s.asmax, (int)o);                              // its trial alpha_s
    if (lane < n_pairs) {
      const uint32_t rk = lane >> lg, k = lane & (K - 1u);
      const uint32_t cyc = sh.cycle[o] + k, bi = sh.best_idx[lane];
      uint32_t f = kPairVeto;
      double l = sh.lt[o], t = 0.0, z = 0.0, wf = 1.0;
      if (cyc >= climit_of(o)) {
        f = kPairLimit;
      } else if (bi == kNoTrial) {
        f = kPairDone;  // no end with phase space above the cutoff
      } else {
        for (uint32_t q = 0; q <= k; ++q) l += sh.best_v[(rk << lg) | q];  // the winners' scales, in cycle order
        if (!(l > sh.ltc[o])) {
          f = kPairDone;
        } else {
          Winner w{0.0, 0.0, 0.0, 0.0, -1, 0, 0};
          w.K = (int)((bi >> 6) & 15u);
          end_from_inverse(sh.cfac[o], sh.tcut[o], w.K, sh.best_c[0][lane], sh.best_c[1][lane], w);
          t = exp(l);
          const U4 a = key_of(o).draw(cyc, kPurposeAccept, 0);
          z = trial_z(w, unit(a.x, a.y));
          const double prob = massless_ratio(w.K, l, t, z, w.rq2, asmax);
          if (prob >= 0.0 && accept_test(prob, a, wf)) f = kPairAccept;
        }
      }
      sh.best_idx[lane] = (bi & ~63u) | f;
      sh.coef[0][lane] = l;  // the cycle's scale (its own reads of coef are over)
      sh.coef[1][lane] = wf;
      sh.best_c[0][lane] = t;
      sh.best_c[1][lane] = z;
    }
    __syncthreads();
    // each event takes its pairs in cycle order up to the first that ends
    // the sequence: the steps of a cycle-by-cycle decision
    if (trial) {
      const uint32_t rk = (uint32_t)__popcll(tmask & ((1ull << lane) - 1ull));
      for (uint32_t k = 0; k < K; ++k) {
        const uint32_t pr = (rk << lg) | k;
        const uint32_t f = sh.best_idx[pr] & 63u;
        if (f == kPairLimit) {
          s.status = kCycleLimitHit;
          break;
        }
        s.trials += sh.counts[pr] & 0xFFFFu;
        s.ends += sh.counts[pr] >> 16;
        const uint32_t this_cycle = s.cycle++;
        if (f == kPairDone) {
          s.status = kDone;
          break;
        }
        s.lt = sh.coef[0][pr];
        wsh() *= sh.coef[1][pr];
        if (f == kPairAccept) {
          if (s.n == s.cap) {
            s.status = kOverflow;
          } else {
            const uint32_t wi = sh.best_idx[pr] >> 6;
            pd = Pending{sh.best_c[0][pr], sh.best_c[1][pr], (int)(wi >> 14), (int)((wi >> 4) & 1023u),
                         (int)(wi & 15u), this_cycle};
            pend = true;
          }
          break;
        }
      }
    }
  } else if (trial && kMassive) {
    s.trials += sh.counts[lane] & 0xFFFFu;
    s.ends += sh.counts[lane] >> 16;
    const uint32_t bi = sh.best_idx[lane];
    MWinner W{Winner{0.0, 0.0, 0.0, 0.0, -1, 0, 0}, 0.0, 0.0, 0.0, 0.0, 1.0, false};
    double best = s.ltc;
    if (bi != kNoTrial) {
      const uint32_t wi = bi >> 6;
      best = sh.best_v[lane];
      W = massive_winner(trial_ctx(s), slots, slot, (int)(wi >> 14), (int)((wi >> 4) & 1023u), (int)(wi & 15u), qm);
    }
    pend = veto_decide_massive(s, best, W, acc, pd, wsh());
  } else if (trial) {
    s.trials += sh.counts[lane] & 0xFFFFu;
    s.ends += sh.counts[lane] >> 16;
    const uint32_t bi = sh.best_idx[lane];
    Winner w{0.0, 0.0, 0.0, 0.0, -1, 0, 0};
    double best = s.ltc;
    if (bi != kNoTrial) {
      const uint32_t wi = bi >> 6;
      w.i = (int)(wi >> 14);
      w.k = (int)((wi >> 4) & 1023u);
      w.K = (int)(wi & 15u);
      best = sh.best_v[lane];
      // the winning end's coefficients, passed on by the item that drew the
      // winner: its cache entry's numbers (or, without a cache, what the item
      // computed from the records, the same numbers)
      end_from_inverse(s.cfac, s.tcut, w.K, sh.best_c[0][lane], sh.best_c[1][lane], w);
    }
    pend = veto_decide_drawn(s, best, w, acc, pd, wsh());
  }
  // --- pending emissions, built together; the new parton's type goes into the mask
  const uint32_t n_pend = __popcll(__ballot(pend));
  const uint32_t n_busy = __popcll(__ballot(busy));
  if (n_pend > 0 && kEmitDiv * n_pend >= n_busy && pend) {
    const int j = s.n;
    // i's and k's colour partners before the emission, loaded beside the
    // emission's own reads: j takes the place of one partner of each, so
    // with i, j and k they are the partners afterwards
    const uint64_t oi = (uint64_t)pd.i * slots.stride + slot, ok = (uint64_t)pd.k * slots.stride + slot;
    const int pci = slots.cpart[oi], pai = slots.apart[oi], pck = slots.cpart[ok], pak = slots.apart[ok];
    if constexpr (kMassive) emit_massive(s, slots, slot, pd, qm);
    else emit(s, slots, slot, pd);
    if (pd.K <= 10) mym[j >> 6] |= 1ull << (j & 63);               // gluon emitted
    else mym[pd.i >> 6] &= ~(1ull << (pd.i & 63));                 // g -> f fbar: i is now a quark
    // ends whose momenta or partners changed: those of i, j, k and of the
    // other colour partners of i and k (partner links are symmetric)
    set_bit(mys, pd.i);
    set_bit(mys, j);
    set_bit(mys, pd.k);
    set_bit(mys, pci);
    set_bit(mys, pai);
    set_bit(mys, pck);
    set_bit(mys, pak);
    pend = false;
  }
  if (busy && !pend && s.status == kRunning && s.cycle >= climit_of(lane)) s.status = kCycleLimitHit;
}

// Plain one-launch form with the flattened mapping: wave w owns events
// 64w .. 64w+63 of the batch (already started by k_me) from start to cutoff,
// with no refill; finished lanes only stop contributing trial work.
// kFour (massless, at most 128 partons): four resident waves per SIMD (128
// registers, a few spilled; 9.2 + 1 KB of LDS), the trial constants
// reloaded from LDS after the rounds (kAhead); otherwise three waves, the
// massive instantiation reloading them too to fit without spilling.
template <bool kMassive, bool kOne, bool kFour = false>
__global__ void __launch_bounds__(64, kFour ? 4 : 3)
    k_shower_plain_flat(Records r, Summary sm, EventInputs in, uint32_t n, EndCache ec) {
  __shared__ FlatShared<kOne, kFour> sh;
  const OneRequest one{in.seed, in.first, in.cycle_limit};
  const uint32_t lane = threadIdx.x;
  const uint32_t words = mask_words(r.cap);
  const uint64_t e = (uint64_t)blockIdx.x * 64 + lane;
  EvState s = {};
  s.status = kDone;
  bool busy = e < n;
  bool pend = false;
  Pending pd{};
  if (busy) {
    init_state(s, r, e, make_keyed(in.seed, in.first + e), in.ecm_of(e), in.tcut_of(e), in.t_over,
               sm.i[kSiN * sm.stride + e], (int)r.cap);
    if constexpr (!kOne) sh.climit[lane] = in.cycle_limit;
    sh.wsh[lane] = 1.0;
    mask_init(flat_gmask + (uint64_t)lane * words, flat_gmask + (uint64_t)(64 + lane) * words, words, r, e, s.n);
  }
  while (__any(busy)) {
    flat_cycle<true, kMassive, kMassive || kFour, !kMassive, kOne>(sh, one, flat_gmask, words, s, busy, pend, pd, r, e, ec,
                                                          e - lane, lane, in.qm);
    if (busy && s.status != kRunning) {
      s.wsh = sh.wsh[lane];
      write_state(s, sm, e);
      busy = false;
    }
    __syncthreads();
  }
}

size_t flat_lds_bytes(uint32_t cap) { return (size_t)2 * 64 * ((cap + 63) / 64) * 8; }

// cache: [event][cap] entries of kCacheWords words (column = event), or null
void launch_shower_plain_flat(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
                              uint64_t* cache, hipStream_t st) {
  if (!n) return;
  const EndCache ec{cache, r.cap};
  const dim3 g((n + 63) / 64), b(64);
  const size_t lds = flat_lds_bytes(r.cap);
  // Massless events: the single-request LDS layout; up to 128 partons per
  // record it leaves room for 3.5 to 4 blocks per SIMD, which the four-wave
  // build fills with 128 registers by reloading its trial constants from
  // LDS after the rounds (and loading the next round's cache entries
  // ahead); above that the masks make LDS the bound and the three-wave
  // build is faster.  With quark masses: the per-event layout up to 64
  // partons, single-request above.
  if (in.massive) {
    if (r.cap > kOneAboveCap) hipLaunchKernelGGL((k_shower_plain_flat<true, true>), g, b, lds, st, r, s, in, n, ec);
    else hipLaunchKernelGGL((k_shower_plain_flat<true, false>), g, b, lds, st, r, s, in, n, ec);
  } else {
    if (r.cap > kFourMaxCap) hipLaunchKernelGGL((k_shower_plain_flat<false, true>), g, b, lds, st, r, s, in, n, ec);
    else hipLaunchKernelGGL((k_shower_plain_flat<false, true, true>), g, b, lds, st, r, s, in, n, ec);
  }
}

// kCached: A.cache holds an end cache per lane (always when in place; the
// serving epochs' staging slots have one unless it could not be allocated).
// In place (one request, kOne): four resident waves per SIMD for massless
// events with at most 128 partons (kFour: 128 registers, no spills; LDS
// allows 3.5 at 128), three with more partons or with quark masses.  Three for
// massless events in the serving epochs' cached staging slots (a few
// spilled registers, outweighed by the third wave: 4000 requests/s of the
// serving mix keep p99 below 40 ms instead of 80); two otherwise.
template <bool kInPlace, bool kMassive, bool kCached, bool kOne = false, bool kFour = false>
__global__ void __launch_bounds__(64, kFour ? 4 : (kInPlace || (kCached && !kMassive) ? 3 : 2))
    k_shower_flat(PersistArgs A) {
  static_assert(kInPlace || !kOne, "one request per launch only in place");
  static_assert(kOne || !kFour, "four waves need the single-request layout");
  // three waves in place: the shower weight in a register and the short
  // item list, so that 256-parton records fit twelve blocks per CU
  constexpr bool kRegW = kOne && !kFour;
  __shared__ FlatShared<kOne, kFour, kRegW> sh;
  const OneRequest one = kOne ? OneRequest{A.reqs[0].seed, A.reqs[0].first, A.reqs[0].cycle_limit}
                              : OneRequest{0ull, 0ull, 0u};
  const uint32_t lane = threadIdx.x;
  const uint32_t words = mask_words(A.slots.cap);
  const uint64_t L = (uint64_t)blockIdx.x * 64 + lane;
  EvState s = {};
  s.status = kDone;
  bool busy = false;
  bool drained = false;
  bool pend = false;
  Pending pd{};
  uint32_t req = 0;
  uint64_t ev = 0;
  uint64_t slot = L;
  uint32_t since = 0;
  while (true) {
    if (refill<(kInPlace ? 16u : 1u)>(A, busy, 64, lane, since, drained, req, ev)) {
      slot = kInPlace ? ev : L;
      start_event<kInPlace>(s, A, A.reqs[req], ev, slot);
      if constexpr (!kOne) sh.climit[lane] = A.reqs[req].cycle_limit;
      if constexpr (kRegW) s.wsh = 1.0;
      else sh.wsh[lane] = 1.0;
      mask_init(flat_gmask + (uint64_t)lane * words, flat_gmask + (uint64_t)(64 + lane) * words, words, A.slots,
                slot, s.n);
      busy = true;
    }
    if (!__any(busy)) break;
    flat_cycle<kCached, kMassive, kInPlace, kCached && !kMassive, kOne>(
        sh, one, flat_gmask, words, s, busy, pend, pd, A.slots, slot, A.cache, L - lane, lane, A.reqs[req].qm);
    if (busy && s.status != kRunning) {
      if constexpr (!kRegW) s.wsh = sh.wsh[lane];
      finish_event<kInPlace>(s, A, A.reqs[req], ev, slot);
      busy = false;
    }
    __syncthreads();
    ++since;
  }
}

// Writes a batch's request and segment descriptors (passed by value, so the
// launch carries them) and zeroes the work counter.
__global__ void k_setup(ReqDev* rd, ReqDev d, Segment* sd, Segment s, unsigned long long* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *rd = d;
    *sd = s;
    *counter = 0ull;
  }
}

__global__ void k_zero(double* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
uint32_t persistent_lanes(const vsh_ctx* ctx) {
  const uint32_t waves = std::max<uint32_t>(1, ctx->tuned.pers_waves_per_cu) * (uint32_t)ctx->n_cu;
  return waves * 64;
}

uint64_t slots_bytes(uint64_t lanes, uint32_t cap) { return lanes * cap * (4 * 8 + 1 + 4 * 2) + 9 * 256; }

uint64_t request_out_bytes(uint64_t n, uint32_t cap, bool partners) {
  return n * cap * (4 * 8 + 1 + 2 * 2 + (partners ? 2 * 2 : 0)) + n * (kNSumD * 8 + kNSumI * 4 + 8) + 2 * n * 8 + 16 * 256 +
         kHistDoubles * 8;
}


Carver::Carver(void* base) : p(static_cast<char*>(base)) {}
char* Carver::take(uint64_t bytes) {
  char* q = p;
  p += align_up(bytes, 256);
  return q;
}

Records carve_slots(Carver& c, uint64_t lanes, uint32_t cap) {
  Records r;
  const uint64_t n = lanes * cap;
  r.E = (double*)c.take(n * 8);
  r.x = (double*)c.take(n * 8);
  r.y = (double*)c.take(n * 8);
  r.z = (double*)c.take(n * 8);
  r.pid = (int8_t*)c.take(n);
  r.col = (uint16_t*)c.take(n * 2);
  r.acol = (uint16_t*)c.take(n * 2);
  r.cpart = (uint16_t*)c.take(n * 2);
  r.apart = (uint16_t*)c.take(n * 2);
  r.stride = lanes;
  r.cap = cap;
  return r;
}

ReqBuffers carve_request(Carver& c, uint64_t n, uint32_t cap, bool partners) {
  ReqBuffers b;
  const uint64_t m = n * cap;
  b.out.E = (double*)c.take(m * 8);
  b.out.x = (double*)c.take(m * 8);
  b.out.y = (double*)c.take(m * 8);
  b.out.z = (double*)c.take(m * 8);
  b.out.pid = (int8_t*)c.take(m);
  b.out.col = (uint16_t*)c.take(m * 2);
  b.out.acol = (uint16_t*)c.take(m * 2);
  b.out.cpart = partners ? (uint16_t*)c.take(m * 2) : nullptr;
  b.out.apart = partners ? (uint16_t*)c.take(m * 2) : nullptr;
  b.out.stride = n;
  b.out.cap = cap;
  // the results in one span, in the order the serving drain copies them
  // back: histogram, integer fields, then the doubles (weight first), hash
  b.hist = (double*)c.take(kHistDoubles * 8);
  b.sum.i = (int32_t*)c.take(kNSumI * n * 4);
  b.sum.d = (double*)c.take(kNSumD * n * 8);
  b.sum.hash = (uint64_t*)c.take(n * 8);
  b.sum.stride = n;
  b.ecm = (double*)c.take(n * 8);
  b.tcut = (double*)c.take(n * 8);
  return b;
}

Scratch carve_scratch(Carver& c, uint64_t n, uint32_t cap) { return carve_obs_scratch(c.p, n, cap); }

// Lanes of the largest persistent grid (16 waves on each of 256 CUs): the
// stride of a batch's end-coefficient cache, whatever the tuning.
constexpr uint64_t kCacheLanes = 16ull * 256 * 64;

uint64_t cache_bytes(uint32_t cap, bool massive) {
  return align_up(kCacheLanes * cap * cache_words(massive) * 8, 256);
}

// A batch is one request, showered in place in its output records.
uint64_t batch_bytes(uint64_t n, uint32_t cap, bool massive) {
  return request_out_bytes(n, cap, true) + cache_bytes(cap, massive) + obs_scratch_bytes(n, cap) + 4096 +
         sizeof(ReqDev) + sizeof(Segment) + 1024;
}

BatchLayout carve_batch(void* base, uint64_t n, uint32_t cap, bool massive) {
  Carver c(base);
  BatchLayout L;
  L.buf = carve_request(c, n, cap, true);
  L.cache.rec = (uint64_t*)c.take(kCacheLanes * cap * cache_words(massive) * 8);
  L.cache.cap = cap;
  L.sc = carve_scratch(c, n, cap);
  L.counter = (unsigned long long*)c.take(256);
  L.reqs = (ReqDev*)c.take(sizeof(ReqDev));
  L.segs = (Segment*)c.take(sizeof(Segment));
  L.end = c.p;
  return L;
}

// The kernel of a mapping, in place or not, for requests with or without
// quark masses; the flattened mapping with or without an end cache (in place
// always has one).
const void* persistent_kernel(uint32_t mapping, bool in_place, bool massive, bool cached, uint32_t cap) {
  if (mapping == kMapFlat) {
    if (in_place && massive) return (const void*)k_shower_flat<true, true, true, true>;
    if (in_place)  // four-wave build up to 128 partons (LDS-bound above)
      return cap > kFourMaxCap ? (const void*)k_shower_flat<true, false, true, true>
                               : (const void*)k_shower_flat<true, false, true, true, true>;
    if (cached)
      return massive ? (const void*)k_shower_flat<false, true, true> : (const void*)k_shower_flat<false, false, true>;
    return massive ? (const void*)k_shower_flat<false, true, false> : (const void*)k_shower_flat<false, false, false>;
  }
  if (massive)
    return in_place ? (const void*)k_shower_persistent<true, true> : (const void*)k_shower_persistent<false, true>;
  return in_place ? (const void*)k_shower_persistent<true> : (const void*)k_shower_persistent<false>;
}

uint32_t persistent_block(uint32_t mapping, uint32_t block) { return mapping == kMapFlat ? 64u : block; }

void launch_persistent(const PersistArgs& A, uint64_t lanes, uint32_t block, uint32_t mapping, bool in_place,
                       bool massive, hipStream_t st) {
  block = persistent_block(mapping, block);
  const dim3 grid((uint32_t)(lanes / block));
  const size_t lds = mapping == kMapFlat ? flat_lds_bytes(A.slots.cap) : 0;
  void* args[] = {const_cast<PersistArgs*>(&A)};
  (void)hipLaunchKernel(persistent_kernel(mapping, in_place, massive, A.cache.rec != nullptr, A.slots.cap), grid,
                        dim3(block), args, lds, st);
}

void launch_setup(ReqDev* rd, const ReqDev& d, Segment* sd, const Segment& s, unsigned long long* counter,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, rd, d, sd, s, counter);
}

void launch_zero(double* p, uint32_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}

// Host-side graph of one batch: [ev0] reset [ev1] persistent [ev2] obs [ev3].
// The event nodes are pointed at the call's timing events (or at the
// context's idle set) before each launch.
static vsh_status build_batch_graph(vsh_ctx* ctx, BatchGraph& g, const PersistArgs& A, const ReqDev& d,
                                    const Segment& sg, uint64_t lanes, uint32_t block, const BatchLayout& L,
                                    const EventInputs& in, uint64_t n, double* hist) {
  hipError_t err;
#define GCHK(x)                                          \
  do {                                                   \
    err = (x);                                           \
    if (err != hipSuccess) return hip_fail(ctx, err, #x); \
  } while (0)
  GCHK(hipGraphCreate(&g.graph, 0));
  hipGraphNode_t prev = nullptr;
  auto add_event = [&](int k) -> hipError_t {
    hipGraphNode_t node;
    hipError_t e = hipGraphAddEventRecordNode(&node, g.graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                              ctx->idle_ev[k]);
    if (e == hipSuccess) {
      g.ev_nodes[k] = node;
      prev = node;
    }
    return e;
  };
  auto add_kernel = [&](const void* fn, dim3 grid, dim3 blk, void** args, unsigned lds = 0) -> hipError_t {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(fn);
    p.gridDim = grid;
    p.blockDim = blk;
    p.sharedMemBytes = lds;
    p.kernelParams = args;
    p.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
    if (e == hipSuccess) prev = node;
    return e;
  };
  g.args = A;
  g.d = d;
  g.s = sg;
  g.rd = L.reqs;
  g.sd = L.segs;
  g.counter = L.counter;
  g.rec = L.buf.out;
  g.sum = L.buf.sum;
  g.in = in;
  g.sc = L.sc;
  g.n = (uint32_t)n;
  g.hist = hist;
  GCHK(add_event(0));
  void* a_setup[] = {&g.rd, &g.d, &g.sd, &g.s, &g.counter};
  GCHK(add_kernel((const void*)k_setup, dim3(1), dim3(64), a_setup));
  void* a_me[] = {&g.rec, &g.sum, &g.in, &g.n, &g.no_hist};
  GCHK(add_kernel((const void*)k_me, dim3((uint32_t)((n + 255) / 256)), dim3(256), a_me));
  GCHK(add_event(1));
  void* a_pers[] = {&g.args};
  const bool massive = g.in.massive != 0;
  GCHK(add_kernel(persistent_kernel(g.mapping, true, massive, true, A.slots.cap), dim3((uint32_t)(lanes / block)),
                  dim3(block),
                  a_pers, g.mapping == kMapFlat ? (unsigned)flat_lds_bytes(A.slots.cap) : 0u));
  GCHK(add_event(2));
  g.nb = L.buf.out.cap + 1;
  g.cap = L.buf.out.cap;
  const bool fixed = g.in.fixed_hist != 0;
  g.ih = fixed ? g.sc.ihist : nullptr;
  g.wm = fixed ? g.sc.wmax : nullptr;
  void* a_zero[] = {&g.sc.cnt, &g.nb, &g.sc.hcopy, &g.ih, &g.wm};
  GCHK(add_kernel((const void*)k_obs_reset, dim3(obs_reset_blocks(g.nb)), dim3(256),
                  a_zero));
  const uint32_t eb = obs_sort_blocks(n);
  void* a_count[] = {&g.sum, &g.n, &g.cap, &g.sc.cnt, &g.wm};
  GCHK(add_kernel((const void*)k_obs_count, dim3(eb), dim3(256), a_count));
  void* a_scan[] = {&g.sc.cnt, &g.nb};
  GCHK(add_kernel((const void*)k_obs_scan, dim3(1), dim3(256), a_scan));
  void* a_scatter[] = {&g.sum, &g.n, &g.cap, &g.sc.cnt, &g.sc.perm};
  GCHK(add_kernel((const void*)k_obs_scatter, dim3(eb), dim3(256), a_scatter));
  void* a_obs[] = {&g.rec, &g.sum, &g.in, &g.sc, &g.n, &g.hist};
  const uint32_t ob = (uint32_t)(std::min<uint64_t>(g.sc.stride, (n + 255) / 256 * 256) / 256);
  GCHK(add_kernel(obs_kernel(massive), dim3(ob), dim3(256), a_obs));
  g.perm_c = g.sc.perm;
  g.cnt_c = g.sc.cnt;
  ObsGroupLaunch gl[3];
  const uint32_t ng = obs_group_launches(g.cap, massive, gl);
  for (uint32_t k = 0; k < ng; ++k) {
    g.glo[k] = gl[k].lo;
    g.ghi[k] = gl[k].hi;
    g.gslots[k] = gl[k].slots;
    void* a_grp[] = {&g.rec, &g.sum, &g.in, &g.perm_c, &g.cnt_c, &g.cap, &g.glo[k], &g.ghi[k], &g.gslots[k], &g.hist,
                     &g.sc};
    const uint32_t wb = (uint32_t)std::min<uint64_t>(n, kObsWaveBlocks);
    GCHK(add_kernel(gl[k].fn, dim3(wb), dim3(64), a_grp, gl[k].lds));
  }
  g.fixed = fixed ? 1u : 0u;
  void* a_fin[] = {&g.sc, &g.hist, &g.fixed};
  GCHK(add_kernel((const void*)k_hist_finalize, dim3(1), dim3(256), a_fin));
  GCHK(add_event(3));
  GCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
#undef GCHK
  return VSH_OK;
}

void destroy_graph(BatchGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = BatchGraph{};
}

static void fill_request_desc(ReqDev& d, const ReqBuffers& b, const vsh_request* req, uint64_t first_idx,
                              const double* ecm_dev, const double* tcut_dev) {
  d.out = b.out;
  d.sum = b.sum;
  d.ecm = ecm_dev;
  d.tcut = tcut_dev;
  d.ecm0 = req->ecm;
  d.tcut0 = req->t_cut;
  d.seed = req->seed;
  d.first = req->first_event + first_idx;
  d.count = b.sum.stride;
  d.cycle_limit = effective_cycle_limit(req->cycle_limit);
  d.t_over = req->t_over;
  d.qm = request_masses(*req);
  d.massive = request_massive(*req);
}

// One batch of `n` events of req (starting at request index first_idx)
// through the persistent form on stream st, with the batch's buffers in the
// workspace at `base`.  Inputs: per-event arrays already on the device (or
// null).  Writes the histogram into hist (accumulates).
vsh_status run_batch(vsh_ctx* ctx, const vsh_request* req, uint64_t first_idx, uint64_t n,
                            hipStream_t st, void* base, const double* ecm_dev, const double* tcut_dev,
                            double* hist, bool use_graph, BatchLayout* out_layout) {
  const uint32_t cap = req->max_partons;
  const uint64_t lanes = persistent_lanes(ctx);
  const uint32_t mapping = ctx->tuned.mapping;
  const uint32_t block = persistent_block(mapping, ctx->tuned.pers_block);
  if (lanes > kCacheLanes) {
    set_error(ctx, "persistent grid of %llu lanes exceeds the %llu the batch layout holds",
              (unsigned long long)lanes, (unsigned long long)kCacheLanes);
    return VSH_E_INTERNAL;
  }
  BatchLayout L = carve_batch(base, n, cap, request_massive(*req) != 0);
  if (out_layout) *out_layout = L;
  ReqDev d;
  fill_request_desc(d, L.buf, req, first_idx, ecm_dev, tcut_dev);
  Segment sg{0, 0, 0, n, 0};
  hipError_t err;
  PersistArgs A;
  A.slots = L.buf.out;  // in place
  A.reqs = L.reqs;
  A.segs = L.segs;
  A.n_segs = 1;
  A.total = n;
  A.next = L.counter;
  A.threshold = ctx->tuned.refill_threshold;
  A.period = ctx->tuned.refill_period;
  A.pad = 0;
  A.cache = L.cache;
  EventInputs in{};
  in.ecm = ecm_dev;
  in.tcut = tcut_dev;
  in.ecm0 = req->ecm;
  in.tcut0 = req->t_cut;
  in.seed = req->seed;
  in.first = req->first_event + first_idx;
  in.cycle_limit = effective_cycle_limit(req->cycle_limit);
  in.t_over = req->t_over;
  in.qm = request_masses(*req);
  in.massive = request_massive(*req);
  in.fixed_hist = (req->flags & VSH_HIST_FIXEDPOINT) ? 1u : 0u;
  hipEvent_t* tev = timing_slot(ctx);
  if (use_graph) {
    BatchGraph& g = ctx->graph;
    const bool same = g.exec && std::memcmp(&g.args, &A, sizeof A) == 0 && g.hist == hist && g.n == n &&
                      std::memcmp(&g.in, &in, sizeof in) == 0 && std::memcmp(&g.d, &d, sizeof d) == 0 &&
                      std::memcmp(&g.s, &sg, sizeof sg) == 0 && g.lanes == lanes && g.block == block &&
                      g.mapping == mapping;
    if (!same) {
      destroy_graph(g);
      g.mapping = mapping;
      vsh_status rc = build_batch_graph(ctx, g, A, d, sg, lanes, block, L, in, n, hist);
      if (rc) {
        destroy_graph(g);
        return rc;
      }
      g.lanes = lanes;
      g.block = block;
    }
    for (int k = 0; k < 4; ++k) {
      err = hipGraphExecEventRecordNodeSetEvent(g.exec, g.ev_nodes[k], tev ? tev[k] : ctx->idle_ev[k]);
      if (err != hipSuccess) return hip_fail(ctx, err, "hipGraphExecEventRecordNodeSetEvent");
    }
    err = hipGraphLaunch(g.exec, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "hipGraphLaunch");
  } else {
    if (tev) (void)hipEventRecord(tev[0], st);
    launch_setup(L.reqs, d, L.segs, sg, L.counter, st);
    launch_me(L.buf.out, L.buf.sum, in, (uint32_t)n, st);
    if (tev) (void)hipEventRecord(tev[1], st);
    launch_persistent(A, lanes, block, mapping, true, in.massive != 0, st);
    if (tev) (void)hipEventRecord(tev[2], st);
    launch_obs(L.buf.out, L.buf.sum, in, L.sc, (uint32_t)n, hist, st);
    if (tev) (void)hipEventRecord(tev[3], st);
    err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(ctx, err, "kernel launch");
  }
  return VSH_OK;
}

uint64_t persistent_workspace_bytes_ctx(const vsh_ctx* ctx, const vsh_request* req) {
  return batch_bytes(req->n_events, req->max_partons, request_massive(*req) != 0);
}

uint64_t persistent_workspace_bytes(const vsh_request* req) {
  return batch_bytes(req->n_events, req->max_partons, request_massive(*req) != 0);
}

vsh_status persistent_into(vsh_ctx* ctx, const vsh_request* req, hipStream_t st, void* ws, double* dev_hist,
                           double* dev_sum_d, int32_t* dev_sum_i, uint64_t* dev_hash) {
  const uint64_t n = req->n_events;
  BatchLayout L;
  vsh_status rc = run_batch(ctx, req, 0, n, st, ws, req->ecm_per_event, req->tcut_per_event, dev_hist, true, &L);
  if (rc) return rc;
  hipError_t err;
  if (dev_sum_d) {
    err = hipMemcpyAsync(dev_sum_d, L.buf.sum.d, kNSumD * n * 8, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "summary copy");
  }
  if (dev_sum_i) {
    err = hipMemcpyAsync(dev_sum_i, L.buf.sum.i, kNSumI * n * 4, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "summary copy");
  }
  if (dev_hash) {
    err = hipMemcpyAsync(dev_hash, L.buf.sum.hash, n * 8, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "summary copy");
  }
  return VSH_OK;
}

vsh_status generate_persistent(vsh_ctx* ctx, const vsh_request* req, vsh_result** out) {
  const auto t0 = std::chrono::steady_clock::now();
  const uint32_t cap = req->max_partons;
  const uint64_t lanes = persistent_lanes(ctx);
  // chunk so that a batch fits the budget (half of it when records are returned)
  uint64_t budget = ctx->budget;
  if (req->flags & VSH_RECORDS) budget /= 2;
  if (lanes > kCacheLanes) {
    set_error(ctx, "persistent grid of %llu lanes exceeds the %llu the batch layout holds",
              (unsigned long long)lanes, (unsigned long long)kCacheLanes);
    return VSH_E_INTERNAL;
  }
  const uint64_t fixed = 64 * 1024 + cache_bytes(cap, request_massive(*req) != 0);
  if (budget <= fixed + request_out_bytes(64, cap, true) + obs_scratch_bytes(64, cap)) {
    set_error(ctx, "memory budget too small for the persistent form at %u partons", cap);
    return VSH_E_NOMEM;
  }
  const uint64_t per_event = request_out_bytes(1, cap, true) + 64 + (uint64_t)cap * 32;
  uint64_t chunk = std::min<uint64_t>(req->n_events, (budget - fixed) / per_event);
  chunk = std::min<uint64_t>(chunk, 1ull << 27);
  ResultBox* box = new_result(req->n_events, req->flags & VSH_SUMMARY);
  if (!box) {
    set_error(ctx, "host allocation failed");
    return VSH_E_NOMEM;
  }
  hipStream_t st = ctx->stream;
  float t_me = 0, t_sh = 0, t_obs = 0;
  for (uint64_t a = 0; a < req->n_events; a += chunk) {
    const uint64_t n = std::min(chunk, req->n_events - a);
    vsh_status rc = ctx->arena.reserve(ctx, batch_bytes(n, cap, request_massive(*req) != 0));
    if (rc) {
      delete box;
      return rc;
    }
    BatchLayout L = carve_batch(ctx->arena.ptr, n, cap, request_massive(*req) != 0);
    hipError_t err;
    const double* ecm_dev = nullptr;
    const double* tcut_dev = nullptr;
    if (req->ecm_per_event) {
      err = hipMemcpyAsync(L.buf.ecm, req->ecm_per_event + a, n * 8, hipMemcpyHostToDevice, st);
      if (err != hipSuccess) { delete box; return hip_fail(ctx, err, "input copy"); }
      ecm_dev = L.buf.ecm;
    }
    if (req->tcut_per_event) {
      err = hipMemcpyAsync(L.buf.tcut, req->tcut_per_event + a, n * 8, hipMemcpyHostToDevice, st);
      if (err != hipSuccess) { delete box; return hip_fail(ctx, err, "input copy"); }
      tcut_dev = L.buf.tcut;
    }
    launch_zero(L.buf.hist, kHistDoubles, st);
    (void)hipEventRecord(ctx->ev[0], st);
    PersistArgs A;
    ReqDev d;
    fill_request_desc(d, L.buf, req, a, ecm_dev, tcut_dev);
    const Segment sg{0, 0, 0, n, 0};
    launch_setup(L.reqs, d, L.segs, sg, L.counter, st);
    EventInputs in{};
    in.ecm = ecm_dev;
    in.tcut = tcut_dev;
    in.ecm0 = req->ecm;
    in.tcut0 = req->t_cut;
    in.seed = req->seed;
    in.first = req->first_event + a;
    in.cycle_limit = effective_cycle_limit(req->cycle_limit);
    in.t_over = req->t_over;
    in.qm = request_masses(*req);
    in.massive = request_massive(*req);
    in.fixed_hist = (req->flags & VSH_HIST_FIXEDPOINT) ? 1u : 0u;
    launch_me(L.buf.out, L.buf.sum, in, (uint32_t)n, st);
    A.slots = L.buf.out;  // in place
    A.reqs = L.reqs;
    A.segs = L.segs;
    A.n_segs = 1;
    A.total = n;
    A.next = L.counter;
    A.threshold = ctx->tuned.refill_threshold;
    A.period = ctx->tuned.refill_period;
    A.pad = 0;
    A.cache = L.cache;
    (void)hipEventRecord(ctx->ev[1], st);
    launch_persistent(A, lanes, ctx->tuned.pers_block, ctx->tuned.mapping, true, in.massive != 0, st);
    (void)hipEventRecord(ctx->ev[2], st);
    launch_obs(L.buf.out, L.buf.sum, in, L.sc, (uint32_t)n, L.buf.hist, st);
    (void)hipEventRecord(ctx->ev[3], st);
    err = hipGetLastError();
    if (err != hipSuccess) { delete box; return hip_fail(ctx, err, "kernel launch"); }
    const bool all_fields = !box->sum_d.empty() || (req->flags & VSH_RECORDS);
    const int32_t* n_host = nullptr;
    rc = copy_back_chunk(ctx, st, L.buf.hist, L.buf.sum, n, n, all_fields, box, a, &n_host);
    if (rc) {
      delete box;
      return rc;
    }
    float ms;
    if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) t_me += ms;
    if (hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]) == hipSuccess) t_sh += ms;
    if (hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) t_obs += ms;
    if (req->flags & VSH_RECORDS) {
      vsh_status rc2 = gather_records(ctx, L.buf.out, L.buf.sum.i + kSiN * n, n_host, n, box);
      if (rc2) {
        delete box;
        return rc2;
      }
    }
  }
  box->pub.t_me_ms = t_me;
  box->pub.t_shower_ms = t_sh;
  box->pub.t_obs_ms = t_obs;
  box->pub.t_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  finish_result(box);
  *out = &box->pub;
  return VSH_OK;
}

}  // namespace vsh
