// vsh_persistent.hpp -- device-visible descriptors of the persistent form and
// the host-side layout helpers shared with the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include "vsh_kernels.hpp"

namespace vsh {

// one request as the persistent kernel sees it: where its events' outputs
// go and how to name its events
struct ReqDev {
  Records out;          // final partons [cap][count]; partner links only when showered in place
  Summary sum;          // [field][count]
  const double* ecm;    // per-event sqrt(s) [count] or null -> ecm0
  const double* tcut;   // per-event t_C [count] or null -> tcut0
  double ecm0, tcut0;
  uint64_t seed, first;  // event ids first .. first + count - 1
  uint64_t count;
  uint32_t cycle_limit;  // veto cycles after which a running event is given up (>= 1)
  double t_over;         // scale of alpha_s in the trial density, 0 = the event's t_C
  QuarkMasses qm;        // quark masses
  uint32_t massive;      // any quark mass above zero
};

// a contiguous range of one request's events inside a launch's work space
struct Segment {
  uint32_t req, pad;
  uint64_t lo, hi;   // request event indices [lo, hi)
  uint64_t start;    // first work index of this segment
};

// Per-lane cache of each parton's dipole ends (flattened mapping): entry
// [(lane * cap) + a] of kCacheWords words holds parton a's id and ordered
// spectators, then per end its trial coefficients (the reciprocals of two;
// four coefficients by kernel class for events with quark masses, in entries
// of kMCacheWords words).  Null: no cache.
constexpr int kCacheWords = 5;
constexpr int kMCacheWords = 9;
inline int cache_words(bool massive) { return massive ? kMCacheWords : kCacheWords; }
struct EndCache {
  uint64_t* rec;
  uint32_t cap;
};

struct PersistArgs {
  Records slots;                  // working records: one slot per lane [cap][lanes], or the
                                  // single request's output records when showered in place
  const ReqDev* reqs;
  const Segment* segs;
  uint32_t n_segs;
  uint32_t threshold;             // refill when at least this many lanes idle (or all)
  uint64_t total;                 // work indices 0 .. total-1
  unsigned long long* next;       // work counter, zeroed before the launch
  uint32_t period;                // veto cycles between refill checks
  uint32_t pad;
  EndCache cache;                 // flattened mapping: per-lane end coefficients, or none
};

struct ReqBuffers {
  Records out;
  Summary sum;
  double *ecm, *tcut, *hist;
};

struct Carver {
  char* p;
  explicit Carver(void* base);
  char* take(uint64_t bytes);
};

struct BatchLayout {
  ReqBuffers buf;
  EndCache cache;
  Scratch sc;
  unsigned long long* counter;
  ReqDev* reqs;
  Segment* segs;
  char* end;
};

// the launch sequence of one batch as an instantiated hipGraph; the kernel
// arguments live here so the graph's parameter pointers stay valid
struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t ev_nodes[4] = {nullptr, nullptr, nullptr, nullptr};
  ReqDev* rd = nullptr;
  ReqDev d{};
  Segment* sd = nullptr;
  Segment s{};
  unsigned long long* counter = nullptr;
  PersistArgs args{};
  Records rec{};
  Summary sum{};
  EventInputs in{};
  Scratch sc{};
  uint32_t n = 0, nb = 0, cap = 0, thr = 0;
  uint32_t glo[3] = {0, 0, 0}, ghi[3] = {0, 0, 0}, gslots[3] = {0, 0, 0};
  const uint32_t* perm_c = nullptr;
  const uint32_t* cnt_c = nullptr;
  double* hist = nullptr;
  double* no_hist = nullptr;  // k_me's histogram to clear: none in a batch
  unsigned long long* ih = nullptr;  // fixed-point cells and largest weight (null: FP64 sums)
  unsigned long long* wm = nullptr;
  uint32_t fixed = 0;  // k_hist_finalize's fixed-point flag
  uint64_t lanes = 0;
  uint32_t block = 0;
  uint32_t mapping = 0;
};

uint64_t slots_bytes(uint64_t lanes, uint32_t cap);
uint64_t request_out_bytes(uint64_t n, uint32_t cap, bool partners);
uint64_t obs_scratch_bytes(uint64_t n, uint32_t cap);
Records carve_slots(Carver& c, uint64_t lanes, uint32_t cap);
ReqBuffers carve_request(Carver& c, uint64_t n, uint32_t cap, bool partners);
Scratch carve_scratch(Carver& c, uint64_t n, uint32_t cap);
enum : uint32_t { kMapLane = 0, kMapFlat = 1 };
void launch_persistent(const PersistArgs& A, uint64_t lanes, uint32_t block, uint32_t mapping, bool in_place,
                       bool massive, hipStream_t st);
void launch_setup(ReqDev* rd, const ReqDev& d, Segment* sd, const Segment& s, unsigned long long* counter,
                  hipStream_t st);
void launch_zero(double* p, uint32_t n, hipStream_t st);
void launch_shower_plain_flat(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
                              uint64_t* cache, hipStream_t st);
void destroy_graph(BatchGraph& g);

}  // namespace vsh
