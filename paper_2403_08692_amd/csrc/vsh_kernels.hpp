// vsh_kernels.hpp -- data layout and kernel declarations of the shower engine.
//
// Layout in HBM (structure of arrays, slot-major so that lane e of a wave
// touching parton slot a of its event reads element [a][e]: consecutive lanes,
// consecutive addresses):
//   E, x, y, z      double   [cap][stride]   four-momenta
//   pid             int8     [cap][stride]
//   col, acol       uint16   [cap][stride]   colour / anticolour line, 0 = none
//   cpart, apart    uint16   [cap][stride]   index of the parton holding the
//                                            other end of this parton's colour
//                                            (anticolour) line, 0xFFFF = none
// plus per-event summaries [field][stride] (see vsh.h for the fields).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vsh_device.hpp"

namespace vsh {

constexpr int kNSumD = 10;
constexpr int kNSumI = 7;
constexpr int kNObs = 8;
constexpr int kNBins = 50;
constexpr int kNHCol = kNBins + 2;
constexpr int kHistDoubles = kNObs * kNHCol * 3;
constexpr uint32_t kMaxCount = 1024;  // largest record capacity

// summary field indices
enum { kSdW = 0, kSdCos = 1, kSdY23 = 2, kSdY34 = 3, kSdTau = 4, kSdC = 5, kSdRho = 6, kSdBT = 7,
       kSdBW = 8, kSdPhi = 9 };
enum { kSiN = 0, kSiStatus = 1, kSiCycles = 2, kSiEmit = 3, kSiFlavour = 4, kSiTrials = 5, kSiEnds = 6 };

struct Records {
  double *E, *x, *y, *z;
  int8_t *pid;
  uint16_t *col, *acol, *cpart, *apart;
  uint64_t stride;  // elements per slot row (>= events in the launch)
  uint32_t cap;

  __device__ __forceinline__ P4 load(uint32_t a, uint64_t e) const {
    const uint64_t o = (uint64_t)a * stride + e;
    return P4{E[o], x[o], y[o], z[o]};
  }
  __device__ __forceinline__ void store(uint32_t a, uint64_t e, const P4& p) const {
    const uint64_t o = (uint64_t)a * stride + e;
    E[o] = p.e;
    x[o] = p.x;
    y[o] = p.y;
    z[o] = p.z;
  }
};

struct Summary {
  double *d;       // [kNSumD][stride]
  int32_t *i;      // [kNSumI][stride]
  uint64_t *hash;  // [stride]
  uint64_t stride;
};

struct EventInputs {
  const double *ecm;   // [n] or null -> ecm0
  const double *tcut;  // [n] or null -> tcut0
  double ecm0, tcut0;
  uint64_t seed, first;
  uint32_t cycle_limit;  // veto cycles after which a running event is given up (>= 1)
  double t_over;         // scale of alpha_s in the trial density, 0 = the event's t_C
  QuarkMasses qm;        // quark masses (massive kernels only when `massive`)
  uint32_t massive;      // any quark mass above zero
  uint32_t fixed_hist;   // histogram sums in int64 fixed point (order-independent)
  __device__ __forceinline__ double ecm_of(uint64_t e) const { return ecm ? ecm[e] : ecm0; }
  __device__ __forceinline__ double tcut_of(uint64_t e) const { return tcut ? tcut[e] : tcut0; }
};

struct HistRanges {
  double lo[kNObs], hi[kNObs];
};

// Scratch of the observables pass: thread slot t keeps its current event's
// partons (and Durham's jets) at element [a][t]; the events are visited in
// order of decreasing parton count (perm), so a wave's lanes hold events of
// the same size.
struct Scratch {
  double *E, *x, *y, *z;    // momenta; Durham merges jets in place
  double *ux, *uy, *uz;     // unit three-vectors of the current jets
  double *dn;               // forward nearest-neighbour y
  uint16_t *nn;             // forward nearest neighbour, 0xFFFF none
  uint8_t *dead;            // merged-away jets
  uint64_t stride;          // thread slots
  uint32_t *perm;           // event indices by decreasing parton count [n]
  uint32_t *cnt;            // per-count offsets [cap + 2]
  uint32_t threshold;       // events with at least this many partons: one wave each
  // the blocks' histograms meet in kHistCopies copies (block b adds into
  // copy b mod kHistCopies, so that no cell's atomics queue up behind every
  // block's), summed into the caller's histogram by k_hist_finalize: FP64
  // cells, or (requests with VSH_HIST_FIXEDPOINT) the cells' int64 sums; the
  // largest |w| of the launch's events (as the bits of a non-negative double,
  // which order like the integers) and L = ceil(log2 n)
  double *hcopy;              // [kHistCopies][kHistDoubles]
  unsigned long long *ihist;  // [kHistCopies][kHistDoubles]
  unsigned long long *wmax;   // [1]
  uint32_t lbits;
};

constexpr uint32_t kObsWaveThreshold = 9;
constexpr int kObsRegSlots = 8;  // events of at most this many partons: observables in registers
constexpr uint32_t kObsWaveMaxCap = 512;
constexpr uint32_t kObsSortPer = 16;  // events per thread of the counting sort by parton count
constexpr uint32_t kHistCopies = 16;  // copies of the histogram set that the blocks' atomics spread over
uint32_t obs_sort_blocks(uint64_t n);
// blocks of the group launches (each block's groups stride over the events
// of their size range): many short blocks end more evenly than a grid of
// one or a few rounds of resident blocks (stress, 10^6 events: 8192 blocks
// 7.3 ms, 32768 blocks 6.9 ms; empty blocks leave at once)
constexpr uint32_t kObsWaveBlocks = 32768;

}  // namespace vsh

// host-side launchers (vsh_kernels.hip)
namespace vsh {
// The observables pass runs a grid-stride loop over obs_threads(n, cap)
// threads (at most 2^25 parton slots of scratch in all).
uint64_t obs_threads(uint64_t n, uint32_t cap);
uint64_t obs_scratch_bytes(uint64_t n, uint32_t cap);
Scratch carve_obs_scratch(char*& p, uint64_t n, uint32_t cap);
// k_obs for requests without (false) or with (true) quark masses
const void* obs_kernel(bool massive);
__global__ void k_obs_count(Summary sm, uint32_t n, uint32_t cap, uint32_t* cnt, unsigned long long* wmax);
__global__ void k_obs_reset(uint32_t* cnt, uint32_t nb, double* hcopy, unsigned long long* ihist,
                            unsigned long long* wmax);
__global__ void k_hist_finalize(Scratch sc, double* hist, uint32_t fixed);
uint32_t obs_reset_blocks(uint32_t nb);
__global__ void k_obs_scan(uint32_t* cnt, uint32_t nb);
__global__ void k_obs_scatter(Summary sm, uint32_t n, uint32_t cap, uint32_t* cnt, uint32_t* perm);
__global__ void k_zero_u32(uint32_t* p, uint32_t n);
__global__ void k_me(Records r, Summary s, EventInputs in, uint32_t n, double* zero_hist);
// one launch of the group observables kernel: function, parton-count range
// [lo, hi), LDS parton slots per group, dynamic LDS bytes
struct ObsGroupLaunch {
  const void* fn;
  uint32_t lo, hi, slots, lds;
};
uint32_t obs_group_launches(uint32_t cap, bool massive, ObsGroupLaunch out[3]);
size_t obs_group_lds(uint32_t g, uint32_t slots);
void launch_me(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
               hipStream_t st, double* zero_hist = nullptr);
void launch_shower_plain(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
                         uint32_t block, uint32_t waves, hipStream_t st);
void launch_obs(const Records& r, const Summary& s, const EventInputs& in, const Scratch& sc,
                uint32_t n, double* hist, hipStream_t st);
void launch_shower_init_records(const Records& r, const Summary& s, const EventInputs& in,
                                uint32_t n, hipStream_t st);
}  // namespace vsh
