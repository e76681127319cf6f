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
  __device__ __forceinline__ double ecm_of(uint64_t e) const { return ecm ? ecm[e] : ecm0; }
  __device__ __forceinline__ double tcut_of(uint64_t e) const { return tcut ? tcut[e] : tcut0; }
};

struct HistRanges {
  double lo[kNObs], hi[kNObs];
};

// jets scratch of the Durham clustering: [4][cap][stride] doubles
struct Scratch {
  double *jE, *jx, *jy, *jz;
  uint64_t stride;
};

}  // namespace vsh

// host-side launchers (vsh_kernels.hip)
namespace vsh {
// k_obs runs a grid-stride loop over at most kObsBlocks x 256 threads; each
// thread owns one Durham scratch slot, so the scratch holds obs_threads(n)
// slots of cap partons.
constexpr uint32_t kObsBlocks = 2048;
uint64_t obs_threads(uint64_t n);
__global__ void k_obs(Records r, Summary sm, EventInputs in, Scratch sc, uint32_t n, double* __restrict__ hist);
void launch_me(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
               hipStream_t st);
void launch_shower_plain(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
                         uint32_t block, hipStream_t st);
void launch_obs(const Records& r, const Summary& s, const EventInputs& in, const Scratch& sc,
                uint32_t n, double* hist, hipStream_t st);
void launch_shower_init_records(const Records& r, const Summary& s, const EventInputs& in,
                                uint32_t n, hipStream_t st);
}  // namespace vsh
