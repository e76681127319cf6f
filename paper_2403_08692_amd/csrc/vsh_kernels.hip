// vsh_kernels.hip -- the plain form of the shower hot path for gfx950 and the
// observables pass shared by both forms.
//
//   k_me             LO matrix element and event initialisation (App. B)
//   k_init_records   colour-partner links for caller-supplied initial states
//   k_shower_plain   thread per event, the whole veto loop in one launch
//                    (App. A / C: select winner, cutoff, alpha_s, veto, split)
//   k_obs            validation, Durham y23/y34, thrust, C, rho_H, B_T/B_W
//                    (Sec. 3.1) and histograms reduced in LDS before the
//                    global atomics
#include "vsh_observables.hpp"
#include "vsh_shower.hpp"

namespace vsh {

__global__ void __launch_bounds__(256) k_me(Records r, Summary s, EventInputs in, uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const MEOut m = me_event(r, e, make_keyed(in.seed, in.first + e), in.ecm_of(e));
  s.d[kSdW * s.stride + e] = m.w;
  s.d[kSdCos * s.stride + e] = m.c;
  s.d[kSdPhi * s.stride + e] = m.phi;
  s.i[kSiN * s.stride + e] = 2;
  s.i[kSiFlavour * s.stride + e] = m.f;
}

// Caller-supplied starts: partner links from the colour labels.
__global__ void __launch_bounds__(256) k_init_records(Records r, Summary s, uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int np = s.i[kSiN * s.stride + e];
  for (int a = 0; a < np; ++a) {
    const uint16_t ca = r.col[(uint64_t)a * r.stride + e];
    const uint16_t aa = r.acol[(uint64_t)a * r.stride + e];
    uint16_t cp = kNoPartner, ap = kNoPartner;
    for (int b = 0; b < np; ++b) {
      if (b == a) continue;
      if (ca != 0 && r.acol[(uint64_t)b * r.stride + e] == ca && cp == kNoPartner) cp = (uint16_t)b;
      if (aa != 0 && r.col[(uint64_t)b * r.stride + e] == aa && ap == kNoPartner) ap = (uint16_t)b;
    }
    r.cpart[(uint64_t)a * r.stride + e] = cp;
    r.apart[(uint64_t)a * r.stride + e] = ap;
  }
  s.d[kSdW * s.stride + e] = 1.0;
}

// Plain form: each thread evolves its event to the cutoff in one launch.
__global__ void __launch_bounds__(256) k_shower_plain(Records r, Summary sm, EventInputs in,
                                                      uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  EvState s;
  init_state(s, r, e, make_keyed(in.seed, in.first + e), in.ecm_of(e), in.tcut_of(e),
             sm.i[kSiN * sm.stride + e], (int)r.cap);
  while (s.status == kRunning) {
    veto_cycle(s, r, e);
    if (s.cycle >= kCycleLimit && s.status == kRunning) s.status = kCycleLimitHit;
  }
  write_state(s, sm, e);
}

// Observables and histograms of events [0, n) held in r (slot-major, stride
// r.stride).  Grid-stride loop: thread t uses Durham scratch slot t.
__global__ void __launch_bounds__(256) k_obs(Records r, Summary sm, EventInputs in, Scratch sc,
                                             uint32_t n, double* __restrict__ hist) {
  __shared__ double lh[kHistDoubles];
  for (int a = threadIdx.x; a < kHistDoubles; a += blockDim.x) lh[a] = 0.0;
  __syncthreads();
  const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = slot; e < n; e += step) {
    const int status = sm.i[kSiStatus * sm.stride + e];
    const int np = sm.i[kSiN * sm.stride + e];
    const ObsOut o = event_observables(r, sc, e, slot, np, in.ecm_of(e), status);
    if (o.status == kDone) hist_fill_lds(lh, o, sm.d[kSdW * sm.stride + e], sm.d[kSdCos * sm.stride + e]);
    for (int h = 0; h < 7; ++h) sm.d[(kSdY23 + h) * sm.stride + e] = o.v[h];
    sm.i[kSiStatus * sm.stride + e] = o.status;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < kHistDoubles; a += blockDim.x) {
    const double v = lh[a];
    if (v != 0.0) unsafeAtomicAdd(&hist[a], v);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline uint32_t blocks_for(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

void launch_me(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
               hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_me, dim3(blocks_for(n, 256)), dim3(256), 0, st, r, s, in, n);
}

void launch_shower_init_records(const Records& r, const Summary& s, const EventInputs& in,
                                uint32_t n, hipStream_t st) {
  (void)in;
  if (!n) return;
  hipLaunchKernelGGL(k_init_records, dim3(blocks_for(n, 256)), dim3(256), 0, st, r, s, n);
}

void launch_shower_plain(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
                         uint32_t block, hipStream_t st) {
  if (!n) return;
  if (block == 0 || block > 256) block = 256;
  hipLaunchKernelGGL(k_shower_plain, dim3(blocks_for(n, block)), dim3(block), 0, st, r, s, in, n);
}

uint64_t obs_threads(uint64_t n) {
  const uint64_t most = (uint64_t)kObsBlocks * 256;
  const uint64_t t = ((n + 255) / 256) * 256;
  return t < most ? t : most;
}

void launch_obs(const Records& r, const Summary& s, const EventInputs& in, const Scratch& sc,
                uint32_t n, double* hist, hipStream_t st) {
  if (!n) return;
  const uint32_t blocks = (uint32_t)(obs_threads(n) / 256);
  hipLaunchKernelGGL(k_obs, dim3(blocks), dim3(256), 0, st, r, s, in, sc, n, hist);
}

}  // namespace vsh
