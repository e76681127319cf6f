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
#include <algorithm>

#include "vsh_observables.hpp"
#include "vsh_shower.hpp"

namespace vsh {

// zero_hist (optional): a histogram set to clear on the way (the first
// min(n, 256) threads clear it), saving its own launch.
__global__ void __launch_bounds__(256) k_me(Records r, Summary s, EventInputs in, uint32_t n, double* zero_hist) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (zero_hist && e < 256u) {
    const uint32_t step = n < 256u ? n : 256u;
    for (uint32_t a = e; a < (uint32_t)kHistDoubles; a += step) zero_hist[a] = 0.0;
  }
  if (e >= n) return;
  const MEOut m = me_event(r, e, make_keyed(in.seed, in.first + e), in.ecm_of(e), in.qm, in.massive != 0);
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
// Compiled for 2, 3 and 4 resident waves per SIMD (register budgets 256,
// 168 and 128); the autotuner picks by timing.  kMassive: each kernel with
// its own massive phase space (requests with quark masses).
template <int kWaves, bool kMassive = false>
__global__ void __launch_bounds__(256, kWaves) k_shower_plain(Records r, Summary sm, EventInputs in,
                                                              uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  EvState s;
  init_state(s, r, e, make_keyed(in.seed, in.first + e), in.ecm_of(e), in.tcut_of(e), in.t_over,
             sm.i[kSiN * sm.stride + e], (int)r.cap);
  while (s.status == kRunning) {
    if constexpr (kMassive) veto_cycle_massive(s, r, e, in.qm);
    else veto_cycle(s, r, e);
    if (s.cycle >= in.cycle_limit && s.status == kRunning) s.status = kCycleLimitHit;
  }
  write_state(s, sm, e);
}

// ---------------------------------------------------------------------------
// Observables pass.  Events are sorted by parton count (largest first) with a
// counting sort, so the lanes of a wave work on events of the same size;
// each thread copies its event into its scratch column (coalesced in every
// later pass), computes the observables and fills an LDS histogram that is
// added to the global one once per block.
// ---------------------------------------------------------------------------
__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Zero the counting sort's counters and, for fixed-point histograms, the
// integer cells and the largest-weight word (a kernel, not a memset, so the
// sequence can be captured in a graph).
__global__ void k_obs_reset(uint32_t* cnt, uint32_t nb, double* hcopy, unsigned long long* ihist,
                            unsigned long long* wmax) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) cnt[i] = 0u;
  if (i < kHistCopies * (uint32_t)kHistDoubles) {
    hcopy[i] = 0.0;
    if (ihist) ihist[i] = 0ull;
  }
  if (wmax && i == 0) *wmax = 0ull;
}

uint32_t obs_reset_blocks(uint32_t nb) { return (std::max<uint32_t>(nb, kHistCopies * kHistDoubles) + 255) / 256; }

// Per-block counts in LDS over kObsSortPer events per thread, one global
// atomic per non-empty count per block (few blocks, so that the atomics of
// the handful of occupied counts do not queue up); with wmax, also the
// largest |w| of the events (the bits of non-negative doubles order like the
// integers, so the maximum does not depend on order).
__global__ void __launch_bounds__(256) k_obs_count(Summary sm, uint32_t n, uint32_t cap, uint32_t* cnt,
                                                   unsigned long long* wmax) {
  __shared__ uint32_t lc[kMaxCount + 1];
  __shared__ unsigned long long lw;
  const uint32_t nb = cap + 1;
  for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x) lc[k] = 0u;
  if (threadIdx.x == 0) lw = 0ull;
  __syncthreads();
  const uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x * kObsSortPer;
  const uint64_t e1 = e0 + (uint64_t)blockDim.x * kObsSortPer < n ? e0 + (uint64_t)blockDim.x * kObsSortPer : n;
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const uint32_t np = (uint32_t)sm.i[kSiN * sm.stride + e];
    atomicAdd(&lc[cap - (np < cap ? np : cap)], 1u);
    if (wmax) atomicMax(&lw, (unsigned long long)__double_as_longlong(fabs(sm.d[kSdW * sm.stride + e])));
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x)
    if (lc[k]) atomicAdd(&cnt[k], lc[k]);
  if (wmax && threadIdx.x == 0 && lw) atomicMax(wmax, lw);
}

// The histogram copies into the caller's histogram (accumulated).  Fixed
// point: the copies' integer cells summed (exactly, in any order), then sum
// w and sum w^2 scaled back by their powers of two, entries as they are, so
// the result does not depend on the order of the events.
__global__ void __launch_bounds__(256) k_hist_finalize(Scratch sc, double* hist, uint32_t fixed) {
  const FixScale fx = fixed ? fix_scale(sc) : FixScale{0, 0};
  for (uint32_t a = threadIdx.x; a < (uint32_t)kHistDoubles; a += blockDim.x) {
    if (fixed) {
      unsigned long long s = 0;
      for (uint32_t c = 0; c < kHistCopies; ++c) s += sc.ihist[c * kHistDoubles + a];
      const double q = (double)(long long)s;
      const int col = (int)(a % 3);
      hist[a] += col == 0 ? ldexp(q, -fx.fw) : (col == 1 ? ldexp(q, -fx.fw2) : q);
    } else {
      double v = 0.0;
      for (uint32_t c = 0; c < kHistCopies; ++c) v += sc.hcopy[c * kHistDoubles + a];
      hist[a] += v;
    }
  }
}

// exclusive prefix sum of nb counters, in place (one block)
__global__ void __launch_bounds__(256) k_obs_scan(uint32_t* cnt, uint32_t nb) {
  __shared__ uint32_t part[256];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + 255) / 256;
  uint32_t sum = 0;
  for (uint32_t k = t * per; k < nb && k < (t + 1) * per; ++k) sum += cnt[k];
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (uint32_t k = 0; k < 256; ++k) {
      const uint32_t v = part[k];
      part[k] = run;
      run += v;
    }
  }
  __syncthreads();
  uint32_t run = part[t];
  for (uint32_t k = t * per; k < nb && k < (t + 1) * per; ++k) {
    const uint32_t v = cnt[k];
    cnt[k] = run;
    run += v;
  }
}

// Each block (kObsSortPer events per thread, as k_obs_count) reserves one
// range per parton count with a single global atomic and places its events
// by their LDS rank inside the range.
__global__ void __launch_bounds__(256) k_obs_scatter(Summary sm, uint32_t n, uint32_t cap, uint32_t* cnt,
                                                     uint32_t* perm) {
  __shared__ uint32_t lc[kMaxCount + 1];
  const uint32_t nb = cap + 1;
  for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x) lc[k] = 0u;
  __syncthreads();
  const uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x * kObsSortPer;
  uint32_t bin[kObsSortPer], rank[kObsSortPer];
#pragma unroll
  for (uint32_t q = 0; q < kObsSortPer; ++q) {
    const uint64_t e = e0 + (uint64_t)q * blockDim.x + threadIdx.x;
    bin[q] = 0;
    rank[q] = 0;
    if (e < n) {
      const uint32_t np = (uint32_t)sm.i[kSiN * sm.stride + e];
      bin[q] = cap - (np < cap ? np : cap);
      rank[q] = atomicAdd(&lc[bin[q]], 1u);
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x)
    if (lc[k]) lc[k] = atomicAdd(&cnt[k], lc[k]);
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kObsSortPer; ++q) {
    const uint64_t e = e0 + (uint64_t)q * blockDim.x + threadIdx.x;
    if (e < n) perm[lc[bin[q]] + rank[q]] = (uint32_t)e;
  }
}

template <bool kMassive>
__global__ void __launch_bounds__(256) k_obs(Records r, Summary sm, EventInputs in, Scratch sc, uint32_t n,
                                             double* __restrict__ hist) {
  __shared__ double lh[kHistDoubles];
  for (int a = threadIdx.x; a < kHistDoubles; a += blockDim.x) lh[a] = 0.0;
  const bool fixed = in.fixed_hist != 0;
  FixScale fxs{0, 0};
  if (fixed) fxs = fix_scale(sc);
  const FixScale* fx = fixed ? &fxs : nullptr;
  __syncthreads();
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t cap = r.cap;
  // After k_obs_scatter, cnt[b] is the end of bin b (bin = cap - parton
  // count), so cnt[cap - m] counts the events with at least m partons; they
  // sit at the front of perm, largest first.
  const uint64_t n_big = sc.threshold <= cap ? sc.cnt[cap - sc.threshold] : 0u;  // done by k_obs_group
  const uint64_t n_mid = (uint32_t)kObsRegSlots < cap ? sc.cnt[cap - (kObsRegSlots + 1)] : n_big;
  // events of at most kObsRegSlots partons, in windows of 256 consecutive
  // events (coalesced counts; the records of a window share cache lines),
  // each window ordered by parton count in LDS so that a wave's events have
  // nearly the same size and its loops stop at the wave's largest
  __shared__ uint16_t order[256];
  __shared__ uint32_t bin_n[kObsRegSlots + 2];  // events per parton count, then the others
  for (uint64_t w0 = (uint64_t)blockIdx.x * 256; w0 < n; w0 += (uint64_t)gridDim.x * 256) {
    const uint64_t e_own = w0 + threadIdx.x;
    const int np_own = e_own < n ? sm.i[kSiN * sm.stride + e_own] : kObsRegSlots + 1;
    const bool mine = np_own <= kObsRegSlots && (uint32_t)np_own < sc.threshold;  // else the lane groups
    const int bin = mine ? np_own : kObsRegSlots + 1;
    if (threadIdx.x < kObsRegSlots + 2) bin_n[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t rank = atomicAdd(&bin_n[bin], 1u);
    __syncthreads();
    uint32_t start = 0;
    for (int b = 0; b < bin; ++b) start += bin_n[b];
    order[start + rank] = (uint16_t)threadIdx.x;
    __syncthreads();
    const uint64_t e = w0 + order[threadIdx.x];
    const int np = e < n ? sm.i[kSiN * sm.stride + e] : kObsRegSlots + 1;
    const bool ok = np <= kObsRegSlots && (uint32_t)np < sc.threshold;
    const int wmax = (int)wave_max(ok ? (uint32_t)np : 0u);
    if (ok) {
      const int status = sm.i[kSiStatus * sm.stride + e];
      const ObsOut o = reg_observables<kObsRegSlots, kMassive>(r, e, np, wmax, in.ecm_of(e), status, in);
      if (o.status == kDone) hist_fill(lh, o, sm.d[kSdW * sm.stride + e], sm.d[kSdCos * sm.stride + e], fx);
      for (int h = 0; h < 7; ++h) sm.d[(kSdY23 + h) * sm.stride + e] = o.v[h];
      sm.i[kSiStatus * sm.stride + e] = o.status;
    }
    __syncthreads();  // order and bin_n serve the next window
  }
  // the rest below the wave threshold, sorted by size, through the scratch
  for (uint64_t q = n_big + t; q < n_mid; q += step) {
    const uint64_t e = sc.perm[q];
    const int status = sm.i[kSiStatus * sm.stride + e];
    const int np = sm.i[kSiN * sm.stride + e];
    for (int a = 0; a < np; ++a) {
      const uint64_t from = (uint64_t)a * r.stride + e, to = (uint64_t)a * sc.stride + t;
      sc.E[to] = r.E[from];
      sc.x[to] = r.x[from];
      sc.y[to] = r.y[from];
      sc.z[to] = r.z[from];
    }
    const ObsOut o = scratch_observables<kMassive>(sc, t, np, in.ecm_of(e), status, in, r, e);
    if (o.status == kDone) hist_fill(lh, o, sm.d[kSdW * sm.stride + e], sm.d[kSdCos * sm.stride + e], fx);
    for (int h = 0; h < 7; ++h) sm.d[(kSdY23 + h) * sm.stride + e] = o.v[h];
    sm.i[kSiStatus * sm.stride + e] = o.status;
  }
  __syncthreads();
  hist_flush(lh, sc, fixed, threadIdx.x, blockDim.x);
}

// ---------------------------------------------------------------------------
// Events of 9 partons and more: a group of G lanes per event (G = 16 for up
// to 31 partons, four events per wave; G = 64 beyond), the group's partons
// in LDS.  Thrust's candidate planes (i < j, four sign choices) and each
// Durham step's pair scan are spread over the group's lanes; ties go to the
// smallest index in the serial scan order (first maximum for thrust, first
// minimum for Durham, as in the one-thread-per-event path).  A block is one
// wave, whose LDS operations take effect in program order, so the groups
// (which may run different numbers of steps) need no barrier between them.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int d = G / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, G);
  return v;
}

// (value, index) -> largest value, smallest index among equal values
template <int G>
__device__ __forceinline__ void group_argmax(double& v, uint32_t& idx) {
#pragma unroll
  for (int d = G / 2; d >= 1; d >>= 1) {
    const double ov = __shfl_xor(v, d, G);
    const uint32_t oi = __shfl_xor(idx, d, G);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

template <int G>
__device__ __forceinline__ void group_argmin(double& v, uint32_t& idx) {
#pragma unroll
  for (int d = G / 2; d >= 1; d >>= 1) {
    const double ov = __shfl_xor(v, d, G);
    const uint32_t oi = __shfl_xor(idx, d, G);
    if (ov < v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// Walk over the pairs (i < j < n) in row-major order: start at linear
// index p, then advance by `by` indices at a time.
struct PairWalk {
  uint32_t i, r, n;  // row i, offset r within the row (j = i + 1 + r)
  __device__ __forceinline__ PairWalk(uint32_t p, uint32_t n_) : i(0), r(p), n(n_) { settle(); }
  __device__ __forceinline__ void settle() {
    while (i + 1 < n && r >= n - 1 - i) {
      r -= n - 1 - i;
      ++i;
    }
  }
  __device__ __forceinline__ void advance(uint32_t by) {
    r += by;
    settle();
  }
  __device__ __forceinline__ uint32_t j() const { return i + 1 + r; }
};

// events with lo_n <= partons < hi_n; `slots` (at most G * MV) LDS parton
// slots per group
// (four waves per SIMD: 128 registers, a few spilled; stress 10^6 events
// 6.9 -> 6.0 ms against the three waves of the unconstrained build, LEP
// unchanged; five waves, 43 spilled, 5.7 ms on stress but 3% slower on LEP)
template <int G, int MV, bool kMassive>
__global__ void __launch_bounds__(64, 4) k_obs_group(Records r, Summary sm, EventInputs in, const uint32_t* perm,
                                                  const uint32_t* cnt, uint32_t cap, uint32_t lo_n, uint32_t hi_n,
                                                  uint32_t slots, double* __restrict__ hist, Scratch sc) {
  constexpr uint32_t kGroups = 64 / G;
  constexpr uint64_t kGroupBits = G == 64 ? ~0ull : ((1ull << (G % 64)) - 1ull);
  extern __shared__ double lds[];
  // this block's copy of the global histogram set (block b: copy b mod
  // kHistCopies), filled with each event's atomics directly: FP64 sums, or
  // the fixed-point integer cells.  A group block holds a few events, so an
  // LDS set would cost more to clear and flush than it saves (k_obs, with
  // 256 events per block, keeps one)
  const uint32_t c0 = (blockIdx.x % kHistCopies) * (uint32_t)kHistDoubles;
  const uint32_t lane = threadIdx.x % G, grp = threadIdx.x / G;
  double* pE = lds + (size_t)grp * 7 * slots;  // [slots] each
  double* px = pE + slots;
  double* py = px + slots;
  double* pz = py + slots;
  double* ux = pz + slots;
  double* uy = ux + slots;
  double* uz = uy + slots;
  uint16_t* list = (uint16_t*)(lds + (size_t)kGroups * 7 * slots) + (size_t)grp * slots;
  // cnt[cap - m] counts the events with at least m partons (see k_obs)
  const uint32_t q_lo = hi_n <= cap ? cnt[cap - hi_n] : 0u;
  const uint32_t q_hi = lo_n <= cap ? cnt[cap - lo_n] : 0u;
  // the grid is sized for the worst case: blocks without an event of this
  // range leave at once (the whole block, before touching LDS)
  if (q_lo + blockIdx.x * kGroups >= q_hi) return;
  const bool fixed = in.fixed_hist != 0;
  FixScale fxs{0, 0};
  if (fixed) fxs = fix_scale(sc);
  const FixScale* fx = fixed ? &fxs : nullptr;
  __syncthreads();
  for (uint32_t q = q_lo + blockIdx.x * kGroups + grp; q < q_hi; q += gridDim.x * kGroups) {
    const uint64_t e = perm[q];
    int status = sm.i[kSiStatus * sm.stride + e];
    const int np = sm.i[kSiN * sm.stride + e];
    const double ecm = in.ecm_of(e), sh = ecm * ecm;
    // nonfin: partons with a non-finite component; offshell: finite partons
    // off their mass shell (kept apart: one non-finite parton makes the
    // event NONFINITE, any number of finite off-shell ones CONSERVATION)
    double tE = 0.0, tx = 0.0, ty = 0.0, tz = 0.0, nonfin = 0.0, offshell = 0.0, sum = 0.0;
    double mxx = 0.0, myy = 0.0, mzz = 0.0, mxy = 0.0, mxz = 0.0, myz = 0.0;
    for (int a = lane; a < np; a += G) {
      const uint64_t o = (uint64_t)a * r.stride + e;
      const P4 p{r.E[o], r.x[o], r.y[o], r.z[o]};
      pE[a] = p.e;
      px[a] = p.x;
      py[a] = p.y;
      pz[a] = p.z;
      if (!(isfinite(p.e) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z))) nonfin += 1.0;
      else if (!(fabs(mdot(p, p) - shell2<kMassive>(in, r, a, e)) <= 1e-10 * sh)) offshell += 1.0;
      tE += p.e;
      tx += p.x;
      ty += p.y;
      tz += p.z;
      const double l = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
      sum += l;
      const double il = 1.0 / l;
      mxx += p.x * p.x * il;
      myy += p.y * p.y * il;
      mzz += p.z * p.z * il;
      mxy += p.x * p.y * il;
      mxz += p.x * p.z * il;
      myz += p.y * p.z * il;
    }
    tE = group_sum<G>(tE);
    tx = group_sum<G>(tx);
    ty = group_sum<G>(ty);
    tz = group_sum<G>(tz);
    nonfin = group_sum<G>(nonfin);
    offshell = group_sum<G>(offshell);
    if (status == kDone) {
      const double tol = 1e-10 * ecm;
      if (nonfin > 0.0) status = kNonFinite;
      else if (fabs(tE - ecm) > tol || fabs(tx) > tol || fabs(ty) > tol || fabs(tz) > tol || offshell > 0.0)
        status = kConservation;
    }
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (status == kDone) {
      sum = group_sum<G>(sum);
      mxx = group_sum<G>(mxx);
      myy = group_sum<G>(myy);
      mzz = group_sum<G>(mzz);
      mxy = group_sum<G>(mxy);
      mxz = group_sum<G>(mxz);
      myz = group_sum<G>(myz);
      // thrust over the candidate planes
      const uint32_t npairs = (uint32_t)np * (np - 1) / 2;
      double best = -1.0;
      uint32_t bidx = 0xFFFFFFFFu;
      double bx = 0.0, by = 0.0, bz = 1.0;
      PairWalk pw(lane, (uint32_t)np);
      for (uint32_t pidx = lane; pidx < npairs; pidx += G, pw.advance(G)) {
        const uint32_t i = pw.i, j = pw.j();
        const double xi = px[i], yi = py[i], zi = pz[i], xj = px[j], yj = py[j], zj = pz[j];
        const double nx = yi * zj - zi * yj, ny = zi * xj - xi * zj, nz = xi * yj - yi * xj;
        double vx = 0.0, vy = 0.0, vz = 0.0;
        for (int k = 0; k < np; ++k) {
          if (k == (int)i || k == (int)j) continue;
          const double xk = px[k], yk = py[k], zk = pz[k];
          const double d = xk * nx + yk * ny + zk * nz;
          if (d > 0.0) { vx += xk; vy += yk; vz += zk; }
          else { vx -= xk; vy -= yk; vz -= zk; }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double si = (c < 2) ? 1.0 : -1.0, sj = (c & 1) ? -1.0 : 1.0;
          const double wx = vx + si * xi + sj * xj, wy = vy + si * yi + sj * yj, wz = vz + si * zi + sj * zj;
          const double m2 = wx * wx + wy * wy + wz * wz;
          if (m2 > best) { best = m2; bidx = 4 * pidx + c; bx = wx; by = wy; bz = wz; }
        }
      }
      double wbest = best;
      uint32_t widx = bidx;
      group_argmax<G>(wbest, widx);
      // the winning lane of the group broadcasts its vector
      const uint64_t who = __ballot(bidx == widx && best == wbest);
      const uint32_t src = (uint32_t)__ffsll((unsigned long long)((who >> (grp * G)) & kGroupBits)) - 1;
      bx = __shfl(bx, (int)src, G);
      by = __shfl(by, (int)src, G);
      bz = __shfl(bz, (int)src, G);
      const double lb = sqrt(wbest);
      double ax = 0.0, ay = 0.0, az = 1.0;
      if (lb > 0.0) { ax = bx / lb; ay = by / lb; az = bz / lb; }
      const double T = sum > 0.0 ? lb / sum : 0.0;
      const double tau = 1.0 - T;
      v[2] = tau > 0.0 ? tau : 0.0;
      const double m2s = mxx * mxx + myy * myy + mzz * mzz + 2.0 * (mxy * mxy + mxz * mxz + myz * myz);
      const double cpar = 1.5 * (sum * sum - m2s) / (sum * sum);
      v[3] = cpar > 0.0 ? cpar : 0.0;
      // hemispheres
      double hpE = 0, hpx = 0, hpy = 0, hpz = 0, hmE = 0, hmx = 0, hmy = 0, hmz = 0, bp = 0, bm = 0;
      for (int a = lane; a < np; a += G) {
        const double x = px[a], y = py[a], z = pz[a], en = pE[a];
        const double d = x * ax + y * ay + z * az;
        const double cx = y * az - z * ay, cy = z * ax - x * az, cz = x * ay - y * ax;
        const double kt = sqrt(cx * cx + cy * cy + cz * cz);
        if (d >= 0.0) { hpE += en; hpx += x; hpy += y; hpz += z; bp += kt; }
        else { hmE += en; hmx += x; hmy += y; hmz += z; bm += kt; }
      }
      hpE = group_sum<G>(hpE); hpx = group_sum<G>(hpx); hpy = group_sum<G>(hpy); hpz = group_sum<G>(hpz);
      hmE = group_sum<G>(hmE); hmx = group_sum<G>(hmx); hmy = group_sum<G>(hmy); hmz = group_sum<G>(hmz);
      bp = group_sum<G>(bp); bm = group_sum<G>(bm);
      const double mp = hpE * hpE - hpx * hpx - hpy * hpy - hpz * hpz;
      const double mm = hmE * hmE - hmx * hmx - hmy * hmy - hmz * hmz;
      const double rho = (mp > mm ? mp : mm) / sh;
      v[4] = rho > 0.0 ? rho : 0.0;
      bp /= 2.0 * sum;
      bm /= 2.0 * sum;
      v[5] = bp + bm;
      v[6] = bp > bm ? bp : bm;
      // Durham: pair scan over the current jets each step
      const double inv_s = 1.0 / sh;
      for (int a = lane; a < np; a += G) {
        list[a] = (uint16_t)a;
        const double l = sqrt(px[a] * px[a] + py[a] * py[a] + pz[a] * pz[a]);
        ux[a] = px[a] / l;
        uy[a] = py[a] / l;
        uz[a] = pz[a] / l;
      }
      int m = np;
      while (m > 2) {
        const uint32_t mp2 = (uint32_t)m * (m - 1) / 2;
        double ymin = INFINITY;
        uint32_t yidx = 0xFFFFFFFFu;
        PairWalk dw(lane, (uint32_t)m);
        for (uint32_t pidx = lane; pidx < mp2; pidx += G, dw.advance(G)) {
          const int ja = list[dw.i], jb = list[dw.j()];
          const double dx = ux[ja] - ux[jb], dy = uy[ja] - uy[jb], dz = uz[ja] - uz[jb];
          const double d2 = (dx * dx + dy * dy) + dz * dz;
          const double em = pE[ja] < pE[jb] ? pE[ja] : pE[jb];
          const double y = em * em * d2 * inv_s;
          if (y < ymin) { ymin = y; yidx = pidx; }
        }
        group_argmin<G>(ymin, yidx);
        const PairWalk win(yidx, (uint32_t)m);
        const uint32_t ia = win.i, ib = win.j();
        if (m == 4) v[1] = ymin;
        if (m == 3) v[0] = ymin;
        const int ja = list[ia], jb = list[ib];
        if (lane == 0) {
          pE[ja] += pE[jb];
          px[ja] += px[jb];
          py[ja] += py[jb];
          pz[ja] += pz[jb];
          const double l = sqrt(px[ja] * px[ja] + py[ja] * py[ja] + pz[ja] * pz[ja]);
          ux[ja] = px[ja] / l;
          uy[ja] = py[ja] / l;
          uz[ja] = pz[ja] / l;
        }
        // drop jet ib from the list: read the entries after it, then write them back one place down
        uint16_t mv[MV];
#pragma unroll
        for (uint32_t k = 0; k < MV; ++k) {
          const uint32_t a = ib + 1 + lane + G * k;
          mv[k] = a < (uint32_t)m ? list[a] : (uint16_t)0;
        }
#pragma unroll
        for (uint32_t k = 0; k < MV; ++k) {
          const uint32_t a = ib + 1 + lane + G * k;
          if (a < (uint32_t)m) list[a - 1] = mv[k];
        }
        --m;
      }
      double* gh = fixed ? reinterpret_cast<double*>(sc.ihist + c0) : sc.hcopy + c0;
      if (lane == 0) hist_fill(gh, ObsOut{{v[0], v[1], v[2], v[3], v[4], v[5], v[6]}, status},
                                   sm.d[kSdW * sm.stride + e], sm.d[kSdCos * sm.stride + e], fx);
    }
#pragma unroll
    for (uint32_t h = 0; h < 7; ++h)  // the group's lanes share the seven stores
      if (h % G == lane) sm.d[(kSdY23 + h) * sm.stride + e] = v[h];
    if (lane == 0) sm.i[kSiStatus * sm.stride + e] = status;
  }
}

// The group launches for records of capacity cap: 16 lanes from
// kObsWaveThreshold to 31 partons, 64 lanes from 32 (smaller events go to
// k_obs).
const void* obs_kernel(bool massive) { return massive ? (const void*)k_obs<true> : (const void*)k_obs<false>; }

uint32_t obs_group_launches(uint32_t cap, bool massive, ObsGroupLaunch out[3]) {
  uint32_t k = 0;
  if (cap > kObsWaveMaxCap || kObsWaveThreshold > cap) return 0;
  const uint32_t t = kObsWaveThreshold;
  {  // 16 lanes up to 31 partons
    const uint32_t slots = std::min<uint32_t>(31, cap);
    const void* fn = massive ? (const void*)k_obs_group<16, 2, true> : (const void*)k_obs_group<16, 2, false>;
    out[k++] = ObsGroupLaunch{fn, std::max<uint32_t>(t, 9), 32, slots, (uint32_t)obs_group_lds(16, slots)};
  }
  if (cap >= 32) {  // a wave from 32
    const void* fn = massive ? (const void*)k_obs_group<64, kObsWaveMaxCap / 64, true>
                             : (const void*)k_obs_group<64, kObsWaveMaxCap / 64, false>;
    out[k++] = ObsGroupLaunch{fn, std::max<uint32_t>(t, 32), cap + 1, cap, (uint32_t)obs_group_lds(64, cap)};
  }
  return k;
}

size_t obs_group_lds(uint32_t g, uint32_t slots) {
  return (size_t)(64 / g) * slots * (7 * 8 + 2) + 64;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline uint32_t blocks_for(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

uint32_t obs_sort_blocks(uint64_t n) { return blocks_for(n, 256u * kObsSortPer); }

void launch_me(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
               hipStream_t st, double* zero_hist) {
  if (!n) return;
  hipLaunchKernelGGL(k_me, dim3(blocks_for(n, 256)), dim3(256), 0, st, r, s, in, n, zero_hist);
}

void launch_shower_init_records(const Records& r, const Summary& s, const EventInputs& in,
                                uint32_t n, hipStream_t st) {
  (void)in;
  if (!n) return;
  hipLaunchKernelGGL(k_init_records, dim3(blocks_for(n, 256)), dim3(256), 0, st, r, s, n);
}

void launch_shower_plain(const Records& r, const Summary& s, const EventInputs& in, uint32_t n,
                         uint32_t block, uint32_t waves, hipStream_t st) {
  if (!n) return;
  if (block == 0 || block > 256) block = 256;
  const dim3 g(blocks_for(n, block)), b(block);
  if (in.massive) hipLaunchKernelGGL((k_shower_plain<2, true>), g, b, 0, st, r, s, in, n);
  else if (waves >= 4) hipLaunchKernelGGL(k_shower_plain<4>, g, b, 0, st, r, s, in, n);
  else if (waves == 3) hipLaunchKernelGGL(k_shower_plain<3>, g, b, 0, st, r, s, in, n);
  else hipLaunchKernelGGL(k_shower_plain<2>, g, b, 0, st, r, s, in, n);
}

// Parton slots of Durham scratch per thread of the one-thread-per-event
// pass: it only sees events below the wave threshold when the wave pass
// runs, else every event up to cap.
static uint32_t thread_slots(uint32_t cap) {
  return (cap <= kObsWaveMaxCap && kObsWaveThreshold <= cap) ? kObsWaveThreshold - 1 : cap;
}

// at most 2^24 parton slots of scratch (1.1 GB) and 2^18 threads (about
// the resident threads of the pass), at most n
uint64_t obs_threads(uint64_t n, uint32_t cap) {
  const uint64_t most =
      std::max<uint64_t>(256, std::min<uint64_t>(1ull << 18, ((1ull << 24) / thread_slots(cap)) / 256 * 256));
  const uint64_t t = ((n + 255) / 256) * 256;
  return t < most ? t : most;
}

static inline uint64_t al256(uint64_t v) { return (v + 255) / 256 * 256; }

uint64_t obs_scratch_bytes(uint64_t n, uint32_t cap) {
  const uint64_t m = obs_threads(n, cap) * thread_slots(cap);
  return 8 * al256(m * 8) + al256(m * 2) + al256(m) + al256(n * 4) + al256((cap + 2) * 4) +
         2 * al256(kHistCopies * kHistDoubles * 8) + al256(8) + 256;
}

Scratch carve_obs_scratch(char*& p, uint64_t n, uint32_t cap) {
  Scratch s;
  s.stride = obs_threads(n, cap);
  const uint64_t m = s.stride * thread_slots(cap);
  auto take = [&](uint64_t bytes) {
    char* q = p;
    p += al256(bytes);
    return q;
  };
  s.E = (double*)take(m * 8);
  s.x = (double*)take(m * 8);
  s.y = (double*)take(m * 8);
  s.z = (double*)take(m * 8);
  s.ux = (double*)take(m * 8);
  s.uy = (double*)take(m * 8);
  s.uz = (double*)take(m * 8);
  s.dn = (double*)take(m * 8);
  s.nn = (uint16_t*)take(m * 2);
  s.dead = (uint8_t*)take(m);
  s.perm = (uint32_t*)take(n * 4);
  s.cnt = (uint32_t*)take((cap + 2) * 4);
  s.hcopy = (double*)take(kHistCopies * kHistDoubles * 8);
  s.ihist = (unsigned long long*)take(kHistCopies * kHistDoubles * 8);
  s.wmax = (unsigned long long*)take(8);
  s.lbits = 0;
  while ((1ull << s.lbits) < n) ++s.lbits;
  // events with at least `threshold` partons go to one wave each (LDS holds
  // up to kObsWaveMaxCap partons); smaller ones to one thread each
  s.threshold = cap <= kObsWaveMaxCap ? kObsWaveThreshold : 0xFFFFFFFFu;
  return s;
}

void launch_obs(const Records& r, const Summary& s, const EventInputs& in, const Scratch& sc,
                uint32_t n, double* hist, hipStream_t st) {
  if (!n) return;
  const uint32_t nb = r.cap + 1;
  const bool fixed = in.fixed_hist != 0;
  unsigned long long* ih = fixed ? sc.ihist : nullptr;
  unsigned long long* wm = fixed ? sc.wmax : nullptr;
  hipLaunchKernelGGL(k_obs_reset, dim3(obs_reset_blocks(nb)), dim3(256), 0, st, sc.cnt, nb, sc.hcopy, ih, wm);
  hipLaunchKernelGGL(k_obs_count, dim3(obs_sort_blocks(n)), dim3(256), 0, st, s, n, r.cap, sc.cnt, wm);
  hipLaunchKernelGGL(k_obs_scan, dim3(1), dim3(256), 0, st, sc.cnt, nb);
  hipLaunchKernelGGL(k_obs_scatter, dim3(obs_sort_blocks(n)), dim3(256), 0, st, s, n, r.cap, sc.cnt, sc.perm);
  const uint32_t blocks = (uint32_t)(std::min<uint64_t>(sc.stride, ((uint64_t)n + 255) / 256 * 256) / 256);
  if (in.massive) hipLaunchKernelGGL(k_obs<true>, dim3(blocks), dim3(256), 0, st, r, s, in, sc, n, hist);
  else hipLaunchKernelGGL(k_obs<false>, dim3(blocks), dim3(256), 0, st, r, s, in, sc, n, hist);
  ObsGroupLaunch gl[3];
  const uint32_t ng = obs_group_launches(r.cap, in.massive != 0, gl);
  for (uint32_t k = 0; k < ng; ++k) {
    const uint32_t wb = (uint32_t)std::min<uint64_t>(n, kObsWaveBlocks);
    const uint32_t* perm = sc.perm;
    const uint32_t* cnt = sc.cnt;
    uint32_t cap = r.cap, lo = gl[k].lo, hi = gl[k].hi, slots = gl[k].slots;
    Records rr = r;
    Summary ss = s;
    EventInputs ii = in;
    double* hh = hist;
    Scratch sc2 = sc;
    void* args[] = {&rr, &ss, &ii, &perm, &cnt, &cap, &lo, &hi, &slots, &hh, &sc2};
    (void)hipLaunchKernel(gl[k].fn, dim3(wb), dim3(64), args, gl[k].lds, st);
  }
  hipLaunchKernelGGL(k_hist_finalize, dim3(1), dim3(256), 0, st, sc, hist, fixed ? 1u : 0u);
}


}  // namespace vsh
