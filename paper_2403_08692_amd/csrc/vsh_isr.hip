// vsh_isr.hip -- the initial-state shower: Drell-Yan q qbar -> V at a hadron
// collider with backward evolution of the incoming lines and the ratio of
// parton densities in the veto (the step to hadron colliders that the
// paper's conclusions name), one lane per event.
//
// No parton-density set is available here, so a closed-form density stands
// in for one: every light quark and antiquark flavour has
// f(x) = (63/128) x^(-1/2) (1 - x)^3 (the ten carry half the momentum; a
// gluon density 3 x^(-1) (1 - x)^5 carries the other half and is not
// needed by this branch), independent of the scale.
//
// Per event: flavour uniform over d, u, s, c, b, the quark from either beam,
// the rapidity of V uniform in |y| < ln(sqrt(S)/Q); x_A x_B = Q^2/S; weight
// (arbitrary units) 10 (2Y) tau f(x_A) f(x_B).  Each incoming line (the
// other incoming parton its spectator) makes one trial per cycle with the
// overestimate 2 C_F x^(-1/2)/(1 - z) of the backward-evolution density
// (alpha_s/2 pi) (dt/t) (dz/z) P_qq(z) f(x/z)/f(x) over x < z < z_max(t_C);
// the largest trial above t_C wins (App. A's competition between trials);
// the veto keeps it with probability alpha_s(t)/alpha_s(t_C) times density
// over overestimate, where (1 - z)^2 >= 4 t z / s~ leaves room for it.  An
// accepted emission uses the Catani-Seymour initial-initial map: the emitter
// becomes p_a/z, the gluon (1 - z - v) p_a/z + v p_b + kT (kT^2 = t, the
// smaller root of v(1 - z - v) = t z / s~) and the final state is carried by
// the Lorentz transformation from the old final-state total to the new one.
// Emitted gluons do not radiate.  The arithmetic is FP64 throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>

#include "../../include/vsh.h"
#include "vsh_internal.hpp"
#include "vsh_math.hpp"

namespace vsh {

struct IsrInputs {
  uint64_t seed, first;
  double sqrt_s, q, tcut;
};

// the stand-in density and its ratio f(x/z)/f(x) as the veto takes it
__device__ __forceinline__ double isr_pdf(double x) {
  return (63.0 / 128.0) / sqrt(x) * ((1.0 - x) * (1.0 - x) * (1.0 - x));
}

constexpr int kIsrKernel = 16;  // the emission hash's kernel id of an initial-state q -> q g

// histogram ranges of the branch: log10(p_T,V / GeV), y_V, emitted gluons,
// log10(p_T / GeV) of the hardest gluon (rows 4-7 unused)
__device__ __forceinline__ double isr_lo(int h) { return h == 1 ? -5.0 : (h == 3 || h == 0 ? -1.0 : 0.0); }
__device__ __forceinline__ double isr_hi(int h) { return h == 1 ? 5.0 : (h == 2 ? 50.0 : (h < 4 ? 3.0 : 1.0)); }

__device__ __forceinline__ int isr_bin(double x, double lo, double hi) {
  if (x != x) return kNBins + 1;
  if (x < lo) return 0;
  if (x >= hi) return kNBins + 1;
  const int b = 1 + (int)((x - lo) / (hi - lo) * kNBins);
  return b > kNBins ? kNBins : b;
}

__global__ void __launch_bounds__(256) k_isr(Records r, Summary sm, IsrInputs in, uint32_t n, double* hist) {
  __shared__ double lh[kHistDoubles];
  for (int a = threadIdx.x; a < kHistDoubles; a += blockDim.x) lh[a] = 0.0;
  __syncthreads();
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    const Keyed key = make_keyed(in.seed, in.first + e);
    // --- the Drell-Yan start
    const U4 m0 = key.draw(0, kPurposeME, 0);
    const int f = 1 + (int)(((uint64_t)m0.x * 5u) >> 32);
    const bool qa = (m0.y & 1u) == 0u;
    const double Y = log(in.sqrt_s / in.q);
    const double y0 = -Y + 2.0 * Y * unit(m0.z, m0.w);
    const double tau = in.q * in.q / (in.sqrt_s * in.sqrt_s);
    double x[2] = {sqrt(tau) * exp(y0), sqrt(tau) * exp(-y0)};
    const double eb = 0.5 * in.sqrt_s;
    const double w = 10.0 * (2.0 * Y) * tau * isr_pdf(x[0]) * isr_pdf(x[1]);
    r.store(0, e, P4{x[0] * eb, 0.0, 0.0, x[0] * eb});
    r.store(1, e, P4{x[1] * eb, 0.0, 0.0, -x[1] * eb});
    r.store(2, e, P4{x[0] * eb + x[1] * eb, 0.0, 0.0, x[0] * eb - x[1] * eb});
    const uint64_t s1 = r.stride, s2 = 2 * r.stride;
    r.pid[e] = (int8_t)(qa ? f : -f);
    r.pid[s1 + e] = (int8_t)(qa ? -f : f);
    r.pid[s2 + e] = 23;
    r.col[e] = qa ? 1 : 0;
    r.acol[e] = qa ? 0 : 1;
    r.col[s1 + e] = qa ? 0 : 1;
    r.acol[s1 + e] = qa ? 1 : 0;
    r.col[s2 + e] = 0;
    r.acol[s2 + e] = 0;
    // --- backward evolution of the two incoming lines
    const double ltc = log_fast(in.tcut);
    const double asmax = alpha_s_of_log(ltc);
    const double cfac = asmax / (2.0 * kPi);
    double lt = log_fast(in.q * in.q);
    int np = 3, next_col = 2, n_emit = 0, status = kRunning;
    uint32_t cycle = 0, trials = 0, ends = 0;
    uint64_t hash = kFnvOffset;
    while (status == kRunning) {
      const P4 pa0 = r.load(0, e), pb0 = r.load(1, e);
      const double st = 2.0 * mdot(pa0, pb0);
      const double a = in.tcut / st;
      const double zmax = 1.0 + 2.0 * a - 2.0 * sqrt(a + a * a);
      double best = ltc, wzlo = 0.0, wL = 0.0;
      int wl = -1;
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        if (!(zmax > x[l])) continue;  // no phase space above the cutoff
        ends += 1;
        const double L = log_fast((1.0 - x[l]) / (1.0 - zmax));
        const double c = cfac * ((2.0 * kCF) / sqrt(x[l]) * L);
        const U4 d = key.draw(cycle, kPurposeTrial, trial_slot((uint32_t)l, (uint32_t)(1 - l), 0));
        const double lt_try = lt + log_fast(unit(d.x, d.y)) / c;
        trials += 1;
        if (lt_try > best) {
          best = lt_try;
          wl = l;
          wzlo = x[l];
          wL = L;
        }
      }
      const uint32_t this_cycle = cycle++;
      if (wl < 0) {
        status = kDone;
        break;
      }
      lt = best;
      const double t = exp(best);
      const U4 acc = key.draw(this_cycle, kPurposeAccept, 0);
      const double z = 1.0 - (1.0 - wzlo) * exp(-unit(acc.x, acc.y) * wL);
      const double xl = x[wl];
      const double disc = (1.0 - z) * (1.0 - z) - 4.0 * t * z / st;
      if (!(disc >= 0.0) || !(z > xl)) continue;  // no room for the emission at this t
      const double dens = kCF * (1.0 + z * z) / (1.0 - z) / z * isr_pdf(xl / z) / isr_pdf(xl);
      const double over = 2.0 * kCF / sqrt(xl) / (1.0 - z);
      const double prob = alpha_s_of_log(best) / asmax * (dens / over);
      if (!(unit(acc.z, acc.w) < prob)) continue;
      if (np == (int)r.cap) {
        status = kOverflow;
        break;
      }
      // --- the emission: initial-initial map and the final state's transformation
      const U4 sd = key.draw(this_cycle, kPurposeSplit, 0);
      const double phi = 2.0 * kPi * unit(sd.x, sd.y);
      double sphi, cphi;
      sincos(phi, &sphi, &cphi);
      const P4 pa = wl == 0 ? pa0 : pb0, pb = wl == 0 ? pb0 : pa0;
      const double v = 0.5 * ((1.0 - z) - sqrt(disc));
      const P4 na{pa.e / z, pa.x / z, pa.y / z, pa.z / z};
      const double kt = sqrt(t);
      const double c1 = 1.0 - z - v;
      const P4 pj{c1 * na.e + v * pb.e, c1 * na.x + v * pb.x + kt * cphi, c1 * na.y + v * pb.y + kt * sphi,
                  c1 * na.z + v * pb.z};
      const P4 Kt{pa.e + pb.e, pa.x + pb.x, pa.y + pb.y, pa.z + pb.z};
      const P4 K{na.e + pb.e - pj.e, na.x + pb.x - pj.x, na.y + pb.y - pj.y, na.z + pb.z - pj.z};
      const P4 S{K.e + Kt.e, K.x + Kt.x, K.y + Kt.y, K.z + Kt.z};
      const double s2n = mdot(S, S), kt2 = mdot(Kt, Kt);
      for (int q = 2; q < np; ++q) {
        const P4 k = r.load((uint32_t)q, e);
        const double sx = mdot(S, k), kx = mdot(Kt, k);
        const double cs = 2.0 * sx / s2n, ck = 2.0 * kx / kt2;
        r.store((uint32_t)q, e, P4{k.e - cs * S.e + ck * K.e, k.x - cs * S.x + ck * K.x, k.y - cs * S.y + ck * K.y,
                                    k.z - cs * S.z + ck * K.z});
      }
      r.store((uint32_t)wl, e, na);
      r.store((uint32_t)np, e, pj);
      x[wl] = xl / z;
      // the gluon goes onto the emitter's colour line
      const uint64_t ow = (uint64_t)wl * r.stride + e, oj = (uint64_t)np * r.stride + e;
      const uint16_t m = (uint16_t)next_col++;
      r.pid[oj] = (int8_t)kGluon;
      if (r.col[ow] != 0) {
        r.col[oj] = r.col[ow];
        r.acol[oj] = m;
        r.col[ow] = m;
      } else {
        r.col[oj] = m;
        r.acol[oj] = r.acol[ow];
        r.acol[ow] = m;
      }
      hash = fnv_step(fnv_step(fnv_step(hash, (uint32_t)kIsrKernel), (uint32_t)wl), (uint32_t)(1 - wl));
      ++np;
      ++n_emit;
      if (cycle >= kCycleLimit) status = kCycleLimitHit;
    }
    // --- validation: finite; the final state carries the incoming total;
    // V on its mass shell, the others massless
    const P4 ia = r.load(0, e), ib = r.load(1, e);
    const P4 tin{ia.e + ib.e, ia.x + ib.x, ia.y + ib.y, ia.z + ib.z};
    P4 tout{0.0, 0.0, 0.0, 0.0};
    bool finite = true, shell = true;
    const double s_in = mdot(tin, tin);
    double ptg = 0.0;
    for (int a2 = 0; a2 < np; ++a2) {
      const P4 p = r.load((uint32_t)a2, e);
      finite = finite && isfinite(p.e) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
      const double m2 = a2 == 2 ? in.q * in.q : 0.0;
      shell = shell && fabs(mdot(p, p) - m2) <= 1e-10 * s_in;
      if (a2 >= 2) {
        tout.e += p.e;
        tout.x += p.x;
        tout.y += p.y;
        tout.z += p.z;
      }
      if (a2 >= 3) {
        const double pt = sqrt(p.x * p.x + p.y * p.y);
        if (pt > ptg) ptg = pt;
      }
    }
    if (status == kDone) {
      const double tol = 1e-10 * tin.e;
      if (!finite) status = kNonFinite;
      else if (fabs(tout.e - tin.e) > tol || fabs(tout.x - tin.x) > tol || fabs(tout.y - tin.y) > tol ||
               fabs(tout.z - tin.z) > tol || !shell)
        status = kConservation;
    }
    const P4 V = r.load(2, e);
    const double ptv = sqrt(V.x * V.x + V.y * V.y);
    const double yv = 0.5 * log((V.e + V.z) / (V.e - V.z));
    if (status == kDone) {
      const double vals[4] = {ptv > 0.0 ? log10(ptv) : -INFINITY, yv, (double)n_emit, ptg > 0.0 ? log10(ptg) : -INFINITY};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        double* cell = &lh[3 * (kNHCol * h + isr_bin(vals[h], isr_lo(h), isr_hi(h)))];
        atomicAdd(&cell[0], w);
        atomicAdd(&cell[1], w * w);
        atomicAdd(&cell[2], 1.0);
      }
    }
    const double dv[kNSumD] = {w, yv, ptv, x[0], x[1], ptg, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kNSumD; ++k) sm.d[k * sm.stride + e] = dv[k];
    sm.i[kSiN * sm.stride + e] = np;
    sm.i[kSiStatus * sm.stride + e] = status;
    sm.i[kSiCycles * sm.stride + e] = (int32_t)cycle;
    sm.i[kSiEmit * sm.stride + e] = n_emit;
    sm.i[kSiFlavour * sm.stride + e] = qa ? f : -f;
    sm.i[kSiTrials * sm.stride + e] = (int32_t)trials;
    sm.i[kSiEnds * sm.stride + e] = (int32_t)ends;
    sm.hash[e] = hash;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < kHistDoubles; a += blockDim.x) {
    const double v = lh[a];
    if (v != 0.0) unsafeAtomicAdd(&hist[a], v);
  }
}

}  // namespace vsh

using namespace vsh;

extern "C" vsh_status vsh_generate_isr(vsh_ctx* ctx, const vsh_request* req, double sqrt_s_hadron,
                                       vsh_result** out) {
  if (!ctx || !out) return VSH_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = nullptr;
  vsh_status rc = validate_request(ctx, req, true);
  if (rc) return rc;
  if (req->max_partons < 3) {
    set_error(ctx, "Drell-Yan records hold the two incoming partons and V: max_partons must be >= 3");
    return VSH_E_INVALID;
  }
  if (req->flags & ~(VSH_SUMMARY | VSH_RECORDS)) {
    set_error(ctx, "vsh_generate_isr takes VSH_SUMMARY and VSH_RECORDS only");
    return VSH_E_INVALID;
  }
  if (req->ecm_per_event || req->tcut_per_event || req->cycle_limit || req->t_over != 0.0 || req->mass_c != 0.0 ||
      req->mass_b != 0.0) {
    set_error(ctx, "vsh_generate_isr takes one Q (ecm) and t_cut, no per-event arrays, tail cut, t_over or masses");
    return VSH_E_INVALID;
  }
  if (!(sqrt_s_hadron > req->ecm) || !std::isfinite(sqrt_s_hadron)) {
    set_error(ctx, "sqrt_s_hadron (%g) must be finite and above Q = ecm (%g)", sqrt_s_hadron, req->ecm);
    return VSH_E_INVALID;
  }
  if (!(req->t_cut < 0.25 * req->ecm * req->ecm)) {
    set_error(ctx, "t_cut must lie below Q^2 / 4");
    return VSH_E_INVALID;
  }
  (void)hipSetDevice(ctx->device);
  const auto t0 = std::chrono::steady_clock::now();
  const uint32_t cap = req->max_partons;
  const uint64_t per_event = (uint64_t)cap * (4 * 8 + 1 + 2 * 2) + kNSumD * 8 + kNSumI * 4 + 8;
  uint64_t budget = ctx->budget;
  if (req->flags & VSH_RECORDS) budget /= 2;
  uint64_t chunk = std::min<uint64_t>(req->n_events, std::min<uint64_t>(budget / (per_event + 64), 1ull << 26));
  if (chunk < req->n_events) chunk &= ~63ull;
  if (chunk == 0) {
    set_error(ctx, "memory budget cannot hold one event of %u partons", cap);
    return VSH_E_NOMEM;
  }
  ResultBox* box = new_result(req->n_events, req->flags & VSH_SUMMARY);
  if (!box) {
    set_error(ctx, "host allocation failed");
    return VSH_E_NOMEM;
  }
  static const double L[kNObs] = {-1.0, -5.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0};
  static const double H[kNObs] = {3.0, 5.0, 50.0, 3.0, 1.0, 1.0, 1.0, 1.0};
  for (int h = 0; h < kNObs; ++h) {
    box->lo[h] = L[h];
    box->hi[h] = H[h];
  }
  hipStream_t st = ctx->stream;
  float t_sh = 0.0f;
  for (uint64_t a = 0; a < req->n_events; a += chunk) {
    const uint64_t count = std::min(chunk, req->n_events - a);
    const uint64_t stride = align_up(count, 64);
    const uint64_t slots = (uint64_t)cap * stride;
    const uint64_t need = slots * (4 * 8 + 1 + 2 * 2) + stride * (kNSumD * 8 + kNSumI * 4 + 8) + kHistDoubles * 8 +
                          16 * 256;
    rc = ctx->arena.reserve(ctx, need);
    if (rc) {
      delete box;
      return rc;
    }
    Carver c(ctx->arena.ptr);
    Records r{};
    r.E = (double*)c.take(slots * 8);
    r.x = (double*)c.take(slots * 8);
    r.y = (double*)c.take(slots * 8);
    r.z = (double*)c.take(slots * 8);
    r.pid = (int8_t*)c.take(slots);
    r.col = (uint16_t*)c.take(slots * 2);
    r.acol = (uint16_t*)c.take(slots * 2);
    r.cpart = r.apart = nullptr;
    r.stride = stride;
    r.cap = cap;
    Summary sm{};
    sm.d = (double*)c.take(kNSumD * stride * 8);
    sm.i = (int32_t*)c.take(kNSumI * stride * 4);
    sm.hash = (uint64_t*)c.take(stride * 8);
    sm.stride = stride;
    double* hist = (double*)c.take(kHistDoubles * 8);
    launch_zero(hist, kHistDoubles, st);
    const IsrInputs in{req->seed, req->first_event + a, sqrt_s_hadron, req->ecm, req->t_cut};
    (void)hipEventRecord(ctx->ev[1], st);
    hipLaunchKernelGGL(k_isr, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, st, r, sm, in, (uint32_t)count,
                       hist);
    (void)hipEventRecord(ctx->ev[2], st);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
      delete box;
      return hip_fail(ctx, err, "k_isr launch");
    }
    const bool all_fields = !box->sum_d.empty() || (req->flags & VSH_RECORDS);
    const int32_t* n_host = nullptr;
    rc = copy_back_chunk(ctx, st, hist, sm, stride, count, all_fields, box, a, &n_host);
    if (rc) {
      delete box;
      return rc;
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]) == hipSuccess) t_sh += ms;
    if (req->flags & VSH_RECORDS) {
      rc = gather_records(ctx, r, sm.i + kSiN * stride, n_host, count, box);
      if (rc) {
        delete box;
        return rc;
      }
    }
  }
  box->pub.t_shower_ms = t_sh;
  box->pub.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  finish_result(box);
  *out = &box->pub;
  return VSH_OK;
}
