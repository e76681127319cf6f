// vsh_shower.hpp -- one event's shower state and one cycle of the veto
// algorithm (App. A SelectWinnerEmission + GenerateEmission; App. C
// SelectWinner / CheckCutoff / alpha_s / AcceptOrVeto / GenerateEmission),
// shared by the plain and the persistent forms; and the LO matrix element
// that starts an event (App. B).
#pragma once

#include "vsh_kernels.hpp"
#include "vsh_massive.hpp"
#include "vsh_math.hpp"

namespace vsh {

// LO event into slot `e` of r: flavour uniform over d,u,s,c,b by a 64-bit
// multiply-shift of one 32-bit word, cos(theta), phi uniform; weight
// 5 |M|^2 / (16 pi s) in pb.  Quark in slot 0 (colour line 1), antiquark in
// slot 1, back to back.  With quark masses the flavour is uniform over those
// open at this sqrt(s) (2 m_f < sqrt(s)), the weight n_open beta |M|^2 /
// (16 pi s) and |p| = beta sqrt(s)/2.
struct MEOut {
  double w, c, phi;
  int f;
};

__device__ __forceinline__ MEOut me_event(const Records& r, uint64_t e, const Keyed& key, double ecm,
                                          const QuarkMasses& qm, bool massive) {
  const U4 a = key.draw(0, kPurposeME, 0);
  const double sh = ecm * ecm;
  int f;
  uint32_t n_open = 5;
  if (!massive) {
    f = 1 + (int)(((uint64_t)a.x * 5u) >> 32);
  } else {
    n_open = 0;
    for (int g = 1; g <= 5; ++g) {
      const double m = quark_mass(qm, g);
      n_open += 4.0 * m * m < sh;
    }
    const uint32_t idx = (uint32_t)(((uint64_t)a.x * (uint64_t)n_open) >> 32);
    f = 0;
    uint32_t seen = 0;
    for (int g = 1; g <= 5; ++g) {
      const double m = quark_mass(qm, g);
      if (4.0 * m * m < sh) {
        if (seen == idx) f = g;
        ++seen;
      }
    }
  }
  const double c = 2.0 * unit(a.z, a.w) - 1.0;
  const U4 b = key.draw(0, kPurposeME, 1);
  const double phi = 2.0 * kPi * unit(b.x, b.y);
  double w, beta = 1.0;
  const double mq = massive ? quark_mass(qm, f) : 0.0;
  if (!massive) {
    w = 5.0 * me2(f, sh, c) / (16.0 * kPi * sh) * kGeV2ToPb;
  } else if (mq == 0.0) {
    w = (double)n_open * me2(f, sh, c) / (16.0 * kPi * sh) * kGeV2ToPb;
  } else {
    beta = sqrt(1.0 - 4.0 * mq * mq / sh);
    w = (double)n_open * beta * me2_massive(f, sh, c, mq) / (16.0 * kPi * sh) * kGeV2ToPb;
  }
  const double st = sqrt((1.0 - c) * (1.0 + c));
  const double en = 0.5 * ecm;
  const double pm = en * beta;
  const double px = pm * st * cos(phi), py = pm * st * sin(phi), pz = pm * c;
  r.store(0, e, P4{en, px, py, pz});
  r.store(1, e, P4{en, -px, -py, -pz});
  r.pid[e] = (int8_t)f;
  r.pid[r.stride + e] = (int8_t)(-f);
  r.col[e] = 1;
  r.acol[e] = 0;
  r.col[r.stride + e] = 0;
  r.acol[r.stride + e] = 1;
  if (r.cpart) {  // output records carry no partner links
    r.cpart[e] = 1;
    r.apart[e] = kNoPartner;
    r.cpart[r.stride + e] = kNoPartner;
    r.apart[r.stride + e] = 0;
  }
  return MEOut{w, c, phi, f};
}

// ---------------------------------------------------------------------------
// Shower state of one event held in registers while it evolves.
// ---------------------------------------------------------------------------
struct EvState {
  Keyed key;
  double lt;  // ln t, the current upper scale
  double tcut, ltc, asmax, cfac;
  uint64_t hash;
  uint32_t cycle, trials, ends;
  int n, next_col, n_emit, status;
  int cap;  // record capacity of this event (its request's)
  double wsh;  // shower weight of the weighted veto (1 while the trial density bounds)
};

// what a trial needs to know about its event
struct TrialCtx {
  Keyed key;
  double lt, tcut, ltc, cfac;
  uint32_t cycle;
};

__device__ __forceinline__ TrialCtx trial_ctx(const EvState& s) {
  return TrialCtx{s.key, s.lt, s.tcut, s.ltc, s.cfac, s.cycle};
}

struct Winner {
  double rq2, zm, zp, L;  // rq2 = 1/Q^2; L = ln((1 - zm)/(1 - zp)), the log of the z range
  int i, k, K;
};

// (splitter, spectator, kernel) in one word whose numeric order is the
// lexicographic order of the paper's loop nest
__device__ __forceinline__ uint32_t pack_trial(int i, int k, int K) {
  return ((uint32_t)i << 14) | ((uint32_t)k << 4) | (uint32_t)K;
}
constexpr uint32_t kNoTrial = 0xFFFFFFFFu;

// Dipole mass and the z range of the overestimate for the end (i, k).
__device__ __forceinline__ bool end_limits(const P4& pi, const P4& pk, double tcut, double& q2, double& zm,
                                           double& zp) {
  q2 = 2.0 * mdot(pi, pk);
  if (!(q2 > 4.0 * tcut)) return false;  // no phase space above the cutoff
  zp = 0.5 * (1.0 + sqrt(1.0 - 4.0 * tcut / q2));
  zm = 1.0 - zp;
  return true;
}

// Trial coefficients c = alpha_s^over/(2 pi) * I of the dipole end (i, k),
// returned as their reciprocals ia = 1/ca, ib = 1/cb, the factors a trial's
// ln(R)/c is taken with: for a quark end ca = its one kernel's; for a gluon
// end ca = g -> g g's; cb = the common one of the five g -> f fbar kernels
// (kept for a quark end too: the decision recovers the end's range from it).
// False (and no coefficients) for an end without phase space above the
// cutoff.
__device__ __forceinline__ bool end_coeffs(double cfac, double tcut, int pid_i, const P4& pi, const P4& pk,
                                           double& q2, double& zm, double& zp, double& L, double& ia,
                                           double& ib) {
  if (!end_limits(pi, pk, tcut, q2, zm, zp)) return false;
  L = log_fast((1.0 - zm) / (1.0 - zp));
  const double ca = pid_i != kGluon ? cfac * ((2.0 * kCF) * L) : cfac * (kCA * L);
  const double cb = cfac * ((0.5 * kTR) * (zp - zm));
  const double r = 1.0 / (ca * cb);  // both reciprocals from one division
  ia = cb * r;
  ib = ca * r;
  return true;
}

// The winning end's z range, mass and log range as the decision takes them:
// recovered from its trial coefficients (the numbers the kernels keep: the
// massive ends' own, the massless ends' reciprocals in end_from_inverse
// below), so that every form decides from the same bits.  cb / (cfac T_R/2)
// = z+ - z- = sqrt(1 - 4 t_C / Q^2), ca / (cfac C) = L with C = 2 C_F or C_A.
// The divisions by cfac and t_C do not wait for the coefficients.  The
// decision's arithmetic (this, trial_z, massless_ratio) is evaluated as
// written, with no multiply-add fused by the compiler, so that the bits do
// not depend on where it is inlined.
__device__ __forceinline__ void end_from_coeffs(double cfac, double tcut, int K, double ca, double cb, Winner& w) {
#pragma clang fp contract(off)
  const double rcf = 1.0 / cfac, rt4 = 0.25 / tcut;
  const double dz = cb * (rcf * (1.0 / (0.5 * kTR)));
  w.zp = 0.5 * (1.0 + dz);
  w.zm = 1.0 - w.zp;
  w.rq2 = ((1.0 - dz) * (1.0 + dz)) * rt4;
  w.L = ca * (rcf * (K <= 9 ? 1.0 / (2.0 * kCF) : 1.0 / kCA));
}

// The same from the reciprocals (ia, ib) that end_coeffs returns and the
// massless forms keep: z+ - z- = cb / (cfac T_R/2) = 1/X with X = ib cfac
// T_R/2, L = ca / (cfac C) = 1/Y with Y = ia cfac C; with 1/(4 t_C) the three
// quotients come from one division, r = 1/(X Y t_C).
__device__ __forceinline__ void end_from_inverse(double cfac, double tcut, int K, double ia, double ib, Winner& w) {
#pragma clang fp contract(off)
  const double X = ib * (cfac * (0.5 * kTR)), Y = ia * (cfac * (K <= 9 ? 2.0 * kCF : kCA));
  const double r = 1.0 / ((X * Y) * tcut);
  const double dz = (Y * tcut) * r;
  w.zp = 0.5 * (1.0 + dz);
  w.zm = 1.0 - w.zp;
  w.rq2 = ((1.0 - dz) * (1.0 + dz)) * ((0.25 * (X * Y)) * r);
  w.L = (X * tcut) * r;
}

// True over trial density of a massless kernel at scale t = e^lt (App. A:
// alpha_s(t)/alpha_s^over x V (1-y) / O) in one division, with y = yn/yd,
// yn = t/Q^2 and yd = z(1-z); the CS w = 1 - z(1-y) = wn/yd.  -1 for
// y >= 1 (outside the phase space).
__device__ __forceinline__ double massless_ratio(int K, double lt, double t, double z, double rq2,
                                                 double asmax) {
#pragma clang fp contract(off)
  const double omz = 1.0 - z;
  const double yn = t * rq2, yd = z * omz;
  if (!(yn < yd)) return -1.0;
  constexpr double b0 = (33.0 - 2.0 * kNf) / (12.0 * kPi);
  constexpr double ln_mz2 = 9.025837845847876;  // ln(91.1876^2), as in alpha_s_of_log
  const double da = 1.0 + kAlphaSMZ * b0 * (lt - ln_mz2);
  double num, den;
  if (K <= 10) {
    const double wn = omz * yd + z * yn;
    const double a = K < 10 ? 1.0 + z : 2.0 - z * omz;  // q -> q g : g -> g g
    num = omz * (yd - yn) * (2.0 * yd - a * wn);
    den = 2.0 * yd * wn;
  } else {
    num = (1.0 - 2.0 * z * omz) * (yd - yn);
    den = yd;
  }
  return kAlphaSMZ * num / (asmax * da * den);
}

// z of the winner from the accept block's uniform uz, by the overestimate's
// inverse integral: for the 1/(1-z) kernels 1 - z = (1 - zm) ((1 - zp)/(1 -
// zm))^uz = (1 - zm) exp(-uz L); uniform in [zm, zp] for g -> f fbar.
__device__ __forceinline__ double trial_z(const Winner& w, double uz) {
#pragma clang fp contract(off)
  return w.K <= 10 ? 1.0 - (1.0 - w.zm) * exp(-uz * w.L) : w.zm + (w.zp - w.zm) * uz;
}

// The trials of an end with coefficients (ca, cb) = (1/ia, 1/ib): t_try = t
// R^(1/c) compared as ln t + ln(R)/c (App. A, trial-scale equation), taken
// as ln t + ln(R) ia (within an ulp of the quotient), strict maximum
// above the running best.  A gluon end's five g -> f fbar kernels share c, so
// only their largest uniform needs a log.  Returns the winning kernel (or -1
// if none beat `best`).  The first block serves a quark end's one kernel and
// a gluon end's g -> g g alike, so lanes with quark and gluon ends share it;
// only the gluon ends go on to blocks 1 and 2.
__device__ __forceinline__ int end_draws(const TrialCtx& c, int i, int k, int pid_i, double ia, double ib,
                                         double& best, uint32_t& trials) {
  // the sums are not fused with the products: a scale drawn ahead (lt = 0)
  // and chained later has the bits of one drawn at its own scale
#pragma clang fp contract(off)
  // kernel list g->gg, g->d dbar, ..., g->b bbar: block g holds kernels 2g, 2g+1
  const bool gluon = pid_i == kGluon;
  const U4 d0 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 0));
  const double l1 = c.lt + log_fast(unit(d0.x, d0.y)) * ia;
  int K = -1;
  if (l1 > best) {
    best = l1;
    K = gluon ? 10 : (pid_i > 0 ? pid_i - 1 : 4 - pid_i);
  }
  trials += gluon ? 6u : 1u;
  if (gluon) {
    // the five uniforms compared by their random bits (unit() is strictly
    // increasing in them): only the largest is converted
    uint64_t bm = unit_bits(d0.z, d0.w);
    int fm = 1;
#pragma unroll  // the two Philox blocks interleave
    for (uint32_t g = 1; g < 3; ++g) {
      const U4 d = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, g));
      const uint64_t b0 = unit_bits(d.x, d.y), b1 = unit_bits(d.z, d.w);
      if (b0 > bm) {  // first flavour wins ties, as in the kernel loop
        bm = b0;
        fm = 2 * g;
      }
      if (b1 > bm) {
        bm = b1;
        fm = 2 * g + 1;
      }
    }
    const double lqq = c.lt + log_fast(unit_of_bits(bm)) * ib;
    if (lqq > best) {
      best = lqq;
      K = 10 + fm;
    }
  }
  return K;
}

// All trials of the dipole end (i, k): one per kernel of the splitter.
__device__ __forceinline__ void end_trials(const TrialCtx& c, int i, int k, int pid_i, const P4& pi,
                                           const P4& pk, double& best, Winner& w, uint32_t& trials,
                                           uint32_t& ends) {
  double q2, zm, zp, L, ia, ib;
  if (!end_coeffs(c.cfac, c.tcut, pid_i, pi, pk, q2, zm, zp, L, ia, ib)) return;
  ends += 1;
  const int K = end_draws(c, i, k, pid_i, ia, ib, best, trials);
  if (K >= 0) {
    w.i = i;
    w.k = k;
    w.K = K;
    end_from_inverse(c.cfac, c.tcut, K, ia, ib, w);
  }
}

// Trials of parton i of the event in slot e: its dipole ends in ascending
// spectator order (a closed two-parton colour loop is one dipole).
__device__ __forceinline__ void parton_trials(const TrialCtx& c, const Records& r, uint64_t e, int i,
                                              double& best, Winner& w, uint32_t& trials, uint32_t& ends) {
  const uint64_t oi = (uint64_t)i * r.stride + e;
  const int pid_i = r.pid[oi];
  int k1 = r.cpart[oi], k2 = r.apart[oi];
  if (k2 == k1) k2 = kNoPartner;
  if (k1 > k2) {
    const int t = k1;
    k1 = k2;
    k2 = t;
  }
  const P4 pi = r.load(i, e);
  if (k1 != kNoPartner) end_trials(c, i, k1, pid_i, pi, r.load(k1, e), best, w, trials, ends);
  if (k2 != kNoPartner) end_trials(c, i, k2, pid_i, pi, r.load(k2, e), best, w, trials, ends);
}

// An accepted emission that has not been built yet: the winner's (i, k, K),
// its t and z, and the cycle that drew it (keys the azimuth).
struct Pending {
  double t, z;
  int i, k, K;
  uint32_t cycle;
};

// AcceptOrVeto's test with the accept block's words (2, 3).  Where the
// trial density undershoots (alpha_s of the trial density taken above t_C,
// ratio prob > 1): the weighted veto, accept with probability r / (2r - 1)
// and weight the event by +-(2r - 1), the least-variance choice.
__device__ __forceinline__ bool accept_test(double prob, const U4& a, double& wsh) {
  if (prob > 1.0) {
    const double g = 2.0 * prob - 1.0;
    const bool acc = unit(a.z, a.w) < prob / g;
    wsh *= acc ? g : -g;
    return acc;
  }
  return unit(a.z, a.w) < prob;
}

// The decision part of one cycle once the winner is known: CheckCutoff,
// alpha_s, AcceptOrVeto (App. C).  `best` is the winner's ln t, `a` the
// cycle's accept block (drawn ahead by the caller).  Returns true for an
// accepted emission that fits the record, described in p.
__device__ __forceinline__ bool veto_decide_drawn(EvState& s, double best, const Winner& w, const U4& a,
                                                  Pending& p, double& wsh) {
  const uint32_t this_cycle = s.cycle++;
  if (w.i < 0) {  // no trial above the cutoff
    s.status = kDone;
    return false;
  }
  s.lt = best;  // the winner's scale bounds every later trial
  const double t = exp(best);
  const double z = trial_z(w, unit(a.x, a.y));
  const double prob = massless_ratio(w.K, best, t, z, w.rq2, s.asmax);
  if (prob < 0.0) return false;  // y >= 1
  if (!accept_test(prob, a, wsh)) return false;
  if (s.n == s.cap) {
    s.status = kOverflow;
    return false;
  }
  p = Pending{t, z, w.i, w.k, w.K, this_cycle};
  return true;
}

__device__ __forceinline__ U4 accept_draw(const EvState& s) { return s.key.draw(s.cycle, kPurposeAccept, 0); }

__device__ __forceinline__ bool veto_decide(EvState& s, double best, const Winner& w, Pending& p) {
  return veto_decide_drawn(s, best, w, accept_draw(s), p, s.wsh);
}

// Colours, flavours, partner links and the hash of an emission whose
// momenta are in place (GenerateEmission, App. C); parton j appended at
// slot n.
__device__ __forceinline__ void emit_colours(EvState& s, const Records& r, uint64_t e, const Winner& w) {
  const int i = w.i, k = w.k, j = s.n;
  const uint64_t oi = (uint64_t)i * r.stride + e;
  const uint64_t ok = (uint64_t)k * r.stride + e;
  const uint64_t oj = (uint64_t)j * r.stride + e;
  const bool via_colour = r.cpart[oi] == k;
  if (w.K <= 10) {  // gluon emitted between i and k on their colour line
    const uint16_t m = (uint16_t)s.next_col++;
    r.pid[oj] = (int8_t)kGluon;
    if (via_colour) {
      r.col[oj] = r.col[oi];
      r.acol[oj] = m;
      r.col[oi] = m;
      r.cpart[oj] = (uint16_t)k;
      r.apart[ok] = (uint16_t)j;
      r.apart[oj] = (uint16_t)i;
      r.cpart[oi] = (uint16_t)j;
    } else {
      r.col[oj] = m;
      r.acol[oj] = r.acol[oi];
      r.acol[oi] = m;
      r.apart[oj] = (uint16_t)k;
      r.cpart[ok] = (uint16_t)j;
      r.cpart[oj] = (uint16_t)i;
      r.apart[oi] = (uint16_t)j;
    }
  } else {  // g -> f fbar: j is the parton colour-adjacent to k
    const int f = w.K - 10;
    if (via_colour) {
      r.pid[oj] = (int8_t)f;
      r.col[oj] = r.col[oi];
      r.acol[oj] = 0;
      r.pid[oi] = (int8_t)(-f);
      r.col[oi] = 0;
      r.cpart[oj] = (uint16_t)k;
      r.apart[ok] = (uint16_t)j;
      r.apart[oj] = kNoPartner;
      r.cpart[oi] = kNoPartner;
    } else {
      r.pid[oj] = (int8_t)(-f);
      r.col[oj] = 0;
      r.acol[oj] = r.acol[oi];
      r.pid[oi] = (int8_t)f;
      r.acol[oi] = 0;
      r.apart[oj] = (uint16_t)k;
      r.cpart[ok] = (uint16_t)j;
      r.cpart[oj] = kNoPartner;
      r.apart[oi] = kNoPartner;
    }
  }
  s.hash = fnv_step(fnv_step(fnv_step(s.hash, (uint32_t)w.K), (uint32_t)i), (uint32_t)k);
  s.n += 1;
  s.n_emit += 1;
}

// GenerateEmission (App. C): kinematics, then colours and flavours.
__device__ __forceinline__ void emit(EvState& s, const Records& r, uint64_t e, const Pending& pe) {
  const double t = pe.t, z = pe.z;
  const uint32_t this_cycle = pe.cycle;
  const Winner w{0.0, 0.0, 0.0, 0.0, pe.i, pe.k, pe.K};
  const U4 sd = s.key.draw(this_cycle, kPurposeSplit, 0);
  const double phi = 2.0 * kPi * unit(sd.x, sd.y);
  double sphi, cphi;
  sincos(phi, &sphi, &cphi);
  const int i = w.i, k = w.k, j = s.n;
  P4 ni, nj, nk;
  split_kinematics(r.load(i, e), r.load(k, e), t, z, cphi, sphi, ni, nj, nk);
  r.store(i, e, ni);
  r.store(k, e, nk);
  r.store(j, e, nj);
  emit_colours(s, r, e, w);
}

// The rest of one cycle once the winner is known: decision, then the
// emission if accepted.
__device__ __forceinline__ void veto_finish(EvState& s, const Records& r, uint64_t e, double best,
                                            const Winner& w) {
  Pending p;
  if (veto_decide(s, best, w, p)) emit(s, r, e, p);
}

// One cycle of the veto algorithm for one event, all in this lane:
// SelectWinnerEmission over every colour-connected (splitter, spectator) in
// lexicographic order, then the veto and the splitting.
__device__ __forceinline__ void veto_cycle(EvState& s, const Records& r, uint64_t e) {
  double best = s.ltc;
  Winner w{0.0, 0.0, 0.0, 0.0, -1, 0, 0};
  const TrialCtx c = trial_ctx(s);
  for (int i = 0; i < s.n; ++i) parton_trials(c, r, e, i, best, w, s.trials, s.ends);
  veto_finish(s, r, e, best, w);
}

// ---------------------------------------------------------------------------
// Massive quarks (vsh_massive.hpp): one cycle with each kernel's own phase
// space.  Kernels whose partons are all massless take exactly the massless
// numbers above, so an event without heavy quarks is the massless event.
// ---------------------------------------------------------------------------
struct MWinner {
  Winner w;
  double Q2, mi, mj, mk, fo;  // (p~ij + p~k)^2, masses, overestimate factor max(F, 1)
  bool massive;
};

// product masses of kernel K (i keeps the splitter's slot)
__device__ __forceinline__ void product_masses(int K, const QuarkMasses& qm, double& mi, double& mj) {
  if (K < 10) {
    mi = quark_mass(qm, K < 5 ? K + 1 : K - 4);
    mj = 0.0;
  } else if (K == 10) {
    mi = 0.0;
    mj = 0.0;
  } else {
    mi = quark_mass(qm, K - 10);
    mj = mi;
  }
}

// Range and trial coefficient of one kernel class of an end, as the trials
// and the decision both take them: z limits, L = ln((1 - zm)/(1 - zp)), the
// coefficient c and the overestimate factor fo = max(F, 1); `massive` for a
// kernel that takes the massive formulas.
struct MRange {
  double zm, zp, L, c, fo;
  bool massive;
};

// A quark end (q -> q g) with splitter mass mi and spectator mass mk.  False
// without phase space above the cutoff.
__device__ __forceinline__ bool mrange_quark(const TrialCtx& c, double q2, double Q2, double mi, double mk,
                                             MRange& R) {
  R.massive = mi > 0.0 || mk > 0.0;
  R.fo = 1.0;
  if (!R.massive) {
    if (!(q2 > 4.0 * c.tcut)) return false;
    R.zp = 0.5 * (1.0 + sqrt(1.0 - 4.0 * c.tcut / q2));
    R.zm = 1.0 - R.zp;
  } else {
    if (!massive_limits(Q2, mi, 0.0, mk, c.tcut, R.zm, R.zp)) return false;
    const double f = massive_flux(Q2, mi, 0.0, mk, mi);
    R.fo = f > 1.0 ? f : 1.0;
  }
  R.L = log_fast((1.0 - R.zm) / (1.0 - R.zp));
  R.c = c.cfac * ((2.0 * kCF) * R.L);
  if (R.massive) R.c *= R.fo;
  return true;
}

// g -> g g and the light g -> q qbar of a gluon end share one z range (only
// the spectator's mass enters): R.c is g -> g g's coefficient, cqq the
// common one of the light flavours.  Zero range and coefficients without
// phase space above the cutoff.
__device__ __forceinline__ bool mrange_light(const TrialCtx& c, double q2, double Q2, double mk, MRange& R,
                                             double& cqq) {
  R.massive = mk > 0.0;
  R.zm = R.zp = R.L = R.c = cqq = 0.0;
  R.fo = 1.0;
  const bool ok = R.massive ? massive_limits(Q2, 0.0, 0.0, mk, c.tcut, R.zm, R.zp) : q2 > 4.0 * c.tcut;
  if (!ok) return false;
  if (!R.massive) {
    R.zp = 0.5 * (1.0 + sqrt(1.0 - 4.0 * c.tcut / q2));
    R.zm = 1.0 - R.zp;
  } else {
    const double f = massive_flux(Q2, 0.0, 0.0, mk, 0.0);  // 1 up to rounding
    R.fo = f > 1.0 ? f : 1.0;
  }
  R.L = log_fast((1.0 - R.zm) / (1.0 - R.zp));
  R.c = c.cfac * (kCA * R.L);
  cqq = c.cfac * ((0.5 * kTR) * (R.zp - R.zm));
  if (R.massive) {
    R.c *= R.fo;
    cqq *= R.fo;
  }
  return true;
}

// g -> Q Qbar of a flavour with mass m: its own range when massive, else the
// light flavours' (G, cqq, light_ok from mrange_light).
__device__ __forceinline__ bool mrange_heavy(const TrialCtx& c, double Q2, double m, double mk, bool light_ok,
                                             const MRange& G, double cqq, MRange& R) {
  R = MRange{G.zm, G.zp, G.L, cqq, G.fo, m > 0.0 || mk > 0.0};
  if (m > 0.0) {
    if (!massive_limits(Q2, m, m, mk, c.tcut, R.zm, R.zp)) return false;
    const double fl = massive_flux(Q2, m, m, mk, 0.0);
    R.fo = fl > 1.0 ? fl : 1.0;
    R.L = log_fast((1.0 - R.zm) / (1.0 - R.zp));
    R.c = c.cfac * ((0.5 * kTR) * (R.zp - R.zm)) * R.fo;
    return true;
  }
  return light_ok;
}

// The winner record of kernel K of the end (i, k) with range R; cgg and cqq
// are the end's g -> g g and light g -> q qbar coefficients (a massless
// kernel's decision recovers its range from them, as the massless forms do).
__device__ __forceinline__ MWinner mwinner_of(const TrialCtx& c, int i, int k, int K, const MRange& R, double cgg,
                                              double cqq, double Q2, double mi, double mj, double mk) {
  Winner wn{0.0, R.zm, R.zp, R.L, i, k, K};
  if (!R.massive) end_from_coeffs(c.cfac, c.tcut, K < 10 ? K : 10, cgg, cqq, wn);
  wn.K = K;
  return MWinner{wn, Q2, mi, mj, mk, R.fo, R.massive};
}

// Every kernel of the end (i, k) in kernel order, strict maximum of ln t.
// Kernels share what their masses let them share: g -> g g and the three
// light g -> q qbar have the same z range (only the spectator's mass enters),
// and the light flavours one coefficient, so only their largest uniform needs
// a log; the c and b kernels have their own range and coefficient.  Each
// Philox block (two kernels) is drawn once.
__device__ __forceinline__ void end_trials_massive(const TrialCtx& c, int i, int k, int pid_i, int pid_k,
                                                   const P4& pi, const P4& pk, const QuarkMasses& qm,
                                                   double& best, MWinner& W, uint32_t& trials,
                                                   uint32_t& ends) {
  const double q2 = 2.0 * mdot(pi, pk);
  const double msp = quark_mass(qm, pid_i), mk = quark_mass(qm, pid_k);
  const double Q2 = q2 + msp * msp + mk * mk;
  bool active = false;
  if (pid_i != kGluon) {
    const int K = pid_i > 0 ? pid_i - 1 : 4 - pid_i;
    MRange R;
    if (mrange_quark(c, q2, Q2, msp, mk, R)) {
      active = true;
      const U4 d = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 0));
      const double lt_try = c.lt + log_fast(unit(d.x, d.y)) / R.c;
      trials += 1;
      if (lt_try > best) {
        best = lt_try;
        W = mwinner_of(c, i, k, K, R, R.c, c.cfac * ((0.5 * kTR) * (R.zp - R.zm)), Q2, msp, 0.0, mk);
      }
    }
  } else {
    // blocks: 0 -> g g, d dbar; 1 -> u ubar, s sbar; 2 -> c cbar, b bbar
    const U4 d0 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 0));
    const U4 d1 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 1));
    const U4 d2 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 2));
    MRange G;
    double cqq;
    const bool ok = mrange_light(c, q2, Q2, mk, G, cqq);
    if (ok) {
      active = true;
      trials += 4;
      const double lgg = c.lt + log_fast(unit(d0.x, d0.y)) / G.c;
      if (lgg > best) {
        best = lgg;
        W = mwinner_of(c, i, k, 10, G, G.c, cqq, Q2, 0.0, 0.0, mk);
      }
      double um = unit(d0.z, d0.w);
      int fm = 1;
      const double uu = unit(d1.x, d1.y), us = unit(d1.z, d1.w);
      if (uu > um) {  // the first flavour wins ties, as in the kernel loop
        um = uu;
        fm = 2;
      }
      if (us > um) {
        um = us;
        fm = 3;
      }
      const double lqq = c.lt + log_fast(um) / cqq;
      if (lqq > best) {
        best = lqq;
        W = mwinner_of(c, i, k, 10 + fm, G, G.c, cqq, Q2, 0.0, 0.0, mk);
      }
    }
#pragma unroll 1
    for (int f = 4; f <= 5; ++f) {  // c cbar, b bbar
      const double m = quark_mass(qm, f);
      MRange H;
      if (!mrange_heavy(c, Q2, m, mk, ok, G, cqq, H)) continue;
      active = true;
      trials += 1;
      const double u = f == 4 ? unit(d2.x, d2.y) : unit(d2.z, d2.w);
      const double lt_try = c.lt + log_fast(u) / H.c;
      if (lt_try > best) {
        best = lt_try;
        W = mwinner_of(c, i, k, 10 + f, H, G.c, cqq, Q2, m, m, mk);
      }
    }
  }
  if (active) ends += 1;
}

// The trial coefficients of the end (i, k) by kernel class, with the
// arithmetic of end_trials_massive: a quark end's in cc[0]; a gluon end's
// g -> g g, light g -> q qbar, g -> c cbar and g -> b bbar in cc[0..3].  0 for a
// class without phase space above the cutoff (an active class's coefficient
// is positive).  The flattened kernels cache them between emissions.
__device__ __forceinline__ void massive_end_coeffs(const TrialCtx& c, int pid_i, int pid_k, const P4& pi,
                                                   const P4& pk, const QuarkMasses& qm, double cc[4]) {
  cc[0] = cc[1] = cc[2] = cc[3] = 0.0;
  const double q2 = 2.0 * mdot(pi, pk);
  const double msp = quark_mass(qm, pid_i), mk = quark_mass(qm, pid_k);
  const double Q2 = q2 + msp * msp + mk * mk;
  if (pid_i != kGluon) {
    MRange R;
    if (mrange_quark(c, q2, Q2, msp, mk, R)) cc[0] = R.c;
    return;
  }
  MRange G;
  double cqq;
  const bool ok = mrange_light(c, q2, Q2, mk, G, cqq);
  if (ok) {
    cc[0] = G.c;
    cc[1] = cqq;
  }
#pragma unroll
  for (int f = 4; f <= 5; ++f) {
    MRange H;
    if (mrange_heavy(c, Q2, quark_mass(qm, f), mk, ok, G, cqq, H)) cc[f - 2] = H.c;
  }
}

// The trials of end_trials_massive from cached coefficients cc (same draws,
// order, counts and winner).  Returns the winning kernel, or -1 if none beat
// `best`.
__device__ __forceinline__ int end_draws_massive(const TrialCtx& c, int i, int k, int pid_i, const double cc[4],
                                                 double& best, uint32_t& trials, uint32_t& ends) {
  int K = -1;
  if (pid_i != kGluon) {
    if (cc[0] == 0.0) return -1;
    ends += 1;
    const U4 d = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 0));
    const double lt_try = c.lt + log_fast(unit(d.x, d.y)) / cc[0];
    trials += 1;
    if (lt_try > best) {
      best = lt_try;
      K = pid_i > 0 ? pid_i - 1 : 4 - pid_i;
    }
    return K;
  }
  if (cc[0] == 0.0 && cc[2] == 0.0 && cc[3] == 0.0) return -1;
  ends += 1;
  const U4 d0 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 0));
  const U4 d1 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 1));
  const U4 d2 = c.key.draw(c.cycle, kPurposeTrial, trial_slot(i, k, 2));
  if (cc[0] != 0.0) {
    trials += 4;
    const double lgg = c.lt + log_fast(unit(d0.x, d0.y)) / cc[0];
    if (lgg > best) {
      best = lgg;
      K = 10;
    }
    double um = unit(d0.z, d0.w);
    int fm = 1;
    const double uu = unit(d1.x, d1.y), us = unit(d1.z, d1.w);
    if (uu > um) {  // the first flavour wins ties, as in the kernel loop
      um = uu;
      fm = 2;
    }
    if (us > um) {
      um = us;
      fm = 3;
    }
    const double lqq = c.lt + log_fast(um) / cc[1];
    if (lqq > best) {
      best = lqq;
      K = 10 + fm;
    }
  }
  if (cc[2] != 0.0) {
    trials += 1;
    const double lt_try = c.lt + log_fast(unit(d2.x, d2.y)) / cc[2];
    if (lt_try > best) {
      best = lt_try;
      K = 14;
    }
  }
  if (cc[3] != 0.0) {
    trials += 1;
    const double lt_try = c.lt + log_fast(unit(d2.z, d2.w)) / cc[3];
    if (lt_try > best) {
      best = lt_try;
      K = 15;
    }
  }
  return K;
}

// The winner record of kernel K of the end (i, k) of the event in column e,
// recomputed from the records with the arithmetic of the trials above (the
// flattened forms, which keep only the winner's (i, k, K)).
__device__ __forceinline__ MWinner massive_winner(const TrialCtx& c, const Records& r, uint64_t e, int i, int k,
                                                  int K, const QuarkMasses& qm) {
  const int pid_i = r.pid[(uint64_t)i * r.stride + e], pid_k = r.pid[(uint64_t)k * r.stride + e];
  const P4 pi = r.load(i, e), pk = r.load(k, e);
  const double q2 = 2.0 * mdot(pi, pk);
  const double msp = quark_mass(qm, pid_i), mk = quark_mass(qm, pid_k);
  const double Q2 = q2 + msp * msp + mk * mk;
  MRange R;
  if (K < 10) {
    mrange_quark(c, q2, Q2, msp, mk, R);
    return mwinner_of(c, i, k, K, R, R.c, c.cfac * ((0.5 * kTR) * (R.zp - R.zm)), Q2, msp, 0.0, mk);
  }
  MRange G;
  double cqq;
  const bool ok = mrange_light(c, q2, Q2, mk, G, cqq);
  if (K <= 13) return mwinner_of(c, i, k, K, G, G.c, cqq, Q2, 0.0, 0.0, mk);
  const double m = quark_mass(qm, K - 10);
  mrange_heavy(c, Q2, m, mk, ok, G, cqq, R);
  return mwinner_of(c, i, k, K, R, G.c, cqq, Q2, m, m, mk);
}

__device__ __forceinline__ void parton_trials_massive(const TrialCtx& c, const Records& r, uint64_t e, int i,
                                                      const QuarkMasses& qm, double& best, MWinner& W,
                                                      uint32_t& trials, uint32_t& ends) {
  const uint64_t oi = (uint64_t)i * r.stride + e;
  const int pid_i = r.pid[oi];
  int k1 = r.cpart[oi], k2 = r.apart[oi];
  if (k2 == k1) k2 = kNoPartner;
  if (k1 > k2) {
    const int t = k1;
    k1 = k2;
    k2 = t;
  }
  const P4 pi = r.load(i, e);
  if (k1 != kNoPartner)
    end_trials_massive(c, i, k1, pid_i, r.pid[(uint64_t)k1 * r.stride + e], pi, r.load(k1, e), qm, best, W,
                       trials, ends);
  if (k2 != kNoPartner)
    end_trials_massive(c, i, k2, pid_i, r.pid[(uint64_t)k2 * r.stride + e], pi, r.load(k2, e), qm, best, W,
                       trials, ends);
}

__device__ __forceinline__ bool veto_decide_massive(EvState& s, double best, const MWinner& W, const U4& a,
                                                    Pending& p, double& wsh) {
  const Winner& w = W.w;
  const uint32_t this_cycle = s.cycle++;
  if (w.i < 0) {
    s.status = kDone;
    return false;
  }
  s.lt = best;
  const double t = exp(best);
  const double z = trial_z(w, unit(a.x, a.y));
  double prob;
  if (!W.massive) {
    prob = massless_ratio(w.K, best, t, z, w.rq2, s.asmax);
    if (prob < 0.0) return false;  // y >= 1
  } else {
    const double ratio = massive_ratio(w.K, t, z, W.Q2, W.mi, W.mj, W.mk, W.fo);
    if (ratio < 0.0) return false;  // outside the phase space
    prob = alpha_s_of_log(best) / s.asmax * ratio;
  }
  if (!accept_test(prob, a, wsh)) return false;
  if (s.n == s.cap) {
    s.status = kOverflow;
    return false;
  }
  p = Pending{t, z, w.i, w.k, w.K, this_cycle};
  return true;
}

__device__ __forceinline__ void emit_massive(EvState& s, const Records& r, uint64_t e, const Pending& pe,
                                             const QuarkMasses& qm) {
  const Winner w{0.0, 0.0, 0.0, 0.0, pe.i, pe.k, pe.K};
  const U4 sd = s.key.draw(pe.cycle, kPurposeSplit, 0);
  const double phi = 2.0 * kPi * unit(sd.x, sd.y);
  double sphi, cphi;
  sincos(phi, &sphi, &cphi);
  const int i = w.i, k = w.k, j = s.n;
  double mi, mj;
  product_masses(w.K, qm, mi, mj);
  const double mk = quark_mass(qm, r.pid[(uint64_t)k * r.stride + e]);
  P4 ni, nj, nk;
  if (mi > 0.0 || mj > 0.0 || mk > 0.0)
    split_massive(r.load(i, e), r.load(k, e), mi, mj, mk, w.K < 10 ? mi : 0.0, pe.t, pe.z, cphi, sphi, ni, nj,
                  nk);
  else
    split_kinematics(r.load(i, e), r.load(k, e), pe.t, pe.z, cphi, sphi, ni, nj, nk);
  r.store(i, e, ni);
  r.store(k, e, nk);
  r.store(j, e, nj);
  emit_colours(s, r, e, w);
}

__device__ __forceinline__ void veto_cycle_massive(EvState& s, const Records& r, uint64_t e,
                                                   const QuarkMasses& qm) {
  double best = s.ltc;
  MWinner W{Winner{0.0, 0.0, 0.0, 0.0, -1, 0, 0}, 0.0, 0.0, 0.0, 0.0, 1.0, false};
  const TrialCtx c = trial_ctx(s);
  for (int i = 0; i < s.n; ++i) parton_trials_massive(c, r, e, i, qm, best, W, s.trials, s.ends);
  Pending p;
  if (veto_decide_massive(s, best, W, accept_draw(s), p, s.wsh)) emit_massive(s, r, e, p, qm);
}

// Fresh state for an event whose n initial partons sit in slot e of r.
// alpha_s of the trial density: alpha_s(t_C), an overestimate at every
// t >= t_C, unless a scale t_over > 0 is given (then the weighted veto)
__device__ __forceinline__ double trial_alpha_s(double ltc, double t_over) {
  return alpha_s_of_log(t_over > 0.0 ? log_fast(t_over) : ltc);
}

__device__ __forceinline__ void init_state(EvState& s, const Records& r, uint64_t e, const Keyed& key,
                                           double ecm, double tcut, double t_over, int n, int cap) {
  s.cap = cap;
  s.key = key;
  s.tcut = tcut;
  s.ltc = log_fast(tcut);
  s.asmax = trial_alpha_s(s.ltc, t_over);
  s.cfac = s.asmax / (2.0 * kPi);
  s.wsh = 1.0;
  s.lt = log_fast(ecm * ecm);  // evolution starts at s
  s.hash = kFnvOffset;
  s.cycle = 0;
  s.trials = 0;
  s.ends = 0;
  s.n = n;
  s.n_emit = 0;
  s.status = kRunning;
  int mc = 0;
  for (int a = 0; a < n; ++a) {
    const int c = r.col[(uint64_t)a * r.stride + e], ac = r.acol[(uint64_t)a * r.stride + e];
    mc = c > mc ? c : mc;
    mc = ac > mc ? ac : mc;
  }
  s.next_col = mc + 1;
}

// State of an event that starts from its two LO partons (colour line 1).
__device__ __forceinline__ void lo_state(EvState& s, const Keyed& key, double ecm, double tcut, double t_over,
                                         int cap) {
  s.key = key;
  s.tcut = tcut;
  s.ltc = log_fast(tcut);
  s.asmax = trial_alpha_s(s.ltc, t_over);
  s.cfac = s.asmax / (2.0 * kPi);
  s.wsh = 1.0;
  s.lt = log_fast(ecm * ecm);
  s.hash = kFnvOffset;
  s.cycle = 0;
  s.trials = 0;
  s.ends = 0;
  s.n = 2;
  s.n_emit = 0;
  s.status = kRunning;
  s.next_col = 2;
  s.cap = cap;
}

// Start the event whose LO partons the matrix-element pass left in slots 0
// and 1 of `from` (column `ev`, no partner links there) in working slot e of r.
__device__ __forceinline__ void start_from_record(EvState& s, const Records& from, uint64_t ev, const Records& r,
                                                  uint64_t e, const Keyed& key, double ecm, double tcut,
                                                  double t_over, int cap) {
  for (uint32_t a = 0; a < 2; ++a) {
    const uint64_t f = (uint64_t)a * from.stride + ev, t = (uint64_t)a * r.stride + e;
    r.E[t] = from.E[f];
    r.x[t] = from.x[f];
    r.y[t] = from.y[f];
    r.z[t] = from.z[f];
    r.pid[t] = from.pid[f];
    r.col[t] = from.col[f];
    r.acol[t] = from.acol[f];
  }
  r.cpart[e] = 1;
  r.apart[e] = kNoPartner;
  r.cpart[r.stride + e] = kNoPartner;
  r.apart[r.stride + e] = 0;
  lo_state(s, key, ecm, tcut, t_over, cap);
}

__device__ __forceinline__ void write_state(const EvState& s, const Summary& sm, uint64_t e) {
  sm.i[kSiN * sm.stride + e] = s.n;
  sm.i[kSiStatus * sm.stride + e] = s.status;
  sm.i[kSiCycles * sm.stride + e] = (int32_t)s.cycle;
  sm.i[kSiEmit * sm.stride + e] = s.n_emit;
  sm.i[kSiTrials * sm.stride + e] = (int32_t)s.trials;
  sm.i[kSiEnds * sm.stride + e] = (int32_t)s.ends;
  sm.hash[e] = s.hash;
  if (s.wsh != 1.0) sm.d[kSdW * sm.stride + e] *= s.wsh;  // event weight = matrix element x shower
}

}  // namespace vsh
