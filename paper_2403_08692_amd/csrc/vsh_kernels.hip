// vsh_kernels.hip -- the shower hot path for gfx950.
//
//   k_me             LO matrix element and event initialisation (App. B)
//   k_init_records   colour-partner links for caller-supplied initial states
//   k_shower_plain   thread per event, the whole veto loop in one launch
//                    (App. A / C: select winner, cutoff, alpha_s, veto, split)
//   k_obs            validation, Durham y23/y34, thrust, C, rho_H, B_T/B_W
//                    (Sec. 3.1) and histograms reduced in LDS before the
//                    global atomics
#include "vsh_kernels.hpp"

namespace vsh {

// ---------------------------------------------------------------------------
// Matrix element: one thread per event.  Flavour uniform over d,u,s,c,b
// (weight x5) by a 64-bit multiply-shift of one 32-bit word, cos(theta) and
// phi uniform; weight = 5 |M|^2 / (16 pi s) in pb.  Quark in slot 0 (colour
// line 1), antiquark in slot 1, back to back.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_me(Records r, Summary s, EventInputs in, uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double ecm = in.ecm_of(e);
  const Keyed key = make_keyed(in.seed, in.first + e);
  const U4 a = key.draw(0, kPurposeME, 0);
  const int f = 1 + (int)(((uint64_t)a.x * 5u) >> 32);
  const double c = 2.0 * unit(a.z, a.w) - 1.0;
  const U4 b = key.draw(0, kPurposeME, 1);
  const double phi = 2.0 * kPi * unit(b.x, b.y);
  const double sh = ecm * ecm;
  const double w = 5.0 * me2(f, sh, c) / (16.0 * kPi * sh) * kGeV2ToPb;
  const double st = sqrt((1.0 - c) * (1.0 + c));
  const double en = 0.5 * ecm;
  const double px = en * st * cos(phi), py = en * st * sin(phi), pz = en * c;
  r.store(0, e, P4{en, px, py, pz});
  r.store(1, e, P4{en, -px, -py, -pz});
  r.pid[e] = (int8_t)f;
  r.pid[r.stride + e] = (int8_t)(-f);
  r.col[e] = 1;
  r.acol[e] = 0;
  r.col[r.stride + e] = 0;
  r.acol[r.stride + e] = 1;
  r.cpart[e] = 1;
  r.apart[e] = kNoPartner;
  r.cpart[r.stride + e] = kNoPartner;
  r.apart[r.stride + e] = 0;
  s.d[kSdW * s.stride + e] = w;
  s.d[kSdCos * s.stride + e] = c;
  s.d[kSdPhi * s.stride + e] = phi;
  s.i[kSiN * s.stride + e] = 2;
  s.i[kSiFlavour * s.stride + e] = f;
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

// ---------------------------------------------------------------------------
// Shower state of one event held in registers while it evolves.
// ---------------------------------------------------------------------------
struct EvState {
  Keyed key;
  double lt;     // ln t, the current upper scale
  double tcut, ltc, asmax, cfac;
  uint64_t hash;
  uint32_t cycle, trials, ends;
  int n, next_col, n_emit, status;
};

struct Winner {
  double q2, zm, zp;
  int i, k, K;
};

// All trials of the dipole end (i, k): one per kernel of the splitter,
// t_try = t R^(1/c) compared as ln t + ln(R)/c (App. A, trial-scale
// equation); strict maximum above the running best.  A gluon end's five
// g -> f fbar kernels share c, so only their largest uniform needs a log.
__device__ __forceinline__ void end_trials(EvState& s, int i, int k, int pid_i, const P4& pi,
                                           const P4& pk, double& best, Winner& w) {
  const double q2 = 2.0 * mdot(pi, pk);
  if (!(q2 > 4.0 * s.tcut)) return;
  const double zp = 0.5 * (1.0 + sqrt(1.0 - 4.0 * s.tcut / q2));
  const double zm = 1.0 - zp;
  const double L = log((1.0 - zm) / (1.0 - zp));
  s.ends += 1;
  if (pid_i != kGluon) {
    const double c = s.cfac * ((2.0 * kCF) * L);
    const U4 d = s.key.draw(s.cycle, kPurposeTrial, trial_slot(i, k, 0));
    const double lt_try = s.lt + log(unit(d.x, d.y)) / c;
    s.trials += 1;
    if (lt_try > best) {
      best = lt_try;
      w = Winner{q2, zm, zp, i, k, pid_i > 0 ? pid_i - 1 : 4 - pid_i};
    }
  } else {
    const double cgg = s.cfac * (kCA * L);
    const double cqq = s.cfac * ((0.5 * kTR) * (zp - zm));
    const U4 d0 = s.key.draw(s.cycle, kPurposeTrial, trial_slot(i, k, 0));
    const U4 d1 = s.key.draw(s.cycle, kPurposeTrial, trial_slot(i, k, 1));
    const U4 d2 = s.key.draw(s.cycle, kPurposeTrial, trial_slot(i, k, 2));
    s.trials += 6;
    const double lgg = s.lt + log(unit(d0.x, d0.y)) / cgg;
    double um = unit(d0.z, d0.w);
    int fm = 1;
    double u = unit(d1.x, d1.y);
    if (u > um) { um = u; fm = 2; }
    u = unit(d1.z, d1.w);
    if (u > um) { um = u; fm = 3; }
    u = unit(d2.x, d2.y);
    if (u > um) { um = u; fm = 4; }
    u = unit(d2.z, d2.w);
    if (u > um) { um = u; fm = 5; }
    const double lqq = s.lt + log(um) / cqq;
    if (lgg > best) {
      best = lgg;
      w = Winner{q2, zm, zp, i, k, 10};
    }
    if (lqq > best) {
      best = lqq;
      w = Winner{q2, zm, zp, i, k, 10 + fm};
    }
  }
}

// One cycle of the veto algorithm for one event: SelectWinnerEmission over
// every colour-connected (splitter, spectator) in lexicographic order,
// CheckCutoff, alpha_s, AcceptOrVeto, GenerateEmission.
__device__ __forceinline__ void veto_cycle(EvState& s, const Records& r, uint64_t e) {
  double best = s.ltc;
  Winner w{0.0, 0.0, 0.0, -1, 0, 0};
  for (int i = 0; i < s.n; ++i) {
    const uint64_t oi = (uint64_t)i * r.stride + e;
    const int pid_i = r.pid[oi];
    int k1 = r.cpart[oi], k2 = r.apart[oi];
    if (k2 == k1) k2 = kNoPartner;  // closed two-parton loop: one dipole
    if (k1 > k2) {
      const int t = k1;
      k1 = k2;
      k2 = t;
    }
    const P4 pi = r.load(i, e);
    if (k1 != kNoPartner) end_trials(s, i, k1, pid_i, pi, r.load(k1, e), best, w);
    if (k2 != kNoPartner) end_trials(s, i, k2, pid_i, pi, r.load(k2, e), best, w);
  }
  const uint32_t this_cycle = s.cycle++;
  if (w.i < 0) {  // no trial above the cutoff
    s.status = kDone;
    return;
  }
  s.lt = best;  // the winner's scale bounds every later trial
  const double t = exp(best);
  const U4 a = s.key.draw(this_cycle, kPurposeAccept, 0);
  const double z = kernel_zgen(w.K, w.zm, w.zp, unit(a.x, a.y));
  const double y = t / (w.q2 * z * (1.0 - z));
  if (!(y < 1.0)) return;
  const double prob = alpha_s(t) / s.asmax * kernel_value(w.K, z, y) * (1.0 - y) / kernel_over(w.K, z);
  if (!(unit(a.z, a.w) < prob)) return;
  if (s.n == (int)r.cap) {
    s.status = kOverflow;
    return;
  }
  // --- splitting: kinematics, colours, flavours, append parton j at slot n
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

__device__ __forceinline__ void init_state(EvState& s, const Records& r, const Summary& sm,
                                           const EventInputs& in, uint64_t e) {
  const double ecm = in.ecm_of(e);
  s.key = make_keyed(in.seed, in.first + e);
  s.tcut = in.tcut_of(e);
  s.ltc = log(s.tcut);
  s.asmax = alpha_s(s.tcut);
  s.cfac = s.asmax / (2.0 * kPi);
  s.lt = log(ecm * ecm);  // evolution starts at s
  s.hash = kFnvOffset;
  s.cycle = 0;
  s.trials = 0;
  s.ends = 0;
  s.n = sm.i[kSiN * sm.stride + e];
  s.n_emit = 0;
  s.status = kRunning;
  int mc = 0;
  for (int a = 0; a < s.n; ++a) {
    const int c = r.col[(uint64_t)a * r.stride + e], ac = r.acol[(uint64_t)a * r.stride + e];
    mc = c > mc ? c : mc;
    mc = ac > mc ? ac : mc;
  }
  s.next_col = mc + 1;
}

__device__ __forceinline__ void write_state(const EvState& s, const Summary& sm, uint64_t e) {
  sm.i[kSiN * sm.stride + e] = s.n;
  sm.i[kSiStatus * sm.stride + e] = s.status;
  sm.i[kSiCycles * sm.stride + e] = (int32_t)s.cycle;
  sm.i[kSiEmit * sm.stride + e] = s.n_emit;
  sm.i[kSiTrials * sm.stride + e] = (int32_t)s.trials;
  sm.i[kSiEnds * sm.stride + e] = (int32_t)s.ends;
  sm.hash[e] = s.hash;
}

// Plain form: each thread evolves its event to the cutoff in one launch.
__global__ void __launch_bounds__(256) k_shower_plain(Records r, Summary sm, EventInputs in,
                                                      uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  EvState s;
  init_state(s, r, sm, in, e);
  while (s.status == kRunning) {
    veto_cycle(s, r, e);
    if (s.cycle >= kCycleLimit && s.status == kRunning) s.status = kCycleLimitHit;
  }
  write_state(s, sm, e);
}

// ---------------------------------------------------------------------------
// Observables, one thread per event (Sec. 3.1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double len3(double x, double y, double z) {
  return sqrt(x * x + y * y + z * z);
}

// exact thrust by the plane enumeration: pairs (i<j) span candidate planes,
// every other momentum sits on one side; i and j take all four sign choices
__device__ double thrust_of(const Records& r, uint64_t e, int n, double sum, double& ax,
                            double& ay, double& az) {
  double best = -1.0, bx = 0.0, by = 0.0, bz = 1.0;
  if (n < 3) {
    for (int m = 0; m < (1 << n); ++m) {
      double vx = 0.0, vy = 0.0, vz = 0.0;
      for (int a = 0; a < n; ++a) {
        const double sg = (m >> a & 1) ? -1.0 : 1.0;
        const uint64_t o = (uint64_t)a * r.stride + e;
        vx += sg * r.x[o];
        vy += sg * r.y[o];
        vz += sg * r.z[o];
      }
      const double m2 = vx * vx + vy * vy + vz * vz;
      if (m2 > best) { best = m2; bx = vx; by = vy; bz = vz; }
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const uint64_t oi = (uint64_t)i * r.stride + e;
      const double xi = r.x[oi], yi = r.y[oi], zi = r.z[oi];
      for (int j = i + 1; j < n; ++j) {
        const uint64_t oj = (uint64_t)j * r.stride + e;
        const double xj = r.x[oj], yj = r.y[oj], zj = r.z[oj];
        const double nx = yi * zj - zi * yj, ny = zi * xj - xi * zj, nz = xi * yj - yi * xj;
        double vx = 0.0, vy = 0.0, vz = 0.0;
        for (int k = 0; k < n; ++k) {
          if (k == i || k == j) continue;
          const uint64_t ok = (uint64_t)k * r.stride + e;
          const double xk = r.x[ok], yk = r.y[ok], zk = r.z[ok];
          const double d = xk * nx + yk * ny + zk * nz;
          if (d > 0.0) { vx += xk; vy += yk; vz += zk; }
          else { vx -= xk; vy -= yk; vz -= zk; }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double si = (c < 2) ? 1.0 : -1.0, sj = (c & 1) ? -1.0 : 1.0;
          const double wx = vx + si * xi + sj * xj, wy = vy + si * yi + sj * yj,
                       wz = vz + si * zi + sj * zj;
          const double m2 = wx * wx + wy * wy + wz * wz;
          if (m2 > best) { best = m2; bx = wx; by = wy; bz = wz; }
        }
      }
    }
  }
  const double l = sqrt(best);
  if (l > 0.0) { ax = bx / l; ay = by / l; az = bz / l; }
  else { ax = 0.0; ay = 0.0; az = 1.0; }
  return sum > 0.0 ? l / sum : 0.0;
}

// Durham clustering, E-scheme; y_ab = min(E_a,E_b)^2 |u_a - u_b|^2 / s
__device__ void durham_of(const Records& r, const Scratch& sc, uint64_t e, int n, double sh,
                          double& y23, double& y34) {
  for (int a = 0; a < n; ++a) {
    const uint64_t o = (uint64_t)a * r.stride + e;
    const uint64_t q = (uint64_t)a * sc.stride + e;
    sc.jE[q] = r.E[o];
    sc.jx[q] = r.x[o];
    sc.jy[q] = r.y[o];
    sc.jz[q] = r.z[o];
  }
  y23 = 0.0;
  y34 = 0.0;
  int m = n;
  while (m > 2) {
    double ymin = 0.0;
    int ba = -1, bb = -1;
    for (int a = 0; a < m; ++a) {
      const uint64_t qa = (uint64_t)a * sc.stride + e;
      const double ea = sc.jE[qa], xa = sc.jx[qa], ya = sc.jy[qa], za = sc.jz[qa];
      const double la = len3(xa, ya, za);
      for (int b = a + 1; b < m; ++b) {
        const uint64_t qb = (uint64_t)b * sc.stride + e;
        const double eb = sc.jE[qb], xb = sc.jx[qb], yb = sc.jy[qb], zb = sc.jz[qb];
        const double lb = len3(xb, yb, zb);
        const double dx = xa / la - xb / lb, dy = ya / la - yb / lb, dz = za / la - zb / lb;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const double em = ea < eb ? ea : eb;
        const double yv = em * em * d2 / sh;
        if (ba < 0 || yv < ymin) { ymin = yv; ba = a; bb = b; }
      }
    }
    if (m == 4) y34 = ymin;
    if (m == 3) y23 = ymin;
    const uint64_t qa = (uint64_t)ba * sc.stride + e;
    const uint64_t qb = (uint64_t)bb * sc.stride + e;
    sc.jE[qa] += sc.jE[qb];
    sc.jx[qa] += sc.jx[qb];
    sc.jy[qa] += sc.jy[qb];
    sc.jz[qa] += sc.jz[qb];
    for (int a = bb; a + 1 < m; ++a) {
      const uint64_t q0 = (uint64_t)a * sc.stride + e, q1 = q0 + sc.stride;
      sc.jE[q0] = sc.jE[q1];
      sc.jx[q0] = sc.jx[q1];
      sc.jy[q0] = sc.jy[q1];
      sc.jz[q0] = sc.jz[q1];
    }
    --m;
  }
}

__device__ __forceinline__ int bin_of(double x, double lo, double hi) {
  if (x != x) return kNBins + 1;
  if (x < lo) return 0;
  if (x >= hi) return kNBins + 1;
  int b = 1 + (int)((x - lo) / (hi - lo) * kNBins);
  return b > kNBins ? kNBins : b;
}

__constant__ HistRanges c_ranges = {{-4.3, -4.3, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0},
                                    {-0.3, -0.3, 0.5, 1.0, 0.5, 0.5, 0.35, 1.0}};

__global__ void __launch_bounds__(256) k_obs(Records r, Summary sm, EventInputs in, Scratch sc,
                                             uint32_t n, double* __restrict__ hist) {
  __shared__ double lh[kHistDoubles];
  for (int a = threadIdx.x; a < kHistDoubles; a += blockDim.x) lh[a] = 0.0;
  __syncthreads();
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    int status = sm.i[kSiStatus * sm.stride + e];
    const int np = sm.i[kSiN * sm.stride + e];
    const double ecm = in.ecm_of(e);
    const double sh = ecm * ecm;
    double obs[7] = {0, 0, 0, 0, 0, 0, 0};
    if (status == kDone) {
      // validation: finite, conserved to 1e-10 sqrt(s), massless to 1e-10 s
      double tE = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
      bool finite = true, massless = true;
      for (int a = 0; a < np; ++a) {
        const P4 p = r.load(a, e);
        finite = finite && isfinite(p.e) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
        tE += p.e;
        tx += p.x;
        ty += p.y;
        tz += p.z;
        massless = massless && fabs(mdot(p, p)) <= 1e-10 * sh;
      }
      const double tol = 1e-10 * ecm;
      if (!finite) status = kNonFinite;
      else if (fabs(tE - ecm) > tol || fabs(tx) > tol || fabs(ty) > tol || fabs(tz) > tol || !massless)
        status = kConservation;
    }
    if (status == kDone) {
      double sum = 0.0;
      for (int a = 0; a < np; ++a) {
        const uint64_t o = (uint64_t)a * r.stride + e;
        sum += len3(r.x[o], r.y[o], r.z[o]);
      }
      double ax, ay, az;
      const double T = thrust_of(r, e, np, sum, ax, ay, az);
      durham_of(r, sc, e, np, sh, obs[0], obs[1]);
      const double tau = 1.0 - T;
      obs[2] = tau > 0.0 ? tau : 0.0;
      // C-parameter
      double dbl = 0.0;
      for (int a = 0; a < np; ++a) {
        const uint64_t oa = (uint64_t)a * r.stride + e;
        const double xa = r.x[oa], ya = r.y[oa], za = r.z[oa], la = len3(xa, ya, za);
        for (int b = 0; b < np; ++b) {
          const uint64_t ob = (uint64_t)b * r.stride + e;
          const double xb = r.x[ob], yb = r.y[ob], zb = r.z[ob], lb = len3(xb, yb, zb);
          const double d = xa * xb + ya * yb + za * zb;
          dbl += d * d / (la * lb);
        }
      }
      const double cpar = 1.5 * (sum * sum - dbl) / (sum * sum);
      obs[3] = cpar > 0.0 ? cpar : 0.0;
      // hemispheres about the thrust axis
      P4 hp{0, 0, 0, 0}, hm{0, 0, 0, 0};
      double bp = 0.0, bm = 0.0;
      for (int a = 0; a < np; ++a) {
        const P4 q = r.load(a, e);
        const double d = q.x * ax + q.y * ay + q.z * az;
        const double kt = len3(q.y * az - q.z * ay, q.z * ax - q.x * az, q.x * ay - q.y * ax);
        if (d >= 0.0) { hp.e += q.e; hp.x += q.x; hp.y += q.y; hp.z += q.z; bp += kt; }
        else { hm.e += q.e; hm.x += q.x; hm.y += q.y; hm.z += q.z; bm += kt; }
      }
      const double mp = mdot(hp, hp), mm = mdot(hm, hm);
      const double rho = (mp > mm ? mp : mm) / sh;
      obs[4] = rho > 0.0 ? rho : 0.0;
      bp /= 2.0 * sum;
      bm /= 2.0 * sum;
      obs[5] = bp + bm;
      obs[6] = bp > bm ? bp : bm;
      // histograms (LDS)
      const double w = sm.d[kSdW * sm.stride + e];
      double vals[kNObs];
      vals[0] = obs[0] > 0.0 ? log10(obs[0]) : -INFINITY;
      vals[1] = obs[1] > 0.0 ? log10(obs[1]) : -INFINITY;
      for (int h = 2; h < 7; ++h) vals[h] = obs[h];
      vals[7] = sm.d[kSdCos * sm.stride + e];
#pragma unroll
      for (int h = 0; h < kNObs; ++h) {
        const int b = bin_of(vals[h], c_ranges.lo[h], c_ranges.hi[h]);
        double* cell = &lh[3 * (kNHCol * h + b)];
        atomicAdd(&cell[0], w);
        atomicAdd(&cell[1], w * w);
        atomicAdd(&cell[2], 1.0);
      }
    }
    for (int h = 0; h < 7; ++h) sm.d[(kSdY23 + h) * sm.stride + e] = obs[h];
    sm.i[kSiStatus * sm.stride + e] = status;
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
static inline uint32_t blocks_for(uint32_t n, uint32_t b) { return (n + b - 1) / b; }

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

void launch_obs(const Records& r, const Summary& s, const EventInputs& in, const Scratch& sc,
                uint32_t n, double* hist, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_obs, dim3(blocks_for(n, 256)), dim3(256), 0, st, r, s, in, sc, n, hist);
}

}  // namespace vsh
