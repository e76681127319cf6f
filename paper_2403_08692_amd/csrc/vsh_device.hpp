// vsh_device.hpp -- device-side building blocks of the shower engine for
// gfx950: counter-based Philox, u(0,1) conversion, one-loop alpha_s, the
// splitting-kernel family and the Catani-Seymour final-final map.
//
// Seymour & Sule, arXiv:2403.08692: the veto algorithm of Appendix A (trial
// scales t = T R^(1/c), z from the inverse of the overestimate's integral,
// acceptance ratio alpha_s/alpha_s^over x P/P^over) and the LO matrix element
// of Appendix B.  Everything is FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vsh {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// QCD colour factors and the electroweak / strong-coupling inputs
constexpr double kCF = 4.0 / 3.0;
constexpr double kCA = 3.0;
constexpr double kTR = 0.5;
constexpr double kNc = 3.0;
constexpr int kNf = 5;
constexpr double kMZ = 91.1876;
constexpr double kGammaZ = 2.4952;
constexpr double kMW = 80.385;
constexpr double kAlphaEM = 1.0 / 128.802;
constexpr double kAlphaSMZ = 0.118;
constexpr double kGeV2ToPb = 0.389379656e9;

// event status codes (shared meaning with the C ABI)
enum : uint8_t { kRunning = 0, kDone = 1, kOverflow = 2, kNonFinite = 3, kConservation = 4,
                 kCycleLimitHit = 5 };
// Every veto cycle lowers the scale or ends the event, so an event finishes
// after a few hundred cycles; this bound only guarantees that every lane of
// a launch exits whatever its inputs.
constexpr uint32_t kCycleLimit = 1u << 20;
// A request's tail cut (0 = none) as the cycle count the kernels compare with.
constexpr uint32_t effective_cycle_limit(uint32_t requested) {
  return requested == 0 || requested > kCycleLimit ? kCycleLimit : requested;
}

// Wave-wide scan and reduction through the device library's cross-lane
// (DPP) sequences; every lane of the wave must call them.
extern "C" __device__ uint64_t __ockl_wfscan_add_u64(uint64_t, bool);
extern "C" __device__ uint32_t __ockl_wfred_max_u32(uint32_t);
__device__ __forceinline__ uint64_t wave_inclusive_sum(uint64_t x) { return __ockl_wfscan_add_u64(x, true); }
__device__ __forceinline__ uint32_t wave_max(uint32_t x) { return __ockl_wfred_max_u32(x); }
__device__ __forceinline__ uint64_t lane63(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Quark masses by flavour (GeV), all zero for the massless shower.
struct QuarkMasses {
  double d, u, s, c, b;
};

__device__ __forceinline__ double quark_mass(const QuarkMasses& q, int pid) {
  const int a = pid < 0 ? -pid : pid;
  return a == 1 ? q.d : a == 2 ? q.u : a == 3 ? q.s : a == 4 ? q.c : a == 5 ? q.b : 0.0;
}

// draw purposes of the random-number contract
enum : uint32_t { kPurposeME = 1, kPurposeTrial = 2, kPurposeAccept = 3, kPurposeSplit = 4 };

constexpr uint16_t kNoPartner = 0xFFFF;
constexpr int kGluon = 21;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Counter = (event lo, event hi,
// cycle, purpose << 24 | slot), key = (seed lo, seed hi).  A draw depends
// only on what it is for, never on which lane or in which order it is made.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t a = (uint64_t)0xD2511F53u * c0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
    // three-input XOR in one gfx950 VALU op (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, k1, 0x96);
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
  }
  return U4{c0, c1, c2, c3};
}

struct Keyed {
  uint32_t ev_lo, ev_hi, k0, k1;
  __device__ __forceinline__ U4 draw(uint32_t cycle, uint32_t purpose, uint32_t slot) const {
    return philox10(ev_lo, ev_hi, cycle, (purpose << 24) | slot, k0, k1);
  }
};

__device__ __forceinline__ Keyed make_keyed(uint64_t seed, uint64_t event) {
  return Keyed{(uint32_t)event, (uint32_t)(event >> 32), (uint32_t)seed, (uint32_t)(seed >> 32)};
}

// 52 random bits m -> (2m+1) 2^-53, exact and strictly inside (0,1): the
// bits give 1 + m 2^-52 in [1, 2), and subtracting 1 - 2^-53 is exact
// (Sterbenz) and leaves m 2^-52 + 2^-53
__device__ __forceinline__ double unit(uint32_t hi, uint32_t lo) {
  const double one_m = __hiloint2double((int)(0x3FF00000u | (hi >> 12)), (int)lo);
  return one_m - 0x1.fffffffffffffp-1;
}

// the same 52 bits as an integer m (unit() is strictly increasing in m, so
// uniforms compare as their m), and unit() of such an m
__device__ __forceinline__ uint64_t unit_bits(uint32_t hi, uint32_t lo) {
  return ((uint64_t)(hi >> 12) << 32) | lo;
}
__device__ __forceinline__ double unit_of_bits(uint64_t m) {
  return unit((uint32_t)(m >> 32) << 12, (uint32_t)m);
}

// trial slot: splitter i, spectator k (both < 1024), block g of the kernel list
__device__ __forceinline__ uint32_t trial_slot(uint32_t i, uint32_t k, uint32_t g) {
  return (i << 14) | (k << 4) | g;
}

// ---------------------------------------------------------------------------
// One-loop alpha_s, n_f = 5, alpha_s(M_Z^2) = 0.118, at the emission's kT^2,
// from lt = ln kT^2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double alpha_s_of_log(double lt) {
  constexpr double b0 = (33.0 - 2.0 * kNf) / (12.0 * kPi);
  constexpr double ln_mz2 = 9.025837845847876;  // ln(91.1876^2)
  return kAlphaSMZ / (1.0 + kAlphaSMZ * b0 * (lt - ln_mz2));
}

// ---------------------------------------------------------------------------
// Splitting kernels (ids): 0-4 q->qg, 5-9 qbar->qbar g, 10 g->gg,
// 11-15 g->f fbar.  CS final-final kernels, leading colour (a gluon's charge
// is shared by its two dipole ends).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double kernel_value(int K, double z, double y) {
  if (K < 10) return kCF * (2.0 / (1.0 - z * (1.0 - y)) - (1.0 + z));
  if (K == 10) return 0.5 * kCA * (2.0 / (1.0 - z * (1.0 - y)) - 2.0 + z * (1.0 - z));
  return 0.5 * kTR * (1.0 - 2.0 * z * (1.0 - z));
}

__device__ __forceinline__ double kernel_over(int K, double z) {
  if (K < 10) return 2.0 * kCF / (1.0 - z);
  if (K == 10) return kCA / (1.0 - z);
  return 0.5 * kTR;
}

__device__ __forceinline__ double kernel_zgen(int K, double zm, double zp, double u) {
  if (K <= 10) return 1.0 - (1.0 - zm) * pow((1.0 - zp) / (1.0 - zm), u);
  return zm + (zp - zm) * u;
}

// ---------------------------------------------------------------------------
// LO e+e- -> q qbar through photon and Z (massless quarks, e- along +z,
// theta between e- and quark): |M|^2 = (4 pi alpha)^2 N_c [A(1+c^2) + B c].
// ---------------------------------------------------------------------------
__device__ __forceinline__ double me2(int flavour, double s, double c) {
  const double sw2 = 1.0 - (kMW / kMZ) * (kMW / kMZ);
  const double kappa = 1.0 / (4.0 * sw2 * (1.0 - sw2));
  const double mz2 = kMZ * kMZ;
  const double den = (s - mz2) * (s - mz2) + kGammaZ * kGammaZ * mz2;
  const double chi1 = kappa * s * (s - mz2) / den;
  const double chi2 = kappa * kappa * s * s / den;
  const double qe = -1.0, ae = -0.5, ve = -0.5 + 2.0 * sw2;
  const bool up = (flavour == 2 || flavour == 4);
  const double qf = up ? 2.0 / 3.0 : -1.0 / 3.0;
  const double af = up ? 0.5 : -0.5;
  const double vf = af - 2.0 * qf * sw2;
  const double A = qe * qe * qf * qf + 2.0 * qe * qf * ve * vf * chi1 +
                   (ae * ae + ve * ve) * (af * af + vf * vf) * chi2;
  const double B = 4.0 * qe * qf * ae * af * chi1 + 8.0 * ae * af * ve * vf * chi2;
  const double e2 = 4.0 * kPi * kAlphaEM;
  return e2 * e2 * kNc * (A * (1.0 + c * c) + B * c);
}

// ---------------------------------------------------------------------------
// Four-vectors (E, px, py, pz), metric (+,-,-,-)
// ---------------------------------------------------------------------------
struct P4 {
  double e, x, y, z;
};

__device__ __forceinline__ double mdot(const P4& a, const P4& b) {
  return a.e * b.e - a.x * b.x - a.y * b.y - a.z * b.z;
}

// v^mu = eps^{mu nu rho sigma} a_nu b_rho c_sigma, eps^{0123} = +1
__device__ __forceinline__ P4 eps4(const P4& a, const P4& b, const P4& c) {
  const double bcx = b.y * c.z - b.z * c.y, bcy = b.z * c.x - b.x * c.z, bcz = b.x * c.y - b.y * c.x;
  const double acx = a.y * c.z - a.z * c.y, acy = a.z * c.x - a.x * c.z, acz = a.x * c.y - a.y * c.x;
  const double abx = a.y * b.z - a.z * b.y, aby = a.z * b.x - a.x * b.z, abz = a.x * b.y - a.y * b.x;
  P4 v;
  v.e = -(a.x * bcx + a.y * bcy + a.z * bcz);
  v.x = -a.e * bcx + b.e * acx - c.e * abx;
  v.y = -a.e * bcy + b.e * acy - c.e * aby;
  v.z = -a.e * bcz + b.e * acz - c.e * abz;
  return v;
}

// CS final-final map: emitter pi (-> i, j) and spectator pk at t = kT^2, z,
// azimuth phi.  Transverse basis from the coordinate axis least aligned with
// E_k p_i - E_i p_k (lower axis on ties), n1 = eps(pi,pk,r), n2 = eps(pi,pk,n1).
__device__ __forceinline__ void split_kinematics(const P4& pi, const P4& pk, double t, double z,
                                                 double cphi, double sphi, P4& oi, P4& oj,
                                                 P4& ok) {
  const double q2 = 2.0 * mdot(pi, pk);
  const double y = t / (q2 * z * (1.0 - z));
  const double kt = sqrt(t);
  const double dx = pk.e * pi.x - pi.e * pk.x;
  const double dy = pk.e * pi.y - pi.e * pk.y;
  const double dz = pk.e * pi.z - pi.e * pk.z;
  int ax = 0;
  double best = fabs(dx);
  if (fabs(dy) < best) {
    ax = 1;
    best = fabs(dy);
  }
  if (fabs(dz) < best) ax = 2;
  const P4 r{0.0, ax == 0 ? 1.0 : 0.0, ax == 1 ? 1.0 : 0.0, ax == 2 ? 1.0 : 0.0};
  P4 n1 = eps4(pi, pk, r);
  const double l1 = sqrt(-mdot(n1, n1));
  n1.e /= l1;
  n1.x /= l1;
  n1.y /= l1;
  n1.z /= l1;
  P4 n2 = eps4(pi, pk, n1);
  const double l2 = sqrt(-mdot(n2, n2));
  n2.e /= l2;
  n2.x /= l2;
  n2.y /= l2;
  n2.z /= l2;
  const double a = z, b = (1.0 - z) * y, c = 1.0 - z, d = z * y, f = 1.0 - y;
  const P4 kp{kt * (cphi * n1.e + sphi * n2.e), kt * (cphi * n1.x + sphi * n2.x),
              kt * (cphi * n1.y + sphi * n2.y), kt * (cphi * n1.z + sphi * n2.z)};
  oi = P4{a * pi.e + b * pk.e + kp.e, a * pi.x + b * pk.x + kp.x, a * pi.y + b * pk.y + kp.y,
          a * pi.z + b * pk.z + kp.z};
  oj = P4{c * pi.e + d * pk.e - kp.e, c * pi.x + d * pk.x - kp.x, c * pi.y + d * pk.y - kp.y,
          c * pi.z + d * pk.z - kp.z};
  ok = P4{f * pk.e, f * pk.x, f * pk.y, f * pk.z};
}

__device__ __forceinline__ uint64_t fnv_step(uint64_t h, uint32_t v) {
  return (h ^ (uint64_t)v) * 0x100000001b3ull;
}
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;

}  // namespace vsh
