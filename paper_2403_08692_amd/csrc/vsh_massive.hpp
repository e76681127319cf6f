// vsh_massive.hpp -- massive final-state quarks: the step the conclusions of
// Seymour & Sule (arXiv:2403.08692) name next.  The veto algorithm of
// App. A is unchanged; the matrix element, the dipole phase space, the
// splitting kernels and the recoil map gain mass terms.
//
// A kernel whose splitter, products and spectator are all massless keeps the
// massless formulas of vsh_device.hpp bit for bit.  For the others, with
// Q = p~ij + p~k, masses mi, mj of the products, mk of the spectator and
// Qb2 = Q^2 - mi^2 - mj^2 - mk^2:
//   evolution variable  t = y Qb2 z (1-z) - (1-z)^2 mi^2 - z^2 mj^2
//                       (the transverse momentum of the splitting when the
//                       spectator is massless), y and z the dipole variables
//                       p_i.p_j / (p_i.p_j + p_i.p_k + p_j.p_k) and
//                       p_i.p_k / (p_i.p_k + p_j.p_k);
//   emission density    alpha_s/(2 pi) F (1-y) dy/y dz V, F = Qb2 / sqrt(
//                       lambda(Q^2, mij^2, mk^2)) from the three-body over the
//                       two-body phase space, dy/y = dt/(t + (1-z)^2 mi^2 +
//                       z^2 mj^2) at fixed z;
//   overestimate        the massless one times max(F, 1), over the z range
//                       where t >= t_C fits below y = 1;
//   kernels             the quasi-collinear mass terms: -m^2/(p_i.p_j) in
//                       Q -> Q g, +2 m^2/s_ij in g -> Q Qbar.
#pragma once

#include "vsh_device.hpp"

namespace vsh {

__device__ __forceinline__ double kallen(double a, double b, double c) {
  return a * a + b * b + c * c - 2.0 * (a * b + a * c + b * c);
}

// |M|^2 of e+e- -> Q Qbar at quark velocity beta: vector current
// 2 - beta^2 (1 - c^2), axial current beta^2 (1 + c^2), their interference
// beta c.  Zero below threshold.
__device__ __forceinline__ double me2_massive(int flavour, double s, double c, double m) {
  const double b2 = 1.0 - 4.0 * m * m / s;
  if (!(b2 > 0.0)) return 0.0;
  const double beta = sqrt(b2);
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
  const double av = qe * qe * qf * qf + 2.0 * qe * qf * ve * vf * chi1 + (ae * ae + ve * ve) * vf * vf * chi2;
  const double aa = (ae * ae + ve * ve) * af * af * chi2;
  const double B = 4.0 * qe * qf * ae * af * chi1 + 8.0 * ae * af * ve * vf * chi2;
  const double e2 = 4.0 * kPi * kAlphaEM;
  return e2 * e2 * kNc * (av * (2.0 - b2 * (1.0 - c * c)) + aa * b2 * (1.0 + c * c) + B * beta * c);
}

// z range of the overestimate: between the roots of
// (mi^2 + mj^2 + Qb2) z^2 - (2 mi^2 + Qb2) z + mi^2 + t_C = 0.
__device__ __forceinline__ bool massive_limits(double Q2, double mi, double mj, double mk, double tcut,
                                               double& zm, double& zp) {
  const double mi2 = mi * mi, mj2 = mj * mj;
  const double qb2 = Q2 - mi2 - mj2 - mk * mk;
  if (!(qb2 > 0.0)) return false;
  const double A = mi2 + mj2 + qb2, B = 2.0 * mi2 + qb2, C = mi2 + tcut;
  const double disc = B * B - 4.0 * A * C;
  if (!(disc > 0.0)) return false;
  const double r = sqrt(disc);
  zm = (B - r) / (2.0 * A);
  zp = (B + r) / (2.0 * A);
  return true;
}

__device__ __forceinline__ double massive_flux(double Q2, double mi, double mj, double mk, double mij) {
  return (Q2 - mi * mi - mj * mj - mk * mk) / sqrt(kallen(Q2, mij * mij, mk * mk));
}

__device__ __forceinline__ double kernel_value_massive(int K, double z, double y, double mi, double qb2,
                                                       double sij) {
  if (K < 10) return kCF * (2.0 / (1.0 - z * (1.0 - y)) - (1.0 + z) - 2.0 * mi * mi / (y * qb2));
  if (K == 10) return kernel_value(K, z, y);
  return 0.5 * kTR * (1.0 - 2.0 * z * (1.0 - z) + 2.0 * mi * mi / sij);
}

// Where an emission at (t, z) lands: y, s_ij = (p_i + p_j)^2 and the
// coefficients of p_i = a p_ij + b p_k + kT in the massive map (the
// spectator p_k rescaled in the Q frame, p_ij = Q - p_k), from p_i^2 = mi^2,
// p_j^2 = mj^2 and p_i.p_k = z p_ij.p_k.  False outside the phase space (m
// is filled either way).
struct MassiveSplit {
  double y, sij, a, b, kt2;
};

__device__ __forceinline__ bool massive_split(double Q2, double mi, double mj, double mk, double t, double z,
                                              MassiveSplit& m) {
  const double mi2 = mi * mi, mj2 = mj * mj, mk2 = mk * mk;
  const double qb2 = Q2 - mi2 - mj2 - mk2;
  const double y = (t + (1.0 - z) * (1.0 - z) * mi2 + z * z * mj2) / (qb2 * z * (1.0 - z));
  const double s = mi2 + mj2 + y * qb2;
  const double lam = kallen(Q2, s, mk2);  // 4 (P^2 - s mk^2), P = p_ij.p_k
  const double P = 0.5 * (Q2 - s - mk2);
  const double b = (mi2 - mj2 - (2.0 * z - 1.0) * s) * P / (0.5 * lam);
  const double a = z - b * mk2 / P;
  const double kt2 = a * a * s + b * b * mk2 + 2.0 * a * b * P - mi2;
  m = MassiveSplit{y, s, a, b, kt2};
  return y < 1.0 && lam > 0.0 && kt2 >= 0.0;
}

// True over trial density without the alpha_s ratio; 0 inside the dead
// cone (kernel not positive), -1 outside the phase space.
__device__ __forceinline__ double massive_ratio(int K, double t, double z, double Q2, double mi, double mj,
                                                double mk, double fover) {
  MassiveSplit m;
  if (!massive_split(Q2, mi, mj, mk, t, z, m)) return -1.0;
  const double qb2 = Q2 - mi * mi - mj * mj - mk * mk;
  const double v = kernel_value_massive(K, z, m.y, mi, qb2, m.sij);
  if (!(v > 0.0)) return 0.0;
  const double f = massive_flux(Q2, mi, mj, mk, K < 10 ? mi : 0.0);
  const double cz = (1.0 - z) * (1.0 - z) * mi * mi + z * z * mj * mj;
  return f * (1.0 - m.y) * (t / (t + cz)) * v / (fover * kernel_over(K, z));
}

// unit vectors orthogonal to pa and pb (the massless map's basis)
__device__ __forceinline__ void transverse_pair(const P4& pa, const P4& pb, P4& n1, P4& n2) {
  const double dx = pb.e * pa.x - pa.e * pb.x;
  const double dy = pb.e * pa.y - pa.e * pb.y;
  const double dz = pb.e * pa.z - pa.e * pb.z;
  int ax = 0;
  double least = fabs(dx);
  if (fabs(dy) < least) {
    ax = 1;
    least = fabs(dy);
  }
  if (fabs(dz) < least) ax = 2;
  const P4 r{0.0, ax == 0 ? 1.0 : 0.0, ax == 1 ? 1.0 : 0.0, ax == 2 ? 1.0 : 0.0};
  n1 = eps4(pa, pb, r);
  const double l1 = sqrt(-mdot(n1, n1));
  n1 = P4{n1.e / l1, n1.x / l1, n1.y / l1, n1.z / l1};
  n2 = eps4(pa, pb, n1);
  const double l2 = sqrt(-mdot(n2, n2));
  n2 = P4{n2.e / l2, n2.x / l2, n2.y / l2, n2.z / l2};
}

__device__ __forceinline__ void split_massive(const P4& pij, const P4& pk, double mi, double mj, double mk,
                                              double mij, double t, double z, double cphi, double sphi,
                                              P4& oi, P4& oj, P4& ok) {
  const P4 Q{pij.e + pk.e, pij.x + pk.x, pij.y + pk.y, pij.z + pk.z};
  const double Q2 = mdot(Q, Q);
  MassiveSplit m;
  massive_split(Q2, mi, mj, mk, t, z, m);
  const double lam = kallen(Q2, m.sij, mk * mk);
  const double scale = sqrt((lam > 0.0 ? lam : 0.0) / kallen(Q2, mij * mij, mk * mk));
  const double along = mdot(Q, pk) / Q2, shift = (Q2 + mk * mk - m.sij) / (2.0 * Q2);
  P4 n1, n2;
  transverse_pair(pij, pk, n1, n2);
  const double kt = sqrt(m.kt2 > 0.0 ? m.kt2 : 0.0);
  const double q[4] = {Q.e, Q.x, Q.y, Q.z}, k[4] = {pk.e, pk.x, pk.y, pk.z};
  const double u1[4] = {n1.e, n1.x, n1.y, n1.z}, u2[4] = {n2.e, n2.x, n2.y, n2.z};
  double vi[4], vj[4], vk[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double nk = scale * (k[c] - along * q[c]) + shift * q[c];
    const double nij = q[c] - nk;
    vk[c] = nk;
    vi[c] = m.a * nij + m.b * nk + kt * (cphi * u1[c] + sphi * u2[c]);
    vj[c] = nij - vi[c];
  }
  oi = P4{vi[0], vi[1], vi[2], vi[3]};
  oj = P4{vj[0], vj[1], vj[2], vj[3]};
  ok = P4{vk[0], vk[1], vk[2], vk[3]};
}

}  // namespace vsh
