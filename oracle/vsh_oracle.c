/*
 * vsh_oracle.c -- serial FP64 reference ("oracle") for the parallel
 * Sudakov-veto parton shower (Seymour & Sule, arXiv:2403.08692).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library, and
 * sharing no source with it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared vsh_oracle.c -lm
 *
 * Structure, in the paper's order:
 *   random numbers ..... Philox4x32-10 from its published definition, keyed
 *                        by (seed, event, cycle, purpose, slot)
 *   matrix element ..... Appendix B: random flavour, LO |M|^2 for
 *                        e+e- -> Z/gamma -> q qbar, differential cross-section
 *   shower ............. Appendix A: SelectWinnerEmission (splitter x
 *                        spectator x kernel, strict maximum above t_C),
 *                        GenerateEmission (veto, kinematics, colours, append),
 *                        main loop from t = s down to t_C
 *   observables ........ Section 3.1: Durham y23/y34, exact thrust by the
 *                        O(N^3) plane enumeration, heavy-jet mass, jet
 *                        broadenings, C-parameter; event validation
 *   histograms ......... 50 uniform bins + under/overflow, weighted
 *
 * Physics inputs the paper does not print (electroweak constants, the
 * splitting kernels, the recoil map, the colour assignment, alpha_s running)
 * are the Catani-Seymour final-final dipole shower in the leading-colour
 * limit with one-loop running; each choice is named where it is used.
 */
#include "vsh_oracle.h"

#include <math.h>
#include <stddef.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------------- */
/* Constants.  QCD colour factors; electroweak inputs at the Z pole.       */
/* ---------------------------------------------------------------------- */
static const double CF = 4.0 / 3.0;
static const double CA = 3.0;
static const double TR = 0.5;
static const double NC = 3.0;
static const int NF = 5;
static const double MZ = 91.1876;
static const double GAMMAZ = 2.4952;
static const double MW = 80.385;
static const double ALPHA_EM = 1.0 / 128.802;
static const double ASMZ = 0.118;
static const double GEV2_TO_PB = 0.389379656e9;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies; the    */
/* key is bumped by the Weyl constants between rounds.                      */
/* ---------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)prod1;
    uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)prod0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

double or_uniform(uint32_t hi, uint32_t lo) {
  uint64_t m = ((uint64_t)(hi >> 12) << 32) | (uint64_t)lo; /* 52 random bits */
  return (double)(2 * m + 1) * 0x1p-53;
}

/* Random-number contract: every draw is one Philox block whose counter is
   (event low word, event high word, cycle, purpose << 24 | slot) and whose
   key is (seed low word, seed high word).  Draws therefore depend only on
   what they are for, never on the order in which anything is evaluated. */
void or_draw(uint64_t seed, uint64_t event, uint32_t cycle, uint32_t purpose,
             uint32_t slot, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)event, (uint32_t)(event >> 32), cycle,
                     (purpose << 24) | (slot & 0xFFFFFFu)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  or_philox4x32_10(ctr, key, out);
}

/* Trial slot of kernel number j (0-based position in the splitter's kernel
   list) of the dipole end with splitter i and spectator k: each Philox block
   serves two consecutive kernels of the list, words (0,1) the even one and
   words (2,3) the odd one. */
static uint32_t trial_slot(int i, int k, int j) {
  return ((uint32_t)i << 14) | ((uint32_t)k << 4) | (uint32_t)(j >> 1);
}

/* ---------------------------------------------------------------------- */
/* Strong coupling: one-loop running with five flavours, fixed at         */
/* alpha_s(M_Z^2) = 0.118 (the value quoted with the jet-rate figure);    */
/* evaluated at the transverse momentum squared of the emission.           */
/* ---------------------------------------------------------------------- */
double or_alpha_s(double t) {
  double b0 = (33.0 - 2.0 * NF) / (12.0 * OR_PI);
  return ASMZ / (1.0 + ASMZ * b0 * log(t / (MZ * MZ)));
}

/* ---------------------------------------------------------------------- */
/* Splitting kernels.  Catani-Seymour final-final dipole kernels with the   */
/* leading-colour split of a gluon's colour charge over its two colour      */
/* partners; y is the dipole recoil variable, z the splitter's momentum     */
/* fraction.  Each kernel has an overestimate that is analytically          */
/* integrable and invertible in z (the P^over of Appendix A).               */
/*   0-4   q -> q g     (splitter d, u, s, c, b)                            */
/*   5-9   qbar -> qbar g                                                   */
/*   10    g -> g g                                                         */
/*   11-15 g -> f fbar  (f = d, u, s, c, b)                                 */
/* ---------------------------------------------------------------------- */
int or_kernel_list(int pid, int out[6]) {
  if (pid >= 1 && pid <= 5) {
    out[0] = pid - 1;
    return 1;
  }
  if (pid <= -1 && pid >= -5) {
    out[0] = 4 - pid;
    return 1;
  }
  if (pid == 21) {
    for (int j = 0; j < 6; ++j) out[j] = 10 + j;
    return 6;
  }
  return 0;
}

double or_kernel_value(int K, double z, double y) {
  if (K < 10) return CF * (2.0 / (1.0 - z * (1.0 - y)) - (1.0 + z));
  if (K == 10) return 0.5 * CA * (2.0 / (1.0 - z * (1.0 - y)) - 2.0 + z * (1.0 - z));
  return 0.5 * TR * (1.0 - 2.0 * z * (1.0 - z));
}

double or_kernel_over(int K, double z) {
  if (K < 10) return 2.0 * CF / (1.0 - z);
  if (K == 10) return CA / (1.0 - z);
  return 0.5 * TR;
}

double or_kernel_integral(int K, double zm, double zp) {
  if (K < 10) return 2.0 * CF * log((1.0 - zm) / (1.0 - zp));
  if (K == 10) return CA * log((1.0 - zm) / (1.0 - zp));
  return 0.5 * TR * (zp - zm);
}

/* inverse of the overestimate's normalised integral from zm (eq. for z) */
double or_kernel_zgen(int K, double zm, double zp, double u) {
  if (K <= 10) return 1.0 - (1.0 - zm) * pow((1.0 - zp) / (1.0 - zm), u);
  return zm + (zp - zm) * u;
}

/* ---------------------------------------------------------------------- */
/* LO matrix element for e+e- -> (gamma or Z) -> q qbar (Appendix B), massless   */
/* quarks; e- along +z and theta the angle between the e- and the quark.   */
/* Summed over final and averaged over initial helicities and colours.     */
/* ---------------------------------------------------------------------- */
static void fermion_couplings(int flavour, double sw2, double *q, double *v, double *a) {
  int up_type = (flavour == 2 || flavour == 4);
  double t3 = up_type ? 0.5 : -0.5;
  *q = up_type ? 2.0 / 3.0 : -1.0 / 3.0;
  *a = t3;
  *v = t3 - 2.0 * (*q) * sw2;
}

static void ew_factors(double s, double *chi1, double *chi2, double *sw2_out) {
  double sw2 = 1.0 - (MW / MZ) * (MW / MZ);
  double kappa = 1.0 / (4.0 * sw2 * (1.0 - sw2));
  double mz2 = MZ * MZ;
  double den = (s - mz2) * (s - mz2) + GAMMAZ * GAMMAZ * mz2;
  *chi1 = kappa * s * (s - mz2) / den;
  *chi2 = kappa * kappa * s * s / den;
  *sw2_out = sw2;
}

/* angular coefficients: |M|^2 = (4 pi alpha)^2 N_c [A (1 + c^2) + B c] */
static void angular_coefficients(int flavour, double s, double *A, double *B) {
  double chi1, chi2, sw2;
  ew_factors(s, &chi1, &chi2, &sw2);
  double qe, ve, ae, qf, vf, af;
  qe = -1.0;
  ae = -0.5;
  ve = -0.5 + 2.0 * sw2;
  fermion_couplings(flavour, sw2, &qf, &vf, &af);
  *A = qe * qe * qf * qf + 2.0 * qe * qf * ve * vf * chi1 +
       (ae * ae + ve * ve) * (af * af + vf * vf) * chi2;
  *B = 4.0 * qe * qf * ae * af * chi1 + 8.0 * ae * af * ve * vf * chi2;
}

double or_me2(int flavour, double s, double cos_theta) {
  double A, B;
  angular_coefficients(flavour, s, &A, &B);
  double e2 = 4.0 * OR_PI * ALPHA_EM;
  return e2 * e2 * NC * (A * (1.0 + cos_theta * cos_theta) + B * cos_theta);
}

/* Quarks of mass m, velocity beta = sqrt(1 - 4 m^2 / s) in the CM frame.
   The vector current gives 1 + beta^2 c^2 + (1 - beta^2) = 2 - beta^2 (1 - c^2),
   the axial current beta^2 (1 + c^2), their interference beta c: the
   c-even coefficient A splits into its vector part A_V (the v_f^2 and
   photon terms) and axial part A_A (the a_f^2 term). */
double or_me2_massive(int flavour, double s, double cos_theta, double m) {
  if (m == 0.0) return or_me2(flavour, s, cos_theta);
  double b2 = 1.0 - 4.0 * m * m / s;
  if (!(b2 > 0.0)) return 0.0;
  double beta = sqrt(b2);
  double chi1, chi2, sw2;
  ew_factors(s, &chi1, &chi2, &sw2);
  double qe = -1.0, ae = -0.5, ve = -0.5 + 2.0 * sw2, qf, vf, af;
  fermion_couplings(flavour, sw2, &qf, &vf, &af);
  double av = qe * qe * qf * qf + 2.0 * qe * qf * ve * vf * chi1 + (ae * ae + ve * ve) * vf * vf * chi2;
  double aa = (ae * ae + ve * ve) * af * af * chi2;
  double B = 4.0 * qe * qf * ae * af * chi1 + 8.0 * ae * af * ve * vf * chi2;
  double c = cos_theta;
  double e2 = 4.0 * OR_PI * ALPHA_EM;
  return e2 * e2 * NC * (av * (2.0 - b2 * (1.0 - c * c)) + aa * b2 * (1.0 + c * c) + B * beta * c);
}

/* sigma_LO over the flavours open at s (2 m_f < sqrt(s)), in pb */
double or_sigma_lo_massive(double s, const double mass[6]) {
  double total = 0.0;
  for (int f = 1; f <= NF; ++f) {
    double m = mass ? mass[f] : 0.0;
    double b2 = 1.0 - 4.0 * m * m / s;
    if (!(b2 > 0.0)) continue;
    double beta = sqrt(b2);
    /* beta times the integral over c of |M|^2 / (32 pi s); the c-even part
       of |M|^2 is a + b c^2 with a = M(0) and b = (M(1) + M(-1))/2 - a */
    double a0 = or_me2_massive(f, s, 0.0, m);
    double b0 = 0.5 * (or_me2_massive(f, s, 1.0, m) + or_me2_massive(f, s, -1.0, m)) - a0;
    total += beta * (2.0 * a0 + 2.0 * b0 / 3.0) / (32.0 * OR_PI * s);
  }
  return total * GEV2_TO_PB;
}

/* total LO cross-section over the five flavours, in pb: the integral of
   |M|^2 / (32 pi s) over cos(theta) in [-1, 1] */
double or_sigma_lo(double s) {
  double total = 0.0;
  for (int f = 1; f <= NF; ++f) {
    double A, B;
    angular_coefficients(f, s, &A, &B);
    total += 4.0 * OR_PI * ALPHA_EM * ALPHA_EM * NC * A / (3.0 * s);
  }
  return total * GEV2_TO_PB;
}

/* One LO event: a uniform flavour (weight x5), uniform cos(theta) and phi;
   the weight is the differential cross-section over the sampling density,
   5 |M|^2 / (16 pi s), in pb.  Outputs p[0..3] quark, p[4..7] antiquark. */
void or_me_event(uint64_t seed, uint64_t event, double ecm, int *flavour,
                 double *cos_theta, double *phi, double *weight, double p[8]) {
  or_me_event_massive(seed, event, ecm, NULL, flavour, cos_theta, phi, weight, p);
}

/* With quark masses: the flavour is uniform over the flavours open at
   this sqrt(s) (2 m_f < sqrt(s); d, u, s always), in the order d, u, s, c,
   b, with weight n_open; the two-body phase space brings a factor beta and
   the quarks have |p| = beta sqrt(s) / 2. */
void or_me_event_massive(uint64_t seed, uint64_t event, double ecm, const double mass[6],
                         int *flavour, double *cos_theta, double *phi, double *weight,
                         double p[8]) {
  uint32_t w[4];
  double s = ecm * ecm;
  int open[5], n_open = 0;
  for (int f = 1; f <= NF; ++f)
    if (!mass || 4.0 * mass[f] * mass[f] < s) open[n_open++] = f;
  or_draw(seed, event, 0, OR_P_ME, 0, w);
  int f = open[(int)(((uint64_t)w[0] * (uint64_t)n_open) >> 32)];
  double c = 2.0 * or_uniform(w[2], w[3]) - 1.0;
  or_draw(seed, event, 0, OR_P_ME, 1, w);
  double ph = 2.0 * OR_PI * or_uniform(w[0], w[1]);
  double m = mass ? mass[f] : 0.0;
  double wt, beta = 1.0;
  if (m == 0.0) {
    wt = (double)n_open * or_me2(f, s, c) / (16.0 * OR_PI * s) * GEV2_TO_PB;
  } else {
    beta = sqrt(1.0 - 4.0 * m * m / s);
    wt = (double)n_open * beta * or_me2_massive(f, s, c, m) / (16.0 * OR_PI * s) * GEV2_TO_PB;
  }
  double st = sqrt((1.0 - c) * (1.0 + c));
  double e = 0.5 * ecm;
  double pm = e * beta;
  double px = pm * st * cos(ph), py = pm * st * sin(ph), pz = pm * c;
  p[0] = e;
  p[1] = px;
  p[2] = py;
  p[3] = pz;
  p[4] = e;
  p[5] = -px;
  p[6] = -py;
  p[7] = -pz;
  *flavour = f;
  *cos_theta = c;
  *phi = ph;
  *weight = wt;
}

/* ---------------------------------------------------------------------- */
/* Minkowski helpers, metric (+,-,-,-)                                      */
/* ---------------------------------------------------------------------- */
static double mdot(const double *a, const double *b) {
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* v^mu = eps^{mu nu rho sigma} a_nu b_rho c_sigma with eps^{0123} = +1,
   written with three-vectors:
     v^0 = -a.(b x c),  v = -a0 (b x c) + b0 (a x c) - c0 (a x b)        */
static void eps4(const double *a, const double *b, const double *c, double *v) {
  double bc[3] = {b[2] * c[3] - b[3] * c[2], b[3] * c[1] - b[1] * c[3], b[1] * c[2] - b[2] * c[1]};
  double ac[3] = {a[2] * c[3] - a[3] * c[2], a[3] * c[1] - a[1] * c[3], a[1] * c[2] - a[2] * c[1]};
  double ab[3] = {a[2] * b[3] - a[3] * b[2], a[3] * b[1] - a[1] * b[3], a[1] * b[2] - a[2] * b[1]};
  v[0] = -(a[1] * bc[0] + a[2] * bc[1] + a[3] * bc[2]);
  for (int m = 0; m < 3; ++m) v[1 + m] = -a[0] * bc[m] + b[0] * ac[m] - c[0] * ab[m];
}

/* ---------------------------------------------------------------------- */
/* Catani-Seymour final-final map.  Emitter ~ij and spectator ~k, both    */
/* massless, Q^2 = 2 p~ij.p~k; t = kT^2 = y z (1-z) Q^2:                   */
/*   p_i = z p~ij + (1-z) y p~k + kT,  p_j = (1-z) p~ij + z y p~k - kT,     */
/*   p_k = (1-y) p~k, with kT^2 = -t and kT orthogonal to both.             */
/* The transverse basis: a reference axis r (the coordinate axis least      */
/* aligned with E_k p_i - E_i p_k, the only spatial direction inside the    */
/* span of the two momenta; ties to the lower axis), n1 = eps(pi,pk,r) and  */
/* n2 = eps(pi,pk,n1), both normalised to n^2 = -1.                         */
/* ---------------------------------------------------------------------- */
void or_split_kinematics(const double pi[4], const double pk[4], double t,
                         double z, double phi, double out_i[4],
                         double out_j[4], double out_k[4]) {
  double q2 = 2.0 * mdot(pi, pk);
  double y = t / (q2 * z * (1.0 - z));
  double kt = sqrt(t);
  double d[3];
  for (int m = 0; m < 3; ++m) d[m] = pk[0] * pi[1 + m] - pi[0] * pk[1 + m];
  int ax = 0;
  if (fabs(d[1]) < fabs(d[ax])) ax = 1;
  if (fabs(d[2]) < fabs(d[ax])) ax = 2;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  r[1 + ax] = 1.0;
  double n1[4], n2[4];
  eps4(pi, pk, r, n1);
  double norm1 = sqrt(-mdot(n1, n1));
  for (int m = 0; m < 4; ++m) n1[m] /= norm1;
  eps4(pi, pk, n1, n2);
  double norm2 = sqrt(-mdot(n2, n2));
  for (int m = 0; m < 4; ++m) n2[m] /= norm2;
  double cphi = cos(phi), sphi = sin(phi);
  for (int m = 0; m < 4; ++m) {
    double kperp = kt * (cphi * n1[m] + sphi * n2[m]);
    out_i[m] = z * pi[m] + (1.0 - z) * y * pk[m] + kperp;
    out_j[m] = (1.0 - z) * pi[m] + z * y * pk[m] - kperp;
    out_k[m] = (1.0 - y) * pk[m];
  }
}

/* ---------------------------------------------------------------------- */
/* Massive quarks (the step the conclusions name: the veto algorithm stays */
/* as it is, the splitting functions gain mass terms).  mass[f] is the     */
/* mass of flavour f = 1..5 (d, u, s, c, b); a NULL table means massless.  */
/* A kernel whose splitter, products and spectator are all massless uses   */
/* the massless formulas above unchanged.                                  */
/*                                                                          */
/* Evolution variable: t = y Qb2 z (1-z) - (1-z)^2 mi^2 - z^2 mj^2 with      */
/* Qb2 = Q^2 - mi^2 - mj^2 - mk^2 (the transverse momentum of i and j when  */
/* the spectator is massless), y = p_i.p_j / (p_i.p_j + p_i.p_k + p_j.p_k)  */
/* and z = p_i.p_k / (p_i.p_k + p_j.p_k); Q = p~ij + p~k.                   */
/* ---------------------------------------------------------------------- */
static double flavour_mass(const double *mass, int pid) {
  if (!mass || pid == 21 || pid == 0) return 0.0;
  return mass[pid > 0 ? pid : -pid];
}

/* masses of the products i and j of kernel K (i keeps the splitter's slot) */
static void kernel_product_masses(int K, const double *mass, double *mi, double *mj) {
  if (K < 10) {
    *mi = flavour_mass(mass, K < 5 ? K + 1 : K - 4);
    *mj = 0.0;
  } else if (K == 10) {
    *mi = 0.0;
    *mj = 0.0;
  } else {
    *mi = flavour_mass(mass, K - 10);
    *mj = *mi;
  }
}

static double kallen(double a, double b, double c) {
  return a * a + b * b + c * c - 2.0 * (a * b + a * c + b * c);
}

/* z range of the overestimate: t >= t_C with y <= 1 holds between the roots
   of (mi^2 + mj^2 + Qb2) z^2 - (2 mi^2 + Qb2) z + mi^2 + t_C = 0.  Returns 0
   when there is no phase space. */
int or_massive_limits(double Q2, double mi, double mj, double mk, double tcut, double *zm,
                      double *zp) {
  double mi2 = mi * mi, mj2 = mj * mj;
  double qb2 = Q2 - mi2 - mj2 - mk * mk;
  if (!(qb2 > 0.0)) return 0;
  double A = mi2 + mj2 + qb2, B = 2.0 * mi2 + qb2, C = mi2 + tcut;
  double disc = B * B - 4.0 * A * C;
  if (!(disc > 0.0)) return 0;
  double r = sqrt(disc);
  *zm = (B - r) / (2.0 * A);
  *zp = (B + r) / (2.0 * A);
  return 1;
}

/* Flux factor of the massive dipole phase space: the three-body phase
   space over the two-body one is Qb2^2 (1 - y) dy dz / (16 pi^2
   sqrt(lambda(Q^2, mij^2, mk^2))) and 2 p_i.p_j = y Qb2, so the emission
   density is alpha_s/(2 pi) F (1 - y) (dy/y) dz V with
   F = Qb2 / sqrt(lambda(Q^2, mij^2, mk^2)); F = 1 when everything is
   massless, and F > 1 only for Q -> Q g with a massive spectator. */
double or_massive_flux(double Q2, double mi, double mj, double mk, double mij) {
  return (Q2 - mi * mi - mj * mj - mk * mk) / sqrt(kallen(Q2, mij * mij, mk * mk));
}

/* Mass terms of the quasi-collinear limit added to the massless kernels:
     Q -> Q g:     C_F [2/(1 - z(1 - y)) - (1 + z) - m^2/(p_i.p_j)]
     g -> Q Qbar:  (T_R/2) [1 - 2 z (1 - z) + 2 m^2 / s_ij]
   with p_i.p_j = y Qb2 / 2 and s_ij = (p_i + p_j)^2 = 2 m^2 + y Qb2 for the
   pair; g -> g g has none. */
double or_kernel_value_massive(int K, double z, double y, double mi, double qb2, double sij) {
  if (K < 10) return CF * (2.0 / (1.0 - z * (1.0 - y)) - (1.0 + z) - 2.0 * mi * mi / (y * qb2));
  if (K == 10) return or_kernel_value(K, z, y);
  return 0.5 * TR * (1.0 - 2.0 * z * (1.0 - z) + 2.0 * mi * mi / sij);
}

/* The emission at (t, z) in the massive map: Q = p~ij + p~k; the spectator
   keeps its direction in the Q frame, rescaled so that (Q - p_k)^2 = s_ij,
     p_k = sqrt(lambda(Q^2, s_ij, mk^2) / lambda(Q^2, mij^2, mk^2))
             (p~k - (Q.p~k / Q^2) Q) + (Q^2 + mk^2 - s_ij) / (2 Q^2) Q,
   and p_ij = Q - p_k.  Then p_i = a p_ij + b p_k + kT, kT orthogonal to
   p_ij and p_k, from p_i^2 = mi^2, p_j^2 = mj^2 and p_i.p_k = z p_ij.p_k:
     b = (mi^2 - mj^2 - (2z - 1) s_ij) P / (2 (P^2 - s_ij mk^2)),
     a = z - b mk^2 / P,   -kT^2 = a^2 s_ij + b^2 mk^2 + 2 a b P - mi^2,
   with P = p_ij.p_k = (Q^2 - s_ij - mk^2)/2 and P^2 - s_ij mk^2 =
   lambda(Q^2, s_ij, mk^2)/4.  With all masses zero, a = z and
   b = (1 - 2z) y / (1 - y): the massless map.  Returns 0 outside the phase
   space (y >= 1, no room for p_k, or kT^2 < 0); the outputs are set either
   way. */
static int massive_vars(double Q2, double mi, double mj, double mk, double t, double z,
                        double *y, double *sij, double *a, double *b, double *kt2) {
  double mi2 = mi * mi, mj2 = mj * mj, mk2 = mk * mk;
  double qb2 = Q2 - mi2 - mj2 - mk2;
  double yy = (t + (1.0 - z) * (1.0 - z) * mi2 + z * z * mj2) / (qb2 * z * (1.0 - z));
  double s = mi2 + mj2 + yy * qb2;
  double lam = kallen(Q2, s, mk2);
  double P = 0.5 * (Q2 - s - mk2);
  double bb = (mi2 - mj2 - (2.0 * z - 1.0) * s) * P / (0.5 * lam);
  double aa = z - bb * mk2 / P;
  double k2 = aa * aa * s + bb * bb * mk2 + 2.0 * aa * bb * P - mi2;
  *y = yy;
  *sij = s;
  *a = aa;
  *b = bb;
  *kt2 = k2;
  return yy < 1.0 && lam > 0.0 && k2 >= 0.0;
}

/* True over trial density of a massive kernel at (t, z), without the
   alpha_s ratio: F (1 - y) t/(t + (1-z)^2 mi^2 + z^2 mj^2) V / (F_over O),
   where t/(t + ...) turns dy/y into dt/t at fixed z and F_over = max(F, 1)
   scales the overestimate; 0 where the kernel is not positive (inside the
   dead cone); -1 outside the phase space. */
double or_massive_ratio(int K, double t, double z, double Q2, double mi, double mj, double mk,
                        double fover) {
  double y, sij, a, b, k2;
  if (!massive_vars(Q2, mi, mj, mk, t, z, &y, &sij, &a, &b, &k2)) return -1.0;
  double qb2 = Q2 - mi * mi - mj * mj - mk * mk;
  double v = or_kernel_value_massive(K, z, y, mi, qb2, sij);
  if (!(v > 0.0)) return 0.0;
  double f = or_massive_flux(Q2, mi, mj, mk, K < 10 ? mi : 0.0);
  double cz = (1.0 - z) * (1.0 - z) * mi * mi + z * z * mj * mj;
  return f * (1.0 - y) * (t / (t + cz)) * v / (fover * or_kernel_over(K, z));
}

/* transverse unit vectors orthogonal to two momenta, as in the massless map */
static void transverse_basis(const double *pa, const double *pb, double n1[4], double n2[4]) {
  double d[3];
  for (int m = 0; m < 3; ++m) d[m] = pb[0] * pa[1 + m] - pa[0] * pb[1 + m];
  int ax = 0;
  if (fabs(d[1]) < fabs(d[ax])) ax = 1;
  if (fabs(d[2]) < fabs(d[ax])) ax = 2;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  r[1 + ax] = 1.0;
  eps4(pa, pb, r, n1);
  double l1 = sqrt(-mdot(n1, n1));
  for (int m = 0; m < 4; ++m) n1[m] /= l1;
  eps4(pa, pb, n1, n2);
  double l2 = sqrt(-mdot(n2, n2));
  for (int m = 0; m < 4; ++m) n2[m] /= l2;
}

void or_split_kinematics_massive(const double pij[4], const double pk[4], double mi, double mj,
                                 double mk, double mij, double t, double z, double phi,
                                 double out_i[4], double out_j[4], double out_k[4]) {
  double Q[4];
  for (int m = 0; m < 4; ++m) Q[m] = pij[m] + pk[m];
  double Q2 = mdot(Q, Q);
  double y, s, a, b, k2;
  massive_vars(Q2, mi, mj, mk, t, z, &y, &s, &a, &b, &k2);
  double lam = kallen(Q2, s, mk * mk);
  double scale = sqrt((lam > 0.0 ? lam : 0.0) / kallen(Q2, mij * mij, mk * mk));
  double along = mdot(Q, pk) / Q2, shift = (Q2 + mk * mk - s) / (2.0 * Q2);
  double n1[4], n2[4];
  transverse_basis(pij, pk, n1, n2);
  double kt = sqrt(k2 > 0.0 ? k2 : 0.0), c1 = cos(phi), s1 = sin(phi);
  for (int m = 0; m < 4; ++m) {
    double newk = scale * (pk[m] - along * Q[m]) + shift * Q[m];
    double newij = Q[m] - newk;
    out_k[m] = newk;
    out_i[m] = a * newij + b * newk + kt * (c1 * n1[m] + s1 * n2[m]);
    out_j[m] = newij - out_i[m];
  }
}

/* ---------------------------------------------------------------------- */
/* Shower (Appendix A)                                                     */
/* ---------------------------------------------------------------------- */
/* leading-colour connection: i's colour flows into k's anticolour, or i's
   anticolour into k's colour */
static int colour_connected(int ci, int ai, int ck, int ak) {
  return (ci != 0 && ci == ak) || (ai != 0 && ai == ck);
}

static uint64_t fnv_step(uint64_t h, uint32_t v) {
  h ^= (uint64_t)v;
  h *= 0x100000001b3ull;
  return h;
}

int or_shower(uint64_t seed, uint64_t event, double ecm, double tcut, int cap,
              int max_cycles, double t_over, const double *mass, int max_emit, int *n,
              double *p, int *pid,
              int *col, int *acol, int *cycles, uint64_t *emit_hash, int *n_emit,
              double *weight, double *emit_log, int max_log, uint64_t *work) {
  int np = *n;
  double t = ecm * ecm;              /* evolution starts at s */
  /* alpha_s of the trial density: alpha_s(t_C) bounds alpha_s(t) at every
     t >= t_C.  A larger scale t_over makes the trial density fall below the
     true one for t < t_over; the weighted veto below corrects for that. */
  double asmax = or_alpha_s(t_over > 0.0 ? t_over : tcut);
  double wgt = 1.0;
  int next_col = 1;
  for (int i = 0; i < np; ++i) {
    if (col[i] >= next_col) next_col = col[i] + 1;
    if (acol[i] >= next_col) next_col = acol[i] + 1;
  }
  int status = OR_RUNNING;
  uint32_t cycle = 0;
  int nemit = 0;
  uint64_t hash = 0xcbf29ce484222325ull;

  while (status == OR_RUNNING) {
    /* --- tail cut: an event still above the cutoff after max_cycles veto
       cycles is given up and vetoed ----------------------------------- */
    if (max_cycles > 0 && cycle >= (uint32_t)max_cycles) {
      status = OR_TRUNCATED;
      break;
    }
    /* --- SelectWinnerEmission: every splitter, spectator, kernel ------- */
    double winner_t = tcut;
    int wi = -1, wk = -1, wK = -1;
    double wq2 = 0.0, wzm = 0.0, wzp = 0.0;
    /* the winner's (p~ij + p~k)^2, masses and overestimate factor, and
       whether its kernel takes the massive formulas */
    double wQ2 = 0.0, wmi = 0.0, wmj = 0.0, wmk = 0.0, wfo = 1.0;
    int wmassive = 0;
    for (int i = 0; i < np; ++i) {
      for (int k = 0; k < np; ++k) {
        if (i == k) continue;
        if (!colour_connected(col[i], acol[i], col[k], acol[k])) continue;
        if (work) work[1]++;
        double q2 = 2.0 * mdot(&p[4 * i], &p[4 * k]);
        double msplit = flavour_mass(mass, pid[i]), mk = flavour_mass(mass, pid[k]);
        double Q2 = q2 + msplit * msplit + mk * mk; /* (p~ij + p~k)^2 */
        int kl[6];
        int nk = or_kernel_list(pid[i], kl);
        int active = 0;
        for (int j = 0; j < nk; ++j) {
          int K = kl[j];
          double mi, mj, zm, zp, fo = 1.0;
          kernel_product_masses(K, mass, &mi, &mj);
          int massive = mi > 0.0 || mj > 0.0 || mk > 0.0;
          if (!massive) {
            if (!(q2 > 4.0 * tcut)) continue; /* no phase space above t_C */
            zp = 0.5 * (1.0 + sqrt(1.0 - 4.0 * tcut / q2));
            zm = 1.0 - zp;
          } else {
            if (!or_massive_limits(Q2, mi, mj, mk, tcut, &zm, &zp)) continue;
            double f = or_massive_flux(Q2, mi, mj, mk, K < 10 ? mi : 0.0);
            fo = f > 1.0 ? f : 1.0;
          }
          active = 1;
          double c = asmax / (2.0 * OR_PI) * or_kernel_integral(K, zm, zp);
          if (massive) c *= fo;
          uint32_t w[4];
          or_draw(seed, event, cycle, OR_P_TRIAL, trial_slot(i, k, j), w);
          double u = (j & 1) ? or_uniform(w[2], w[3]) : or_uniform(w[0], w[1]);
          double t_try = t * pow(u, 1.0 / c);
          if (work) work[3]++;
          if (t_try > winner_t) {
            winner_t = t_try;
            wi = i;
            wk = k;
            wK = K;
            wq2 = q2;
            wzm = zm;
            wzp = zp;
            wQ2 = Q2;
            wmi = mi;
            wmj = mj;
            wmk = mk;
            wfo = fo;
            wmassive = massive;
          }
        }
        if (active && work) work[2]++; /* an end with phase space above t_C */
      }
    }
    uint32_t this_cycle = cycle++;
    if (work) work[0]++;

    /* --- cutoff ------------------------------------------------------ */
    if (wi < 0) {
      t = tcut;
      status = OR_DONE;
      break;
    }
    t = winner_t; /* the winner's scale bounds every later trial */

    /* --- veto -------------------------------------------------------- */
    uint32_t a[4];
    or_draw(seed, event, this_cycle, OR_P_ACCEPT, 0, a);
    double uz = or_uniform(a[0], a[1]);
    double uv = or_uniform(a[2], a[3]);
    double z = or_kernel_zgen(wK, wzm, wzp, uz);
    double y, prob = 0.0;
    int inside; /* inside the true phase space at this t */
    if (!wmassive) {
      y = t / (wq2 * z * (1.0 - z));
      inside = y < 1.0;
      if (inside)
        prob = or_alpha_s(t) / asmax * or_kernel_value(wK, z, y) * (1.0 - y) /
               or_kernel_over(wK, z);
    } else {
      double qb2 = wQ2 - wmi * wmi - wmj * wmj - wmk * wmk;
      y = (t + (1.0 - z) * (1.0 - z) * wmi * wmi + z * z * wmj * wmj) / (qb2 * z * (1.0 - z));
      double r = or_massive_ratio(wK, t, z, wQ2, wmi, wmj, wmk, wfo);
      inside = r >= 0.0;
      prob = or_alpha_s(t) / asmax * r;
    }
    int accept = 0;
    if (inside) {
      if (work) work[5]++;
      if (prob > 1.0) {
        /* weighted veto where the true density exceeds the trial density:
           accept with probability e, weight the event by prob / e if
           accepted and (1 - prob) / (1 - e) if not; e = prob / (2 prob - 1)
           minimises the variance of that factor, which is then
           +-(2 prob - 1) */
        double e = prob / (2.0 * prob - 1.0);
        accept = uv < e;
        wgt *= accept ? 2.0 * prob - 1.0 : -(2.0 * prob - 1.0);
      } else {
        accept = uv < prob;
      }
    }
    if (!accept) continue;

    /* --- splitting --------------------------------------------------- */
    if (np == cap) {
      status = OR_OVERFLOW;
      break;
    }
    uint32_t sdraw[4];
    or_draw(seed, event, this_cycle, OR_P_SPLIT, 0, sdraw);
    double phi = 2.0 * OR_PI * or_uniform(sdraw[0], sdraw[1]);
    double ni[4], nj[4], nk4[4];
    if (wmassive)
      or_split_kinematics_massive(&p[4 * wi], &p[4 * wk], wmi, wmj, wmk, wK < 10 ? wmi : 0.0, t, z,
                                  phi, ni, nj, nk4);
    else
      or_split_kinematics(&p[4 * wi], &p[4 * wk], t, z, phi, ni, nj, nk4);
    for (int m = 0; m < 4; ++m) {
      p[4 * wi + m] = ni[m];
      p[4 * wk + m] = nk4[m];
      p[4 * np + m] = nj[m];
    }
    /* colours and flavours; the colour side takes precedence */
    int via_colour = (col[wi] != 0 && col[wi] == acol[wk]);
    int jpid, jcol, jacol;
    if (wK <= 10) { /* gluon emission: j sits between i and k */
      int m = next_col++;
      jpid = 21;
      if (via_colour) {
        jcol = col[wi];
        jacol = m;
        col[wi] = m;
      } else {
        jcol = m;
        jacol = acol[wi];
        acol[wi] = m;
      }
    } else { /* g -> f fbar: j is the parton colour-adjacent to k */
      int f = wK - 10;
      if (via_colour) {
        jpid = f;
        jcol = col[wi];
        jacol = 0;
        pid[wi] = -f;
        col[wi] = 0;
      } else {
        jpid = -f;
        jcol = 0;
        jacol = acol[wi];
        pid[wi] = f;
        acol[wi] = 0;
      }
    }
    pid[np] = jpid;
    col[np] = jcol;
    acol[np] = jacol;
    if (emit_log && nemit < max_log) {
      double *e = &emit_log[OR_NLOG * nemit];
      e[0] = t;
      e[1] = z;
      e[2] = y;
      e[3] = (double)wK;
      e[4] = (double)wi;
      e[5] = (double)wk;
      e[6] = phi;
    }
    hash = fnv_step(hash, (uint32_t)wK);
    hash = fnv_step(hash, (uint32_t)wi);
    hash = fnv_step(hash, (uint32_t)wk);
    ++np;
    ++nemit;
    if (work) work[4]++;
    if (max_emit >= 0 && nemit >= max_emit) status = OR_STOPPED;
  }
  *n = np;
  if (cycles) *cycles = (int)cycle;
  if (emit_hash) *emit_hash = hash;
  if (n_emit) *n_emit = nemit;
  if (weight) *weight = wgt;
  return status;
}

/* ---------------------------------------------------------------------- */
/* Observables (Section 3.1)                                               */
/* ---------------------------------------------------------------------- */
static double norm3(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* Exact thrust T = max_n sum|p.n| / sum|p|.  The optimal hemisphere split is
   a plane through the origin; turning it until it touches two momenta
   shows that it is one of the planes spanned by a pair (i, j), with i and j
   themselves on either side: N(N-1)/2 planes x N dot products, plus the
   four sign choices of i and j.  First maximum wins. */
double or_thrust(int n, const double *p, double axis[3]) {
  double sum = 0.0;
  for (int a = 0; a < n; ++a) sum += norm3(&p[4 * a + 1]);
  double best = -1.0, bv[3] = {0.0, 0.0, 1.0};
  if (n < 3) {
    /* all 2^n sign vectors directly */
    for (int mask = 0; mask < (1 << n); ++mask) {
      double v[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < n; ++a) {
        double sg = (mask >> a & 1) ? -1.0 : 1.0;
        for (int m = 0; m < 3; ++m) v[m] += sg * p[4 * a + 1 + m];
      }
      double m2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      if (m2 > best) {
        best = m2;
        bv[0] = v[0];
        bv[1] = v[1];
        bv[2] = v[2];
      }
    }
  } else {
    static const double sgn[4][2] = {{1.0, 1.0}, {1.0, -1.0}, {-1.0, 1.0}, {-1.0, -1.0}};
    for (int i = 0; i < n; ++i) {
      for (int j = i + 1; j < n; ++j) {
        const double *pi = &p[4 * i + 1], *pj = &p[4 * j + 1];
        double nrm[3] = {pi[1] * pj[2] - pi[2] * pj[1], pi[2] * pj[0] - pi[0] * pj[2],
                         pi[0] * pj[1] - pi[1] * pj[0]};
        double v[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < n; ++k) {
          if (k == i || k == j) continue;
          const double *pk = &p[4 * k + 1];
          double d = pk[0] * nrm[0] + pk[1] * nrm[1] + pk[2] * nrm[2];
          double sg = d > 0.0 ? 1.0 : -1.0;
          for (int m = 0; m < 3; ++m) v[m] += sg * pk[m];
        }
        for (int c = 0; c < 4; ++c) {
          double w[3];
          for (int m = 0; m < 3; ++m) w[m] = v[m] + sgn[c][0] * pi[m] + sgn[c][1] * pj[m];
          double m2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
          if (m2 > best) {
            best = m2;
            bv[0] = w[0];
            bv[1] = w[1];
            bv[2] = w[2];
          }
        }
      }
    }
  }
  double len = sqrt(best);
  if (axis) {
    if (len > 0.0) {
      for (int m = 0; m < 3; ++m) axis[m] = bv[m] / len;
    } else {
      axis[0] = 0.0;
      axis[1] = 0.0;
      axis[2] = 1.0;
    }
  }
  return sum > 0.0 ? len / sum : 0.0;
}

/* Durham (k_T) clustering with E-scheme recombination:
   y_ab = 2 min(E_a^2, E_b^2) (1 - cos theta_ab) / s, written with
   1 - cos theta = |u_a - u_b|^2 / 2 for unit vectors u.  y_{n,n+1} is the
   smallest y at the step from n+1 to n pseudo-jets (0 if the event never
   had n+1 partons).  Ties go to the lowest (a, b). */
void or_durham(int n, const double *p, double s, double *y23, double *y34) {
  enum { MAXJ = 1024 };
  static double jet[MAXJ][4];
  int m = n < MAXJ ? n : MAXJ;
  for (int a = 0; a < m; ++a)
    for (int c = 0; c < 4; ++c) jet[a][c] = p[4 * a + c];
  *y23 = 0.0;
  *y34 = 0.0;
  while (m > 2) {
    double ymin = 0.0;
    int ba = -1, bb = -1;
    for (int a = 0; a < m; ++a) {
      double la = norm3(&jet[a][1]);
      for (int b = a + 1; b < m; ++b) {
        double lb = norm3(&jet[b][1]);
        double d2 = 0.0;
        for (int c = 1; c < 4; ++c) {
          double dc = jet[a][c] / la - jet[b][c] / lb;
          d2 += dc * dc;
        }
        double emin = jet[a][0] < jet[b][0] ? jet[a][0] : jet[b][0];
        double y = emin * emin * d2 / s;
        if (ba < 0 || y < ymin) {
          ymin = y;
          ba = a;
          bb = b;
        }
      }
    }
    if (m == 4) *y34 = ymin;
    if (m == 3) *y23 = ymin;
    for (int c = 0; c < 4; ++c) jet[ba][c] += jet[bb][c];
    for (int a = bb; a + 1 < m; ++a)
      for (int c = 0; c < 4; ++c) jet[a][c] = jet[a + 1][c];
    --m;
  }
}

/* C = 3 (l1 l2 + l2 l3 + l3 l1) of the linearised momentum tensor
     = (3/2) [ (sum|p|)^2 - sum_{a,b} (p_a.p_b)^2 / (|p_a||p_b|) ] / (sum|p|)^2 */
double or_cparameter(int n, const double *p) {
  double sum = 0.0, dbl = 0.0;
  for (int a = 0; a < n; ++a) sum += norm3(&p[4 * a + 1]);
  for (int a = 0; a < n; ++a) {
    double la = norm3(&p[4 * a + 1]);
    for (int b = 0; b < n; ++b) {
      double lb = norm3(&p[4 * b + 1]);
      double d = p[4 * a + 1] * p[4 * b + 1] + p[4 * a + 2] * p[4 * b + 2] + p[4 * a + 3] * p[4 * b + 3];
      dbl += d * d / (la * lb);
    }
  }
  double c = 1.5 * (sum * sum - dbl) / (sum * sum);
  return c > 0.0 ? c : 0.0;
}

/* hemispheres split by the plane normal to the thrust axis (p.n >= 0 is the
   "+" side): heavy-jet mass rho_H = max(M+^2, M-^2)/s; broadenings
   B_pm = sum_pm |p x n| / (2 sum|p|), B_T = B+ + B-, B_W = max. */
void or_hemispheres(int n, const double *p, const double axis[3], double s,
                    double *rho_h, double *b_t, double *b_w) {
  double hp[4] = {0, 0, 0, 0}, hm[4] = {0, 0, 0, 0};
  double bp = 0.0, bm = 0.0, sum = 0.0;
  for (int a = 0; a < n; ++a) {
    const double *q = &p[4 * a];
    sum += norm3(&q[1]);
    double d = q[1] * axis[0] + q[2] * axis[1] + q[3] * axis[2];
    double cr[3] = {q[2] * axis[2] - q[3] * axis[1], q[3] * axis[0] - q[1] * axis[2],
                    q[1] * axis[1] - q[2] * axis[0]};
    double kt = norm3(cr);
    if (d >= 0.0) {
      for (int c = 0; c < 4; ++c) hp[c] += q[c];
      bp += kt;
    } else {
      for (int c = 0; c < 4; ++c) hm[c] += q[c];
      bm += kt;
    }
  }
  double mp = mdot(hp, hp), mm = mdot(hm, hm);
  double rho = (mp > mm ? mp : mm) / s;
  *rho_h = rho > 0.0 ? rho : 0.0;
  bp /= 2.0 * sum;
  bm /= 2.0 * sum;
  *b_t = bp + bm;
  *b_w = bp > bm ? bp : bm;
}

/* Validate (Table 1, "Validate Events"; the criterion is not printed, this is
   the reading taken): every component finite; the total four-momentum equal
   to (ecm, 0, 0, 0) within 1e-10 ecm per component; every parton on its mass
   shell (massless unless the table gives its flavour a mass) within
   1e-10 s.  Finiteness is checked first, so an event with a non-finite
   component is NONFINITE whatever else is wrong with it.  pid may be NULL
   when mass is NULL (every parton massless). */
int or_validate_massive(int n, const double *p, const int *pid, double ecm, const double *mass) {
  double tot[4] = {0, 0, 0, 0};
  for (int a = 0; a < 4 * n; ++a)
    if (!isfinite(p[a])) return OR_NONFINITE;
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < 4; ++c) tot[c] += p[4 * a + c];
  double tol = 1e-10 * ecm;
  if (fabs(tot[0] - ecm) > tol || fabs(tot[1]) > tol || fabs(tot[2]) > tol || fabs(tot[3]) > tol)
    return OR_CONSERVATION;
  for (int a = 0; a < n; ++a) {
    double m = mass ? flavour_mass(mass, pid[a]) : 0.0;
    if (fabs(mdot(&p[4 * a], &p[4 * a]) - m * m) > 1e-10 * ecm * ecm) return OR_CONSERVATION;
  }
  return OR_DONE;
}

int or_validate(int n, const double *p, double ecm) { return or_validate_massive(n, p, NULL, ecm, NULL); }

/* ---------------------------------------------------------------------- */
/* Initial-state shower (the step to hadron colliders that the conclusions */
/* name: an extra step to evaluate PDFs).  No PDF set is available here, so */
/* a closed-form density stands in for one: every light quark and          */
/* antiquark flavour has f(x) = (63/128) x^(-1/2) (1 - x)^3 and the gluon   */
/* g(x) = 3 x^(-1) (1 - x)^5, independent of the scale; the ten quark and   */
/* antiquark densities carry half the momentum and the gluon the other      */
/* half (momentum sum rule).                                               */
/*                                                                          */
/* Hard process: q qbar -> colour singlet V of mass Q (Drell-Yan) at hadron */
/* centre-of-mass energy sqrt(S): flavour uniform over d, u, s, c, b, the   */
/* quark from either beam, rapidity y of V uniform in |y| < ln(sqrt(S)/Q),  */
/* x_A = sqrt(tau) e^y, x_B = sqrt(tau) e^-y, tau = Q^2/S; weight (arbitrary */
/* units: the rapidity density of the parton luminosity for a unit partonic */
/* cross-section) 10 (2 Y) tau f(x_A) f(x_B).                               */
/*                                                                          */
/* Shower: each incoming line evolves backwards from t = Q^2 with the       */
/* density (alpha_s(t)/2 pi) (dt/t) (dz/z) P_qq(z) f(x/z)/f(x), P_qq(z) =    */
/* C_F (1 + z^2)/(1 - z), x the line's current momentum fraction; the other */
/* incoming parton is the spectator; the two lines' trials compete (largest */
/* t wins) as the dipole ends of the final-state shower do.  An emission at */
/* (t, z) uses the Catani-Seymour initial-initial map: the emitter becomes  */
/* p_a/z (fraction x/z), the gluon p_j = (1 - z - v) p_a/z + v p_b + kT with */
/* kT^2 = -t and v(1 - z - v) = t z / s~ (s~ = 2 p_a.p_b before the emission, */
/* smaller root), and every final-state momentum is carried by the Lorentz  */
/* transformation that takes the old final-state total to the new one.  The */
/* emitted gluons do not radiate (this branch evolves the incoming lines    */
/* only).  The overestimate 2 C_F x^(-1/2)/(1 - z) bounds the density      */
/* (z^(-1/2) ((1 - x/z)/(1 - x))^3 <= x^(-1/2) for x <= z <= 1).            */
/* ---------------------------------------------------------------------- */
double or_pdf_q(double x) { return x > 0.0 && x < 1.0 ? (63.0 / 128.0) / sqrt(x) * pow(1.0 - x, 3.0) : 0.0; }
double or_pdf_g(double x) { return x > 0.0 && x < 1.0 ? 3.0 / x * pow(1.0 - x, 5.0) : 0.0; }

/* z range of the overestimate for a line at fraction x in a dipole of
   s~ = 2 p_a.p_b: from x (the parent's fraction stays below 1) up to where
   kT^2 = t_C needs (1 - z)^2 = 4 t_C z / s~.  Returns 0 without phase space. */
int or_isr_zlimits(double x, double st, double tcut, double *zlo, double *zhi) {
  double a = tcut / st;
  double zmax = 1.0 + 2.0 * a - 2.0 * sqrt(a + a * a);
  if (!(zmax > x)) return 0;
  *zlo = x;
  *zhi = zmax;
  return 1;
}

/* true over trial density of an emission at (t, z) of a line at fraction x
   (without alpha_s): P_qq(z)/z f(x/z)/f(x) / O(z); -1 outside the phase
   space (no real v at this t) */
double or_isr_ratio(double t, double z, double x, double st) {
  double disc = (1.0 - z) * (1.0 - z) - 4.0 * t * z / st;
  if (!(disc >= 0.0) || !(z > x)) return -1.0;
  double p = CF * (1.0 + z * z) / (1.0 - z);
  double dens = p / z * or_pdf_q(x / z) / or_pdf_q(x);
  double over = 2.0 * CF / sqrt(x) / (1.0 - z);
  return dens / over;
}

/* Catani-Seymour initial-initial map of an emission at (t, z) off the
   incoming pa with spectator pb: new incoming pa/z, the gluon, and the
   transformation of the final state (applied to k[0..nk-1] in place). */
static void isr_map(double *pa, const double *pb, double t, double z, double phi, double *pj, double *k, int nk) {
  double st = 2.0 * mdot(pa, pb);
  double v = 0.5 * ((1.0 - z) - sqrt((1.0 - z) * (1.0 - z) - 4.0 * t * z / st));
  double Kt[4], K[4], na[4];
  for (int m = 0; m < 4; ++m) {
    Kt[m] = pa[m] + pb[m];
    na[m] = pa[m] / z;
  }
  /* transverse basis: both incoming momenta are along the beam axis */
  double kt = sqrt(t);
  double kp[4] = {0.0, kt * cos(phi), kt * sin(phi), 0.0};
  for (int m = 0; m < 4; ++m) {
    pj[m] = (1.0 - z - v) * na[m] + v * pb[m] + kp[m];
    K[m] = na[m] + pb[m] - pj[m];
  }
  /* Lambda = g - 2 (K + Kt)(K + Kt)/(K + Kt)^2 + 2 K Kt / Kt^2 */
  double S[4];
  for (int m = 0; m < 4; ++m) S[m] = K[m] + Kt[m];
  double s2 = mdot(S, S), kt2 = mdot(Kt, Kt);
  for (int q = 0; q < nk; ++q) {
    double *x = &k[4 * q];
    double sx = mdot(S, x), ktx = mdot(Kt, x);
    double y[4];
    for (int m = 0; m < 4; ++m) y[m] = x[m] - 2.0 * S[m] * sx / s2 + 2.0 * K[m] * ktx / kt2;
    for (int m = 0; m < 4; ++m) x[m] = y[m];
  }
  for (int m = 0; m < 4; ++m) pa[m] = na[m];
}

/* Start of a Drell-Yan event (above): partons [from beam A, from beam B, V]. */
void or_isr_me(uint64_t seed, uint64_t event, double sqrt_s_had, double q, int *flavour, int *quark_from_a,
               double *rapidity, double *weight, double *xa, double *xb, double p[12]) {
  uint32_t w[4];
  or_draw(seed, event, 0, OR_P_ME, 0, w);
  int f = 1 + (int)(((uint64_t)w[0] * 5u) >> 32);
  int qa = (w[1] & 1u) == 0;
  double Y = log(sqrt_s_had / q);
  double y = -Y + 2.0 * Y * or_uniform(w[2], w[3]);
  double tau = q * q / (sqrt_s_had * sqrt_s_had);
  double a = sqrt(tau) * exp(y), b = sqrt(tau) * exp(-y);
  double e = 0.5 * sqrt_s_had;
  double pa[4] = {a * e, 0.0, 0.0, a * e}, pb[4] = {b * e, 0.0, 0.0, -b * e};
  for (int m = 0; m < 4; ++m) {
    p[m] = pa[m];
    p[4 + m] = pb[m];
    p[8 + m] = pa[m] + pb[m];
  }
  *flavour = f;
  *quark_from_a = qa;
  *rapidity = y;
  *xa = a;
  *xb = b;
  *weight = 10.0 * (2.0 * Y) * tau * or_pdf_q(a) * or_pdf_q(b);
}

/* Shower of one Drell-Yan event whose n partons (incoming a, incoming b,
   then the final state) are in p/pid/col/acol (length cap), with the
   current fractions *xa, *xb; updated in place.  Kernel id 16 marks an
   initial-state q -> q g in the emission hash.  Returns the status. */
int or_isr_shower(uint64_t seed, uint64_t event, double q, double tcut, int cap, int max_emit, int *n,
                  double *p, int *pid, int *col, int *acol, double *xa, double *xb, int *cycles,
                  uint64_t *emit_hash, int *n_emit, double *emit_log, int max_log, uint64_t *work) {
  int np = *n;
  double t = q * q;
  double asmax = or_alpha_s(tcut);
  int next_col = 1;
  for (int i = 0; i < np; ++i) {
    if (col[i] >= next_col) next_col = col[i] + 1;
    if (acol[i] >= next_col) next_col = acol[i] + 1;
  }
  double x[2] = {*xa, *xb};
  int status = OR_RUNNING;
  uint32_t cycle = 0;
  int nemit = 0;
  uint64_t hash = 0xcbf29ce484222325ull;
  while (status == OR_RUNNING) {
    double st = 2.0 * mdot(&p[0], &p[4]);
    double winner_t = tcut;
    int wl = -1;
    double wzlo = 0.0, wzhi = 0.0;
    for (int l = 0; l < 2; ++l) { /* line l (slot l) with spectator slot 1 - l */
      if (work) work[1]++;
      double zlo, zhi;
      if (!or_isr_zlimits(x[l], st, tcut, &zlo, &zhi)) continue;
      if (work) work[2]++;
      double c = asmax / (2.0 * OR_PI) * 2.0 * CF / sqrt(x[l]) * log((1.0 - zlo) / (1.0 - zhi));
      uint32_t w[4];
      or_draw(seed, event, cycle, OR_P_TRIAL, trial_slot(l, 1 - l, 0), w);
      double t_try = t * pow(or_uniform(w[0], w[1]), 1.0 / c);
      if (work) work[3]++;
      if (t_try > winner_t) {
        winner_t = t_try;
        wl = l;
        wzlo = zlo;
        wzhi = zhi;
      }
    }
    uint32_t this_cycle = cycle++;
    if (work) work[0]++;
    if (wl < 0) {
      status = OR_DONE;
      break;
    }
    t = winner_t;
    uint32_t a4[4];
    or_draw(seed, event, this_cycle, OR_P_ACCEPT, 0, a4);
    double z = 1.0 - (1.0 - wzlo) * pow((1.0 - wzhi) / (1.0 - wzlo), or_uniform(a4[0], a4[1]));
    double r = or_isr_ratio(t, z, x[wl], st);
    if (r < 0.0) continue;
    if (work) work[5]++;
    if (!(or_uniform(a4[2], a4[3]) < or_alpha_s(t) / asmax * r)) continue;
    if (np == cap) {
      status = OR_OVERFLOW;
      break;
    }
    uint32_t sd[4];
    or_draw(seed, event, this_cycle, OR_P_SPLIT, 0, sd);
    double phi = 2.0 * OR_PI * or_uniform(sd[0], sd[1]);
    double pj[4];
    isr_map(&p[4 * wl], &p[4 * (1 - wl)], t, z, phi, pj, &p[8], np - 2);
    for (int m = 0; m < 4; ++m) p[4 * np + m] = pj[m];
    x[wl] /= z;
    /* the gluon goes onto the emitter's colour line */
    int m = next_col++;
    pid[np] = 21;
    if (col[wl] != 0) {
      col[np] = col[wl];
      acol[np] = m;
      col[wl] = m;
    } else {
      col[np] = m;
      acol[np] = acol[wl];
      acol[wl] = m;
    }
    if (emit_log && nemit < max_log) {
      double *e = &emit_log[OR_NLOG * nemit];
      e[0] = t;
      e[1] = z;
      e[2] = x[wl];
      e[3] = 16.0;
      e[4] = (double)wl;
      e[5] = (double)(1 - wl);
      e[6] = phi;
    }
    hash = fnv_step(hash, 16u);
    hash = fnv_step(hash, (uint32_t)wl);
    hash = fnv_step(hash, (uint32_t)(1 - wl));
    ++np;
    ++nemit;
    if (work) work[4]++;
    if (max_emit >= 0 && nemit >= max_emit) status = OR_STOPPED;
  }
  *n = np;
  *xa = x[0];
  *xb = x[1];
  if (cycles) *cycles = (int)cycle;
  if (emit_hash) *emit_hash = hash;
  if (n_emit) *n_emit = nemit;
  return status;
}

/* Validation of a Drell-Yan event: finite; the final state (slots 2..n-1)
   carries the incoming total to 1e-10 of its energy per component; V on its
   mass shell Q and the others massless within 1e-10 of the incoming s. */
int or_isr_validate(int n, const double *p, double q) {
  for (int a = 0; a < 4 * n; ++a) {
    if (isfinite(p[a])) continue;
    return OR_NONFINITE;
  }
  double in[4], out[4] = {0, 0, 0, 0};
  for (int m = 0; m < 4; ++m) in[m] = p[m] + p[4 + m];
  for (int a = 2; a < n; ++a)
    for (int m = 0; m < 4; ++m) out[m] += p[4 * a + m];
  double tol = 1e-10 * in[0], s = mdot(in, in);
  for (int m = 0; m < 4; ++m)
    if (fabs(out[m] - in[m]) > tol) return OR_CONSERVATION;
  for (int a = 0; a < n; ++a) {
    double m2 = a == 2 ? q * q : 0.0;
    if (fabs(mdot(&p[4 * a], &p[4 * a]) - m2) > 1e-10 * s) return OR_CONSERVATION;
  }
  return OR_DONE;
}

/* Histogram ranges of the Drell-Yan branch: log10(p_T,V / GeV), y_V,
   emitted gluons, log10(p_T / GeV) of the hardest gluon; the other four
   rows are unused. */
void or_isr_hist_ranges(double lo[OR_NOBS], double hi[OR_NOBS]) {
  static const double L[OR_NOBS] = {-1.0, -5.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0};
  static const double H[OR_NOBS] = {3.0, 5.0, 50.0, 3.0, 1.0, 1.0, 1.0, 1.0};
  for (int h = 0; h < OR_NOBS; ++h) {
    lo[h] = L[h];
    hi[h] = H[h];
  }
}

static void hist_fill(double *hist, int h, double x, double w, const double *lo, const double *hi);

/* Whole Drell-Yan pipeline over events first .. first+n_events-1: start,
   shower, validation, observables (p_T,V, y_V, gluons, hardest gluon p_T),
   histograms.  sum_d per event: w, y_V, p_T,V, x_A, x_B, hardest gluon p_T,
   then 0; sum_i as or_generate (flavour = +f for the quark from beam A, -f
   from beam B). */
int or_isr_generate(uint64_t seed, uint64_t first, uint64_t n_events, double sqrt_s_had, double q, double tcut,
                    int cap, double *sum_d, int32_t *sum_i, uint64_t *sum_hash, double *hist, int32_t *rec_n,
                    double *rec_p, int32_t *rec_pid, int32_t *rec_col, int32_t *rec_acol, uint64_t *work) {
  enum { MAXCAP = 1024 };
  if (cap < 3 || cap > MAXCAP || !(sqrt_s_had > q) || !(q > 0.0)) return -1;
  static double p[4 * MAXCAP];
  static int pid[MAXCAP], col[MAXCAP], acol[MAXCAP];
  double lo[OR_NOBS], hi[OR_NOBS];
  or_isr_hist_ranges(lo, hi);
  for (uint64_t e = 0; e < n_events; ++e) {
    uint64_t ev = first + e;
    int f, qa;
    double y, w, xa, xb;
    or_isr_me(seed, ev, sqrt_s_had, q, &f, &qa, &y, &w, &xa, &xb, p);
    pid[0] = qa ? f : -f;
    pid[1] = qa ? -f : f;
    pid[2] = 23;
    col[0] = qa ? 1 : 0;
    acol[0] = qa ? 0 : 1;
    col[1] = qa ? 0 : 1;
    acol[1] = qa ? 1 : 0;
    col[2] = acol[2] = 0;
    int n = 3, cycles = 0, nemit = 0;
    uint64_t hash = 0;
    uint64_t ew[OR_NWORK] = {0, 0, 0, 0, 0, 0};
    int status = or_isr_shower(seed, ev, q, tcut, cap, -1, &n, p, pid, col, acol, &xa, &xb, &cycles, &hash, &nemit,
                               NULL, 0, ew);
    if (work)
      for (int k = 0; k < OR_NWORK; ++k) work[k] += ew[k];
    if (status == OR_DONE) status = or_isr_validate(n, p, q);
    double ptv = sqrt(p[9] * p[9] + p[10] * p[10]);
    double yv = 0.5 * log((p[8] + p[11]) / (p[8] - p[11]));
    double ptg = 0.0;
    for (int a = 3; a < n; ++a) {
      double pt = sqrt(p[4 * a + 1] * p[4 * a + 1] + p[4 * a + 2] * p[4 * a + 2]);
      if (pt > ptg) ptg = pt;
    }
    if (status == OR_DONE && hist) {
      hist_fill(hist, 0, ptv > 0.0 ? log10(ptv) : -INFINITY, w, lo, hi);
      hist_fill(hist, 1, yv, w, lo, hi);
      hist_fill(hist, 2, (double)nemit, w, lo, hi);
      hist_fill(hist, 3, ptg > 0.0 ? log10(ptg) : -INFINITY, w, lo, hi);
    }
    if (sum_d) {
      double *d = &sum_d[OR_NSUM_D * e];
      for (int k = 0; k < OR_NSUM_D; ++k) d[k] = 0.0;
      d[0] = w;
      d[1] = yv;
      d[2] = ptv;
      d[3] = xa;
      d[4] = xb;
      d[5] = ptg;
    }
    if (sum_i) {
      int32_t *si = &sum_i[OR_NSUM_I * e];
      si[0] = n;
      si[1] = status;
      si[2] = cycles;
      si[3] = nemit;
      si[4] = qa ? f : -f;
      si[5] = (int32_t)ew[3];
      si[6] = (int32_t)ew[2];
    }
    if (sum_hash) sum_hash[e] = hash;
    if (rec_n) rec_n[e] = n;
    if (rec_p)
      for (int a = 0; a < 4 * n; ++a) rec_p[(size_t)4 * cap * e + a] = p[a];
    for (int a = 0; a < n; ++a) {
      if (rec_pid) rec_pid[(size_t)cap * e + a] = pid[a];
      if (rec_col) rec_col[(size_t)cap * e + a] = col[a];
      if (rec_acol) rec_acol[(size_t)cap * e + a] = acol[a];
    }
  }
  return 0;
}

/* obs = {y23, y34, tau = 1 - T, C, rho_H, B_T, B_W} */
void or_observables(int n, const double *p, double ecm, double obs[7]) {
  double s = ecm * ecm;
  double axis[3];
  double thrust = or_thrust(n, p, axis);
  or_durham(n, p, s, &obs[0], &obs[1]);
  double tau = 1.0 - thrust;
  obs[2] = tau > 0.0 ? tau : 0.0;
  obs[3] = or_cparameter(n, p);
  or_hemispheres(n, p, axis, s, &obs[4], &obs[5], &obs[6]);
}

/* histogram ranges: log10 y23, log10 y34, tau, C, rho_H, B_T, B_W, cos(theta) */
void or_hist_ranges(double lo[OR_NOBS], double hi[OR_NOBS]) {
  static const double L[OR_NOBS] = {-4.3, -4.3, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0};
  static const double H[OR_NOBS] = {-0.3, -0.3, 0.5, 1.0, 0.5, 0.5, 0.35, 1.0};
  for (int h = 0; h < OR_NOBS; ++h) {
    lo[h] = L[h];
    hi[h] = H[h];
  }
}

static void hist_fill(double *hist, int h, double x, double w, const double *lo, const double *hi) {
  int b;
  if (x != x) {
    b = OR_NBINS + 1;
  } else if (x < lo[h]) {
    b = 0;
  } else if (x >= hi[h]) {
    b = OR_NBINS + 1;
  } else {
    b = 1 + (int)((x - lo[h]) / (hi[h] - lo[h]) * OR_NBINS);
    if (b > OR_NBINS) b = OR_NBINS;
  }
  double *cell = &hist[3 * (OR_NHCOL * h + b)];
  cell[0] += w;
  cell[1] += w * w;
  cell[2] += 1.0;
}

int or_generate(uint64_t seed, uint64_t first, uint64_t n_events,
                const double *ecm, double ecm0, const double *tcut,
                double tcut0, int cap, int max_cycles, double t_over, const double *mass,
                double *sum_d, int32_t *sum_i,
                uint64_t *sum_hash, double *hist, int32_t *rec_n,
                double *rec_p, int32_t *rec_pid, int32_t *rec_col,
                int32_t *rec_acol, uint64_t *work) {
  enum { MAXCAP = 1024 };
  if (cap < 2 || cap > MAXCAP || max_cycles < 0 || t_over < 0.0) return -1;
  static double p[4 * MAXCAP];
  static int pid[MAXCAP], col[MAXCAP], acol[MAXCAP];
  double lo[OR_NOBS], hi[OR_NOBS];
  or_hist_ranges(lo, hi);
  for (uint64_t e = 0; e < n_events; ++e) {
    uint64_t ev = first + e;
    double E = ecm ? ecm[e] : ecm0;
    double tc = tcut ? tcut[e] : tcut0;
    int flavour;
    double cth, phi, w;
    or_me_event_massive(seed, ev, E, mass, &flavour, &cth, &phi, &w, p);
    pid[0] = flavour;
    col[0] = 1;
    acol[0] = 0;
    pid[1] = -flavour;
    col[1] = 0;
    acol[1] = 1;
    int n = 2, cycles = 0, nemit = 0;
    uint64_t hash = 0;
    uint64_t ew[OR_NWORK] = {0, 0, 0, 0, 0, 0};
    double wsh = 1.0;
    int status = or_shower(seed, ev, E, tc, cap, max_cycles, t_over, mass, -1, &n, p, pid, col, acol,
                           &cycles, &hash, &nemit, &wsh, NULL, 0, ew);
    w *= wsh; /* the event weight: matrix element times weighted veto */
    if (work)
      for (int k = 0; k < OR_NWORK; ++k) work[k] += ew[k];
    double obs[7] = {0, 0, 0, 0, 0, 0, 0};
    if (status == OR_DONE) status = mass ? or_validate_massive(n, p, pid, E, mass) : or_validate(n, p, E);
    if (status == OR_DONE) {
      or_observables(n, p, E, obs);
      if (hist) {
        hist_fill(hist, 0, obs[0] > 0.0 ? log10(obs[0]) : -INFINITY, w, lo, hi);
        hist_fill(hist, 1, obs[1] > 0.0 ? log10(obs[1]) : -INFINITY, w, lo, hi);
        for (int h = 2; h < 7; ++h) hist_fill(hist, h, obs[h], w, lo, hi);
        hist_fill(hist, 7, cth, w, lo, hi);
      }
    }
    if (sum_d) {
      double *d = &sum_d[OR_NSUM_D * e];
      d[0] = w;
      d[1] = cth;
      for (int h = 0; h < 7; ++h) d[2 + h] = obs[h];
      d[9] = phi;
    }
    if (sum_i) {
      int32_t *si = &sum_i[OR_NSUM_I * e];
      si[0] = n;
      si[1] = status;
      si[2] = cycles;
      si[3] = nemit;
      si[4] = flavour;
      si[5] = (int32_t)ew[3]; /* trial emissions */
      si[6] = (int32_t)ew[2]; /* dipole ends with phase space above t_C */
    }
    if (sum_hash) sum_hash[e] = hash;
    if (rec_n) rec_n[e] = n;
    if (rec_p) {
      for (int a = 0; a < 4 * n; ++a) rec_p[(size_t)4 * cap * e + a] = p[a];
    }
    for (int a = 0; a < n; ++a) {
      if (rec_pid) rec_pid[(size_t)cap * e + a] = pid[a];
      if (rec_col) rec_col[(size_t)cap * e + a] = col[a];
      if (rec_acol) rec_acol[(size_t)cap * e + a] = acol[a];
    }
  }
  return 0;
}
