/*
 * vsh_oracle.h -- serial FP64 reference implementation ("the oracle") of the
 * parallel Sudakov-veto parton shower of Seymour & Sule, "An Algorithm to
 * Parallelise Parton Showers on a GPU" (arXiv:2403.08692).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path: every
 * function here (Philox, matrix element, shower, observables, histograms) is
 * written independently from the paper and the published physics it cites.
 *
 * Everything is FP64, one event at a time, in the order of the serial
 * algorithm of Appendix A (SelectWinnerEmission / GenerateEmission / main
 * loop), with the LO matrix element of Appendix B and the observables of
 * Section 3.1.  Compiled with -ffp-contract=off and no fast-math.
 *
 * Momenta are stored as (E, px, py, pz) in GeV; scales t in GeV^2.
 *
 * Pins (tests/test_oracle_*.py check each function against something other
 * than itself): Philox against the published known-answer vectors; alpha_s
 * against closed-form values and the one-loop running; the kernels against
 * the DGLAP collinear limits, their overestimates, integrals and z inverses
 * by quadrature; the matrix element against sigma_LO, the R ratio and the
 * angular shape; the dipole map against its invariants; the first emission
 * and the no-emission probability against the Sudakov factor by quadrature;
 * thrust against brute force over every hemisphere split; C against the
 * eigenvalues of the momentum tensor; Durham against three-parton closed
 * forms and four-parton brute force; hemisphere masses against brute force;
 * the tail cut (max_cycles) against the first cycles of the uncut shower;
 * the weighted veto against the Sudakov factor by quadrature; massive
 * quarks against the vector-current threshold factor and a Dirac-trace spin
 * sum (matrix element), the Dalitz-plot Jacobian and invariants (map), the
 * massive eikonal factor (soft limit), the massless limit, and the first
 * emission off a heavy pair against a Dalitz-plot quadrature.  The g -> Q
 * Qbar mass term is pinned only by its bound and massless limit.
 * Whole showered events beyond the first emission have no external
 * reference: parity unpinned there (colour, flavour and momentum
 * conservation are checked, the distributions are not).
 */
#ifndef VSH_ORACLE_H
#define VSH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* event status codes (same meaning as the product library's) */
enum {
  OR_RUNNING = 0,     /* still showering                                   */
  OR_DONE = 1,        /* reached the cutoff                                */
  OR_OVERFLOW = 2,    /* an accepted emission found the record full        */
  OR_NONFINITE = 3,   /* a non-finite momentum component                   */
  OR_CONSERVATION = 4,/* momentum conservation or masslessness violated    */
  OR_TRUNCATED = 5,   /* still above the cutoff after max_cycles veto cycles:
                         the event is vetoed (the tail cut that the caption
                         of Fig. 7 suggests studying)                      */
  OR_STOPPED = 6      /* stopped after max_emit emissions (test runs only) */
};

enum { OR_NOBS = 8, OR_NBINS = 50, OR_NHCOL = OR_NBINS + 2 };
enum { OR_NSUM_D = 10, OR_NSUM_I = 7 };
enum { OR_NLOG = 7 };
enum { OR_NWORK = 6 };

/* Philox4x32-10 block function (Salmon et al., SC'11) */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* (2m+1) 2^-53 with m = ((hi >> 12) << 32) | lo: exact, strictly inside (0,1) */
double or_uniform(uint32_t hi, uint32_t lo);
/* the four draw purposes of the random-number contract */
enum { OR_P_ME = 1, OR_P_TRIAL = 2, OR_P_ACCEPT = 3, OR_P_SPLIT = 4 };
void or_draw(uint64_t seed, uint64_t event, uint32_t cycle, uint32_t purpose,
             uint32_t slot, uint32_t out[4]);

double or_alpha_s(double t);

/* splitting kernels: id 0-4 q->qg (d,u,s,c,b), 5-9 qbar->qbar g,
   10 g->gg, 11-15 g->f fbar (f = d,u,s,c,b) */
int    or_kernel_list(int pid, int out[6]);
double or_kernel_value(int K, double z, double y);
double or_kernel_over(int K, double z);
double or_kernel_integral(int K, double zm, double zp);
double or_kernel_zgen(int K, double zm, double zp, double u);

/* LO e+e- -> q qbar */
double or_me2(int flavour, double s, double cos_theta);
double or_sigma_lo(double s);
void   or_me_event(uint64_t seed, uint64_t event, double ecm, int *flavour,
                   double *cos_theta, double *phi, double *weight, double p[8]);

/* Massive quarks: mass[f] is the mass of flavour f = 1..5 (d, u, s, c, b;
   mass[0] unused); NULL means five massless flavours. */
double or_me2_massive(int flavour, double s, double cos_theta, double m);
double or_sigma_lo_massive(double s, const double mass[6]);
void   or_me_event_massive(uint64_t seed, uint64_t event, double ecm, const double mass[6],
                           int *flavour, double *cos_theta, double *phi, double *weight,
                           double p[8]);
int    or_massive_limits(double Q2, double mi, double mj, double mk, double tcut, double *zm,
                         double *zp);
double or_massive_flux(double Q2, double mi, double mj, double mk, double mij);
double or_kernel_value_massive(int K, double z, double y, double mi, double qb2, double sij);
double or_massive_ratio(int K, double t, double z, double Q2, double mi, double mj, double mk,
                        double fover);
void   or_split_kinematics_massive(const double pij[4], const double pk[4], double mi, double mj,
                                   double mk, double mij, double t, double z, double phi,
                                   double out_i[4], double out_j[4], double out_k[4]);
int    or_validate_massive(int n, const double *p, const int *pid, double ecm, const double *mass);

/* Catani-Seymour final-final map */
void or_split_kinematics(const double pi[4], const double pk[4], double t,
                         double z, double phi, double out_i[4],
                         double out_j[4], double out_k[4]);

/* Shower one event from the n0 partons given in p/pid/col/acol (arrays of
   length cap, updated in place).  Returns the final status.  max_cycles > 0
   stops an event that has used that many veto cycles without reaching the
   cutoff (status OR_TRUNCATED); 0 means no limit.  t_over > 0 takes
   alpha_s(t_over) for the trial density instead of alpha_s(t_C): below
   t_over that is no overestimate, and the weighted veto (where the ratio r
   exceeds 1: accept with probability r / (2r - 1), weight the event by
   +-(2r - 1)) keeps every distribution exact on average; *weight returns
   the product of those factors (1 with t_over = 0).  mass (NULL = massless)
   gives quark masses: kernels with a massive splitter, product or spectator
   take the massive phase space, kernels and map.
   max_emit >= 0 stops after that many emissions (test runs). */
int or_shower(uint64_t seed, uint64_t event, double ecm, double tcut, int cap,
              int max_cycles, double t_over, const double *mass, int max_emit, int *n,
              double *p, int *pid,
              int *col, int *acol, int *cycles, uint64_t *emit_hash, int *n_emit,
              double *weight, double *emit_log, int max_log, uint64_t *work);

/* Initial-state shower of Drell-Yan events with a closed-form stand-in
   parton density (no PDF set is available); see vsh_oracle.c. */
double or_pdf_q(double x);
double or_pdf_g(double x);
int    or_isr_zlimits(double x, double st, double tcut, double *zlo, double *zhi);
double or_isr_ratio(double t, double z, double x, double st);
void   or_isr_me(uint64_t seed, uint64_t event, double sqrt_s_had, double q, int *flavour, int *quark_from_a,
                 double *rapidity, double *weight, double *xa, double *xb, double p[12]);
int    or_isr_shower(uint64_t seed, uint64_t event, double q, double tcut, int cap, int max_emit, int *n,
                     double *p, int *pid, int *col, int *acol, double *xa, double *xb, int *cycles,
                     uint64_t *emit_hash, int *n_emit, double *emit_log, int max_log, uint64_t *work);
int    or_isr_validate(int n, const double *p, double q);
void   or_isr_hist_ranges(double lo[OR_NOBS], double hi[OR_NOBS]);
int    or_isr_generate(uint64_t seed, uint64_t first, uint64_t n_events, double sqrt_s_had, double q, double tcut,
                       int cap, double *sum_d, int32_t *sum_i, uint64_t *sum_hash, double *hist, int32_t *rec_n,
                       double *rec_p, int32_t *rec_pid, int32_t *rec_col, int32_t *rec_acol, uint64_t *work);

/* observables */
double or_thrust(int n, const double *p, double axis[3]);
void   or_durham(int n, const double *p, double s, double *y23, double *y34);
double or_cparameter(int n, const double *p);
void   or_hemispheres(int n, const double *p, const double axis[3], double s,
                      double *rho_h, double *b_t, double *b_w);
int    or_validate(int n, const double *p, double ecm);
void   or_observables(int n, const double *p, double ecm, double obs[7]);
void   or_hist_ranges(double lo[OR_NOBS], double hi[OR_NOBS]);

/* Whole pipeline over events first .. first+n_events-1.  Per-event
   ecm/tcut arrays may be NULL (then ecm0/tcut0 are used).  Any output
   pointer may be NULL.  hist is [OR_NOBS][OR_NHCOL][3] (sum w, sum w^2,
   entries), accumulated (not cleared); only events that reach the cutoff
   and validate fill it.  max_cycles, t_over and mass as for or_shower; the event
   weight (summary field 0, histograms) is the matrix-element weight times
   the shower's.  Returns 0, or -1 on bad arguments. */
int or_generate(uint64_t seed, uint64_t first, uint64_t n_events,
                const double *ecm, double ecm0, const double *tcut,
                double tcut0, int cap, int max_cycles, double t_over, const double *mass,
                double *sum_d, int32_t *sum_i,
                uint64_t *sum_hash, double *hist, int32_t *rec_n,
                double *rec_p, int32_t *rec_pid, int32_t *rec_col,
                int32_t *rec_acol, uint64_t *work);

#ifdef __cplusplus
}
#endif
#endif
