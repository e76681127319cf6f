/*
 * vsh.h -- C ABI of libvsh, an MI355X (gfx950) engine for the parallel
 * Sudakov-veto parton shower of Seymour & Sule, "An Algorithm to Parallelise
 * Parton Showers on a GPU" (arXiv:2403.08692).
 *
 * What one call computes (Section 3 and Appendices A-C of the paper):
 * generate N events e+e- -> q qbar at sqrt(s) from the LO matrix element
 * (App. B), shower each to the cutoff t_C with the veto algorithm run for all
 * events at once (Sec. 2; App. A and C), then compute Durham jet rates and
 * event shapes (Sec. 3.1) into histograms, returning per-event summaries and,
 * on request, the event records.
 *
 * Conventions
 *  - Every call returns vsh_status: VSH_OK (0) or a negative error code.
 *    No C++ exception crosses this interface.  After an error,
 *    vsh_last_error(ctx) describes it (valid until the next call on ctx).
 *  - Units: GeV for energies and momenta, GeV^2 for t and t_C, pb for
 *    weights.  Momenta are (E, px, py, pz).
 *  - An event is a pure function of (seed, event id, sqrt(s), t_C, cap) and
 *    the request's physics options (cycle_limit, t_over, quark masses):
 *    every random number is Philox4x32-10 keyed by (seed, event id) with a
 *    counter naming the draw, so results do not depend on batching, launch
 *    form, lane mapping or on which other requests share the device.
 *  - Per-event problems (record overflow, non-finite momenta, violated
 *    momentum conservation) and the tail cut (cycle_limit) are not call
 *    errors: they set the event's status and are counted in the result;
 *    such events are left out of histograms.
 *  - Threading: one context per device.  A context is internally locked:
 *    calls from several host threads are serialised.
 */
#ifndef VSH_H
#define VSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VSH_VERSION_MAJOR 1
#define VSH_VERSION_MINOR 3

typedef enum {
  VSH_OK = 0,
  VSH_E_INVALID = -1,   /* bad argument (message names it)                     */
  VSH_E_NOMEM = -2,     /* the request can never fit the memory budget, or an
                           allocation (device arena, pinned staging) failed      */
  VSH_E_DEVICE = -3,    /* no usable gfx950 device, or a HIP runtime error      */
  VSH_E_BUSY = -4,      /* not finished yet (vsh_poll) / serving loop owns it   */
  VSH_E_NOTFOUND = -5,  /* unknown ticket                                       */
  VSH_E_CANCELLED = -6, /* the request was cancelled                            */
  VSH_E_INTERNAL = -7
} vsh_status;

/* event status codes, per event */
enum {
  VSH_EV_RUNNING = 0,
  VSH_EV_DONE = 1,         /* showered to the cutoff, validated                  */
  VSH_EV_OVERFLOW = 2,     /* an accepted emission found the record full         */
  VSH_EV_NONFINITE = 3,    /* a momentum component is not finite                 */
  VSH_EV_CONSERVATION = 4, /* |sum p - (sqrt s, 0)| > 1e-10 sqrt s, or |p_i^2| > 1e-10 s */
  VSH_EV_CYCLE_LIMIT = 5   /* still above the cutoff after the request's cycle_limit veto cycles
                              (2^20 when 0: a guard, not reached in practice); vetoed: no
                              observables, left out of the histograms                */
};

/* observables / histograms: 50 uniform bins [lo, hi) plus underflow (bin 0)
   and overflow (bin 51); each cell holds (sum w, sum w^2, entries).
     0 log10 y23 (Durham)  [-4.3, -0.3]      4 rho_H (heavy-jet mass^2 / s) [0, 0.5]
     1 log10 y34 (Durham)  [-4.3, -0.3]      5 B_T (total broadening)     [0, 0.5]
     2 tau = 1 - T (thrust) [0, 0.5]          6 B_W (wide broadening)      [0, 0.35]
     3 C-parameter          [0, 1]            7 cos(theta) of the quark    [-1, 1]
   log10 y is filled only for y > 0; y = 0 (fewer than 3 or 4 partons) goes
   to the underflow bin. */
#define VSH_NOBS 8
#define VSH_NBINS 50
#define VSH_NHCOL (VSH_NBINS + 2)
#define VSH_HIST_DOUBLES (VSH_NOBS * VSH_NHCOL * 3)

/* per-event summary, structure of arrays [field][n_events]
   double fields: 0 w (pb), 1 cos(theta), 2 y23, 3 y34, 4 tau, 5 C, 6 rho_H,
                  7 B_T, 8 B_W, 9 phi (of the quark)
   int32 fields : 0 partons n, 1 status, 2 veto cycles (SelectWinner calls,
                  the last empty one included), 3 accepted emissions,
                  4 flavour (1..5 = d,u,s,c,b), 5 trial emissions generated,
                  6 dipole ends with phase space above t_C, summed over cycles
   hash         : FNV-1a over the sequence of accepted (kernel, splitter,
                  spectator) triples, 32-bit words, offset basis
                  0xcbf29ce484222325, prime 0x100000001b3 */
#define VSH_NSUM_D 10
#define VSH_NSUM_I 7

/* request flags */
#define VSH_SUMMARY 0x1u           /* return per-event summaries                       */
#define VSH_RECORDS 0x2u           /* return the final partons of every event (CSR)     */
#define VSH_FORM_PLAIN 0x0u        /* one launch; each wave keeps its events (one lane
                                      each, or 64 with their trials spread over the
                                      lanes) from start to the cutoff                   */
#define VSH_FORM_PERSISTENT 0x4u   /* persistent waves with ballot compaction + refill,
                                      events evolving in their output records           */
#define VSH_INPUTS_ON_DEVICE 0x8u  /* ecm_per_event / tcut_per_event are device pointers
                                      (vsh_generate_into only)                          */
#define VSH_HIST_FIXEDPOINT 0x10u  /* histogram sums in int64 fixed point, so that they do
                                      not depend on the order in which events are added
                                      (the atomic histogramming of Sec. 3.2 / Table 1,
                                      made order-independent): sum w is accumulated as
                                      integers in units of 2^-fw with 2^(62 - fw) above
                                      n |w|max (n the events of the request, |w|max the
                                      largest event weight), sum w^2 likewise, and both
                                      converted to FP64 once at the end.  The result is
                                      then the same bits served alone, served in a mix,
                                      through vsh_generate in either form or
                                      vsh_generate_into, whenever the request is
                                      processed in one piece (vsh_generate splits only
                                      requests larger than its memory budget; each
                                      piece then has its own scale).  The sums are
                                      within 2^-(62 - ceil(log2 n)) |w|max per event of
                                      the FP64 ones.  Weights must be finite.          */

typedef struct vsh_ctx vsh_ctx; /* device arena, stream, kernel cache, serving state */

typedef struct {
  int device;                /* HIP device ordinal                                      */
  uint64_t mem_budget_bytes; /* device memory the context may hold; 0 = 80% of free      */
  uint32_t flags;            /* reserved, 0                                              */
  const char *tuner_cache_path; /* optional file of earlier vsh_autotune choices (read
                                   by vsh_autotune, which appends each new choice);
                                   NULL or "" = none.  Copied at vsh_create.        */
} vsh_ctx_opts;

/* Create a context on opts->device (opts may be NULL: device 0, default
   budget).  The context holds what the paper's "device preparation" stage
   (Table 1) allocates once: the device arena, reused by every later call and
   grown on demand, the stream and the stage events.  Fails with VSH_E_DEVICE
   when the device is not gfx950 or HIP reports an error.  *out is owned by
   the caller; release with vsh_destroy. */
vsh_status vsh_create(const vsh_ctx_opts *opts, vsh_ctx **out);
void vsh_destroy(vsh_ctx *ctx);
/* Last error message of ctx (or of the last failed vsh_create if ctx is
   NULL); never NULL. */
const char *vsh_last_error(const vsh_ctx *ctx);

typedef struct {
  uint64_t n_events;     /* >= 1                                                    */
  uint64_t seed;         /* Philox key                                              */
  uint64_t first_event;  /* event ids are first_event .. first_event + n_events - 1 */
  double ecm;            /* sqrt(s) in GeV, > 0; used when ecm_per_event is NULL      */
  double t_cut;          /* t_C in GeV^2, > 0.01; used when tcut_per_event is NULL    */
  const double *ecm_per_event;  /* optional [n_events]; host memory, read during the call
                                   (copied by vsh_submit)                              */
  const double *tcut_per_event; /* optional [n_events]; likewise                       */
  uint32_t max_partons;  /* record capacity per event, 2..1024 (64, 128, 256 typical)  */
  uint32_t flags;        /* VSH_SUMMARY | VSH_RECORDS | VSH_FORM_*                     */
  uint32_t cycle_limit;  /* tail cut (the study suggested with Fig. 7): an event still
                            above the cutoff after this many veto cycles stops with
                            VSH_EV_CYCLE_LIMIT and is vetoed.  0 = no cut (2^20 guard);
                            values above 2^20 act as 2^20.  Events that end within the
                            limit are exactly those of the uncut run.                */
  double t_over;         /* scale (GeV^2) of alpha_s in the trial density: 0 = t_cut, an
                            overestimate (App. A), every shower weight 1.  A larger value
                            makes fewer trials; below t_over the trial density undershoots,
                            and the weighted veto (the extension for bounded ratios that
                            App. A notes) keeps every distribution exact on average: where
                            the ratio r of true to trial density exceeds 1 the emission is
                            accepted with probability r/(2r - 1) and the event weight
                            multiplied by +(2r - 1), or by -(2r - 1) on rejection.  Event
                            weights (summary field 0, histograms, sum_w) include it.
                            0 or > 0.01                                               */
  double mass_c, mass_b; /* charm and bottom quark masses in GeV (0 = massless, the
                            default; d, u, s stay massless): the extension to massive
                            final-state quarks that the conclusions name.  The matrix
                            element then carries the quark velocity and draws only
                            flavours open at sqrt(s); kernels with a massive parton
                            take the massive dipole phase space, the quasi-collinear
                            mass terms and the massive recoil map; events validate on
                            their mass shells.  Such requests run the massive kernels
                            of the tuned mapping.  0 <= mass, finite                  */
} vsh_request;

/* Result of one request.  Library-owned host memory; release with
   vsh_result_free.  Optional arrays are NULL unless their flag was set. */
typedef struct {
  uint64_t n_events, n_done, n_overflow, n_nonfinite, n_conservation;
  double sum_w, sum_w2;       /* over all events: sigma estimate = sum_w / n_events */
  uint32_t n_obs, n_bins;     /* VSH_NOBS, VSH_NBINS                               */
  const double *hist_lo, *hist_hi; /* [VSH_NOBS]                                    */
  const double *hist;         /* [VSH_NOBS][VSH_NHCOL][3]                           */
  const double *sum_d;        /* [VSH_NSUM_D][n_events]                             */
  const int32_t *sum_i;       /* [VSH_NSUM_I][n_events]                             */
  const uint64_t *sum_hash;   /* [n_events]                                         */
  const uint64_t *rec_offsets;/* [n_events + 1]; event e owns partons
                                 rec_offsets[e] .. rec_offsets[e+1]-1               */
  const double *rec_p;        /* [total][4]                                         */
  const int8_t *rec_pid;      /* [total]: 1..5 quarks, -1..-5 antiquarks, 21 gluon   */
  const uint16_t *rec_col, *rec_acol; /* [total]: colour / anticolour line, 0 = none */
  uint64_t total_cycles;      /* sum over events of veto cycles                     */
  uint64_t total_trials;      /* sum over events of trial emissions                  */
  uint64_t total_ends;        /* sum over events and cycles of active dipole ends    */
  uint64_t total_emissions;   /* sum over events of accepted emissions               */
  uint32_t max_cycles;        /* longest event, in veto cycles                       */
  double t_me_ms, t_shower_ms, t_obs_ms, t_total_ms; /* device time per stage; total is
                                                        host wall clock of the call  */
  uint64_t n_cycle_limit;     /* events stopped by the request's cycle_limit        */
  uint32_t queue_ahead;       /* served requests: requests waiting for admission ahead
                                 of this one when it was submitted (0 otherwise)     */
  double t_queue_ms;          /* served requests: submission to admission (memory
                                 reserved), host wall clock (0 otherwise)            */
} vsh_result;

/* Blocking generation (Sec. 3 problem statement; App. C for the shower).
   Allocates from the context arena (grow-only, reused across calls), runs
   matrix element, shower and observables on the context's stream, copies the
   results to pinned host memory.  Requests larger than the budget allows at
   once are processed in event-id chunks (identical results).
   Errors: VSH_E_INVALID (n_events = 0, ecm <= 0, t_cut <= 0.01, max_partons
   outside 2..1024, unknown flags, t_over neither 0 nor a finite value above
   0.01, a negative or non-finite quark mass), VSH_E_NOMEM (not even one
   chunk fits), VSH_E_DEVICE. */
vsh_status vsh_generate(vsh_ctx *ctx, const vsh_request *req, vsh_result **out);
void vsh_result_free(vsh_result *res);

/* The main loop of App. A (select the winning trial emission, veto, emit,
   until the cutoff) from caller-supplied initial states instead of LO events
   (a q g qbar start, say), followed by the validation and observables of
   Sec. 3.1.  offsets [n_events+1] index into p [total][4], pid, col,
   acol [total] (host memory, read during the call); the event's sqrt(s) is
   taken from the sum of its momenta' energies, t_cut from req; req->ecm and
   the per-event arrays are ignored.  Weights are 1.  The evolution starts at
   t = s of each event.  Same errors as vsh_generate, plus VSH_E_INVALID for an
   event with more partons than max_partons or an inconsistent colour flow. */
vsh_status vsh_shower_records(vsh_ctx *ctx, const vsh_request *req, const uint64_t *offsets,
                              const double *p, const int8_t *pid, const uint16_t *col,
                              const uint16_t *acol, vsh_result **out);

/* Initial-state shower (the step to hadron colliders that the paper's
   conclusions name: PDFs evaluated in the shower).  Drell-Yan events
   q qbar -> V at hadron centre-of-mass energy sqrt_s_hadron with V of mass
   Q = req->ecm: flavour uniform over d, u, s, c, b, the quark from either
   beam, the rapidity of V uniform in |y| < ln(sqrt_s_hadron / Q); each
   incoming line evolves backwards from t = Q^2 to req->t_cut with the
   density (alpha_s/2 pi) (dt/t) (dz/z) P_qq(z) f(x/z)/f(x), the other
   incoming parton its spectator, emissions through the Catani-Seymour
   initial-initial map (the final state takes the recoil); the emitted
   gluons do not radiate.  No parton-density set is available, so f is a
   closed-form stand-in, f(x) = (63/128) x^(-1/2) (1 - x)^3 for every quark
   and antiquark (with a gluon 3 x^(-1) (1 - x)^5 the momentum sum rule holds).
   Records: slot 0 the incoming parton from beam A (+z), 1 from beam B,
   2 V (pid 23), then the emitted gluons.  Weights (arbitrary units): the
   parton luminosity's rapidity density for a unit partonic cross-section,
   10 (2Y) tau f(x_A) f(x_B).  Summary double fields: 0 w, 1 y_V, 2 p_T,V,
   3 x_A, 4 x_B (final fractions), 5 p_T of the hardest gluon; int fields
   as vsh_generate's (flavour +f with the quark from beam A, -f from B).
   Histograms: 0 log10(p_T,V / GeV) [-1, 3], 1 y_V [-5, 5], 2 emitted gluons
   [0, 50], 3 log10(p_T / GeV) of the hardest gluon [-1, 3] (rows 4-7 unused;
   hist_lo / hist_hi give the ranges).  One lane per event, plain form.
   Errors: those of vsh_generate, and VSH_E_INVALID for flags other than
   VSH_SUMMARY | VSH_RECORDS, per-event arrays, a cycle limit, t_over or
   masses, max_partons < 3, sqrt_s_hadron <= Q, or t_cut >= Q^2 / 4. */
vsh_status vsh_generate_isr(vsh_ctx *ctx, const vsh_request *req, double sqrt_s_hadron, vsh_result **out);

/* Device-side generation into caller-owned device memory, on the caller's
   HIP stream, with no allocation and no host synchronisation: the launch
   sequence of vsh_generate without its copies, i.e. the problem statement of
   Sec. 3 (matrix element of App. B, shower of App. A / C, observables of
   Sec. 3.1 into histograms) with every result left on the device.
     stream      hipStream_t of the caller (NULL = the null stream)
     workspace   device buffer of at least vsh_workspace_size() bytes
     dev_hist    [VSH_HIST_DOUBLES] device doubles, accumulated into (clear first)
     dev_sum_d   optional [VSH_NSUM_D][n_events] device doubles
     dev_sum_i   optional [VSH_NSUM_I][n_events] device int32
     dev_hash    optional [n_events] device uint64
   With VSH_INPUTS_ON_DEVICE, ecm_per_event / tcut_per_event are device
   pointers.  The call returns once the kernels are enqueued. */
vsh_status vsh_generate_into(vsh_ctx *ctx, const vsh_request *req, void *stream, void *workspace,
                             uint64_t workspace_bytes, double *dev_hist, double *dev_sum_d,
                             int32_t *dev_sum_i, uint64_t *dev_hash);
/* Workspace bytes vsh_generate_into needs for req (0 on invalid input). */
uint64_t vsh_workspace_size(const vsh_request *req);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops that must not call hipMalloc, harnesses that forbid
   it): vsh_generate_into in the plain form, with its workspace in a device
   array the library owns instead of a caller buffer.  The array holds
   VSH_STATIC_SCRATCH_BYTES (64 MiB: about 10^4 LEP events at 64 partons;
   vsh_workspace_size(req) must not exceed it); every device that runs the
   library holds its own copy until the process ends.  The call allocates
   nothing (no hipMalloc, no pinned memory, no library allocation), only
   enqueues kernels and device-to-device copies on `stream`, and returns.
   Arguments, outputs and per-event inputs as for vsh_generate_into.
   All calls on one device share that device's array and nothing in it needs
   to start at zero, but calls whose work overlaps on one device (two host
   threads, or two streams without an ordering between them) race on it:
   order them on one stream.
   Errors: those of vsh_generate_into; VSH_E_INVALID for VSH_FORM_PERSISTENT
   or VSH_RECORDS; VSH_E_NOMEM when the request needs more than the array. */
#define VSH_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
vsh_status vsh_generate_into_static(vsh_ctx *ctx, const vsh_request *req, void *stream, double *dev_hist,
                                    double *dev_sum_d, int32_t *dev_sum_i, uint64_t *dev_hash);

/* Stage timing of vsh_generate_into, per stage as in the paper's Table 1
   and Fig. 6 (matrix element, shower, observables).  After vsh_timing_start, each
   vsh_generate_into call (at most VSH_TIMING_MAX_CALLS) records HIP events on
   its own stream before and after each of its three stages: matrix element,
   shower, observables + histograms.  vsh_timing_read waits for those events
   and writes ms[3 * c + stage] for calls c = 0 .. *n_calls - 1 (at most
   max_calls), then stops recording.  Errors: VSH_E_INVALID when timing was
   not started. */
#define VSH_TIMING_MAX_CALLS 1024
vsh_status vsh_timing_start(vsh_ctx *ctx);
vsh_status vsh_timing_read(vsh_ctx *ctx, float *ms, uint32_t max_calls, uint32_t *n_calls);

/* Launch parameters of the two forms of the parallel veto loop of Sec. 2
   (one launch per batch, or persistent waves refilled from a work counter).  vsh_autotune picks them by timing
   candidates on a sample request; vsh_set_tuning sets them directly (values
   are clamped to the ranges below).  They change speed only: every event
   is the same for any setting. */
typedef struct {
  uint32_t plain_block;      /* threads per block, plain form: 64, 128 or 256          */
  uint32_t mapping;          /* persistent form: 0 = one lane per event,
                                1 = each cycle's trials spread over the wave's lanes   */
  uint32_t waves_per_cu;     /* persistent waves launched per compute unit, 1..16 (the
                                flattened kernel keeps 8 resident per CU; later waves
                                start as earlier ones exit)                           */
  uint32_t block;            /* threads per block of mapping 0: 64, 128 or 256          */
  uint32_t refill_threshold; /* idle lanes a wave waits for before refilling, 1..64;
                                batches evolve in their output records and claim whole
                                multiples of 16 events, so there it is at least 16    */
  uint32_t refill_period;    /* veto cycles between refill checks, 1..64               */
  uint32_t plain_waves;      /* register budget of the plain kernel, as resident waves
                                per SIMD: 2, 3 or 4 (more waves, fewer registers)     */
  uint32_t plain_mapping;    /* plain form: 0 = one lane per event, 1 = each wave's 64
                                events with their cycle's trials spread over its lanes */
  uint32_t from_cache;       /* set by vsh_autotune: 1 when the settings came from the
                                context's tuner cache file (nothing was timed)       */
} vsh_tuning;
vsh_status vsh_get_tuning(vsh_ctx *ctx, vsh_tuning *out);
vsh_status vsh_set_tuning(vsh_ctx *ctx, const vsh_tuning *t);
/* Time the candidate settings of the persistent form (or, with
   VSH_FORM_PLAIN in sample->flags, the plain mapping, block size and register
   budget) on `sample`
   (its first min(n_events, 2^18) events) and keep the fastest in ctx;
   *chosen (optional) receives it.  Candidates whose summaries differ from
   the first candidate's are rejected (VSH_E_INTERNAL).  With a tuner cache
   (vsh_ctx_opts.tuner_cache_path), a sample whose key (library version,
   device, form, capacity, sample size, sqrt(s), t_C or a hash of the
   per-event arrays, masses, t_over, cycle limit) is in the file takes the
   cached settings without timing (chosen->from_cache = 1); otherwise the new
   choice is appended to the file.  An unreadable or unwritable cache file is
   ignored. */
vsh_status vsh_autotune(vsh_ctx *ctx, const vsh_request *sample, vsh_tuning *chosen);

/* Serving (continuous batching).  Sec. 2's parallel form needs nothing but
   independent events, so events of different requests (each its own sqrt(s),
   t_C, seed and size) share the same launches; the per-request results are
   those of the problem statement of Sec. 3.  vsh_submit copies the request (and its
   per-event arrays) and returns at once with a ticket; the context's serving
   loop admits requests by event-record memory, runs their events together in
   persistent launches as slots free up, and keeps one histogram set per
   request.  Per-request results equal those of vsh_generate on the same
   request up to the summation order of the histograms.
   vsh_poll: *done = 1 once finished.  vsh_wait blocks until finished and
   hands over the result (once; the ticket is then forgotten).
   vsh_cancel: stops admitting the request's events; vsh_wait then returns
   VSH_E_CANCELLED.  A HIP error while a request is admitted, showered or
   measured fails that request alone: it finishes (vsh_poll reports it done),
   and vsh_wait returns VSH_E_DEVICE (VSH_E_NOMEM when the observables'
   scratch cannot be allocated) with the HIP error in vsh_last_error.
   Errors: VSH_E_NOTFOUND for unknown tickets, and those of vsh_generate at
   submission. */
vsh_status vsh_submit(vsh_ctx *ctx, const vsh_request *req, uint64_t *ticket);
vsh_status vsh_poll(vsh_ctx *ctx, uint64_t ticket, int *done);
vsh_status vsh_wait(vsh_ctx *ctx, uint64_t ticket, vsh_result **out);
vsh_status vsh_cancel(vsh_ctx *ctx, uint64_t ticket);

/* Testing hook for the serving error path (for test suites, not part of the
   method): the next `count` serving launches of ctx report a HIP launch
   failure to the loop instead of launching, so the requests they hold fail
   as described above while the device stays healthy.  Starts the serving
   loop if needed. */
vsh_status vsh_test_fail_epochs(vsh_ctx *ctx, uint32_t count);

#ifdef __cplusplus
}
#endif
#endif /* VSH_H */
