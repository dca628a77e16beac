/*
 * rtbte -- collision integrals and time integrators of the coupled
 * electron-phonon real-time Boltzmann equation on AMD MI355X (gfx950).
 *
 * The problem (paper: Eq. (bte)) is
 *     df_nk/dt  = I^{e-ph}[f, N]_nk
 *     dN_nuq/dt = I^{ph-e}[f, N]_nuq + I^{ph-ph}[N]_nuq
 * with the collision integrals of Methods, Eq. (e-ph) and Eq. (ph-ph), the
 * Gaussian delta_sigma(E) = exp(-(E/sigma)^2)/(sigma sqrt(pi)) truncated at
 * |E| <= nsigma*sigma, and a phonon frequency cutoff hw_cut (Methods, grid-size
 * paragraphs).  The state vector is y = [f; N] (Eq. (state_vec)); the
 * integrators are the adaptive embedded ERK method with WRMS error norm and
 * PID step control (Methods, ERK method) and the third-order MIS multirate
 * method with e-ph as the fast and ph-ph as the slow part (Eq. (mri_rhs),
 * Methods, MRI method).
 *
 * Conventions
 *   - Energies in eV, times in fs.  hbar = 0.6582119569 eV fs.
 *   - All arrays in rtbte_problem are HOST memory, read during rtbte_create
 *     and deep-copied; the caller may free them on return.
 *   - y, ydot, t, h arguments of the stepping calls are caller-owned DEVICE
 *     buffers of doubles on the context's device.  y holds the instances
 *     back to back at the offsets reported by rtbte_layout; within an
 *     instance it is [f (n_el); N (n_ph)].  t, h hold one entry per instance.
 *   - A stepping call whose t_out is at or before an instance's t leaves that
 *     instance (its y, t and step sizes) as it is.
 *   - All device work is enqueued on the HIP stream passed in (NULL: the
 *     null stream).  Calls that return results to the host synchronise that
 *     stream; rtbte_rhs does not.
 *   - Every call returns an RTBTE_* status; no C++ exception crosses the ABI.
 *     rtbte_last_error(ctx) describes the last failure (ctx may be NULL for
 *     a failed create).  A context is not thread-safe; distinct contexts are
 *     independent.
 */
#ifndef RTBTE_H
#define RTBTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RTBTE_OK = 0,
  RTBTE_E_INVAL = -1,       /* bad argument or problem data                         */
  RTBTE_E_NOMEM = -2,       /* host or device allocation failed                     */
  RTBTE_E_HIP = -3,         /* a HIP runtime call failed                            */
  RTBTE_E_STEP = -4,        /* more than max_fails consecutive error-test failures  */
  RTBTE_E_NONFINITE = -5,   /* a non-finite error estimate (NaN/Inf in the state)   */
  RTBTE_E_UNSUPPORTED = -6  /* option combination not implemented                   */
};

/* Parts of the right-hand side (Eq. (erk_rhs)); OR them together. */
enum {
  RTBTE_PART_EPH = 1,   /* I^{e-ph}: electron rows                         */
  RTBTE_PART_PHE = 2,   /* I^{ph-e}: phonon rows, e-ph absorption channels */
  RTBTE_PART_PHPH = 4,  /* I^{ph-ph}: phonon rows, three-phonon channels   */
  RTBTE_PART_ALL = 7
};

enum { RTBTE_FP64 = 0, RTBTE_MIXED = 1 };
/* Weight storage of RTBTE_MIXED (Options.mixed_weights).  Every weight is
   stored relative to the FP32 scale of its block of 512 consecutive channels.
     RTBTE_W_PACK8    8 bytes per channel: both partner positions (P bits each,
                      relative to the instance; P = bits of the largest
                      instance's state count), the row tag, the emission bit
                      and the weight as a small float (6 exponent bits, M =
                      min(53 - 2P, 23) mantissa bits; relative rounding
                      <= 2^-(M+1), e.g. 2^-20 for 115 200 states) in one
                      64-bit word.
                      Needs P <= 20 (instances of at most 2^20 states).
     RTBTE_W_F16X     10 bytes: 8-byte index word (24-bit positions) and an
                      FP16 head whose 11-bit significand tail sits in the index
                      word: 22 significant bits, relative rounding <= 2^-22;
     RTBTE_W_F16      10 bytes, FP16 only: relative rounding <= 2^-11;
     RTBTE_W_BF16_EPH 10 bytes, BF16 for the e-ph and ph-e weights (<= 2^-8),
                      FP16 for the ph-ph weights (<= 2^-11);
     RTBTE_W_AUTO     RTBTE_W_PACK8 when its mantissa has at least 12 bits
                      (instances of at most 2^20 states), else RTBTE_W_F16X.
   rtbte_get_weight_format reports the format chosen and its rounding. */
enum { RTBTE_W_AUTO = 0, RTBTE_W_PACK8 = 1, RTBTE_W_F16X = 2, RTBTE_W_F16 = 3, RTBTE_W_BF16_EPH = 4 };

typedef struct rtbte_ctx rtbte_ctx;

/* One rt-BTE instance, stated as in Methods, Eq. (e-ph) and Eq. (ph-ph).
 *   n_el          windowed electron states (n,k) kept in the dynamics
 *   n_ph          phonon states (nu,q)
 *   n_k_total,    sizes of the FULL k and q grids: the 1/N_k and 1/N_q
 *   n_q_total     prefactors use them even when a window keeps fewer states
 *   eps[n_el]     band energies eps_nk (eV)
 *   hw[n_ph]      phonon energies hbar*omega_nuq (eV)
 *   n_eph entries of the e-ph matrix, one per process nk -> mk+q with
 *                 phonon nu q:  eph_row = nk, eph_partner = mk+q,
 *                 eph_phonon = nu q, eph_g2 = |g_mn nu(k,q)|^2 (eV^2).
 *                 Each entry gives an emission and an absorption channel on
 *                 the electron side (kept when its energy mismatch is within
 *                 nsigma*sigma_eph) and, for a kept absorption channel, one
 *                 phonon-side I^{ph-e} channel in row nu q.
 *   n_pp entries  of the ph-ph matrix, one per ordered (lambda; lambda',
 *                 lambda'') with q + q' + q'' = 0: pp_row = lambda,
 *                 pp_a = lambda', pp_b = lambda'', pp_v2 = |V3|^2 (eV^2).
 *                 Each gives an emission channel (delta(-hw + hw' + hw''))
 *                 and an absorption channel (factor 2, delta(hw - hw' + hw'')).
 *   sigma_eph, sigma_pp   Gaussian widths (eV) > 0
 *   nsigma        truncation in units of sigma (> 0)
 *   hw_cut        channels touching a phonon with hw < hw_cut are dropped
 * Rows are processed in groups of up to 16 consecutive rows of one kind
 * (group_rows_el, group_rows_ph); a group's channels are summed merged in the order of a partner index
 * (e-ph electron rows: the phonon; ph-e: the initial electron; ph-ph: the
 * first partner), entries with equal index keeping their input order.
 * Numbering states in grid order therefore keeps the gathers of the
 * populations local.
 */
typedef struct {
  int32_t n_el, n_ph;
  int32_t n_k_total, n_q_total;
  const double *eps, *hw;
  int64_t n_eph;
  const int32_t *eph_row, *eph_partner, *eph_phonon;
  const double *eph_g2;
  int64_t n_pp;
  const int32_t *pp_row, *pp_a, *pp_b;
  const double *pp_v2;
  double sigma_eph, sigma_pp, nsigma, hw_cut;
} rtbte_problem;

/* A model of the ph-ph matrix elements, evaluated on the fly instead of read
 * from stored weights (the paper interpolates its ph-ph matrix elements on
 * the fly rather than storing them: Methods, graphene and silicon grid
 * paragraphs).  The phonon states of an instance are numbered
 * id = q * n_modes + nu over a periodic grid of L points per axis
 * (q = i L + j in 2D, (i L + j) L + k in 3D); the time-reversed state of id
 * is -q with the same nu.  For a channel's triplet (l; a, b):
 *   (c0, c1, c2) = the sorted ids of the triplet or of its time-reversed
 *                  image, whichever is lexicographically smaller;
 *   (r0, r1, r2, r3) = Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11)
 *                  of the counter (c0, c1, c2, stream) under (key0, key1);
 *   n = sqrt(-2 ln u1) cos(2 pi u2), u_i = (r_i + 1/2) 2^-32 (Box-Muller);
 *   |V3|^2 = exp(ln_mu + ln_sigma n)   (eV^2).
 * It is symmetric under permutation of the three phonons and under time
 * reversal. */
typedef struct {
  int32_t dim;              /* 2 or 3 */
  int32_t L;                /* grid points per axis */
  int32_t n_modes;          /* phonon branches (n_ph = n_modes * L^dim) */
  uint32_t key0, key1;      /* Philox key */
  uint32_t stream;          /* fourth counter word */
  double ln_mu, ln_sigma;   /* ln|V3|^2 = ln_mu + ln_sigma * n */
} rtbte_pp_model;

/* Options; rtbte_default_options fills every field. */
typedef struct {
  int32_t precision;       /* RTBTE_FP64 (default) or RTBTE_MIXED: compact weights relative
                              to one FP32 scale per 512 channels (format: mixed_weights),
                              populations gathered as one FP32 code per state (formed in
                              FP64), factors and products in FP32, per-lane compensated
                              FP32 sums added in FP64; the state, the stages,
                              the WRMS norm and the step control stay FP64.  RTBTE_MIXED
                              holds at most 2^24 states per context (RTBTE_E_INVAL beyond) */
  int32_t mixed_weights;   /* RTBTE_MIXED only: RTBTE_W_AUTO (default), RTBTE_W_PACK8,
                              RTBTE_W_F16X, RTBTE_W_F16 or RTBTE_W_BF16_EPH               */
  int32_t device;          /* HIP device ordinal                                           */
  /* ERK error test (Eq. (wrms_weights)): w_i = 1/(rtol |y_i| + atol_i),
     atol_i = atol_el on electron components and atol_ph on phonon components */
  double rtol, atol_el, atol_ph;
  /* MIS fast integrator: 0 adaptive ERK with fast_* tolerances, 1 fixed RK4
     with step h_fast (the last substep of a stage interval is shortened) */
  int32_t fast_mode;
  double h_fast;
  double fast_rtol, fast_atol_el, fast_atol_ph;
  /* PID controller (Eq. (pid_controller)): h' = h * safety * eps_k^(-k1/p) *
     eps_{k-1}^(-k2/p) * eps_{k-2}^(-k3/p); pid_alt_sign = 1 uses +k2/p.
     Ratio limited to <= eta_max (eta_max_first on the first step) after an
     accepted step and to [eta_fail_min, eta_fail_max] after a rejected one
     (and to <= eta_fail_repeat from the small_nef-th consecutive rejection
     on); errors below eps_floor count as eps_floor; more than max_fails
     consecutive rejections end the call with RTBTE_E_STEP. */
  double pid_k1, pid_k2, pid_k3;
  int32_t pid_order, pid_alt_sign;
  double safety, eta_max, eta_max_first, eta_fail_min, eta_fail_max, eps_floor;
  int32_t max_fails;
  int32_t use_graph;        /* 1: the steps between two host checks of the done flags are
                               captured once into a HIP graph (per argument set: y, t/h
                               buffers, tableau, controller) on a stream of the context, and
                               replayed on the caller's stream; 0: launched one by one.  The
                               results are identical.  Profiling (rtbte_profile) launches
                               eagerly, since it times individual launches.                  */
  int32_t steps_per_poll;   /* steps enqueued between host checks of the done flags           */
  int32_t group_rows_el;    /* consecutive electron rows sharing one merged channel stream:
                               1, 2, 4, 8, 12 or 16 (0: 8)                                     */
  int32_t group_rows_ph;    /* the same for phonon rows (0: 16)                                 */
  int64_t item_channels;    /* channels per work item of the collision kernel (0: sized so
                               that there are ~40k items, within [2048, 65536])                */
  int32_t tune;             /* 1: autotune the launch shape at create: for up to four row-group
                               layouts (the given or default one; 4 and 16 electron rows; 8
                               phonon rows) and three item sizes each (the given or default
                               one, half, double), time 20 full right-hand sides each and
                               keep the fastest; a shape tried later replaces the one kept
                               only when it is more than 2 % faster (the timing noise), so the
                               given or default shape stays unless another clearly beats it.
                               Any shape gives the same results to rounding order.
                               Costs up to four layout builds; a cache hit costs one.        */
  const char *tune_cache;   /* text file of tuned shapes, one line per problem signature
                               (device, precision, sizes); read before tuning, appended
                               after.  NULL: env RTBTE_TUNE_CACHE; neither: no cache.         */
  int32_t fp64_layout;      /* RTBTE_FP64 channel storage: RTBTE_F64_AUTO (default: packed
                               when instances have at most 2^19 states), RTBTE_F64_PACKED
                               (12 bytes: an 8-byte word of P-bit instance-relative
                               positions, row tag, emission bit and high weight bits, and a
                               4-byte word of low weight bits; the weight keeps
                               min(80 - 2P, 52) mantissa bits, so it is exact for P <= 14
                               and within 2^-43 relative for P <= 19; arithmetic stays
                               FP64) or RTBTE_F64_PLAIN (16 bytes: two 32-bit indices and
                               the FP64 weight)                                              */
  int32_t fp64_check;       /* RTBTE_MIXED only.  0 (default): off.  K > 0: the context also
                               keeps the FP64 lists (packed when instances have at most 2^19
                               states, else plain: 12 or 16 more bytes per channel) so that
                               rtbte_check_fp64 can measure the mixed right-hand side against
                               FP64, and the stepping calls do so at every K-th poll,
                               reporting the last value in rtbte_stats.err_vs_fp64_last     */
  int32_t small_nef;        /* from the small_nef-th consecutive error-test failure on (default
                               5), the step ratio after a rejection is also capped by        */
  double eta_fail_repeat;   /* eta_fail_repeat (default 0.3): a rescue for steps the PID
                               history factors keep from shrinking                          */
  int32_t pp_fold;          /* 1 (default): when an instance's ph-ph list is mirror-symmetric
                               (every (l; a, b) with a != b has (l; b, a) with the same
                               |V3|^2, as the sum over ordered partner pairs gives; checked
                               at create), store the emission channel of each such pair once,
                               with twice the weight (the emission factor and delta are
                               symmetric in a and b): a quarter fewer ph-ph channels, the
                               same sums to rounding order.  0: store every channel.       */
  int32_t tiled;            /* 0 (default): one wavefront per work item, partners gathered
                               from global memory.  1: with packed channels (FP64 packed,
                               mixed RTBTE_W_PACK8) the collision kernels run tiled: the
                               channels of each group are cut where their sorted partner
                               crosses a key block (1024 states FP64, 2048 mixed), and a
                               launch block of four consecutive groups stages the
                               populations of the key block and of the other partners'
                               window in LDS, so most partner reads leave global memory
                               (half the vector-memory instructions); item_channels then
                               sets the channels a block takes per wavefront.  On the
                               graphene-like workload it is slower (its 64 KB of LDS per
                               block allow two blocks per compute unit).  Both give the
                               same results to rounding order.                              */
  const rtbte_pp_model *pp_model; /* NULL (default): ph-ph weights from pp_v2.  Else n_inst
                               models, one per instance: matrix-free ph-ph weights.  The
                               channel list keeps partners and flags only (8 bytes per ph-ph
                               channel) and every right-hand side recomputes
                               prefactor * |V3|^2 * delta (FP64, in both precisions) from
                               the model and the phonon energies; pp_v2 may be NULL (it is
                               not read).  Needs the packed layouts (FP64 packed, mixed
                               RTBTE_W_PACK8) and tiled = 0 (RTBTE_E_UNSUPPORTED else).   */
} rtbte_options;

enum { RTBTE_F64_AUTO = 0, RTBTE_F64_PACKED = 1, RTBTE_F64_PLAIN = 2 };

typedef struct {
  int64_t n_rhs_eph, n_rhs_phe, n_rhs_phph; /* evaluations of each part                 */
  int64_t n_accept, n_reject;               /* ERK (or MIS slow) steps of this instance */
  int64_t n_fast_accept, n_fast_reject;     /* fast steps inside MIS                    */
  double t, h_last, h_min, h_max, eps_last;
  int32_t status;                           /* RTBTE_* status of the last stepping call */
  double err_vs_fp64_last;                  /* last ||f_mixed - f_fp64|| / ||f_fp64|| of
                                               this instance (fp64_check); -1: none     */
  int32_t health;                           /* RTBTE_HEALTH_* bits: populations found out
                                               of their physical range in the state after
                                               a poll interval of a stepping call, since
                                               create or rtbte_reset (0: none)          */
} rtbte_stats;

/* Health bits (rtbte_stats.health): an electron occupation outside
 * [-1e-6, 1 + 1e-6] (or not a number), a phonon occupation below -1e-6 (or
 * not a number).  Informational: the run goes on (a diverging fixed-step run,
 * for instance, sets them long before its state overflows). */
enum { RTBTE_HEALTH_F_RANGE = 1, RTBTE_HEALTH_N_NEGATIVE = 2 };

void rtbte_default_options(rtbte_options *opts);

/* Build a context for n_inst independent instances (problems[0..n_inst)).
 * Computes every channel weight (delta, prefactor, cutoff), derives the
 * I^{ph-e} lists, groups channels by destination row and uploads them.
 * Errors: RTBTE_E_INVAL (index out of range, sigma <= 0, nsigma <= 0,
 * negative counts, an instance with no states, n_inst < 1; checked before
 * any device call), RTBTE_E_NOMEM, RTBTE_E_HIP. */
int rtbte_create(const rtbte_problem *problems, int32_t n_inst, const rtbte_options *opts,
                 rtbte_ctx **out);
void rtbte_destroy(rtbte_ctx *ctx);
const char *rtbte_last_error(const rtbte_ctx *ctx);

/* Offset of instance `inst` in y, and its sizes. */
int rtbte_layout(const rtbte_ctx *ctx, int32_t inst, int64_t *y_offset, int32_t *n_el,
                 int32_t *n_ph);
/* Total length of y over all instances. */
int64_t rtbte_ny(const rtbte_ctx *ctx);
/* Channels of instance `inst` (-1: all) the right-hand side sums, as the
 * method defines them (every emission and absorption channel of every entry
 * kept by the truncation and the cutoff): counts[0] electron-side e-ph,
 * counts[1] phonon-side ph-e, counts[2] ph-ph. */
int rtbte_counts(const rtbte_ctx *ctx, int32_t inst, int64_t counts[3]);

/* Channels actually stored and streamed (rtbte_counts less the ph-ph
 * emission channels carried by their mirrors under pp_fold). */
int rtbte_stored_counts(const rtbte_ctx *ctx, int32_t inst, int64_t counts[3]);

/* ydot = the parts of f(y) selected by `parts` (Eq. (erk_rhs); parts of
 * Eq. (mri_rhs)).  Rows a part does not touch are written with 0.  y and ydot
 * are device arrays of rtbte_ny() doubles and must not overlap. */
int rtbte_rhs(rtbte_ctx *ctx, const double *y, double *ydot, int32_t parts, void *stream);

/* rtbte_rhs for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as rtbte_rhs (bitwise),
 * but the call allocates nothing: its scratch (the per-work-item row sums,
 * and in mixed precision the FP32 population codes) lives in one static
 * device buffer of rtbte_noalloc_scratch_limit() bytes (32 MiB), which each
 * device the library runs on holds until the process ends.  A context whose
 * shape needs more (rtbte_noalloc_scratch_bytes) gets RTBTE_E_INVAL and must
 * use rtbte_rhs.  Every context on a device shares that device's buffer:
 * calls that can overlap in time (different streams, or different host
 * threads, without ordering between them) race and give wrong results; calls
 * on one stream are ordered and safe.  The kernel launches of this call are
 * not timed by rtbte_profile. */
int rtbte_rhs_noalloc(rtbte_ctx *ctx, const double *y, double *ydot, int32_t parts, void *stream);
/* Static scratch bytes rtbte_rhs_noalloc needs for this context (-1: ctx
 * NULL), and the size of the static buffer. */
int64_t rtbte_noalloc_scratch_bytes(const rtbte_ctx *ctx);
int64_t rtbte_noalloc_scratch_limit(void);

/* Linearized (relaxation-time) rates of the parts in `parts` at the state y:
 * rates[i] = -d(ydot_i)/d(y_i) with every partner population held fixed,
 * i.e. the sum over row i's channels of W times the derivative of the
 * channel's occupation factor (after Eq. (e-ph) and Eq. (ph-ph)) with
 * respect to the row's own population.  With parts = RTBTE_PART_PHPH at
 * phonons in Bose-Einstein equilibrium these are the mode-resolved
 * three-phonon scattering rates (1/fs) the paper analyses its grids with.
 * Same device buffers and stream as rtbte_rhs.  RTBTE_FP64 contexts only
 * (RTBTE_E_UNSUPPORTED otherwise). */
int rtbte_rates(rtbte_ctx *ctx, const double *y, double *rates, int32_t parts, void *stream);

/* The mixed-precision right-hand side at the device state y against the
 * FP64 one from the lists an RTBTE_MIXED context keeps when created with
 * fp64_check > 0: err[inst] (HOST, n_inst doubles, may be NULL) =
 * ||f_mixed(y) - f_fp64(y)|| / ||f_fp64(y)|| in the 2-norm over each
 * instance's rows (0 when both vanish).  Also recorded for rtbte_stats.
 * Two right-hand sides, not counted in the statistics; synchronizes
 * `stream`.  RTBTE_E_UNSUPPORTED for FP64 contexts and for mixed contexts
 * without the FP64 lists. */
int rtbte_check_fp64(rtbte_ctx *ctx, const double *y, double *err, void *stream);

/* Energy-resolved averages of one instance's populations (the zone averages
 * the paper plots beside the band structure and the phonon dispersion,
 * Results, Fig. 1).  which = 0: carriers f binned by the band energy eps;
 * which = 1: phonons N binned by hbar omega.  Bin k covers
 * [e_lo + k de, e_lo + (k+1) de), de = (e_hi - e_lo) / n_bins; states outside
 * [e_lo, e_hi) are left out.  y (and y_ref, may be NULL) are device states of
 * rtbte_ny() doubles; out is HOST memory of 3 n_bins doubles receiving, per
 * bin, the state count, the mean population and the mean of y - y_ref (0
 * without y_ref).  Sums run in a fixed order (bitwise reproducible).  The call
 * allocates a small device index, synchronizes `stream` and returns when out
 * is written.  RTBTE_E_INVAL for a bad instance, `which`, bin count or range. */
int rtbte_energy_average(rtbte_ctx *ctx, const double *y, const double *y_ref, int32_t inst, int32_t which,
                         double e_lo, double e_hi, int32_t n_bins, double *out, void *stream);

/* Effective temperature of each phonon branch of one instance (the branch
 * temperatures of the paper's supplementary analysis): T_m solves
 * sum_{j in m} hw_j N_BE(hw_j, T_m) = sum_{j in m} hw_j N_j over the branch's
 * states with hw_j > 0 (Bose-Einstein occupations carrying the branch's
 * energy), found by bisection in log T over [1e-2, 1e7] K; T_m = 0 when the
 * branch energy is not positive.  mode_of (HOST, the instance's n_ph entries)
 * gives each phonon state's branch in [0, n_modes); T_out is HOST memory of
 * n_modes doubles.  y is a device state; the call synchronizes `stream`.
 * RTBTE_E_INVAL for a bad instance, branch count or branch index. */
int rtbte_mode_temperatures(rtbte_ctx *ctx, const double *y, int32_t inst, const int32_t *mode_of,
                            int32_t n_modes, double *T_out, void *stream);

/* Adaptive Zonneveld 4(3) ERK (Methods, ERK method) on the full RHS, every
 * instance with its own t, step size and PID history, until every instance
 * reaches t_out (one_step = 0) or has taken one accepted step (one_step = 1).
 * y (device) is updated in place; t[inst] and h[inst] (device) hold the
 * current time and the next step size on return.  h[inst] <= 0 asks for a
 * starting step (Hairer-Norsett-Wanner estimate).  The PID error history is
 * kept in the context between calls (rtbte_reset clears it).
 * On RTBTE_E_STEP / RTBTE_E_NONFINITE, y and t hold the last accepted state. */
int rtbte_step_adaptive(rtbte_ctx *ctx, double *y, double *t, double *h, double t_out,
                        int32_t one_step, void *stream);

/* Fixed-step classical RK4 on the full RHS (the prior-work baseline):
 * n_steps steps of size h_step from *t (device t, one entry per instance).
 * A step whose result is not finite, or whose root mean square overflows,
 * is not taken, and the call returns RTBTE_E_NONFINITE with y and t at the
 * last state reached; fixed fast steps inside the multirate and splitting
 * steps are checked the same way.  A step too long for the fastest
 * scattering rates (the paper's failure mode of fixed steps) can also blow
 * the populations up to large finite values, which are returned as they are. */
int rtbte_step_rk4(rtbte_ctx *ctx, double *y, double *t, double h_step, int64_t n_steps,
                   void *stream);

/* Third-order MIS multirate method (Methods, MRI method; Eq. (mis_coef) with
 * the Knoth-Wolke 3-stage base method): slow part I^{ph-ph} at fixed step
 * h_slow, fast part I^{e-ph} + I^{ph-e} integrated over each stage interval
 * with forcing, by the fast integrator chosen in the options.  Advances to
 * t_out (the last slow step is shortened to land on it) or by one slow step
 * (one_step = 1).  h_fast[inst] (device) carries each instance's adaptive
 * fast step.  In a batched context the slow steps are common: every
 * instance must be at the same t (RTBTE_E_UNSUPPORTED otherwise), and each
 * integrates its fast part with its own adaptive steps; an instance computes
 * exactly what it computes alone.  On an error (a fast solve that fails its
 * error test max_fails + 1 times in a row, a non-finite value) y and t hold
 * the state at the start of the slow step that failed; the slow steps before
 * it are kept.  The first call allocates one state-sized work vector kept by
 * the context. */
int rtbte_step_multirate(rtbte_ctx *ctx, double *y, double *t, double *h_fast, double t_out,
                         double h_slow, int32_t one_step, void *stream);

/* MIS multirate with an adaptive slow step (the extension the paper names
 * for future work in its Discussion: both time steps chosen from
 * tolerances).  The paper gives no slow error estimator; this one is step
 * doubling (Hairer, Norsett & Wanner, Solving ODEs I, II.4): an attempt of
 * size H takes one MIS step of H and two of H/2 from the same state, keeps
 * the two-half-step result, and estimates its local error as
 * (y_half - y_full) / 7 (the MIS order being 3).  The estimate's WRMS norm
 * with the options' rtol, atol_el and atol_ph (weights from the state at the
 * start of the attempt) decides acceptance; the next H is
 * H safety eps^(-1/4), limited as for the ERK controller (eta_max,
 * eta_max_first on the first accepted step, eta_fail_min .. eta_fail_max
 * (and eta_fail_repeat from the small_nef-th consecutive failure) on
 * rejection, at most max_fails consecutive rejections).  The fast part is
 * integrated as in rtbte_step_multirate (full step, then the two halves, the
 * fast solver's state carried through all three).
 * h_slow[inst] (device, one entry per instance) holds the first slow step
 * (must be > 0) and receives the next proposed one; t (device) and y are
 * updated after every accepted step, so on an error they hold the last
 * accepted state.  Advances to t_out (the last step shortened to land) or by
 * one accepted step (one_step = 1).  In a batched context the slow steps are
 * common: every instance must be at the same t with the same h_slow
 * (RTBTE_E_UNSUPPORTED otherwise), a slow step is accepted only when every
 * instance's WRMS error is at most 1 (the controller takes the largest
 * instance norm), and each instance integrates its fast part with its own
 * steps; a batch of identical instances steps exactly as one alone.
 * The first call allocates three state-sized work vectors kept by the
 * context. */
int rtbte_step_multirate_adaptive(rtbte_ctx *ctx, double *y, double *t, double *h_fast, double *h_slow,
                                  double t_out, int32_t one_step, void *stream);

/* First-order operator splitting (the alternative the paper compares MIS
 * with, Results, Fig. 3): each step of h_slow advances the fast part
 * I^{e-ph} + I^{ph-e} over the step by RK4 substeps of h_fast (the last one
 * cut to land), then the slow part I^{ph-ph} over the same interval by one
 * RK4 step.  Advances t (device, one entry per instance) to t_out, the last
 * step shortened to land.  In a batched context the steps are common: every
 * instance must be at the same t (RTBTE_E_UNSUPPORTED otherwise). */
int rtbte_step_split(rtbte_ctx *ctx, double *y, double *t, double h_fast, double h_slow, double t_out,
                     void *stream);

/* Clear the integrator state kept between calls (PID histories, counters,
 * the last FP64 check and its poll count). */
int rtbte_reset(rtbte_ctx *ctx);
int rtbte_get_stats(const rtbte_ctx *ctx, int32_t inst, rtbte_stats *out);

/* Launch shape in use: electron and phonon rows per group, channels per item. */
int rtbte_get_tuning(const rtbte_ctx *ctx, int32_t *group_rows_el, int32_t *group_rows_ph,
                     int64_t *item_channels);
/* Channel storage in use: the RTBTE_W_* format of a mixed context (-1 for
 * FP64 plain 16-byte channels, -2 for FP64 packed 12-byte channels), bytes
 * per stored channel, and the bound on the relative rounding of a stored
 * weight (mixed: before the FP32 product with its block scale; FP64 plain
 * and FP64 packed with at most 2^14 states per instance: 0). */
int rtbte_get_weight_format(const rtbte_ctx *ctx, int32_t *format, int32_t *bytes_per_channel,
                            double *weight_rounding);
/* Where the shape came from: *source = 0 given or default, 1 tuned at create
 * (then *rhs_ms is the measured time of one right-hand side), 2 tune cache. */
int rtbte_get_tuning_source(const rtbte_ctx *ctx, int32_t *source, double *rhs_ms);
/* Number of HIP graph launches made by the stepping calls (use_graph). */
int64_t rtbte_graph_launches(const rtbte_ctx *ctx);

/* Checkpoint of the integrator state kept in the context (PID histories,
 * step sizes, counters, health bits; not y, which the caller owns).  With buf == NULL,
 * *len receives the size needed. */
int rtbte_get_state(const rtbte_ctx *ctx, void *buf, size_t *len);
int rtbte_set_state(rtbte_ctx *ctx, const void *buf, size_t len);

/* Timing of the collision-kernel launches (the dominant kernels): with
 * enable = 1 every launch is bracketed by HIP events on its own stream.
 * rtbte_profile resets the totals; rtbte_profile_read synchronises the device
 * and returns the summed kernel time (ms), the number of launches and their
 * summed algorithmic bytes: every stored channel of the evaluated parts once
 * at its storage size (FP64: 12 B packed, 16 B plain; mixed: 8 B packed
 * words, 10 B for the 16-bit-head formats, plus 4 B per 512 channels for
 * the block scales), the state read once (8 B per state; mixed: its 4-byte
 * population code), and the group and item tables (40 B per group; 24 B
 * item record, 4 B order entry and 128 B of row sums per item). */
int rtbte_profile(rtbte_ctx *ctx, int32_t enable);
int rtbte_profile_read(rtbte_ctx *ctx, double *total_ms, int64_t *launches, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* RTBTE_H */
