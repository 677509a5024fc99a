/*
 * fstat.h -- C ABI of libfstat: batched semi-coherent F-statistic for eccentric
 * inspirals in one TDI-X channel, on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Fu, Wang & Mohanty, "Hierarchical search method for
 * gravitational waves from stellar-mass binary black holes in noisy
 * space-based detector data" (arXiv:2407.10797):
 *   - inner product <a,b> = 4 Re int a conj(b) / S_n df        (Sec. II.A)
 *   - F(Theta_I) = 1/2 N^T M^{-1} N, N^i = <s|A^i>, M^ij = <A^i|A^j>
 *                                   (Sec. II.A, Eq. coherent_F_stat)
 *   - semi-coherent mean over N_seg frequency partitions whose outer limits
 *     are the template's lowest/highest instantaneous frequency during the
 *     observation                  (Sec. II.B, Eq. semi-cohF)
 *   - restricted-PN eccentric waveform (App. A) seen through the zeroth-order
 *     frequency-domain TDI response evaluated at the SPA time (Sec. IV)
 *   - PSO with ring local best and let-them-fly boundaries (Sec. III.A).
 *
 * Conventions shared by every entry point
 *   - Intrinsic parameters theta6 = {t_c [s], Mc [solar masses], delta_mu,
 *     theta [rad] (ecliptic colatitude), phi [rad] (ecliptic longitude),
 *     e0 (eccentricity at 10 mHz GW frequency)}, row-major [n][6] doubles.
 *   - Frequency grid f_j = (k_lo + j) * df, 0 <= j < nbins.
 *   - Complex arrays are interleaved (re, im) doubles.
 *   - Calls are ordered on the HIP stream passed in (NULL = default stream).
 *     With host pointers the call returns after results are copied back;
 *     with FSTAT_DEVICE_PTRS it returns after enqueueing, and results are
 *     valid once the stream is synchronised.
 *   - Return value: FSTAT_OK (0) or a negative FSTAT_E* code; the message of
 *     the most recent failure in the calling thread is fstat_last_error().
 *   - Per-particle physics outcomes are values, not errors: a template whose
 *     instantaneous frequency never enters the band during the observation
 *     gets F_hat = -inf (the let-them-fly fitness of Sec. III.A); a particle
 *     with non-finite or unphysical parameters (Mc <= 0, |delta_mu| >= 1,
 *     e0 < 0) passed through device pointers gets F_hat = NaN (with host
 *     pointers the call fails with FSTAT_EINVAL instead).
 *   - One plan may be used by one stream at a time.
 */
#ifndef FSTAT_H
#define FSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSTAT_OK 0
#define FSTAT_EINVAL (-1)      /* bad argument                         */
#define FSTAT_ENOMEM (-2)      /* device allocation failed             */
#define FSTAT_EDEVICE (-3)     /* HIP runtime / kernel launch failure  */
#define FSTAT_EUNSUPPORTED (-4)

/* precision selectors (fstat_opts.precision is a mask of these bits) */
#define FSTAT_FP64 1   /* everything in FP64                                   */
#define FSTAT_MIXED 2  /* FP64 phase, SPA time, response and solve; the response
                          rounded (or interpolated) in FP32, FP32 products and
                          partition sums of the N-terms                       */

/* flags */
#define FSTAT_DEVICE_PTRS 1u  /* all array arguments are device pointers    */
#define FSTAT_EVAL_MIXED 2u   /* fstat_eval: use the mixed-precision path   */
#define FSTAT_PROFILE 4u      /* fstat_opts.flags: time the bin-loop kernel  */
#define FSTAT_EVAL_SURROGATE 8u /* fstat_eval / pso_stage: learned eccentric
                                   phase for particles with Np >= 16        */
#define FSTAT_AUTOTUNE_FORCE 16u /* fstat_autotune: ignore the cache         */
#define FSTAT_AUTOTUNE_MODE 64u  /* fstat_autotune: also time the exact loop and
                                    keep it for the plan's later evaluations
                                    of that precision when it is faster     */
#define FSTAT_EVAL_EXACT 32u  /* fstat_eval / pso_stage / fstat_autotune: the
                                 exact template at every bin instead of the
                                 per-work-item interpolation of its smooth
                                 factors (same result to ~1e-12)             */

typedef struct fstat_plan_s *fstat_plan_t;

/* TDI channels (Sec. II.A names them; the paper's search uses X alone):
 * first-generation equal-arm Michelson combinations at spacecraft 1, 2, 3 and
 * the combinations with independent instrumental noise
 * A = (Z - X)/sqrt 2, E = (X - 2Y + Z)/sqrt 6, T = (X + Y + Z)/sqrt 3.     */
#define FSTAT_CHANNEL_X 0
#define FSTAT_CHANNEL_Y 1
#define FSTAT_CHANNEL_Z 2
#define FSTAT_CHANNEL_A 3
#define FSTAT_CHANNEL_E 4
#define FSTAT_CHANNEL_T 5
/* fstat_waveform flags: the channel to synthesise (default X)               */
#define FSTAT_WAVEFORM_CHANNEL(c) ((uint32_t)(c) << 8)

typedef struct {
  double T_obs;        /* observation length [s] (support = [0, T_obs])        */
  double df;           /* bin spacing [Hz], > 0                                */
  int64_t k_lo;        /* first bin index, >= 1                                */
  int64_t nbins;       /* number of bins per channel, >= 1                     */
  const double *data;  /* s_c(f_j), complex [n_channels][nbins] (interleaved)  */
  const double *psd;   /* one-sided S_c(f_j) > 0, [n_channels][nbins]          */
  int32_t n_channels;  /* channels with independent noise, 1..6; 0 = 1         */
  int32_t reserved;
  const int32_t *channels; /* [n_channels] FSTAT_CHANNEL_* codes, distinct, or
                          NULL for a single TDI-X channel.  The statistic sums
                          N and M over the channels (Sec. II.A, Eq. aandMN
                          with the inner product summed over channels)       */
} fstat_data_desc;

typedef struct {
  int32_t precision;   /* mask of FSTAT_FP64 | FSTAT_MIXED; 0 = both           */
  uint32_t flags;      /* FSTAT_DEVICE_PTRS: data/psd are device pointers      */
  int32_t chunk;       /* bins per work item (bin tile); 0 = 2048              */
  int32_t reserved;
  double refine_budget; /* FP64 interpolating loop: partitions where the
                           interpolation error could move F by more than this
                           (relative to max(|F|, 1); a first-order estimate
                           from the maximising amplitudes beta = M^{-1} N,
                           the noise-weighted norm of each item's template
                           error and the error of its quadrature M-terms)
                           get their largest-error items evaluated again
                           exactly.  0 = 5e-10; < 0 = never                 */
} fstat_opts;

/* Create a plan: validates the grid (EINVAL on nbins < 1, df <= 0, k_lo < 1,
 * non-finite data or PSD <= 0 when host pointers are given), copies data and
 * PSD to device memory the plan owns, and precomputes the per-bin factors
 * that do not depend on the template (the noise weighting 1/S_n, the f^{-7/6}
 * amplitude of App. A, the bin width factor 4 df of Eq. inner_product, and the
 * template-independent part of the TDI-X transfer).  The caller keeps
 * ownership of `data`; it may be freed after this call returns.            */
int fstat_plan_create(fstat_plan_t *plan, const fstat_data_desc *data, const fstat_opts *opts,
                      void *hip_stream);

/* Batched semi-coherent F-statistic (Sec. II.B, Eq. semi-cohF).
 *   params   [n][6] theta6 per particle
 *   np       [n] partition counts (N_seg) >= 1, or NULL to use np_uniform for all
 *   F_hat    [n]   out: (1/Np) sum_l F_l
 *   F_part   [n][part_stride] out: per-partition F_l (entries l >= Np untouched),
 *            or NULL; part_stride must be >= max Np when given
 *   amps     [n][part_stride][4] out: per-partition maximum-likelihood
 *            amplitudes a_1..a_4 = M^{-1} N (Eq. aandMN3) in the App. B basis
 *            of fstat_waveform (unit template amplitude), the minimum-norm
 *            maximiser when M is singular; 0 for empty partitions and NaN for
 *            invalid particles (entries l >= Np untouched), or NULL
 *   flags    FSTAT_DEVICE_PTRS and/or FSTAT_EVAL_MIXED
 * Partition l covers e_l <= f < e_{l+1}, e_l = f_lo + (f_hi - f_lo) l / Np,
 * with [f_lo, f_hi] the template's frequency range during [0, T_obs] clipped
 * to the band; the last partition is closed.  Empty partitions give F_l = 0.
 * A partition whose 4x4 matrix M has eigenvalue ratio below 1e-12 is solved
 * with the pseudo-inverse.  n = 0 is a no-op.  EINVAL: n < 0, np < 1,
 * part_stride too small, precision not built into the plan.               */
int fstat_eval(fstat_plan_t plan, const double *params, int64_t n, const int32_t *np,
               int32_t np_uniform, double *F_hat, double *F_part, double *amps,
               int64_t part_stride, uint32_t flags, void *hip_stream);

/* Scratch of fstat_eval_noalloc on each device: 128 MiB (fixed). */
#define FSTAT_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* Allocation-free variant of fstat_eval, for callers that cannot allocate
 * device memory during an evaluation: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same statistic, kernels,
 * arguments and results as fstat_eval with FSTAT_DEVICE_PTRS (bit for bit),
 * but the work lists, per-item records and partial sums live in a fixed
 * scratch array of FSTAT_NOALLOC_SCRATCH_BYTES per device, part of the
 * library's device code (it stays allocated until the process ends); the call
 * itself allocates nothing and does not synchronize.
 *   params, np, F_hat, F_part, amps: device pointers, as fstat_eval's
 *   flags    FSTAT_EVAL_MIXED and/or FSTAT_EVAL_EXACT (FSTAT_DEVICE_PTRS is
 *            implied)
 * The scratch holds n x (ceil(nbins / chunk) x channels + part_stride) work
 * items at about 565 bytes each (chunk: the plan's work-item size); with the
 * default 2048-bin items that is e.g. 320 particles at Np = 256 on 20,972
 * bins, or 16,384 particles at Np = 1; larger calls fail with EINVAL and a
 * message giving the bytes needed.
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents (each call initialises what it reads): calls that overlap
 * on one device race, whatever their plans and streams, so serialise them
 * (one stream, or events).  The plan must have been created on the current
 * device (fstat_plan_create takes the scratch's device address there).  The
 * plan's profiling (FSTAT_PROFILE) and fstat_interp_stats do not see these
 * calls.  EINVAL as fstat_eval, and for a plan of another device or a call
 * beyond the scratch; EUNSUPPORTED with FSTAT_EVAL_SURROGATE.              */
int fstat_eval_noalloc(fstat_plan_t plan, const double *params, int64_t n, const int32_t *np,
                       int32_t np_uniform, double *F_hat, double *F_part, double *amps,
                       int64_t part_stride, uint32_t flags, void *hip_stream);

/* Numerical spacecraft orbit for the plan's templates (Sec. IV: a numerical
 * orbit interpolated with Chebyshev polynomials instead of the analytic one).
 *   nodes  [n_seg][3][3][10]: positions of spacecraft 1..3 (x, y, z in
 *          seconds of light travel, the frame of the analytic orbit) at the
 *          Chebyshev points t = t0 + dt (seg + (1 + s_k)/2),
 *          s_k = cos(pi (k + 1/2) / 10), of each segment of length dt
 * Positions between the points are the degree-9 interpolant of the segment
 * that holds t (outside the table, the end segment's).  The table must cover
 * [0, T_obs].  Delays and sinc arguments keep the nominal arm length; the
 * link phases take the tabulated arm vectors.  The plan converts the table to
 * Chebyshev coefficients and keeps its own device copy (the caller's buffer
 * may be reused on return); later fstat_eval, pso_stage and fstat_search
 * calls on this plan use it (fstat_waveform, which takes no plan, does not).
 * n_seg = 0 returns to the analytic orbit.  Flags: FSTAT_DEVICE_PTRS (nodes
 * on the device).  Waits for completion.  Must not overlap an evaluation on
 * the same plan.  EINVAL: null plan or nodes, n_seg < 0, dt <= 0, coverage,
 * non-finite values; ENOMEM / HIP errors leave the previous table in place.  */
int fstat_plan_set_orbit(fstat_plan_t plan, double t0, double dt, int32_t n_seg,
                         const double *nodes, uint32_t flags, void *hip_stream);

/* Extrinsic parameters from the amplitudes (App. B, Eq. extrinPara).
 *   amps    [n][4] a_1..a_4 as fstat_eval writes them
 *   params  [n][6] theta6 of the same rows, or NULL
 *   out     [n][4] out: D_L, iota in [0, pi], psi in (-pi/2, pi/2], phi_c in
 *           (-pi, pi]
 * The arctangents are two-argument: psi = atan2(A+ a4 - Ax a1, -(Ax a2 +
 * A+ a3)) / 2, c = sgn(sin 2 psi) (+1 at 0), phi_c = atan2(c (A+ a4 - Ax a1),
 * -c (Ax a3 + A+ a2)); (psi + pi/2, phi_c + pi) describes the same a.  At
 * iota = 0 or pi only 2 psi +- phi_c is defined and psi = 0 is returned.
 * Without params D_L is in the units of 1/a (the unit template amplitude);
 * with params it is in metres, through the App. A amplitude constant
 * A = -sqrt(5/24) Mc^{5/6} / (pi^{2/3} D_L), whose sign turns phi_c by pi.
 * All-zero a gives (inf, NaN, NaN, NaN).  Flags: FSTAT_DEVICE_PTRS (amps,
 * params and out on the device; the call is then stream-ordered, otherwise
 * it waits).  EINVAL: n < 0, null amps or out, invalid chirp mass (host).  */
int fstat_extrinsic(const double *amps, const double *params, int64_t n, double *out,
                    uint32_t flags, void *hip_stream);

/* Template signal x_X(f_j) = sum_i a_i A^i(f_j) on a grid (for injections):
 * the App. A waveform with phi_c = 0, amplitude f^{-7/6}, through the TDI-X
 * response at the SPA time, with the four real amplitudes a_1..a_4 of
 * Sec. II.A (Eq. response) in the App. B basis; zero outside the template's
 * support during [0, T_obs].  out: complex [nbins] (interleaved).  Flags:
 * FSTAT_DEVICE_PTRS (params, amps and out all on the device),
 * FSTAT_WAVEFORM_CHANNEL(c) for a channel other than X.                   */
int fstat_waveform(double T_obs, double df, int64_t k_lo, int64_t nbins, const double *params6,
                   const double *amps4, double *out, uint32_t flags, void *hip_stream);

/* Autotuner for the bin loop: times fstat_eval of `params` (device pointers,
 * n particles; np [n] partition counts (device) with part_stride their
 * maximum, or np NULL and np_uniform for all) for work items of 256, 512,
 * 1024, 2048, 2560, 4096, 4608 and 8192 bins (those above the interpolating
 * loop's LDS tile, 2560 bins FP64 and 4608 mixed, for the exact loop only) and
 * persistent grids of 1, 2, 4 times the resident occupancy, keeps
 * the fastest for the precision selected by flags (FSTAT_EVAL_MIXED) in the
 * plan, and returns it.  With FSTAT_AUTOTUNE_MODE it times the exact per-bin
 * loop as well and, when that is faster (small batches, where the
 * interpolating loop's node evaluations are a latency chain), makes the
 * plan's later evaluations of that precision use it (the statistic is the
 * same within the parity bars; FSTAT_EVAL_EXACT tunes the exact loop only).
 * Results are cached in the text file named by $FSTAT_TUNE_CACHE (if set),
 * keyed by GPU architecture, band size, Np class (and whether Np varies),
 * precision and mode; FSTAT_AUTOTUNE_FORCE re-measures.  Requires
 * FSTAT_DEVICE_PTRS; waits for completion.  best_ms is -1 when the value came
 * from the cache.                                                          */
int fstat_autotune(fstat_plan_t plan, const double *params, int64_t n, int32_t np_uniform,
                   const int32_t *np, int32_t part_stride, uint32_t flags, int32_t *best_chunk,
                   int32_t *best_mult, double *best_ms, void *hip_stream);

/* ---- particle swarm stage (Sec. III.A; batched runs of Sec. III.B) -------- */
typedef struct {
  int32_t n_runs;      /* independent PSO runs in this launch, >= 1            */
  int32_t n_part;      /* particles per run, 1..1024                           */
  int32_t iters;       /* iterations (fixed-iteration termination), >= 0       */
  int32_t ring_k;      /* neighbours on each side in the ring (lbest); <= 0 or
                          >= n_part/2 selects the global best                  */
  double w_start, w_end; /* inertia weight, linear in the iteration index      */
  double c1, c2;       /* acceleration constants                                */
  double vmax;         /* |v_j| <= vmax in the normalised [0,1]^6 space        */
  uint64_t seed;       /* Philox4x64-10 key word 0 (key word 1 = run index)    */
  const double *box;   /* [n_runs][6][2] search box per run (host pointer)     */
  const int32_t *np;   /* [n_runs] partition count per run (host pointer)      */
  uint32_t flags;      /* FSTAT_EVAL_MIXED selects the mixed-precision F        */
  int32_t use_graph;   /* 1: capture one iteration in a hipGraph and replay    */
} pso_stage_desc;

typedef struct {
  double *best_x;      /* [n_runs][6] physical parameters of each run's gbest   */
  double *best_F;      /* [n_runs] its F_hat                                    */
  double *trace;       /* [iters][n_runs] gbest fitness after each iteration, or NULL */
  double *final_x;     /* [n_runs][n_part][6] final particle positions (normalised), or NULL */
} pso_result;

/* Run `iters` PSO iterations for all runs at once.  Per run r the search box
 * box[r] is mapped to [0,1]^6; initial x ~ U[0,1], v ~ U[-x, 1-x]; each
 * iteration evaluates F_hat for every particle in one batch (particles outside
 * [0,1]^6 get -inf and are not evaluated: let-them-fly), updates personal
 * and ring-local bests (strict improvement, lowest index wins ties), then
 *   v <- w v + c1 r1 (p - x) + c2 r2 (l - x),  v clamped to [-vmax, vmax],
 *   x <- x + v,
 * with r1, r2 ~ U[0,1) drawn per particle, dimension and iteration from
 * Philox4x64-10.  All state stays on the device; results (host pointers)
 * are written when the call returns.  With the environment variable
 * FSTAT_PROGRESS = N > 0 the call waits for the device every N iterations
 * and prints one progress line to stderr.  EINVAL on bad sizes or boxes.  */
int pso_stage(fstat_plan_t plan, const pso_stage_desc *desc, pso_result *result, void *hip_stream);

/* ---- hierarchical search (Sec. III.B, Fig. 2) ------------------------------ */
typedef struct {
  double box[6][2];    /* full search range {lo, hi}: t_c [s], Mc [Msun], delta_mu,
                          theta [rad], phi [rad], e0                              */
  int32_t n_slices;    /* stage 1: the t_c range cut into this many equal,
                          contiguous intervals (paper: 24)                        */
  int32_t runs[3];     /* PSO runs per search space in stages 1..3 (24, 8, 48)  */
  int32_t iters[3];    /* PSO iterations per run (8000, 8000, 15000)            */
  int32_t np[3];       /* N_seg of the statistic (16, 16, 1)                    */
  int32_t n_part;      /* particles per run, 1..1024 (128)                      */
  int32_t ring_k;      /* ring radius of the local best; <= 0: global best      */
  double w_start, w_end, c1, c2, vmax;   /* PSO constants as in pso_stage_desc */
  double width2[2];    /* stage-2 box widths in t_c [s] and Mc [Msun]
                          (0.01 yr, 0.6)                                          */
  double width3[5];    /* stage-3 box widths in t_c [s], Mc [Msun], theta, phi,
                          e0 (0.004 yr, 0.3, 0.4, 0.4, 0.006)                     */
  uint64_t seed;       /* stage s uses PSO seed  seed + s * 0x9E3779B97F4A7C15  */
  uint32_t flags[3];   /* per stage: FSTAT_EVAL_MIXED / _SURROGATE / _EXACT     */
  int32_t use_graph;   /* as in pso_stage_desc                                  */
  int32_t max_stage;   /* stop after this stage (1..3); 0 = 3                   */
  const char *checkpoint; /* text file that keeps the results of finished stages
                          (written after each stage, read to resume), or NULL  */
} fstat_search_desc;

typedef struct {
  int32_t stages_done;      /* out: stages finished (resumed ones included)   */
  int32_t stages_resumed;   /* out: stages taken from the checkpoint           */
  double *stage1_x;         /* [n_slices][6] best of each t_c interval, or NULL */
  double *stage1_F;         /* [n_slices], or NULL                              */
  double *stage2_x;         /* [n_slices][6] best of each stage-2 space, or NULL */
  double *stage2_F;         /* [n_slices], or NULL                              */
  double stage3_x[2][6];    /* best of the stage-3 spaces around theta, pi - theta */
  double stage3_F[2];
  double best_x[6];         /* final intrinsic estimate (stage 3, else the last
                               finished stage's best)                          */
  double best_F;            /* its F_hat at that stage's N_seg                  */
  double amps[4];           /* a_1..a_4 at best_x, fully coherent (N_seg = 1)  */
  double extrinsic[4];      /* D_L [m], iota, psi, phi_c from amps (App. B)    */
  double stage_ms[3];       /* wall time of each stage run here (0: resumed)   */
  int64_t evals[3];         /* template evaluations per stage (runs x n_part x
                               iters over all spaces)                          */
} fstat_search_result;

/* The three-stage search: stage 1 runs runs[0] PSO runs in each of n_slices
 * equal t_c intervals of the full box and keeps the best of each interval;
 * stage 2 centres a box of widths width2 in (t_c, Mc) on each of those, keeps
 * the other parameters' full ranges, runs runs[1] runs in each and keeps the
 * single best over all of them; stage 3 centres boxes of widths width3 in
 * (t_c, Mc, theta, phi, e0) on that point and on its mirror theta -> pi - theta
 * (delta_mu keeps its full range), runs runs[2] runs in each, and the best of
 * the two is the estimate.  Boxes are clipped to the full box, except phi when
 * the full box spans the whole circle (the statistic is periodic in phi).
 * Every MAX takes the first of equal values.  Then the amplitudes a at the
 * estimate (fstat_eval, N_seg = 1, FP64) and the extrinsic parameters
 * (fstat_extrinsic with the chirp mass) are filled in.  All runs of a stage
 * go to one pso_stage call (run index = space * runs + k).  With a checkpoint
 * path, finished stages are read back if the file was written for the same
 * descriptor and grid (else EINVAL) and each newly finished stage is
 * written; max_stage stops early so that a long search can be split over
 * several processes.  Waits for completion.  EINVAL on bad sizes or
 * widths; errors of pso_stage pass through.                               */
int fstat_search(fstat_plan_t plan, const fstat_search_desc *desc, fstat_search_result *result,
                 void *hip_stream);

/* The boxes one stage of fstat_search would search (host arithmetic only, no
 * device call): stage 1 ignores `centres` and gives n_slices boxes; stage 2
 * gives one box per centre (n_centres of them); stage 3 gives the two boxes
 * around centres[0] (theta and pi - theta).  boxes_out: [n][6][2].  Returns
 * the number of boxes, or a negative error code.                          */
int fstat_search_boxes(const fstat_search_desc *desc, int32_t stage, const double *centres,
                       int32_t n_centres, double *boxes_out);

/* Diagnostics for plans created with FSTAT_PROFILE, accumulated since the
 * last reset, from HIP events recorded on the caller's stream: kernel_ms =
 * the whole bin-loop stage (interpolation nodes, tile grouping, the
 * interpolating loop, the exact passes), main_ms = its main kernel alone (the
 * interpolating loop, or the exact loop under FSTAT_EVAL_EXACT); the number
 * of evaluations; the bin-template evaluations performed (sum over particles
 * of their support size).  Waits for the recorded events.  EINVAL without
 * profiling.                                                               */
int fstat_profile_read(fstat_plan_t plan, int reset, double *kernel_ms, double *main_ms,
                       int64_t *launches, int64_t *bin_templates);

/* Work items of the plan's last evaluation and how many took the exact
 * per-bin loop: `rejected` = items the interpolating loop handed over (fewer
 * than 32 bins, or interpolants that missed an end point; all items after an
 * FSTAT_EVAL_EXACT evaluation), `refined` = interpolated items evaluated again
 * exactly because their partition's matrix is ill-conditioned enough for the
 * interpolation error to matter (FP64 path only).  bin_mix [14] (or NULL):
 * bins of the items by the interpolating loop's per-bin work, [0..2] phase
 * polynomial and sine at every bin, at transfer degree 5, 7, 9, [3..5] the
 * FP64 loop's difference recurrence for the template factor, at degree 5, 7,
 * 9 (on the mixed path [0] degree 4 and [2] degree 6 with the phase carried
 * by all nine forward differences, [3] degree 4 and [5] degree 6 with four),
 * [6] handed to the exact loop;
 * [7 + k] (k < 6) the lanes with bins (runs) of the items of kind k, each of
 * which does the kind's per-lane work once, [13] the items handed to the exact
 * loop (EINVAL after an FSTAT_EVAL_EXACT evaluation).  Waits for hip_stream.
 * EINVAL before the first evaluation.                                      */
int fstat_interp_stats(fstat_plan_t plan, int64_t *items, int64_t *rejected, int64_t *refined,
                       int64_t *bin_mix, void *hip_stream);

/* ---- learned surrogate for the eccentric phase (App. A) ------------------- */
/* One forward and backward pass of the surrogate network on the device, for
 * checking its training kernels: 3 -> 256 -> 256 -> 256 -> 256 -> 1 with SiLU,
 * BF16 MFMA operands and FP32 accumulation, mean squared error.
 *   params [198657] FP32 (layout W1[256][3] b1 | W2[256][256] b2 | W3 b3 |
 *          W4 b4 | w5[256] b5), x [B][3], t [B] (host pointers), B a
 *          positive multiple of 64; out: loss, grad [198657], y [B] or NULL.
 * EINVAL on bad sizes.  Allocates and frees its own device buffers.        */
int fstat_mlp_grad(const float *params, const float *x, const float *t, int32_t B, double *loss,
                   float *grad, float *y);

/* Inference-only forward of the same network (the fused kernel that evaluates
 * the surrogate's knots): y[r] for R rows of x [R][3] (host pointers), any
 * R in 1..2^31.  Same operand rounding as the training forward.  EINVAL on
 * bad arguments.  Allocates and frees its own device buffers.             */
int fstat_mlp_forward(const float *params, const float *x, int64_t R, float *y);

/* Train the plan's surrogate for the eccentric phase correction Psi_e
 * (App. A) on the device: n_samples (f, Mc, e0) points uniform over
 * f in [10, 100] mHz, Mc in [10, 50] Msun, e0 in [0, 0.15], targets from the
 * plain template code (Psi_e in units of e0^2 times the Newtonian phase), the
 * last 1/16 held out; `steps` Adam steps of `batch` samples with a cosine
 * step-size decay from `lr`.  Afterwards fstat_eval / pso_stage accept
 * FSTAT_EVAL_SURROGATE: for particles with Np >= 16 the network is evaluated
 * at four knots per partition and interpolated to every bin; a particle keeps
 * it only if, in every partition, the residual against the analytic term at
 * the knots and mid-points (mean removed) implies a mismatch <= 1e-3, else it
 * falls back to the analytic template.  Np = 1 never uses it.
 * EINVAL: batch not a positive multiple of 64, n_samples < 17 batches,
 * steps < 1 or lr <= 0.  Waits for completion.                           */
typedef struct {
  int64_t n_samples;   /* training + held-out samples                           */
  int32_t batch;       /* samples per step, a multiple of 64                    */
  int32_t steps;       /* optimiser steps                                       */
  double lr;           /* initial Adam step size                                */
  uint64_t seed;       /* sample and initialisation seed                        */
  double *loss_trace;  /* [steps] training loss per step (host), or NULL        */
  double val_rmse;     /* out: held-out root-mean-square error (network units)  */
  double val_max;      /* out: held-out max |error| (network units)             */
} fstat_surrogate_desc;
int fstat_surrogate_train(fstat_plan_t plan, fstat_surrogate_desc *desc, void *hip_stream);

/* Particles of the last FSTAT_EVAL_SURROGATE evaluation that used the
 * surrogate and that fell back to the analytic template; flags [n] (host, or
 * NULL): 1 where particle i of that evaluation used the surrogate, else 0
 * (n at most that evaluation's particle count).  EINVAL before any surrogate
 * evaluation or for n beyond the last evaluation.                         */
int fstat_surrogate_stats(fstat_plan_t plan, int64_t *used, int64_t *fallback, int32_t *flags,
                          int64_t n);

/* The surrogate network's weights (host arrays of 198,657 floats in the flat
 * layout of fstat_mlp_grad): `out` (or NULL) receives the plan's trained
 * weights; `in` (or NULL) replaces them and marks the surrogate trained, for
 * reuse of one training across plans.  Waits for completion.  EINVAL: null
 * plan, `out` without a trained surrogate, non-finite weights in `in`.    */
int fstat_surrogate_params(fstat_plan_t plan, const float *in, float *out, void *hip_stream);

/* Measured peaks for the roofline (not part of the statistic): kind
 *   FSTAT_CALIB_FMA64  chains of FP64 fused multiply-adds, `size` rounds of
 *                      128 per lane, 16 blocks of 256 per compute unit;
 *                      rate in TFLOP/s (FMA = 2)
 *   FSTAT_CALIB_FMA32  the same in FP32 (scalar, unpacked instructions)
 *   FSTAT_CALIB_COPY   device-to-device copy of `size` bytes; rate in GB/s
 *                      counting bytes read plus bytes written
 * Each is launched once to warm up, then `reps` times between two events;
 * ms is the average launch.  Allocates (and frees) its own buffers and waits
 * for completion.  EINVAL: unknown kind, size or reps < 1, size above 2^24
 * rounds or 64 GiB.                                                       */
#define FSTAT_CALIB_FMA64 0
#define FSTAT_CALIB_FMA32 1
#define FSTAT_CALIB_COPY 2
int fstat_calibrate(int32_t kind, int64_t size, int32_t reps, double *rate, double *ms,
                    void *hip_stream);

/* Release the plan and its device memory (NULL is ignored). */
void fstat_plan_destroy(fstat_plan_t plan);

/* Message for the most recent failure in this thread ("" if none). */
const char *fstat_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSTAT_H */
