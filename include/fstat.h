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
#define FSTAT_MIXED 2  /* FP64 phase + SPA time + solve; FP32 response, products
                          and Kahan-compensated partition sums                */

/* flags */
#define FSTAT_DEVICE_PTRS 1u  /* all array arguments are device pointers    */
#define FSTAT_EVAL_MIXED 2u   /* fstat_eval: use the mixed-precision path   */
#define FSTAT_PROFILE 4u      /* fstat_opts.flags: time the bin-loop kernel  */
#define FSTAT_EVAL_SURROGATE 8u /* fstat_eval / pso_stage: learned eccentric
                                   phase for particles with Np >= 16        */
#define FSTAT_AUTOTUNE_FORCE 16u /* fstat_autotune: ignore the cache         */
#define FSTAT_EVAL_EXACT 32u  /* fstat_eval / pso_stage / fstat_autotune: the
                                 exact template at every bin instead of the
                                 per-work-item interpolation of its smooth
                                 factors (same result to ~1e-12)             */

typedef struct fstat_plan_s *fstat_plan_t;

typedef struct {
  double T_obs;        /* observation length [s] (support = [0, T_obs])        */
  double df;           /* bin spacing [Hz], > 0                                */
  int64_t k_lo;        /* first bin index, >= 1                                */
  int64_t nbins;       /* number of bins, >= 1                                 */
  const double *data;  /* s(f_j), complex [nbins] (interleaved)                */
  const double *psd;   /* one-sided S_n(f_j) > 0, [nbins]                      */
} fstat_data_desc;

typedef struct {
  int32_t precision;   /* mask of FSTAT_FP64 | FSTAT_MIXED; 0 = both           */
  uint32_t flags;      /* FSTAT_DEVICE_PTRS: data/psd are device pointers      */
  int32_t chunk;       /* bins per work item (bin tile); 0 = 2048              */
  int32_t reserved;
  double refine_budget; /* FP64 interpolating loop: partitions where the
                           interpolation error could move F by more than this
                           (relative; bound 2 cond(M) e) are evaluated again
                           exactly.  0 = 1e-9; < 0 = never                   */
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
 * FSTAT_DEVICE_PTRS (params, amps and out all on the device).           */
int fstat_waveform(double T_obs, double df, int64_t k_lo, int64_t nbins, const double *params6,
                   const double *amps4, double *out, uint32_t flags, void *hip_stream);

/* Autotuner for the bin loop: times fstat_eval of `params` (device pointers,
 * n particles, uniform np) for work items of 256..8192 bins and persistent
 * grids of 1, 2, 4 times the resident occupancy, keeps the fastest for the
 * precision selected by flags (FSTAT_EVAL_MIXED) in the plan, and returns it.
 * Results are cached in the text file named by $FSTAT_TUNE_CACHE (if set),
 * keyed by GPU architecture, band size, Np class and precision;
 * FSTAT_AUTOTUNE_FORCE re-measures.  Requires FSTAT_DEVICE_PTRS; waits for
 * completion.  best_ms is -1 when the value came from the cache.          */
int fstat_autotune(fstat_plan_t plan, const double *params, int64_t n, int32_t np_uniform,
                   uint32_t flags, int32_t *best_chunk, int32_t *best_mult, double *best_ms,
                   void *hip_stream);

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
 * are written when the call returns.  EINVAL on bad sizes or boxes.       */
int pso_stage(fstat_plan_t plan, const pso_stage_desc *desc, pso_result *result, void *hip_stream);

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
 * interpolation error to matter (FP64 path only).  Waits for hip_stream.
 * EINVAL before the first evaluation.                                      */
int fstat_interp_stats(fstat_plan_t plan, int64_t *items, int64_t *rejected, int64_t *refined,
                       void *hip_stream);

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
 * surrogate and that fell back to the analytic template.                  */
int fstat_surrogate_stats(fstat_plan_t plan, int64_t *used, int64_t *fallback);

/* Release the plan and its device memory (NULL is ignored). */
void fstat_plan_destroy(fstat_plan_t plan);

/* Message for the most recent failure in this thread ("" if none). */
const char *fstat_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSTAT_H */
