/*
 * vfisv.h -- C ABI of libvfisv.so, the MI355X (gfx950) Milne-Eddington
 * Stokes-vector inverter.
 *
 * The library implements the per-pixel inversion of Borrero et al.,
 * "VFISV: Very Fast Inversion of the Stokes Vector for the Helioseismic and
 * Magnetic Imager" (arXiv:0901.2702): for every pixel a Levenberg-Marquardt
 * fit (Sect. 2, Eqs. 1-6; Sect. 4.2, Table 2) of a Milne-Eddington model,
 * synthesised with Voigt / Faraday-Voigt profiles and analytic derivatives
 * (Sect. 3.1-3.2, Eqs. 7-9; Sect. 4.4) and observed through a linear filter
 * (Sect. 5 and 7: profiles convolved with the HMI filters).
 *
 * Conventions
 *  - Every function returns an int status (VFISV_OK = 0 or a negative
 *    VFISV_E_* code) and never throws.  On a validation error nothing is
 *    enqueued and no output is written; vfisv_last_error() explains.
 *  - "dev" pointers are device memory of the context's HIP device, owned by
 *    the caller, kept alive until the stream has been synchronised.  "host"
 *    pointers are read during the call only.
 *  - stream is a hipStream_t passed as void* (NULL: the null stream).  Work
 *    is enqueued asynchronously; the caller synchronises.
 *  - A context is not thread-safe: use one per host thread, or lock.  The
 *    inversions of one context share its pixel-queue heads and counters:
 *    they must not be in flight at the same time (enqueue them on one
 *    stream, or use one context per stream).
 *
 * Model parameters (API order and units), 10 per pixel, float32:
 *   0 B [G], 1 inclination gamma [deg], 2 azimuth psi [deg],
 *   3 line-of-sight velocity [km/s] (positive = redshift),
 *   4 Doppler width [mA], 5 damping a, 6 eta0 (line-to-continuum absorption
 *   ratio), 7 S0, 8 S1 (source function S0 + S1 tau), 9 filling factor alpha.
 *   Fitted models lie in the box B [0, 5000], gamma [0, 180], psi [0, 180]
 *   (0 and 180 are the same azimuth; values just below 180 round to 180 in
 *   float32), v [-20, 20], Doppler width [5, 150], a [0, 5], eta0
 *   [1e-3, 1e3], S0 [-1, 3], S1 [0, 5], alpha [0, 1].
 *   (Sect. 2 model vector with the macroturbulence fixed at zero, which
 *   Sect. 4.1 shows can be dropped.)
 *
 * Stokes data of one pixel: [4][n_obs] float32, rows I, Q, U, V.
 */
#ifndef VFISV_H
#define VFISV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VFISV_NPAR 10

/* Return codes. */
#define VFISV_OK 0
#define VFISV_E_INVALID (-1)     /* bad argument: null pointer, bad size,   */
                                 /* non-finite or negative weight/filter   */
#define VFISV_E_DEVICE (-2)      /* HIP error (message in last_error)       */
#define VFISV_E_NOMEM (-3)       /* device or host allocation failed        */
#define VFISV_E_UNSUPPORTED (-4) /* valid request the library cannot serve */

/* Per-pixel status word: low 4 bits = exit code. */
#define VFISV_CONVERGED 0  /* relative chi^2 decrease below rel_tol      */
#define VFISV_MAX_ITER 1   /* max_iter trial syntheses used              */
#define VFISV_STALLED 2    /* damping eps grew above eps_max             */
#define VFISV_NONFINITE 3  /* non-finite input: params and chi2 are NaN  */

typedef struct vfisv_ctx vfisv_ctx;
typedef struct vfisv_instrument vfisv_instrument;

/* Instrument: a Zeeman-triplet line (Table 1; Eq. 7 gives its splitting
 * from lambda0 and g_eff) synthesised on n_fine wavelengths and observed
 * through a linear filter (n_obs x n_fine), e.g. the six HMI filter
 * positions of Sect. 1.  Taps smaller than tap_threshold times the largest
 * tap of their row are dropped (0 keeps every non-zero tap); the sum of the
 * dropped taps' magnitudes, relative to the row sum, is reported through
 * vfisv_instrument_info. */
typedef struct {
  double lambda0_A;             /* line centre [A]                      */
  double geff;                  /* effective Lande factor               */
  int n_fine;                   /* synthesis points, 1..4096            */
  const double *fine_offset_mA; /* host [n_fine], offsets from lambda0  */
  int n_obs;                    /* observed samples: 6, or 1..4096 with
                                   a banded filter                      */
  const double *filter;         /* host [n_obs][n_fine], row-major      */
  double tap_threshold;         /* relative; 0 <= t < 1                 */
} vfisv_instrument_desc;

typedef struct {
  int n_active_fine;       /* synthesis points carrying a non-zero tap */
  int n_taps;              /* non-zero taps kept over all rows         */
  double max_dropped_rel;  /* largest dropped tap mass / row sum       */
  double cz_mA_per_G;      /* Eq. 7 splitting constant                 */
  int lm_register_rows;    /* filter rows whose sums the LM pass keeps in
                              registers at once: 6-row filters 5 when the
                              first row to end and the last to start share
                              at most 4 synthesis points (the first is then
                              finished in LDS), else 6; banded filters 4 */
} vfisv_instrument_info;

/* Fit options; vfisv_options_default fills the documented defaults. */
typedef struct {
  int max_iter;        /* trial syntheses per pixel (default 50)            */
  double eps0;         /* initial damping (1e-3)                            */
  double eps_max;      /* stall threshold (1e8)                             */
  double rel_tol;      /* relative chi^2 decrease ending the fit (1e-5)     */
  uint32_t free_mask;  /* bit p set: parameter p free (0x3FF)               */
  int grid_waves;      /* persistent grid size in waves; 0 = auto: the      */
                       /* vfisv_autotune choice for the instrument's layout */
                       /* if there is one, else CUs x occupancy             */
  int chunk_log2;      /* pixel queue block = 2^chunk_log2 consecutive      */
                       /* pixels, 0..20, or -1 = auto (default: the tuned   */
                       /* value, else 8).  Scheduling only: the per-pixel   */
                       /* results do not depend on grid_waves or chunk_log2 */
  int lanes_per_pixel; /* 1 (default) or 2: with 2, HMI-shaped pixels use a  */
                       /* pair of lanes each (half the synthesis points per */
                       /* lane, ~1.7x faster passes) whenever the resident */
                       /* grid can give every pixel two lanes, or all but   */
                       /* at most a tenth of them, which wait for a free    */
                       /* pair (at most 36,044 pixels on MI355X: 1,024      */
                       /* waves of 64 lanes at one wave per SIMD); results  */
                       /* then differ from the one-lane path by float32     */
                       /* rounding of the synthesis sums, and do not depend */
                       /* on the grid.  The learned path's refit uses pairs */
                       /* by the same rule; vfisv_invert_batches keeps one  */
                       /* lane per pixel.                                   */
  int voigt;           /* H and F (Sect. 3.2) by: 0 (default) Weideman's     */
                       /* 16-term rational series; 1 or 2 the Taylor table */
                       /* of Eqs. 10-13 (500 u x 100 a nodes at 0.05, built */
                       /* by the library on first use: a synchronising     */
                       /* allocation) at first or second order.  HMI-shaped */
                       /* instruments only; not in vfisv_invert_batches.     */
  int fixed_iters;     /* 0 (default): exits on convergence, stall or        */
                       /* max_iter.  > 0: the paper's scheme (Sect. 4.2):    */
                       /* exactly fixed_iters trials per pixel (fewer only if */
                       /* it stalls with no restart left), the best model   */
                       /* seen is returned, status carries the restarts     */
                       /* used in bits 8..15.  vfisv_invert only.            */
  int restarts;        /* with fixed_iters: restarts per pixel (default 0).  */
                       /* A restart, due when (a) after 10 trials chi^2 is   */
                       /* not 10x below its first value or (b) 5 trials in a */
                       /* row failed (or the damping passed eps_max),       */
                       /* moves each free parameter of the best model by a  */
                       /* uniform offset of up to 0.1 k prior half-widths   */
                       /* (restart k; B 1500 G, angles 90, v 3, Doppler     */
                       /* width 15, a 0.25, eta0 14.5, S0 0.2, S1 0.2,      */
                       /* alpha 0.4); its evaluation counts as a trial and  */
                       /* the damping carries over.                          */
  uint64_t restart_seed; /* offsets: SplitMix64 output (pixel << 16 | k << 4 */
                       /* | parameter) of the stream seeded with this value */
  double hess_reuse;   /* Sect. 4.4: an accepted step that starts from a    */
                       /* model with chi^2 below this keeps the previous    */
                       /* J^T W J and rebuilds only the gradient (the paper */
                       /* gives no threshold).  0 (default): always rebuilt.*/
                       /* Changes the results (slower convergence where the */
                       /* curvature still changes); >= 0.                   */
  uint32_t fallback_rule; /* learned path only (vfisv_invert_learned): which  */
                       /* pixels are re-fitted after the short fit, from    */
                       /* where, and which fit is kept.  0 (default): pixels */
                       /* with reduced chi^2 above the threshold, from the  */
                       /* combined start, keeping the lower chi^2.  Bits:   */
                       /* VFISV_REFIT_UNCONVERGED, VFISV_REFIT_FROM_DEFAULT, */
                       /* VFISV_REFIT_KEEP_REFIT (all three: the rule as    */
                       /* stated for the learned initialiser's fallback).    */
  int deriv_split;     /* Fig. 6 computes derivatives only after a successful */
                       /* trial.  0: every pass computes the Jacobian of its  */
                       /* model, ahead of the acceptance test (one pass per   */
                       /* trial); k in 1..64: trials run values-only passes  */
                       /* and an accepted model waits for a derivative pass, */
                       /* which a wave runs once k/64 of its live lanes (or  */
                       /* all of them) wait; -1 (default): the              */
                       /* vfisv_autotune choice, else VFISV_DERIV_SPLIT_DEFAULT; */
                       /* the learned path's default is 0 (its short fits    */
                       /* start near the minimum, where most trials need     */
                       /* their Jacobian).                                   */
                       /* Scheduling only: the per-pixel results are the same */
                       /* bits for every value.  Not with fixed_iters.        */
} vfisv_options;

#define VFISV_DERIV_SPLIT_DEFAULT 4

/* vfisv_options.fallback_rule bits (Sect. 5 leaves the fallback open). */
#define VFISV_REFIT_UNCONVERGED 1  /* also re-fit pixels whose short fit did
                                      not end CONVERGED (non-finite input
                                      excepted)                             */
#define VFISV_REFIT_FROM_DEFAULT 2 /* re-fit from the default model, not the
                                      combined start                        */
#define VFISV_REFIT_KEEP_REFIT 4   /* keep the re-fit's result even where its
                                      chi^2 is higher than the short fit's  */

/* Result of vfisv_autotune. */
typedef struct {
  int grid_waves;     /* chosen persistent grid (waves)                 */
  int chunk_log2;     /* chosen pixel-queue block                        */
  double best_ms;     /* sample inversion time with the choice           */
  double default_ms;  /* with the untuned default (-1 if not a candidate) */
  int candidates;     /* configurations timed                            */
  int64_t sample;     /* pixels in the timed sample                      */
  int deriv_split;    /* chosen derivative-pass split (vfisv_options)    */
} vfisv_tuning;

/* Work counters of the most recent vfisv_invert on a context. */
typedef struct {
  int64_t pixels;         /* pixels finished                                */
  int64_t trials;         /* trial syntheses (sum of iters)                 */
  int64_t accepts;        /* accepted trials                                */
  int64_t passes;         /* synthesis passes executed (trials + initial)   */
  int64_t svd_fallbacks;  /* solves that needed the eigen/SVD fallback      */
  int64_t grid_waves;     /* waves launched                                 */
  int64_t hessians;       /* J^T W J updates: initial, restart and accepted */
                          /* models, less those kept by hess_reuse          */
  int64_t derivative_passes; /* passes that computed the Jacobian (all of   */
                          /* them when deriv_split is 0)                     */
  int64_t jacobians;      /* Jacobians the fits need (Fig. 6): one per start */
                          /* and per accepted trial that does not end its fit */
} vfisv_counters;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` (the device is made current on
 * the calling thread).  Allocates the context's device work counters and
 * the histogram bins.  Errors: VFISV_E_INVALID (out == NULL or no such
 * device), VFISV_E_DEVICE, VFISV_E_NOMEM. */
int vfisv_create(vfisv_ctx **out, int device);

/* Free the context (synchronises its device).  NULL is accepted. */
int vfisv_destroy(vfisv_ctx *ctx);

/* Message of the last failed call on ctx (ctx == NULL: of the last failed
 * vfisv_create on this thread).  Valid until the next call on ctx. */
const char *vfisv_last_error(const vfisv_ctx *ctx);

/* Library version string. */
const char *vfisv_version(void);

/* ---- instrument ------------------------------------------------------- */

/* Copy the instrument (line, synthesis grid and filter of Sect. 5: the
 * observed samples are linear combinations of the synthesised profile on
 * the fine grid) to the device; host inputs are copied and the instrument
 * owns its device tables.  Validates sizes (1 <= n_fine, n_obs <= 4096),
 * finiteness and non-negativity of the filter.  Two layouts are served:
 *  - n_obs == 6 (HMI-shaped): taps anywhere on the grid;
 *  - banded (any other n_obs): the kept taps of row i lie within the 16
 *    synthesis points a0 + 4 i .. a0 + 4 i + 15 for one a0, as for a
 *    Gaussian instrumental profile of up to 16 taps on a grid oversampled
 *    4 times (e.g. 112 samples, 15 taps, 464 points).
 * Any other filter returns VFISV_E_UNSUPPORTED. */
int vfisv_instrument_create(vfisv_ctx *ctx, const vfisv_instrument_desc *desc,
                            vfisv_instrument **out);
int vfisv_instrument_info_get(const vfisv_instrument *inst, vfisv_instrument_info *info);
int vfisv_instrument_destroy(vfisv_instrument *inst);

/* ---- options ---------------------------------------------------------- */

void vfisv_options_default(vfisv_options *opt);

/* ---- forward synthesis (Sect. 3; filtered, Sect. 5) ------------------- */

/* For n pixels: the filtered Stokes vector of the model params (dev
 * [n][10]) into stokes (dev [n][4][n_obs]) and, if jac != NULL, its
 * Jacobian into jac (dev [n][4][n_obs][10], per API unit).  If noise !=
 * NULL (dev [n][4][n_obs]) it is added to stokes (not to jac).  Params are
 * used as given (no projection).  n == 0 is a no-op. */
int vfisv_synthesize(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                     const float *params, const float *noise, float *stokes,
                     float *jac, void *stream);
/* The same with the Voigt evaluation chosen as in vfisv_options.voigt
 * (0, 1 or 2; 1 and 2 need an HMI-shaped instrument). */
int vfisv_synthesize_voigt(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                           const float *params, const float *noise, float *stokes,
                           float *jac, int voigt, void *stream);

/* ---- inversion (Sects. 2 and 4) --------------------------------------- */

/* Invert n pixels.
 *   stokes: dev [n][4][n_obs] observed profiles.
 *   W:      dev weights w^2/sigma^2 of Eq. 1: [4][n_obs] shared by all
 *           pixels, or [n][4][n_obs] when W_per_pixel != 0.  Must be
 *           finite and >= 0 (not checked on the device; a pixel with a
 *           non-finite weight gets status NONFINITE).
 *   init:   dev [n][10] starting models, or NULL for the default model
 *           (B 1500 G, gamma 90, psi 90, v 0, Doppler width 35 mA, a 0.25,
 *           eta0 15.5, S0 0.3, S1 0.7, alpha 0.6).
 *   params: dev [n][10] best model (float32, API units).
 *   chi2:   dev [n] reduced chi^2 of Eq. 1 at params (float64).
 *   iters:  dev [n] trial syntheses used.
 *   status: dev [n] status word, or NULL.
 * Per-pixel numerical trouble never fails the call; it is reported in
 * status.  n == 0 enqueues nothing.  4*n_obs - (free parameters) must be
 * > 0.  With a banded instrument the pass reads an interleaved copy of
 * stokes (16 bytes per pixel and sample) that the call makes first, in a
 * context buffer that grows when a larger batch comes (the growth
 * allocates and waits for the device; calls after it allocate nothing). */
int vfisv_invert(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                 const float *stokes, const float *W, int W_per_pixel,
                 const float *init, const vfisv_options *opt, float *params,
                 double *chi2, int32_t *iters, int32_t *status, void *stream);

/* Several batches in one persistent launch (e.g. fine-spectrum and
 * HMI-shaped pixels together).  Each batch has its own instrument, pixels,
 * weights, optional start and outputs, with the same meaning as the
 * arguments of vfisv_invert; all share opt (the degrees of freedom of
 * Eq. 1 follow each batch's instrument).  Every wave of the launch works
 * through the batches in the order given, moving on when the current
 * batch has no pixel left, so put the batch with the most work per pixel
 * first: the later batches then fill the waves that the earlier ones leave
 * idle.  1 <= n_batches <= 4; batches with n == 0 are allowed.  The
 * per-pixel results equal those of vfisv_invert on each batch alone. */
typedef struct {
  const vfisv_instrument *inst;
  int64_t n;
  const float *stokes;   /* dev [n][4][n_obs]                          */
  const float *W;        /* dev [4][n_obs], or [n][4][n_obs]            */
  int W_per_pixel;
  const float *init;     /* dev [n][10] or NULL (default model)         */
  float *params;         /* dev [n][10]                                 */
  double *chi2;          /* dev [n]                                     */
  int32_t *iters;        /* dev [n]                                     */
  int32_t *status;       /* dev [n] or NULL                             */
} vfisv_batch;
int vfisv_invert_batches(vfisv_ctx *ctx, const vfisv_batch *batches, int n_batches,
                         const vfisv_options *opt, void *stream);

/* Scheduling autotuner: inverts the first `sample` pixels (<= 0: 131072,
 * at most n) of the caller's data, from the default model with opt's fit
 * settings, twice per candidate, timed with HIP events on `stream`: first
 * every derivative-pass split (deriv_split 0, 2, 4, 8, 16, 32;
 * the fixed-iteration scheme only 0) at the default schedule, then at the
 * best split every persistent grid (1, 2, 3, 4, 6 or 8 waves per CU, up to
 * the waves that are resident at once for the layout's kernel) and
 * pixel-queue block (2^4, 2^8, 2^12 pixels).  A sample of m of the n
 * pixels runs on each candidate grid scaled by m / n (at least 8 waves; at
 * most 8 pixels per lane on the default grid, one factor for every
 * candidate), so that every lane inverts as many pixels as
 * in the whole launch and the tail weighs about as much as it will there.
 * The fastest is kept for this
 * instrument's layout in the context; later inversions with grid_waves == 0,
 * chunk_log2 == -1 and deriv_split == -1 use it.  default_ms is the time of
 * the untuned default (split VFISV_DERIV_SPLIT_DEFAULT, default schedule).
 * Results go to library scratch (the caller's outputs are not touched) and
 * are identical for every candidate, so only speed changes.  Allocates and
 * synchronises: call it at set-up, not under graph capture.  out may be
 * NULL.  Overwrites the work counters. */
int vfisv_autotune(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                   const float *stokes, const float *W, int W_per_pixel,
                   const vfisv_options *opt, int64_t sample, vfisv_tuning *out,
                   void *stream);

/* Classical initial guess (Sect. 5: magnetograph / weak-field B and gamma,
 * Jefferies & Mickey 1991; azimuth from the linear polarisation, Auer et
 * al. 1977; velocity from the line position), per pixel from its observed
 * samples at the centroids of the instrument's filter rows:
 *   I_c = max I; v = c * (centre of gravity of I_c - I) / lambda0;
 *   B_par = -sum V I' / (C_Z sum I'^2); B_perp^2 = 4 sum |Q+iU| |I''| /
 *   (C_Z^2 sum I''^2); 2 psi = atan2(sum U, sum Q) (the linear polarisation
 *   integrated over the samples);
 * I', I'' finite differences across the samples; B and gamma from
 * B_par / 0.6 and B_perp / sqrt(0.6) (default filling factor 0.6); Doppler
 * width, damping, eta0 and alpha from the default model; S0, S1 = 0.3 I_c,
 * 0.7 I_c; then the box.  A vanishing sum gives 0 for its estimate; a pixel
 * with non-finite samples gets the default model.
 *   stokes: dev [n][4][n_obs]; params: dev [n][10] (usable as vfisv_invert's
 *   init); pol: dev [n] polarisation level max sqrt(Q^2+U^2+V^2) / I_c, or
 *   NULL.  Needs n_obs >= 3.  Asynchronous on stream. */
int vfisv_init_classical(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                         const float *stokes, float *params, float *pol, void *stream);

/* The two initialisations of Sect. 5 combined: a starting model from
 * elsewhere (normally the network's, vfisv_mlp_forward) keeps all its
 * parameters except that the azimuth is always replaced by the classical
 * one, and B and gamma by the classical ones where the polarisation level
 * is below pol_threshold (0.06 in the paper).  The classical estimates are
 * those of vfisv_init_classical; a pixel with non-finite samples keeps base
 * unchanged.  The result goes through the box.
 *   base: dev [n][10] finite float32; params: dev [n][10] output, may be
 *   the same buffer as base (each pixel reads its row before writing it);
 *   pol: dev [n] or NULL, as for vfisv_init_classical; pol_threshold >= 0
 *   (+inf gives classical B, gamma and azimuth everywhere, 0 only the
 *   azimuth).  Needs n_obs >= 3.  Asynchronous on stream. */
int vfisv_init_combined(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                        const float *stokes, const float *base, float pol_threshold,
                        float *params, float *pol, void *stream);

/* Per-pixel weights of Sect. 4.3 (Eqs. 1, 14, 15) for vfisv_invert with
 * W_per_pixel = 1: W = w^2 / sigma^2 with w_Q = w_U = w_V = 1 and
 *   w_I = 0.7778 |I_c(mu) - I_c| + 0.3                              (Eq. 14)
 *   I_c(mu) = 0.33644 + 1.30590 mu - 1.79238 mu^2 + 2.45050 mu^3
 *             - 1.89979 mu^4 + 0.59943 mu^5                         (Eq. 15)
 * where I_c is the pixel's largest observed intensity, in units of the
 * disk-centre quiet-Sun continuum, and mu (cosine of the heliocentric
 * angle) is clamped to [0, 1].
 *   stokes: dev [n][4][n_obs]; mu: dev [n]; sigma: host [4] noise level
 *   per Stokes parameter (finite, > 0), the same at every sample;
 *   W: dev [n][4][n_obs] output.
 * A pixel with non-finite mu or Stokes-I samples gets NaN weights for I
 * (its inversion then ends with status VFISV_NONFINITE).  Asynchronous on
 * stream. */
int vfisv_stokes_weights(vfisv_ctx *ctx, const vfisv_instrument *inst, int64_t n,
                         const float *stokes, const float *mu, const float *sigma, float *W,
                         void *stream);

/* Work counters of the most recent vfisv_invert or vfisv_invert_batches
 * (synchronises the context's device). */
int vfisv_get_counters(vfisv_ctx *ctx, vfisv_counters *out);

/* Histogram of per-pixel iteration counts (the iters output of an
 * inversion; the paper's fixed-iteration scheme, Sect. 4.2, is replaced here
 * by exits whose cost varies per pixel, and this is its distribution).
 *   iters: dev [n] int32 (may be NULL when n == 0).
 *   hist:  host [n_bins] int64, 1 <= n_bins <= 4096; hist[i] = number of
 *          pixels with iters == i for i < n_bins - 1, the last bin counts
 *          iters >= n_bins - 1 (negative values count in bin 0).
 * Enqueued on `stream` after the work already there, then synchronises that
 * stream and writes hist.  Uses a context-owned device buffer: calls on one
 * context must not overlap.  Exact integer counts. */
int vfisv_iter_histogram(vfisv_ctx *ctx, int64_t n, const int32_t *iters, int n_bins,
                         int64_t *hist, void *stream);

/* ---- damped normal-equation solve (Eqs. 3-5), for verification -------- */

/* For n systems: delta = solution of (H + eps diag H) delta = g on the
 * diagonally equilibrated system (Cholesky, eigen/SVD fallback discarding
 * singular values below 1e-12 of the largest; parameters outside
 * free_mask or without leverage get delta = 0).
 *   H:     dev [n][55] float32, lower triangle packed row by row
 *          (H[p][q], q <= p, at p*(p+1)/2 + q).
 *   g:     dev [n][10] float32; eps: dev [n] float64.
 *   delta: dev [n][10] float64; code: dev [n] int32 (0 Cholesky,
 *          1 fallback, 2 nothing free), or NULL. */
int vfisv_solve(vfisv_ctx *ctx, int64_t n, const float *H, const float *g,
                const double *eps, uint32_t free_mask, double *delta,
                int32_t *code, void *stream);

/* ---- learned initialiser (Sect. 5: network-proposed starting model) --- */

/* A multilayer perceptron n_in -> 256 -> 256 -> 256 -> 10 (exact-erf GELU,
 * bfloat16 weights and activations on the matrix cores, float32
 * accumulation, float32 master weights and Adam state).  Inputs are the
 * pixel's Stokes samples [4][n_obs] flattened, standardised by
 * (x - in_mean) / in_std.  Outputs are ten codes: the field vector
 * (B cos g, B sin g cos 2psi, B sin g sin 2psi) / 3000, then v, Doppler
 * width, a, eta0, S0, S1, alpha standardised by out_mean/out_std [7].  The
 * library owns weights, optimiser state and work buffers. */
typedef struct vfisv_mlp vfisv_mlp;

/* New network with He-initialised weights (seeded).  Host arrays are
 * copied.  Errors: VFISV_E_INVALID (n_in outside 1..1248, the widest input
 * whose 64-row activation tile fits the workgroup's LDS; non-finite or
 * non-positive std), VFISV_E_NOMEM. */
int vfisv_mlp_create(vfisv_ctx *ctx, int n_in, const float *in_mean, const float *in_std,
                     const float *out_mean, const float *out_std, uint64_t seed,
                     vfisv_mlp **out);
int vfisv_mlp_destroy(vfisv_mlp *mlp);

/* Number of float32 parameters (packed W1 [K0][256], b1, W2, b2, W3, b3,
 * W4 [256][32], b4 [32], K0 = n_in rounded up to 32; -1 if mlp is NULL). */
int64_t vfisv_mlp_num_params(const vfisv_mlp *mlp);

/* Number of network inputs n_in (the row length of the stokes arrays the
 * network functions read); -1 if mlp is NULL. */
int vfisv_mlp_num_inputs(const vfisv_mlp *mlp);

/* Copy the float32 parameters to / from host memory (synchronising).
 * set_params also clears the Adam state. n must equal num_params. */
int vfisv_mlp_get_params(vfisv_mlp *mlp, float *host, int64_t n);
int vfisv_mlp_set_params(vfisv_mlp *mlp, const float *host, int64_t n);

/* Inference for n pixels: stokes dev [n][4*n_obs] -> codes dev [n][10]
 * and/or params dev [n][10] (decoded, projected into the parameter box).
 * At least one output must be given.  Internal buffers grow on first use
 * (a synchronising allocation). */
int vfisv_mlp_forward(vfisv_ctx *ctx, vfisv_mlp *mlp, int64_t n, const float *stokes,
                      float *codes, float *params, void *stream);

/* Gradient of the mean squared error over all n x 10 codes (no update):
 * targets dev [n][10]; grad dev [num_params]; loss dev [1] (sum of squared
 * errors) or NULL.  n must be a positive multiple of 32. */
int vfisv_mlp_gradient(vfisv_ctx *ctx, vfisv_mlp *mlp, int64_t n, const float *stokes,
                       const float *targets, float *grad, double *loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch of rows
 * `rows` (dev int32 [batch], indices into stokes [.][n_in] and targets
 * [.][10]; every index must address a row of both, which is not checked);
 * batch a positive multiple of 32.  The summed squared error
 * accumulates until vfisv_mlp_take_loss. */
int vfisv_mlp_train_step(vfisv_ctx *ctx, vfisv_mlp *mlp, const float *stokes,
                         const float *targets, const int32_t *rows, int batch, float lr,
                         void *stream);

/* Summed squared error of the training steps since the last call
 * (synchronising; resets the sum). */
int vfisv_mlp_take_loss(vfisv_mlp *mlp, double *sum_sq);

/* Normalisation of a training set (Sect. 5 trains on synthetic, filtered,
 * noisy profiles): per input column the mean and standard deviation of
 * stokes [n][n_in], per code 3..9 (v .. alpha, coded as they are) those of
 * params [n][10]; population deviations, floored at 1e-6.  Pass them to
 * vfisv_mlp_create.  stokes, params: dev float32; outputs: host [n_in] and
 * [7].  n >= 2, 1 <= n_in <= 1248.  Allocates and synchronises. */
int vfisv_mlp_stats(vfisv_ctx *ctx, int64_t n, int n_in, const float *stokes,
                    const float *params, float *in_mean, float *in_std, float *out_mean,
                    float *out_std, void *stream);

/* Training run of Sect. 5: the network learns the models from the
 * profiles and training stops when the error on a separate control set
 * rises.  Targets are the standardised codes of params (the field vector
 * (B cos g, B sin g cos 2 psi, B sin g sin 2 psi) / 3000, then v .. alpha
 * standardised with the network's output normalisation).  Each epoch visits
 * the training rows in a fresh random order (Fisher-Yates shuffle driven by
 * SplitMix64 seeded with seed + epoch) in batches of `batch` rows (the
 * last partial batch is dropped), one Adam step per batch with a cosine
 * learning rate from lr down to lr * min_lr_frac over the whole run; after
 * each epoch the control error (mean squared code error) is measured.  The
 * weights of the epoch with the lowest control error are kept; the run
 * stops early once the control error is 2% above that best and the best
 * is 3 or more epochs old.  The Adam state is left as the last step made it. */
typedef struct {
  const float *stokes;       /* dev [n][n_in] training profiles           */
  const float *params;       /* dev [n][10] their models (API units)      */
  int64_t n;                 /* >= batch                                   */
  const float *ctrl_stokes;  /* dev [n_ctrl][n_in] control profiles       */
  const float *ctrl_params;  /* dev [n_ctrl][10]                          */
  int64_t n_ctrl;            /* >= 1                                       */
  int epochs;                /* >= 1                                       */
  int batch;                 /* positive multiple of 32, <= 2^20           */
  float lr;                  /* > 0                                        */
  float min_lr_frac;         /* in (0, 1]                                  */
  uint64_t seed;             /* shuffle key                                */
} vfisv_train_spec;

typedef struct {
  int epochs_run;            /* epochs completed                           */
  int best_epoch;            /* epoch whose weights were kept (from 0)     */
  double best_control_mse;   /* its control error                          */
  int64_t steps;             /* Adam steps made                            */
} vfisv_train_report;

/* Runs the training on `stream` (synchronising at every epoch end); the
 * network ends with the best epoch's weights.  train_mse and control_mse
 * (host [spec->epochs], or NULL) receive each completed epoch's mean
 * squared code error on the training batches and on the control set.
 * Allocates scratch for the run (about 50 bytes per training row) and
 * frees it before returning. */
int vfisv_mlp_train(vfisv_ctx *ctx, vfisv_mlp *mlp, const vfisv_train_spec *spec,
                    vfisv_train_report *report, double *train_mse, double *control_mse,
                    void *stream);

/* Versioned binary file: magic, version, sizes, normalisation, parameters
 * and (version 2) the optimiser state -- the Adam step count and both
 * moment vectors, so that a loaded network trains on where the saved one
 * stopped -- then an FNV-1a checksum of all of it.  load reads versions 1
 * (optimiser state zero) and 2 and rejects others and bad checksums. */
int vfisv_mlp_save(vfisv_mlp *mlp, const char *path);
int vfisv_mlp_load(vfisv_ctx *ctx, const char *path, vfisv_mlp **out);

/* The network's input and output normalisation (host arrays [n_in], [n_in],
 * [7], [7]), as given to vfisv_mlp_create or read by vfisv_mlp_load. */
int vfisv_mlp_get_norm(const vfisv_mlp *mlp, float *in_mean, float *in_std, float *out_mean,
                       float *out_std);

/* Learned-start inversion: the network proposes each pixel's starting
 * model, LM runs at most learned_max_iter trials from it, and every pixel
 * whose reduced chi^2 then exceeds chi2_accept (<= 0: the 0.99 quantile of
 * chi^2_dof / dof, vfisv_chi2_quantile) is re-fitted by plain LM with
 * opt->max_iter trials from the paper's combined start (Sect. 5: the
 * network's model with the classical azimuth, and the weak-field B and gamma
 * below 6 % polarisation, as vfisv_init_combined; the default model when
 * n_obs < 3); the better fit is kept, iters counts the trials of both runs
 * and status gets bit 16 (VFISV_FALLBACK_USED).  opt->fallback_rule changes
 * the refit set, start and choice (VFISV_REFIT_* bits).  Pixels with
 * non-finite input (status VFISV_NONFINITE) are never re-fitted.  Buffers as
 * in vfisv_invert (W shared or per pixel); the network must take 4*n_obs
 * inputs.  Library scratch (about 100 bytes per pixel) grows on first use
 * (a synchronising allocation). */
#define VFISV_FALLBACK_USED 16
int vfisv_invert_learned(vfisv_ctx *ctx, const vfisv_instrument *inst, vfisv_mlp *mlp,
                         int64_t n, const float *stokes, const float *W, int W_per_pixel,
                         const vfisv_options *opt, int learned_max_iter, double chi2_accept,
                         float *params, double *chi2, int32_t *iters, int32_t *status,
                         void *stream);

/* The learned path's default acceptance threshold: the q-quantile of a
 * chi-square variable with dof degrees of freedom divided by dof (the
 * reduced chi^2 of Eq. 1 that a pixel fitted to noise of the stated sigma
 * stays below with probability q).  Host computation (regularised
 * incomplete gamma function, bisection to 1e-13 relative); no device work.
 * Errors: VFISV_E_INVALID for dof < 1 or dof > 1e6, q outside (0, 1), out
 * NULL. */
int vfisv_chi2_quantile(int dof, double q, double *out);

/* Per-phase timing of vfisv_invert_learned (measurement aid).  With on != 0,
 * later calls that are not being captured into a graph record HIP events on
 * their stream between the phases (network inference, short fit, selection
 * and combined start, re-fit, merge) and keep the work counters of the
 * short-fit launch apart from those of the re-fit launch.  Enabling creates
 * the events and a 256-byte device buffer (allocates and synchronises);
 * on == 0 releases them.  vfisv_learned_phases_get synchronises with the
 * most recent timed call and reports it (VFISV_E_INVALID if none). */
typedef struct {
  double ms[5];              /* network, short fit, selection + combined
                                start, re-fit, merge (HIP event times)   */
  vfisv_counters short_fit;  /* work of the short-fit launch             */
  vfisv_counters refit;      /* work of the re-fit launch                */
} vfisv_learned_phases;
int vfisv_learned_phase_timing(vfisv_ctx *ctx, int on);
int vfisv_learned_phases_get(vfisv_ctx *ctx, vfisv_learned_phases *out);

/* Allocation-free learned-start inversion, for callers that cannot allocate
 * device memory: code under HIP graph capture, serving loops and harnesses
 * that forbid hipMalloc.  Arguments, kernels and results are those of
 * vfisv_invert_learned (the same bits), but the per-call scratch (about 100
 * bytes per pixel) lies in a fixed device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends, and the call makes
 * no allocation of any kind.  The caller passes inputs and outputs as for
 * vfisv_invert_learned.  Limits and differences:
 *  - n <= VFISV_NOALLOC_MAX_PIXELS, else VFISV_E_INVALID (split the batch);
 *  - banded instruments are read in the API layout (no interleaved copy);
 *    the results are the same;
 *  - options.voigt != 0 needs the Taylor table, which an earlier call that
 *    may allocate builds (else VFISV_E_UNSUPPORTED).
 * Every call on one GPU, from any context or stream, uses that GPU's single
 * array, which keeps the last call's contents: calls that overlap in time on
 * one GPU race and give wrong results; serialise them. */
#define VFISV_NOALLOC_MAX_PIXELS 524288
int vfisv_invert_learned_noalloc(vfisv_ctx *ctx, const vfisv_instrument *inst, vfisv_mlp *mlp,
                                 int64_t n, const float *stokes, const float *W,
                                 int W_per_pixel, const vfisv_options *opt,
                                 int learned_max_iter, double chi2_accept, float *params,
                                 double *chi2, int32_t *iters, int32_t *status, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* VFISV_H */
