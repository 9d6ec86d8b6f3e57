/*
 * FP64 CPU oracle for the per-pixel Milne-Eddington Stokes inversion of
 * Borrero et al., "VFISV: Very Fast Inversion of the Stokes Vector for the
 * Helioseismic and Magnetic Imager" (arXiv:0901.2702).
 *
 * THIS IS TEST INFRASTRUCTURE.  It is a plain, slow, double-precision
 * restatement of what the inversion computes, used only by the tests, by the
 * package smoke check and by the CPU-baseline leg of the benchmark.  The GPU
 * library never links, includes or calls it, and it shares no code, header,
 * table or constant with the GPU library.
 *
 * Parameter order (API order, units):
 *   0 B [G], 1 gamma [deg], 2 psi [deg], 3 v_los [km/s], 4 Doppler width
 *   [mA], 5 damping a, 6 eta0, 7 S0, 8 S1, 9 filling factor alpha.
 * (Sect. 2 lists the Milne-Eddington model vector; the macroturbulence is
 * held at zero, Sect. 4.1.)
 *
 * Stokes arrays of one pixel are laid out [4][n_obs] (I, Q, U, V rows).
 */
#ifndef VFISV_ORACLE_H
#define VFISV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NPAR 10

enum {
  ORC_B = 0, ORC_GAMMA, ORC_PSI, ORC_VLOS, ORC_DLD, ORC_A, ORC_ETA0,
  ORC_S0, ORC_S1, ORC_ALPHA
};

/* Exit codes of one pixel (low bits of the status word). */
enum { ORC_CONVERGED = 0, ORC_MAX_ITER = 1, ORC_STALLED = 2, ORC_NONFINITE = 3 };

/* A spectral line observed through a linear instrument (Sect. 3.1, Table 1,
 * Eq. 7; the filter is the instrument's linear map from the synthesis grid
 * to the observed samples). */
typedef struct {
  double lambda0_A;              /* line centre [A] */
  double geff;                   /* effective Lande factor */
  int n_fine;                    /* synthesis grid points */
  const double *fine_offset_mA;  /* [n_fine] offsets from lambda0 [mA] */
  int n_obs;                     /* observed wavelengths L */
  const double *filter;          /* [n_obs][n_fine] row-major */
  int voigt;                     /* H, F by: 0 the Faddeeva function itself,
                                    1 or 2 the Taylor table of Eqs. 12-13 at
                                    first or second order */
} orc_instrument;

typedef struct {
  int max_iter;        /* trial syntheses allowed */
  double eps0;         /* initial Levenberg-Marquardt damping */
  double eps_max;      /* damping above which the pixel is declared stalled */
  double rel_tol;      /* relative chi^2 decrease that ends the fit */
  uint32_t free_mask;  /* bit p set: parameter p is free */
  int fixed_iters;     /* > 0: the paper's scheme (Sect. 4.2): exactly this
                          many trials per pixel, no exit on convergence, the
                          best model seen is the result */
  int restarts;        /* with fixed_iters: restarts from a perturbed best
                          model allowed per pixel (triggers (a) and (b) of
                          Sect. 4.2) */
  uint64_t seed;       /* key of the restart perturbations */
  double hess_reuse;   /* Sect. 4.4: an accepted step from a model whose chi^2
                          is below this keeps the previous J^T W J and only
                          rebuilds the gradient; 0 rebuilds every time */
} orc_options;

typedef struct {
  int64_t trials;       /* trial syntheses (values only) */
  int64_t derivs;       /* syntheses with derivatives (initial + accepted) */
  int64_t solves;       /* damped normal-equation solves */
  int64_t svd_fallbacks;/* solves that needed the eigen/SVD fallback */
  int64_t hessians;     /* J^T W J built (initial, restarts, accepted steps
                           not covered by hess_reuse) */
} orc_counters;

/* Faddeeva function w(u + i a) = H + i F for a >= 0 (Sect. 3.2). */
void orc_faddeeva(double u, double a, double *H, double *F);
void orc_faddeeva_batch(int64_t n, const double *u, const double *a, double *H, double *F);

/* Taylor-table evaluation of H and F (Sect. 3.2, Eqs. 10-13): a table of H
 * and F at u = 0.05 i (i < 500) and a = 0.05 j (j < 100), built from
 * orc_faddeeva; H and F at (u, a) are extrapolated from the nearest node
 * with the first (order 1) or the first and second (order 2) derivatives of
 * Eqs. 8-11.  H is even and F odd in u.  Where |u| is beyond the last
 * node's cell (>= 24.975) the asymptotic series of w(z) for large |z| is
 * used instead; a is clamped to the last node (the model's box ends at
 * a = 5).  The table is built once per process, on first use. */
enum { ORC_VT_NU = 500, ORC_VT_NA = 100 };
#define ORC_VT_STEP 0.05
void orc_voigt_taylor(int order, double u, double a, double *H, double *F);
void orc_voigt_taylor_batch(int order, int64_t n, const double *u, const double *a, double *H,
                            double *F);
/* The table node values (for tests): H and F at (u_i, a_j). */
void orc_voigt_table_node(int i, int j, double *H, double *F);

/* Zeeman splitting constant of Eq. 7 [mA per G]. */
double orc_zeeman_constant(double lambda0_A, double geff);

/* Stokes vector on the synthesis grid and, if dS != NULL, its derivatives.
 * S: [4][n_fine]; dS: [4][n_fine][10] (derivatives per API unit). */
void orc_synth_fine(const orc_instrument *inst, const double *M, double *S, double *dS);

/* Observed (filtered) Stokes vector and optional Jacobian.
 * S: [4][n_obs]; J: [4][n_obs][10]. */
void orc_forward(const orc_instrument *inst, const double *M, double *S, double *J);

/* Box projection with the exact symmetries of the model. */
void orc_project(double *M);

/* Damping update of Table 2. */
double orc_eps_decrease(double eps);
double orc_eps_increase(double eps);

/* Damped solve (H + eps diag H) delta = g on the equilibrated system.
 * Returns 0 if the Cholesky factorisation succeeded, 1 if the eigen/SVD
 * fallback was used, 2 if nothing was free. */
int orc_solve(const double *H, const double *g, double eps, uint32_t free_mask,
              double *delta);

/* Default initial model (prior midpoints). */
void orc_default_init(double *M);

/* One pixel: Levenberg-Marquardt from M0.
 * obs: [4][n_obs] (float, promoted); W: [4][n_obs] weights w^2/sigma^2.
 * M0 may be NULL (default model).  pixel keys the restart perturbations.
 * In the fixed-iteration mode the status word carries the restarts used in
 * bits 8..15. */
void orc_lm_pixel(const orc_instrument *inst, const orc_options *opt,
                  const float *obs, const float *W, const double *M0, int64_t pixel,
                  double *M_out, double *chi2_out, int32_t *iters_out,
                  int32_t *status_out, orc_counters *cnt);

/* SplitMix64 (Steele, Lea and Flood 2014) used as a counter-based
 * generator: the c-th output (c >= 0) of the stream seeded with seed. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t c);
/* Uniform in [0, 1) for restart k of a pixel and parameter p: output number
 * (pixel << 16 | k << 4 | p) of the stream, top 53 bits. */
double orc_restart_uniform(uint64_t seed, int64_t pixel, int k, int p);

/* Batch over pixels with a pool of nthreads (<=0: all hardware threads).
 * stokes: [n][4][n_obs]; W: [4][n_obs] or [n][4][n_obs] if W_per_pixel;
 * init: [n][10] or NULL.  Returns the number of threads used. */
int orc_invert(const orc_instrument *inst, const orc_options *opt, int64_t n,
               const float *stokes, const float *W, int W_per_pixel,
               const double *init, double *params, double *chi2,
               int32_t *iters, int32_t *status, orc_counters *cnt,
               int nthreads);

/* Operation census (built only into liboracle_census.so, with ORC_CENSUS
 * defined; oracle/census.py): the arithmetic of every routine is counted
 * as it runs, one count per +, -, * or / on a double, in these categories.
 * Gradient work counts only the components that are not identically zero
 * (an operation whose derivative operands are both zero does nothing). */
enum {
  ORC_CEN_VALUE = 0,    /* synthesis and filter, values */
  ORC_CEN_GRADIENT,     /* synthesis and filter, derivatives (Eqs. 8-9, chain rule) */
  ORC_CEN_VOIGT_CALLS,  /* H, F evaluations */
  ORC_CEN_VOIGT,        /* arithmetic of the Taylor-table evaluations (Eqs. 10-13) */
  ORC_CEN_CHI2,         /* residuals and chi^2 (Eq. 1) */
  ORC_CEN_NORMAL,       /* J^T W J (one triangle) and J^T W r */
  ORC_CEN_SOLVE,        /* equilibration, damping, Cholesky, substitutions, step */
  ORC_CEN_SPECIAL,      /* sqrt, sin, cos, rounding calls (not in the counts above) */
  ORC_CEN_N
};
#ifdef ORC_CENSUS
extern uint64_t orc_census[ORC_CEN_N];
/* Copies the counters into out[ORC_CEN_N] and clears them. */
void orc_census_take(uint64_t *out);
#define ORC_COUNT(cat, n) (orc_census[(cat)] += (uint64_t)(n))
#else
#define ORC_COUNT(cat, n) ((void)0)
#endif

/* Batch forward synthesis (values only), for building synthetic inputs.
 * params: [n][10]; out: [n][4][n_obs]. */
int orc_forward_batch(const orc_instrument *inst, int64_t n, const double *params,
                      double *out, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
