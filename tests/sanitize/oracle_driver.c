/*
 * Driver for the sanitizer builds of the FP64 oracle (AddressSanitizer +
 * UndefinedBehaviorSanitizer, ThreadSanitizer): runs every oracle routine on
 * an HMI-shaped instrument (six Gaussian filters on a 101-point grid) and on
 * edge cases -- values-only and derivative syntheses for the three H, F
 * evaluations, LM fits from the default and a given start, the fixed-
 * iteration scheme with restarts, the kept Hessian, a non-finite
 * observation, solves that need the eigen fallback or freeze every
 * parameter, and the threaded batch routines.  Exits non-zero on a result
 * that is not finite where it must be.  Test infrastructure only.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define NF 101
#define NO 6

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double uniform(double lo, double hi) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return lo + (hi - lo) * (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void draw_model(double *M) {
  M[ORC_B] = uniform(0.0, 3000.0);
  M[ORC_GAMMA] = acos(uniform(-1.0, 1.0)) * 180.0 / 3.14159265358979323846;
  M[ORC_PSI] = uniform(0.0, 180.0);
  M[ORC_VLOS] = uniform(-3.0, 3.0);
  M[ORC_DLD] = uniform(20.0, 50.0);
  M[ORC_A] = uniform(0.0, 0.5);
  M[ORC_ETA0] = uniform(1.0, 30.0);
  M[ORC_S0] = uniform(0.1, 0.5);
  M[ORC_S1] = 1.0 - M[ORC_S0];
  M[ORC_ALPHA] = uniform(0.2, 1.0);
}

static int check_finite(const char *what, const double *x, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) {
      fprintf(stderr, "%s: element %d is not finite\n", what, i);
      return 1;
    }
  return 0;
}

int main(int argc, char **argv) {
  const int threads = argc > 1 ? atoi(argv[1]) : 4;
  double fine[NF], filt[NO * NF];
  const double centres[NO] = {-172.0, -103.2, -34.4, 34.4, 103.2, 172.0};
  const double sig = 76.0 / (2.0 * sqrt(2.0 * log(2.0)));
  for (int k = 0; k < NF; ++k) fine[k] = -600.0 + 12.0 * k;
  for (int i = 0; i < NO; ++i) {
    double s = 0.0;
    for (int k = 0; k < NF; ++k) {
      const double x = (fine[k] - centres[i]) / sig;
      filt[i * NF + k] = exp(-0.5 * x * x);
      s += filt[i * NF + k];
    }
    for (int k = 0; k < NF; ++k) filt[i * NF + k] /= s;
  }
  orc_instrument inst = {6173.3356, 2.5, NF, fine, NO, filt, 0};
  int bad = 0;

  /* syntheses: values and Jacobians with each H, F evaluation */
  double M[ORC_NPAR], S[4 * NO], J[4 * NO * ORC_NPAR], Sf[4 * NF], dSf[4 * NF * ORC_NPAR];
  for (int v = 0; v < 3; ++v) {
    inst.voigt = v;
    for (int t = 0; t < 8; ++t) {
      draw_model(M);
      orc_forward(&inst, M, S, NULL);
      orc_forward(&inst, M, S, J);
      orc_synth_fine(&inst, M, Sf, dSf);
      bad |= check_finite("forward", S, 4 * NO) | check_finite("jacobian", J, 4 * NO * ORC_NPAR);
    }
  }
  inst.voigt = 0;
  /* H, F over a wide range of (u, a), including the asymptotic region */
  for (int i = 0; i < 200; ++i) {
    double h, f, u = uniform(-400.0, 400.0), a = uniform(0.0, 6.0);
    orc_faddeeva(u, a, &h, &f);
    orc_voigt_taylor(1, u, a, &h, &f);
    orc_voigt_taylor(2, u, a, &h, &f);
    bad |= !isfinite(h) || !isfinite(f);
  }

  /* fits: default start, given start, fixed iterations with restarts, kept
   * Hessian, a non-finite sample */
  enum { NPX = 48 };
  float *obs = malloc(sizeof(float) * NPX * 4 * NO);
  float W[4 * NO];
  double *P = malloc(sizeof(double) * NPX * ORC_NPAR);
  for (int r = 0; r < 4 * NO; ++r) W[r] = 1e6f;
  for (int p = 0; p < NPX; ++p) {
    draw_model(P + p * ORC_NPAR);
    orc_forward(&inst, P + p * ORC_NPAR, S, NULL);
    for (int r = 0; r < 4 * NO; ++r) obs[p * 4 * NO + r] = (float)(S[r] + uniform(-1e-3, 1e-3));
  }
  obs[5 * 4 * NO + 3] = NAN;
  orc_options opt = {50, 1e-3, 1e8, 1e-5, 0x3FF, 0, 0, 7, 0.0};
  orc_counters cnt;
  memset(&cnt, 0, sizeof cnt);
  double Mo[ORC_NPAR], chi2;
  int32_t it, st;
  for (int p = 0; p < 8; ++p) {
    orc_lm_pixel(&inst, &opt, obs + p * 4 * NO, W, NULL, p, Mo, &chi2, &it, &st, &cnt);
    if (p != 5) bad |= check_finite("fit", Mo, ORC_NPAR);
    orc_lm_pixel(&inst, &opt, obs + p * 4 * NO, W, P + p * ORC_NPAR, p, Mo, &chi2, &it, &st,
                 &cnt);
  }
  orc_options fixed = opt;
  fixed.fixed_iters = 30;
  fixed.restarts = 3;
  orc_options keep = opt;
  keep.hess_reuse = 10.0;
  orc_options frozen = opt;
  frozen.free_mask = 0x1F7; /* v and alpha held */
  for (int p = 0; p < 4; ++p) {
    orc_lm_pixel(&inst, &fixed, obs + p * 4 * NO, W, NULL, p, Mo, &chi2, &it, &st, &cnt);
    orc_lm_pixel(&inst, &keep, obs + p * 4 * NO, W, NULL, p, Mo, &chi2, &it, &st, &cnt);
    orc_lm_pixel(&inst, &frozen, obs + p * 4 * NO, W, NULL, p, Mo, &chi2, &it, &st, &cnt);
  }

  /* solves: singular (rank one) -> eigen fallback; all parameters frozen */
  double H[ORC_NPAR * ORC_NPAR], g[ORC_NPAR], d[ORC_NPAR];
  for (int i = 0; i < ORC_NPAR; ++i) {
    g[i] = uniform(-1.0, 1.0);
    for (int j = 0; j < ORC_NPAR; ++j) H[i * ORC_NPAR + j] = (i + 1.0) * (j + 1.0);
  }
  const int c1 = orc_solve(H, g, 0.0, 0x3FF, d);
  const int c2 = orc_solve(H, g, 1e-3, 0x0, d);
  bad |= check_finite("fallback solve", d, ORC_NPAR);
  if (c1 != 1 || c2 != 2) {
    fprintf(stderr, "solve codes %d %d\n", c1, c2);
    bad = 1;
  }
  for (int i = 0; i < 50; ++i) {
    double e = uniform(1e-9, 1e9);
    e = orc_eps_decrease(e) + orc_eps_increase(e);
    double Mp[ORC_NPAR];
    draw_model(Mp);
    Mp[ORC_B] = uniform(-6000.0, 6000.0);
    Mp[ORC_GAMMA] = uniform(-720.0, 720.0);
    Mp[ORC_PSI] = uniform(-720.0, 720.0);
    orc_project(Mp);
    bad |= check_finite("projection", Mp, ORC_NPAR);
  }

  /* threaded batches: per-pixel weights, given starts */
  double *par = malloc(sizeof(double) * NPX * ORC_NPAR), *c2v = malloc(sizeof(double) * NPX);
  int32_t *its = malloc(sizeof(int32_t) * NPX), *sts = malloc(sizeof(int32_t) * NPX);
  float *Wp = malloc(sizeof(float) * NPX * 4 * NO);
  for (int i = 0; i < NPX * 4 * NO; ++i) Wp[i] = (float)uniform(5e5, 1.5e6);
  double *fwd = malloc(sizeof(double) * NPX * 4 * NO);
  orc_forward_batch(&inst, NPX, P, fwd, threads);
  orc_invert(&inst, &opt, NPX, obs, W, 0, NULL, par, c2v, its, sts, &cnt, threads);
  orc_invert(&inst, &opt, NPX, obs, Wp, 1, P, par, c2v, its, sts, &cnt, threads);
  orc_invert(&inst, &fixed, NPX, obs, W, 0, NULL, par, c2v, its, sts, &cnt, threads);
  if (sts[5] != ORC_NONFINITE) {
    fprintf(stderr, "non-finite pixel status %d\n", sts[5]);
    bad = 1;
  }
  free(obs);
  free(P);
  free(par);
  free(c2v);
  free(its);
  free(sts);
  free(Wp);
  free(fwd);
  printf("oracle driver: %s (trials %lld)\n", bad ? "FAILED" : "ok", (long long)cnt.trials);
  return bad;
}
