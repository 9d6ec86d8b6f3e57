/*
 * Oracle Levenberg-Marquardt inversion (test infrastructure; see oracle.h).
 *
 * Follows Sect. 2 (Eqs. 1-6), Sect. 4.2 (Table 2 and the exits) and
 * Sect. 4.4 (derivatives only after a successful iteration, Fig. 6):
 *
 *   chi^2 = 1/(4L - F) sum_ij (I_obs - I_syn)^2 w_ij^2 / sigma_i^2   (Eq. 1)
 *
 * with W = w^2 / sigma^2 supplied by the caller.  The modified Hessian of
 * Eqs. 3-4 is read as the Gauss-Newton matrix J^T W J with its diagonal
 * multiplied by (1 + eps); the gradient of Eq. 2 is -2/(4L-F) J^T W r; the
 * common factor 2/(4L-F) cancels in the step of Eq. 5.
 *
 * The step solves (H + eps diag H) delta = g on the diagonally equilibrated
 * system C = D^-1/2 H D^-1/2 by Cholesky.  The paper uses an SVD to avoid
 * singular systems; here the SVD (for this symmetric matrix, the Jacobi
 * eigen-decomposition, whose pseudo-inverse is the SVD one) is the fallback
 * when the factorisation breaks down, with singular values below 1e-12 of
 * the largest discarded.
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include "oracle.h"

#define NP ORC_NPAR

void orc_default_init(double *M) {
  /* midpoints of the synthetic priors */
  const double m0[NP] = {1500.0, 90.0, 90.0, 0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6};
  memcpy(M, m0, sizeof m0);
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

void orc_project(double *M) {
  /* exact symmetries: (-B, gamma) == (B, 180 - gamma); gamma and -gamma give
   * the same profiles; psi is defined modulo 180 degrees */
  if (M[ORC_B] < 0.0) {
    M[ORC_B] = -M[ORC_B];
    M[ORC_GAMMA] = 180.0 - M[ORC_GAMMA];
  }
  double g = fmod(M[ORC_GAMMA], 360.0);
  if (g < 0.0) g += 360.0;
  if (g > 180.0) g = 360.0 - g;
  M[ORC_GAMMA] = g;
  double p = fmod(M[ORC_PSI], 180.0);
  if (p < 0.0) p += 180.0;
  M[ORC_PSI] = p;
  M[ORC_B] = clampd(M[ORC_B], 0.0, 5000.0);
  M[ORC_VLOS] = clampd(M[ORC_VLOS], -20.0, 20.0);
  M[ORC_DLD] = clampd(M[ORC_DLD], 5.0, 150.0);
  M[ORC_A] = clampd(M[ORC_A], 0.0, 5.0);
  M[ORC_ETA0] = clampd(M[ORC_ETA0], 1e-3, 1e3);
  M[ORC_S0] = clampd(M[ORC_S0], -1.0, 3.0);
  M[ORC_S1] = clampd(M[ORC_S1], 0.0, 5.0);
  M[ORC_ALPHA] = clampd(M[ORC_ALPHA], 0.0, 1.0);
}

/* Table 2: the first row that matches, read top-down. */
double orc_eps_decrease(double eps) {
  if (eps > 1e4) return eps / 100.0;
  if (eps >= 1e-4) return eps / 10.0;
  return eps / 2.0;
}
double orc_eps_increase(double eps) {
  if (eps < 1e-4) return eps * 100.0;
  if (eps > 1e4) return eps * 10.0;
  return eps * 2.0;
}

/* Cholesky of the n x n SPD matrix A (row-major, lower factor in place).
 * Returns 0 on success. */
static int cholesky(int n, double *A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    ORC_COUNT(ORC_CEN_SOLVE, 2 * j);
    if (!(d > 0.0) || !isfinite(d)) return 1;
    const double ljj = sqrt(d);
    ORC_COUNT(ORC_CEN_SPECIAL, 1);
    A[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / ljj;
      ORC_COUNT(ORC_CEN_SOLVE, 2 * j + 1);
    }
  }
  return 0;
}

/* Cyclic Jacobi eigen-decomposition of the symmetric n x n matrix A:
 * on return A's diagonal holds the eigenvalues and V the eigenvectors
 * (columns). */
static void jacobi_eigen(int n, double *A, double *V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i != j) off += A[i * n + j] * A[i * n + j];
        else diag += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* A <- R^T A R with R the rotation in the (p, q) plane */
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

int orc_solve(const double *H, const double *g, double eps, uint32_t free_mask,
              double *delta) {
  int idx[NP], n = 0;
  double maxd = 0.0;
  for (int p = 0; p < NP; ++p) {
    delta[p] = 0.0;
    if ((free_mask >> p) & 1u)
      if (H[p * NP + p] > maxd) maxd = H[p * NP + p];
  }
  /* parameters with no leverage on chi^2 are frozen for this step */
  for (int p = 0; p < NP; ++p)
    if (((free_mask >> p) & 1u) && H[p * NP + p] > 1e-30 * maxd && maxd > 0.0) idx[n++] = p;
  if (n == 0) return 2;

  double sc[NP], C[NP * NP], b[NP];
  for (int i = 0; i < n; ++i) sc[i] = 1.0 / sqrt(H[idx[i] * NP + idx[i]]);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) C[i * n + j] = sc[i] * H[idx[i] * NP + idx[j]] * sc[j];
    C[i * n + i] += eps; /* (1 + eps) on the equilibrated unit diagonal */
    b[i] = sc[i] * g[idx[i]];
  }
  /* census: n reciprocals (and square roots), one triangle of C (2 each),
   * the damping and the scaled gradient */
  ORC_COUNT(ORC_CEN_SOLVE, n + n * (n + 1) + n + n);
  ORC_COUNT(ORC_CEN_SPECIAL, n);

  double L[NP * NP], y[NP];
  memcpy(L, C, sizeof(double) * n * n);
  int used_fallback = 0;
  if (cholesky(n, L) == 0) {
    for (int i = 0; i < n; ++i) { /* L z = b */
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
      y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) { /* L^T y = z */
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * y[k];
      y[i] = s / L[i * n + i];
    }
    ORC_COUNT(ORC_CEN_SOLVE, 2 * (n * (n - 1) + n)); /* the two substitutions */
  } else {
    used_fallback = 1;
    double A[NP * NP], V[NP * NP];
    memcpy(A, C, sizeof(double) * n * n);
    jacobi_eigen(n, A, V);
    double smax = 0.0;
    for (int i = 0; i < n; ++i)
      if (fabs(A[i * n + i]) > smax) smax = fabs(A[i * n + i]);
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    for (int j = 0; j < n; ++j) {
      const double lam = A[j * n + j];
      if (!(fabs(lam) >= 1e-12 * smax) || lam == 0.0) continue;
      double proj = 0.0;
      for (int i = 0; i < n; ++i) proj += V[i * n + j] * b[i];
      for (int i = 0; i < n; ++i) y[i] += V[i * n + j] * proj / lam;
    }
  }
  for (int i = 0; i < n; ++i) delta[idx[i]] = sc[i] * y[i];
  ORC_COUNT(ORC_CEN_SOLVE, n);
  return used_fallback;
}

static int popcount10(uint32_t m) {
  int c = 0;
  for (int p = 0; p < NP; ++p) c += (m >> p) & 1u;
  return c;
}

/* chi^2 of Eq. 1 and, with J, the normal equations H = J^T W J and
 * g = J^T W r, r = obs - syn (H NULL: the gradient only). */
static double chi2_and_normal(int rows, const float *obs, const float *W, const double *S,
                              const double *J, double dof, double *H, double *g) {
  double chi = 0.0;
  if (J) {
    if (H) memset(H, 0, sizeof(double) * NP * NP);
    memset(g, 0, sizeof(double) * NP);
  }
  for (int r = 0; r < rows; ++r) {
    const double res = (double)obs[r] - S[r];
    const double w = (double)W[r];
    chi += w * res * res;
    ORC_COUNT(ORC_CEN_CHI2, 4);
    if (J) {
      const double *j = J + (size_t)r * NP;
      /* census: w r once; per non-zero J entry a multiply-add into g and w J
       * once; per pair of non-zero entries of one triangle a multiply-add */
      ORC_COUNT(ORC_CEN_NORMAL, 1);
      for (int p = 0; p < NP; ++p) {
        g[p] += w * res * j[p];
        if (H)
          for (int q = 0; q < NP; ++q) H[p * NP + q] += w * j[p] * j[q];
        if (j[p] != 0.0) {
          ORC_COUNT(ORC_CEN_NORMAL, 2);
          if (H) {
            ORC_COUNT(ORC_CEN_NORMAL, 1);
            for (int q = p; q < NP; ++q) ORC_COUNT(ORC_CEN_NORMAL, 2 * (j[q] != 0.0));
          }
        }
      }
    }
  }
  ORC_COUNT(ORC_CEN_CHI2, 1);
  return chi / dof;
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t c) {
  /* state after c + 1 increments by the golden gamma, then the mix */
  uint64_t z = seed + (c + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double orc_restart_uniform(uint64_t seed, int64_t pixel, int k, int p) {
  const uint64_t c = ((uint64_t)pixel << 16) | ((uint64_t)(k & 0xFFF) << 4) | (uint64_t)(p & 15);
  return (double)(orc_splitmix64(seed, c) >> 11) * (1.0 / 9007199254740992.0);
}

/* Half-widths of the synthetic priors: the scale of restart perturbations. */
static const double RESTART_HALF[NP] = {1500.0, 90.0, 90.0, 3.0, 15.0, 0.25, 14.5, 0.2, 0.2, 0.4};

/* The paper's scheme (Sect. 4.2): a fixed number of trials; a restart from
 * the best model seen, its free parameters perturbed by uniform offsets of
 * up to 0.1 k prior half-widths on restart k (the damping carries over),
 * when (a) after the first 10 trials chi^2 has not fallen by a
 * factor 10 from its first value, or (b) 5 trials in a row brought no
 * improvement (or the damping passed eps_max).  A restart's evaluation is
 * itself a trial, so every pixel runs exactly fixed_iters trials unless it
 * stalls with no restart left. */
static void lm_pixel_fixed(const orc_instrument *inst, const orc_options *opt,
                           const float *obs, const float *W, const double *M0, int64_t pixel,
                           double *M_out, double *chi2_out, int32_t *iters_out,
                           int32_t *status_out, orc_counters *cnt, int rows, double dof) {
  double M[NP], Mt[NP], Mg[NP], delta[NP], H[NP * NP], g[NP];
  double *S = (double *)malloc(sizeof(double) * rows);
  double *J = (double *)malloc(sizeof(double) * rows * NP);
  if (M0) memcpy(M, M0, sizeof M);
  else orc_default_init(M);
  orc_project(M);
  orc_forward(inst, M, S, J);
  cnt->derivs++;
  cnt->hessians++;
  double chi2 = chi2_and_normal(rows, obs, W, S, J, dof, H, g);
  const double chi2_first = chi2;
  memcpy(Mg, M, sizeof M);
  double chig = chi2;
  double eps = opt->eps0;
  int status = ORC_MAX_ITER, it = 0, bad = 0, k = 0, pending = 0;
  if (!isfinite(chi2)) status = ORC_NONFINITE;
  while (status != ORC_NONFINITE && it < opt->fixed_iters) {
    ++it;
    if (pending) {  /* restart: evaluate the perturbed best model */
      ++k;
      for (int p = 0; p < NP; ++p)  /* frozen parameters keep their value */
        M[p] = ((opt->free_mask >> p) & 1u)
                   ? Mg[p] + (2.0 * orc_restart_uniform(opt->seed, pixel, k, p) - 1.0) * 0.1 *
                                 k * RESTART_HALF[p]
                   : Mg[p];
      orc_project(M);
      orc_forward(inst, M, S, J);
      cnt->derivs++;
      cnt->hessians++;
      cnt->trials++;
      chi2 = chi2_and_normal(rows, obs, W, S, J, dof, H, g);
      if (isfinite(chi2) && chi2 < chig) {
        memcpy(Mg, M, sizeof M);
        chig = chi2;
      }
      bad = 0;
      pending = 0;
      continue;
    }
    const int sres = orc_solve(H, g, eps, opt->free_mask, delta);
    cnt->solves++;
    if (sres == 1) cnt->svd_fallbacks++;
    for (int p = 0; p < NP; ++p) Mt[p] = M[p] + delta[p];
    orc_project(Mt);
    orc_forward(inst, Mt, S, NULL);
    cnt->trials++;
    const double chi2_t = chi2_and_normal(rows, obs, W, S, NULL, dof, NULL, NULL);
    if (isfinite(chi2_t) && chi2_t < chi2) {
      /* near the minimum the curvature barely changes: keep H (Sect. 4.4) */
      const int keep_h = chi2 < opt->hess_reuse;
      memcpy(M, Mt, sizeof M);
      chi2 = chi2_t;
      orc_forward(inst, M, S, J);
      cnt->derivs++;
      if (!keep_h) cnt->hessians++;
      chi2_and_normal(rows, obs, W, S, J, dof, keep_h ? NULL : H, g);
      eps = orc_eps_decrease(eps);
      bad = 0;
      if (chi2 < chig) {
        memcpy(Mg, M, sizeof M);
        chig = chi2;
      }
    } else {
      eps = orc_eps_increase(eps);
      ++bad;
    }
    const int stalled = eps > opt->eps_max;
    if (k < opt->restarts &&
        ((it == 10 && !(chig <= chi2_first / 10.0)) || bad >= 5 || stalled)) {
      pending = 1;
    } else if (stalled) {
      status = ORC_STALLED;
      break;
    }
  }
  memcpy(M_out, Mg, sizeof Mg);
  *chi2_out = chig;
  *iters_out = it;
  *status_out = status | (k << 8);
  free(S);
  free(J);
}

void orc_lm_pixel(const orc_instrument *inst, const orc_options *opt,
                  const float *obs, const float *W, const double *M0, int64_t pixel,
                  double *M_out, double *chi2_out, int32_t *iters_out,
                  int32_t *status_out, orc_counters *cnt) {
  const int rows = 4 * inst->n_obs;
  const double dof = (double)(rows - popcount10(opt->free_mask & 0x3FFu));
  for (int r = 0; r < rows; ++r)
    if (!isfinite(obs[r]) || !isfinite(W[r])) {
      for (int p = 0; p < NP; ++p) M_out[p] = NAN;
      *chi2_out = NAN;
      *iters_out = 0;
      *status_out = ORC_NONFINITE;
      return;
    }
  if (opt->fixed_iters > 0) {
    lm_pixel_fixed(inst, opt, obs, W, M0, pixel, M_out, chi2_out, iters_out, status_out, cnt,
                   rows, dof);
    return;
  }

  double M[NP], Mt[NP], delta[NP], H[NP * NP], g[NP];
  double *S = (double *)malloc(sizeof(double) * rows);
  double *J = (double *)malloc(sizeof(double) * rows * NP);
  if (M0) memcpy(M, M0, sizeof M);
  else orc_default_init(M);
  orc_project(M);

  /* initial model: synthesis with derivatives */
  orc_forward(inst, M, S, J);
  cnt->derivs++;
  cnt->hessians++;
  double chi2 = chi2_and_normal(rows, obs, W, S, J, dof, H, g);
  double eps = opt->eps0;
  int status = ORC_MAX_ITER, it = 0;
  if (!isfinite(chi2)) {
    status = ORC_NONFINITE;
  } else {
    while (it < opt->max_iter) {
      ++it;
      const int sres = orc_solve(H, g, eps, opt->free_mask, delta);
      cnt->solves++;
      if (sres == 1) cnt->svd_fallbacks++;
      for (int p = 0; p < NP; ++p) Mt[p] = M[p] + delta[p];
      ORC_COUNT(ORC_CEN_SOLVE, NP);
      orc_project(Mt);
      /* trial: values only (Fig. 6) */
      orc_forward(inst, Mt, S, NULL);
      cnt->trials++;
      const double chi2_t = chi2_and_normal(rows, obs, W, S, NULL, dof, NULL, NULL);
      if (isfinite(chi2_t) && chi2_t < chi2) {
        const double dec = chi2 - chi2_t;
        /* Sect. 4.4: when the model the step started from was already near
         * the minimum (chi^2 below hess_reuse), the Hessian is kept and
         * only the gradient is rebuilt */
        const int keep_h = chi2 < opt->hess_reuse;
        memcpy(M, Mt, sizeof M);
        chi2 = chi2_t;
        /* success: derivatives at the new best model */
        orc_forward(inst, M, S, J);
        cnt->derivs++;
        if (!keep_h) cnt->hessians++;
        chi2_and_normal(rows, obs, W, S, J, dof, keep_h ? NULL : H, g);
        eps = orc_eps_decrease(eps);
        if (dec < opt->rel_tol * (chi2 + dec)) {
          status = ORC_CONVERGED;
          break;
        }
      } else {
        eps = orc_eps_increase(eps);
        if (eps > opt->eps_max) {
          status = ORC_STALLED;
          break;
        }
      }
    }
  }
  memcpy(M_out, M, sizeof M);
  *chi2_out = chi2;
  *iters_out = it;
  *status_out = status;
  free(S);
  free(J);
}

/* ------------------------------------------------------------------ */
/* Thread pool over pixels (one pixel at a time from a shared counter). */

typedef struct {
  const orc_instrument *inst;
  const orc_options *opt;
  int64_t n;
  const float *stokes, *W;
  int W_per_pixel;
  const double *init;
  double *params, *chi2;
  int32_t *iters, *status;
  const double *fwd_params;
  double *fwd_out;
  atomic_llong next;
  orc_counters cnt[256];
} pool_job;

typedef struct {
  pool_job *job;
  int tid;
} pool_arg;

static void *invert_worker(void *p) {
  pool_arg *a = (pool_arg *)p;
  pool_job *jb = a->job;
  const int rows = 4 * jb->inst->n_obs;
  orc_counters *cnt = &jb->cnt[a->tid];
  for (;;) {
    const int64_t start = atomic_fetch_add(&jb->next, 1);
    if (start >= jb->n) break;
    const int64_t end = start + 1;
    for (int64_t i = start; i < end; ++i) {
      const float *w = jb->W_per_pixel ? jb->W + i * rows : jb->W;
      orc_lm_pixel(jb->inst, jb->opt, jb->stokes + i * rows, w,
                   jb->init ? jb->init + i * NP : NULL, i, jb->params + i * NP,
                   &jb->chi2[i], &jb->iters[i], &jb->status[i], cnt);
    }
  }
  return NULL;
}

static void *forward_worker(void *p) {
  pool_arg *a = (pool_arg *)p;
  pool_job *jb = a->job;
  const int rows = 4 * jb->inst->n_obs;
  for (;;) {
    const int64_t start = atomic_fetch_add(&jb->next, 1);
    if (start >= jb->n) break;
    const int64_t end = start + 1;
    for (int64_t i = start; i < end; ++i)
      orc_forward(jb->inst, jb->fwd_params + i * NP, jb->fwd_out + i * rows, NULL);
  }
  return NULL;
}

static int resolve_threads(int nthreads) {
  if (nthreads <= 0) {
    long hc = sysconf(_SC_NPROCESSORS_ONLN);
    nthreads = hc > 0 ? (int)hc : 1;
  }
  if (nthreads > 256) nthreads = 256;
  return nthreads;
}

static void run_pool(pool_job *job, int nthreads, void *(*fn)(void *)) {
  pthread_t th[256];
  pool_arg args[256];
  for (int t = 0; t < nthreads; ++t) {
    args[t].job = job;
    args[t].tid = t;
    pthread_create(&th[t], NULL, fn, &args[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

int orc_invert(const orc_instrument *inst, const orc_options *opt, int64_t n,
               const float *stokes, const float *W, int W_per_pixel,
               const double *init, double *params, double *chi2,
               int32_t *iters, int32_t *status, orc_counters *cnt,
               int nthreads) {
  nthreads = resolve_threads(nthreads);
  pool_job *job = (pool_job *)calloc(1, sizeof(pool_job));
  job->inst = inst;
  job->opt = opt;
  job->n = n;
  job->stokes = stokes;
  job->W = W;
  job->W_per_pixel = W_per_pixel;
  job->init = init;
  job->params = params;
  job->chi2 = chi2;
  job->iters = iters;
  job->status = status;
  atomic_init(&job->next, 0);
  run_pool(job, nthreads, invert_worker);
  if (cnt) {
    memset(cnt, 0, sizeof *cnt);
    for (int t = 0; t < nthreads; ++t) {
      cnt->trials += job->cnt[t].trials;
      cnt->derivs += job->cnt[t].derivs;
      cnt->solves += job->cnt[t].solves;
      cnt->svd_fallbacks += job->cnt[t].svd_fallbacks;
      cnt->hessians += job->cnt[t].hessians;
    }
  }
  free(job);
  return nthreads;
}

int orc_forward_batch(const orc_instrument *inst, int64_t n, const double *params,
                      double *out, int nthreads) {
  nthreads = resolve_threads(nthreads);
  pool_job *job = (pool_job *)calloc(1, sizeof(pool_job));
  job->inst = inst;
  job->n = n;
  job->fwd_params = params;
  job->fwd_out = out;
  atomic_init(&job->next, 0);
  run_pool(job, nthreads, forward_worker);
  free(job);
  return nthreads;
}
