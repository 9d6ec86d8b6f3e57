/*
 * Oracle Faddeeva function (test infrastructure; see oracle.h).
 *
 * The Voigt and Faraday-Voigt functions of Sect. 3.2 are the real and
 * imaginary parts of w(z) = exp(-z^2) erfc(-iz) at z = u + i a, a >= 0:
 *   H(a,u) = (a/pi)  Int exp(-y^2) / ((u-y)^2 + a^2) dy
 *   F(a,u) = (1/pi)  Int (u-y) exp(-y^2) / ((u-y)^2 + a^2) dy
 * (F taken as Im w: this is the normalisation for which Eqs. 8-9 hold.)
 *
 * The paper evaluates w with the rational approximation of Hui et al.
 * (1977).  The oracle instead uses three textbook representations, each in
 * the region where it is accurate to double precision:
 *   1. small |z|: the Maclaurin series  w = sum_n (iz)^n / Gamma(n/2 + 1);
 *   2. large |x| or y: the Laplace continued fraction
 *        w = (1/sqrt(pi)) / (zeta + (1/2)/(zeta + (2/2)/(zeta + ...))),
 *      zeta = -i z, evaluated bottom-up;
 *   3. in between: Gautschi's (1970) scheme, i.e. the Taylor series of w
 *      about the shifted point z + i h, whose normalised derivatives are
 *      products of the continued-fraction tails evaluated at z + i h.
 * w(-x + iy) = conj(w(x + iy)) reduces everything to x >= 0.
 * Accuracy against arbitrary-precision evaluation is ~1e-15 relative.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>

#include "oracle.h"

static const double ORC_SQRT_PI = 1.7724538509055160273;

/* Region 1: sum of the two interleaved power series. */
static double complex w_maclaurin(double complex z) {
  double complex mz2 = -z * z;
  double complex even = 1.0;                       /* (iz)^{2m} / m!            */
  double complex odd = 2.0 * I * z / ORC_SQRT_PI;  /* (iz)^{2m+1}/Gamma(m+3/2)  */
  double complex sum = even + odd;
  for (int m = 1; m < 400; ++m) {
    even *= mz2 / (double)m;
    odd *= mz2 / ((double)m + 0.5);
    sum += even + odd;
    if (cabs(even) + cabs(odd) < 1e-18 * cabs(sum)) break;
  }
  return sum;
}

/* Regions 2 and 3.  With h = 0 this is the plain continued fraction
 * truncated after n_cf levels; with h > 0 the Taylor sum about z + i h is
 * truncated after n_taylor terms. */
static double complex w_shifted(double complex z, double h, int n_taylor, int n_cf) {
  double complex zeta = -I * z + h;  /* -i (z + i h) */
  double complex r = 0.0;            /* tail r_{n+1} */
  double complex s = 0.0;
  double lam[128];                   /* (2h)^n */
  if (n_taylor > 127) n_taylor = 127;
  lam[0] = 1.0;
  for (int n = 1; n <= n_taylor; ++n) lam[n] = lam[n - 1] * 2.0 * h;
  for (int n = n_cf; n >= 0; --n) {
    r = 1.0 / (2.0 * (zeta + (double)(n + 1) * r));
    if (h > 0.0) {
      if (n <= n_taylor) s = r * (lam[n] + s);
    } else if (n == 0) {
      s = r;
    }
  }
  return (2.0 / ORC_SQRT_PI) * s;
}

void orc_faddeeva(double u, double a, double *H, double *F) {
  const double x = fabs(u), y = a;
  const double complex z = x + I * y;
  const double r2 = x * x + y * y;
  double complex w;
  if (r2 < 1.0) {
    w = w_maclaurin(z);
  } else if (x >= 7.0 || y >= 3.0) {
    const int n_cf = (int)(8.0 + 600.0 / sqrt(r2));
    w = w_shifted(z, 0.0, 0, n_cf);
  } else {
    const double h = 1.9 * (1.0 - y / 3.0);
    w = w_shifted(z, h, (int)lround(10.0 + 34.0 * h), (int)lround(30.0 + 30.0 * h));
  }
  *H = creal(w);
  *F = (u < 0.0) ? -cimag(w) : cimag(w);
}

void orc_faddeeva_batch(int64_t n, const double *u, const double *a, double *H, double *F) {
  for (int64_t i = 0; i < n; ++i) orc_faddeeva(u[i], a[i], &H[i], &F[i]);
}

/* ---- Taylor table (Sect. 3.2, Eqs. 10-13) -------------------------------- */

static double vt_H[ORC_VT_NA][ORC_VT_NU], vt_F[ORC_VT_NA][ORC_VT_NU];
static pthread_once_t vt_once = PTHREAD_ONCE_INIT;

static void vt_build(void) {
  for (int j = 0; j < ORC_VT_NA; ++j)
    for (int i = 0; i < ORC_VT_NU; ++i)
      orc_faddeeva(ORC_VT_STEP * i, ORC_VT_STEP * j, &vt_H[j][i], &vt_F[j][i]);
}

void orc_voigt_table_node(int i, int j, double *H, double *F) {
  pthread_once(&vt_once, vt_build);
  *H = vt_H[j][i];
  *F = vt_F[j][i];
}

/* w(z) ~ (i / sqrt(pi)) (1/z) (1 + 1/(2 z^2) + 3/(4 z^4) + 15/(8 z^6)) for
 * large |z| (the next term is below 1e-10 relative for |z| >= 24.975). */
static void w_asymptotic(double x, double y, double *H, double *F) {
  const double complex z = x + I * y;
  const double complex iz2 = 1.0 / (z * z);
  const double complex s = 1.0 + iz2 * (0.5 + iz2 * (0.75 + iz2 * 1.875));
  const double complex w = (I / ORC_SQRT_PI) * s / z;
  /* census: z^2 (5), its reciprocal (5), the Horner sum (2 + 1 + 6 + 1 + 6
   * + 1), the factor i/sqrt(pi) (2), the division by z (11) */
  ORC_COUNT(ORC_CEN_VOIGT, 40);
  *H = creal(w);
  *F = cimag(w);
}

void orc_voigt_taylor(int order, double u, double a, double *H, double *F) {
  const double x = fabs(u);
  const double sgn = u < 0.0 ? -1.0 : 1.0;
  if (x >= ORC_VT_STEP * (ORC_VT_NU - 0.5)) {
    w_asymptotic(x, a, H, F);
    *F *= sgn;
    return;
  }
  pthread_once(&vt_once, vt_build);
  const int i = (int)lround(x / ORC_VT_STEP);
  long jl = lround(a / ORC_VT_STEP);
  ORC_COUNT(ORC_CEN_VOIGT, 2);
  ORC_COUNT(ORC_CEN_SPECIAL, 2);
  if (jl < 0) jl = 0;
  if (jl > ORC_VT_NA - 1) jl = ORC_VT_NA - 1;
  const int j = (int)jl;
  const double u0 = ORC_VT_STEP * i, a0 = ORC_VT_STEP * j;
  const double h = vt_H[j][i], f = vt_F[j][i];
  /* Eqs. 8-9 at the node */
  const double al = -2.0 / ORC_SQRT_PI + 2.0 * a0 * h + 2.0 * u0 * f;
  const double be = 2.0 * a0 * f - 2.0 * u0 * h;
  const double du = x - u0, da = a - a0;
  double Ht = h + al * da + be * du;
  double Ft = f + be * da - al * du;
  /* census: the node (2), alpha (6), beta (5), the offsets (2), H and F (4 + 4) */
  ORC_COUNT(ORC_CEN_VOIGT, 2 + 6 + 5 + 2 + 4 + 4);
  if (order >= 2) {
    /* Eqs. 10-11: the second derivatives are multiples of these two */
    const double P = h + a0 * al + u0 * be;
    const double Q = f + a0 * be - u0 * al;
    Ht += P * (da * da - du * du) + 2.0 * Q * da * du;
    Ft += Q * (da * da - du * du) - 2.0 * P * da * du;
    /* census: P and Q (4 + 4), da^2 - du^2 and da du once each (3 + 1), the
     * two second-order terms (5 + 5) */
    ORC_COUNT(ORC_CEN_VOIGT, 22);
  }
  *H = Ht;
  *F = sgn * Ft;
}

void orc_voigt_taylor_batch(int order, int64_t n, const double *u, const double *a, double *H,
                            double *F) {
  for (int64_t i = 0; i < n; ++i) orc_voigt_taylor(order, u[i], a[i], &H[i], &F[i]);
}
