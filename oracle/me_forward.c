/*
 * Oracle Milne-Eddington forward model with exact derivatives
 * (test infrastructure; see oracle.h).
 *
 * What is computed (Sect. 2, Sect. 3.1-3.2, Eqs. 7-9):
 *  - Zeeman triplet: one pi and two sigma components, the sigma components
 *    shifted by -/+ Delta lambda_B = C_Z B with C_Z from Eq. 7 (blue at
 *    shorter wavelength, red at longer);
 *  - Doppler shift lambda0 v / c; reduced frequencies
 *    u_c = (Delta lambda - lambda0 v/c -/+ shift_c) / Delta lambda_D;
 *  - profiles phi_c = H(a, u_c), psi_c = F(a, u_c) with the analytic
 *    derivatives of Eqs. 8-9;
 *  - absorption-matrix elements eta_I,Q,U,V and rho_Q,U,V of the
 *    Milne-Eddington atmosphere, and the Unno-Rachkovsky solution for a
 *    source function S0 + S1 tau at disk centre (both only cited by the
 *    paper: Landolfi & Landi Degl'Innocenti 1982; Del Toro Iniesta 2003);
 *  - filling factor: a non-magnetic component (same atmosphere, B = 0) fills
 *    1 - alpha of the resolution element;
 *  - the instrument's linear filter maps the synthesis grid to the observed
 *    samples (Sect. 5: profiles are convolved with the HMI filters).
 *
 * Derivatives are carried in forward mode: every intermediate is a value
 * with its gradient with respect to the 10 parameters in API units, and the
 * four rules below (sum, product, quotient, sin/cos) plus Eqs. 8-9 for
 * H and F propagate them.  That is the analytic Jacobian of Sect. 4.4,
 * obtained from the same evaluation as the Stokes vector.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define NP ORC_NPAR
static const double ORC_C_KMS = 299792.458;
static const double ORC_PI = 3.14159265358979323846;
static const double ORC_TWO_OVER_SQRT_PI = 1.1283791670955125739;

typedef struct {
  double v;
  double d[NP];
} dual;

#ifdef ORC_CENSUS
uint64_t orc_census[ORC_CEN_N];
void orc_census_take(uint64_t *out) {
  memcpy(out, orc_census, sizeof orc_census);
  memset(orc_census, 0, sizeof orc_census);
}
#endif

/* Census of one gradient component of a sum (x + y), a product (x y') + x' y)
 * or a quotient ((x' - r y') / y): operations on components that are not
 * identically zero. */
#define NZ(x) ((x) != 0.0)
#define CEN_SUM(x, y) ORC_COUNT(ORC_CEN_GRADIENT, NZ(x) && NZ(y))
#define CEN_PROD(x, y) ORC_COUNT(ORC_CEN_GRADIENT, NZ(x) + NZ(y) + (NZ(x) && NZ(y)))
#define CEN_QUOT(x, y) ORC_COUNT(ORC_CEN_GRADIENT, (NZ(x) || NZ(y)) ? 1 + NZ(y) + (NZ(x) && NZ(y)) : 0)

/* nd = number of live gradient components (0 = values only, NP = all). */
static dual d_const(double v) {
  dual r;
  memset(&r, 0, sizeof r);
  r.v = v;
  return r;
}
static dual d_var(double v, int idx, double seed) {
  dual r = d_const(v);
  r.d[idx] = seed;
  return r;
}
static dual d_add(dual a, dual b, int nd) {
  dual r;
  r.v = a.v + b.v;
  ORC_COUNT(ORC_CEN_VALUE, 1);
  for (int k = 0; k < nd; ++k) {
    CEN_SUM(a.d[k], b.d[k]);
    r.d[k] = a.d[k] + b.d[k];
  }
  return r;
}
static dual d_sub(dual a, dual b, int nd) {
  dual r;
  r.v = a.v - b.v;
  ORC_COUNT(ORC_CEN_VALUE, 1);
  for (int k = 0; k < nd; ++k) {
    CEN_SUM(a.d[k], b.d[k]);
    r.d[k] = a.d[k] - b.d[k];
  }
  return r;
}
static dual d_mul(dual a, dual b, int nd) {
  dual r;
  r.v = a.v * b.v;
  ORC_COUNT(ORC_CEN_VALUE, 1);
  for (int k = 0; k < nd; ++k) {
    CEN_PROD(a.d[k], b.d[k]);
    r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  }
  return r;
}
static dual d_div(dual a, dual b, int nd) {
  dual r;
  r.v = a.v / b.v;
  ORC_COUNT(ORC_CEN_VALUE, 1);
  for (int k = 0; k < nd; ++k) {
    CEN_QUOT(a.d[k], b.d[k]);
    r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  }
  return r;
}
static dual d_scale(dual a, double c, int nd) {
  dual r;
  r.v = a.v * c;
  ORC_COUNT(ORC_CEN_VALUE, 1);
  for (int k = 0; k < nd; ++k) {
    ORC_COUNT(ORC_CEN_GRADIENT, NZ(a.d[k]));
    r.d[k] = a.d[k] * c;
  }
  return r;
}
static dual d_addc(dual a, double c) {
  a.v += c;
  ORC_COUNT(ORC_CEN_VALUE, 1);
  return a;
}
static dual d_sin(dual a, int nd) {
  dual r;
  r.v = sin(a.v);
  const double c = cos(a.v);
  ORC_COUNT(ORC_CEN_SPECIAL, nd > 0 ? 2 : 1);
  for (int k = 0; k < nd; ++k) {
    ORC_COUNT(ORC_CEN_GRADIENT, NZ(a.d[k]));
    r.d[k] = c * a.d[k];
  }
  return r;
}
static dual d_cos(dual a, int nd) {
  dual r;
  r.v = cos(a.v);
  const double s = -sin(a.v);
  ORC_COUNT(ORC_CEN_SPECIAL, nd > 0 ? 2 : 1);
  for (int k = 0; k < nd; ++k) {
    ORC_COUNT(ORC_CEN_GRADIENT, NZ(a.d[k]));
    r.d[k] = s * a.d[k];
  }
  return r;
}

/* H and F at (a, u) with Eqs. 8-9:
 *   dH/da = -dF/du = -2/sqrt(pi) + 2aH + 2uF   (alpha)
 *   dH/du =  dF/da =  2aF - 2uH                (beta)            */
static void d_voigt(int variant, dual u, dual a, int nd, dual *H, dual *F) {
  double h, f;
  if (variant == 0)
    orc_faddeeva(u.v, a.v, &h, &f);
  else
    orc_voigt_taylor(variant, u.v, a.v, &h, &f);
  const double al = -ORC_TWO_OVER_SQRT_PI + 2.0 * a.v * h + 2.0 * u.v * f;
  const double be = 2.0 * a.v * f - 2.0 * u.v * h;
  ORC_COUNT(ORC_CEN_VOIGT_CALLS, 1);
  if (nd > 0) ORC_COUNT(ORC_CEN_GRADIENT, 6 + 5);  /* alpha and beta, Eqs. 8-9 */
  H->v = h;
  F->v = f;
  for (int k = 0; k < nd; ++k) {
    /* H' = alpha a' + beta u', F' = beta a' - alpha u': a product pair each */
    ORC_COUNT(ORC_CEN_GRADIENT, 2 * (NZ(a.d[k]) + NZ(u.d[k]) + (NZ(a.d[k]) && NZ(u.d[k]))));
    H->d[k] = al * a.d[k] + be * u.d[k];
    F->d[k] = be * a.d[k] - al * u.d[k];
  }
}

static dual d_sq(dual a, int nd) { return d_mul(a, a, nd); }

double orc_zeeman_constant(double lambda0_A, double geff) {
  /* Eq. 7: Delta lambda_B = 4.66685e-10 g_eff B lambda0^2 [mA], lambda0 in A */
  return 4.66685e-10 * geff * lambda0_A * lambda0_A;
}

/* Stokes vector (I,Q,U,V) and its gradient at one synthesis-grid point. */
static void synth_point(double lambda0_mA, double cz, int voigt, const double *M, double dlam,
                        int nd, dual out[4]) {
  const double deg = ORC_PI / 180.0;
  ORC_COUNT(ORC_CEN_VALUE, 2); /* the two angles in radians */
  dual B = d_var(M[ORC_B], ORC_B, 1.0);
  dual gam = d_var(M[ORC_GAMMA] * deg, ORC_GAMMA, deg);
  dual chi = d_var(M[ORC_PSI] * deg, ORC_PSI, deg);
  dual v = d_var(M[ORC_VLOS], ORC_VLOS, 1.0);
  dual dld = d_var(M[ORC_DLD], ORC_DLD, 1.0);
  dual a = d_var(M[ORC_A], ORC_A, 1.0);
  dual eta0 = d_var(M[ORC_ETA0], ORC_ETA0, 1.0);
  dual S0 = d_var(M[ORC_S0], ORC_S0, 1.0);
  dual S1 = d_var(M[ORC_S1], ORC_S1, 1.0);
  dual alpha = d_var(M[ORC_ALPHA], ORC_ALPHA, 1.0);

  /* reduced frequencies of the pi, blue and red components */
  dual shift_v = d_scale(v, lambda0_mA / ORC_C_KMS, nd);
  dual u_p = d_div(d_sub(d_const(dlam), shift_v, nd), dld, nd);
  dual zee = d_div(d_scale(B, cz, nd), dld, nd);
  dual u_b = d_add(u_p, zee, nd);
  dual u_r = d_sub(u_p, zee, nd);

  dual Hp, Fp, Hb, Fb, Hr, Fr;
  d_voigt(voigt, u_p, a, nd, &Hp, &Fp);
  d_voigt(voigt, u_b, a, nd, &Hb, &Fb);
  d_voigt(voigt, u_r, a, nd, &Hr, &Fr);

  dual sg = d_sin(gam, nd), cg = d_cos(gam, nd);
  dual sin2g = d_sq(sg, nd);
  dual one_p_cos2g = d_addc(d_sq(cg, nd), 1.0);
  dual c2c = d_cos(d_scale(chi, 2.0, nd), nd);
  dual s2c = d_sin(d_scale(chi, 2.0, nd), nd);
  dual half = d_scale(eta0, 0.5, nd);

  dual Hs = d_scale(d_add(Hb, Hr, nd), 0.5, nd);
  dual Fs = d_scale(d_add(Fb, Fr, nd), 0.5, nd);

  /* absorption matrix */
  dual etaI = d_addc(d_mul(half, d_add(d_mul(Hp, sin2g, nd), d_mul(Hs, one_p_cos2g, nd), nd), nd), 1.0);
  dual lin_e = d_mul(half, d_mul(d_sub(Hp, Hs, nd), sin2g, nd), nd);
  dual lin_r = d_mul(half, d_mul(d_sub(Fp, Fs, nd), sin2g, nd), nd);
  dual etaQ = d_mul(lin_e, c2c, nd);
  dual etaU = d_mul(lin_e, s2c, nd);
  dual etaV = d_mul(half, d_mul(d_sub(Hr, Hb, nd), cg, nd), nd);
  dual rhoQ = d_mul(lin_r, c2c, nd);
  dual rhoU = d_mul(lin_r, s2c, nd);
  dual rhoV = d_mul(half, d_mul(d_sub(Fr, Fb, nd), cg, nd), nd);

  /* Unno-Rachkovsky solution */
  dual Pi = d_add(d_add(d_mul(etaQ, rhoQ, nd), d_mul(etaU, rhoU, nd), nd), d_mul(etaV, rhoV, nd), nd);
  dual eI2 = d_sq(etaI, nd);
  dual rho2 = d_add(d_add(d_sq(rhoQ, nd), d_sq(rhoU, nd), nd), d_sq(rhoV, nd), nd);
  dual eta2 = d_add(d_add(d_sq(etaQ, nd), d_sq(etaU, nd), nd), d_sq(etaV, nd), nd);
  dual Delta = d_sub(d_mul(eI2, d_add(d_sub(eI2, eta2, nd), rho2, nd), nd), d_sq(Pi, nd), nd);

  dual numI = d_mul(etaI, d_add(eI2, rho2, nd), nd);
  dual numQ = d_add(d_add(d_mul(eI2, etaQ, nd),
                          d_mul(etaI, d_sub(d_mul(etaV, rhoU, nd), d_mul(etaU, rhoV, nd), nd), nd), nd),
                    d_mul(rhoQ, Pi, nd), nd);
  dual numU = d_add(d_add(d_mul(eI2, etaU, nd),
                          d_mul(etaI, d_sub(d_mul(etaQ, rhoV, nd), d_mul(etaV, rhoQ, nd), nd), nd), nd),
                    d_mul(rhoU, Pi, nd), nd);
  dual numV = d_add(d_add(d_mul(eI2, etaV, nd),
                          d_mul(etaI, d_sub(d_mul(etaU, rhoQ, nd), d_mul(etaQ, rhoU, nd), nd), nd), nd),
                    d_mul(rhoV, Pi, nd), nd);

  dual Im = d_add(S0, d_div(d_mul(S1, numI, nd), Delta, nd), nd);
  dual Qm = d_scale(d_div(d_mul(S1, numQ, nd), Delta, nd), -1.0, nd);
  dual Um = d_scale(d_div(d_mul(S1, numU, nd), Delta, nd), -1.0, nd);
  dual Vm = d_scale(d_div(d_mul(S1, numV, nd), Delta, nd), -1.0, nd);

  /* non-magnetic component: same atmosphere with B = 0 */
  dual I0 = d_add(S0, d_div(S1, d_addc(d_mul(eta0, Hp, nd), 1.0), nd), nd);

  dual one_m_alpha = d_addc(d_scale(alpha, -1.0, nd), 1.0);
  out[0] = d_add(d_mul(alpha, Im, nd), d_mul(one_m_alpha, I0, nd), nd);
  out[1] = d_mul(alpha, Qm, nd);
  out[2] = d_mul(alpha, Um, nd);
  out[3] = d_mul(alpha, Vm, nd);
}

void orc_synth_fine(const orc_instrument *inst, const double *M, double *S, double *dS) {
  const int nf = inst->n_fine;
  const int nd = dS ? NP : 0;
  const double lambda0_mA = inst->lambda0_A * 1000.0;
  const double cz = orc_zeeman_constant(inst->lambda0_A, inst->geff);
  for (int k = 0; k < nf; ++k) {
    dual out[4];
    synth_point(lambda0_mA, cz, inst->voigt, M, inst->fine_offset_mA[k], nd, out);
    for (int s = 0; s < 4; ++s) {
      S[s * nf + k] = out[s].v;
      if (dS)
        for (int p = 0; p < NP; ++p) dS[((size_t)s * nf + k) * NP + p] = out[s].d[p];
    }
  }
}

void orc_forward(const orc_instrument *inst, const double *M, double *S, double *J) {
  const int nf = inst->n_fine, no = inst->n_obs;
  double *Sf = (double *)malloc(sizeof(double) * 4 * nf);
  double *dSf = J ? (double *)malloc(sizeof(double) * 4 * nf * NP) : NULL;
  orc_synth_fine(inst, M, Sf, dSf);
  /* observed samples: S_obs = F . S_fine (a plain matrix product) */
  for (int s = 0; s < 4; ++s)
    for (int i = 0; i < no; ++i) {
      const double *Fi = inst->filter + (size_t)i * nf;
      double acc = 0.0;
      for (int k = 0; k < nf; ++k) acc += Fi[k] * Sf[s * nf + k];
      S[s * no + i] = acc;
      /* census: a multiply-add per tap that is not zero */
      for (int k = 0; k < nf; ++k) ORC_COUNT(ORC_CEN_VALUE, 2 * NZ(Fi[k]));
      if (J) {
        for (int p = 0; p < NP; ++p) {
          double aj = 0.0;
          for (int k = 0; k < nf; ++k) aj += Fi[k] * dSf[((size_t)s * nf + k) * NP + p];
          J[((size_t)s * no + i) * NP + p] = aj;
          for (int k = 0; k < nf; ++k)
            ORC_COUNT(ORC_CEN_GRADIENT, 2 * (NZ(Fi[k]) && NZ(dSf[((size_t)s * nf + k) * NP + p])));
        }
      }
    }
  free(Sf);
  free(dSf);
}
