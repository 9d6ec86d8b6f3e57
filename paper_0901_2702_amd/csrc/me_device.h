// Device-side Milne-Eddington synthesis, Jacobian, normal equations and
// damped solve for the gfx950 inverter.  One pixel per lane: everything a
// pixel needs per pass lives in that lane's registers; wave-uniform data
// (fine-grid offsets, filter taps, Faddeeva coefficients) comes through the
// scalar cache.
//
// Physics (Borrero et al. 2009, arXiv:0901.2702):
//  * Zeeman triplet of Sect. 3.1: pi component at the (Doppler-shifted) line
//    centre, blue/red sigma components shifted by -/+ C_Z B (Eq. 7).
//  * Voigt H and Faraday-Voigt F (Sect. 3.2) as Re/Im of the Faddeeva
//    function w(u + i a), with the analytic derivatives of Eqs. 8-9.
//  * Milne-Eddington absorption matrix and Unno-Rachkovsky solution for a
//    source function S0 + S1 tau at disk centre (the paper's cited
//    Landolfi & Landi Degl'Innocenti 1982 solution); the magnetised
//    fraction alpha mixes with a field-free component of the same
//    atmosphere (Sect. 2 model vector).
//  * Instrument filter (Sect. 5/7): a linear map from the synthesis grid to
//    the observed samples, applied to values and derivatives alike.
//
// Evaluation choices that differ from the paper's CPU code:
//  * w(z) uses Weideman's (1994) rational series with N = 16 terms, which is
//    branch-free (every lane runs the same instructions) and accurate to
//    ~6e-7 relative in float32, instead of Hui et al. (1977) or the Taylor
//    table of Eqs. 12-13 (~1e-4).
//  * Q and U are synthesised in the frame psi = 0 (eta_U = rho_U = 0) and
//    rotated by 2 psi after filtering; the psi derivatives then follow
//    exactly from dQ/dpsi = -2U, dU/dpsi = 2Q.
//  * The derivatives of the Stokes outputs are taken with respect to the
//    five absorption-matrix elements once per point and chained to the six
//    profile/angle/strength parameters; per-pixel factors (1/Doppler width,
//    C_Z, lambda0/c, degrees) are applied after filtering.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace vfisv {

constexpr int NPAR = 10;
constexpr int NW = 16;          // Weideman series length
constexpr int NOBS_HMI = 6;     // observed samples of the HMI-shaped path
constexpr int NACC = 29;        // per-row accumulators (see synth_pass)
constexpr float INV_SQRT_PI = 0.56418958354775628695f;
constexpr float TWO_OVER_SQRT_PI = 1.1283791670955125739f;
constexpr float DEG = 0.017453292519943295769f;
constexpr double DEG_D = 0.017453292519943295769;
constexpr double C_KMS = 299792.458;

// Wave-uniform constants of one launch (kernel argument -> SGPRs).
constexpr int OV_MAX = 4;  // records shared by the two rows of the register slot 4

struct Consts {
  float wc[NW + 1];      // 2 * a_n, n = 1..NW (index 0 unused)
  float wL, wL2, w2L;    // Weideman L, L^2, 2L
  float lam_over_c;      // lambda0 [mA] / c [km/s]
  float cz;              // Eq. 7 splitting constant [mA/G]
  int n_pts;             // synthesis points with a non-zero tap
  int n_obs;
  float row_sum[8];      // sum of the kept taps of each filter row
  // Dense layout, windowed records (slot order): from record sw_k on, the
  // register slot 4 takes a row that starts there, and the row it held
  // (one that ends within OV_MAX records) is parked in LDS; -1 when the
  // filter has no such pair of rows.  slot_row / slot_rs: filter row and row
  // sum of each slot (slot 5: the parked row).
  int sw_k;
  int slot_row[6];
  float slot_rs[6];
  const float2* vtab;    // Taylor table {H, F} [VT_NA][VT_NU] (Voigt variants 1, 2)
};

// One synthesis point: offset and the taps of the (up to 6) filter rows;
// w[6] carries the bit mask of rows with a non-zero tap.  32 bytes.  In the
// windowed records w[0..4] are the taps of the five register slots and w[5]
// the tap of the parked row.
struct __attribute__((aligned(32))) Point {
  float dl;
  float w[7];
};

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Instrument tables are written once, before any launch, and only read by
// the kernels: reading them through the constant address space lets the
// compiler use scalar loads (one per wave, through the scalar cache) for
// these wave-uniform records instead of per-lane vector loads.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p, int i) {
  static_assert(sizeof(T) % 4 == 0, "records are made of 32-bit words");
  typedef const __attribute__((address_space(4))) float* ConstWords;
  const ConstWords src = (ConstWords)(p + i);
  T out;
  float* dst = reinterpret_cast<float*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
  return out;
}

// Per-pixel quantities of one synthesis pass.
struct Pix {
  float vsi, invD, zs, a, denr, denr2, c0;
  float hs2, hc, hI, hq, hsin2g, hsg, s2h, cgh;
  float eta0, alpha, oma;
  int ja;          // Taylor table: damping node of this pixel
  float a0, da;    //   its damping and the offset a - a0
};

__device__ __forceinline__ void pix_setup(const float* M, const Consts& C, Pix& p) {
  const float B = M[0], g = M[1] * DEG, v = M[3], dld = M[4], a = M[5], eta0 = M[6],
              al = M[9];
  p.invD = frcp(dld);
  p.vsi = C.lam_over_c * v * p.invD;
  p.zs = C.cz * B * p.invD;
  p.a = a;
  p.denr = C.wL + a;
  p.denr2 = p.denr * p.denr;
  p.c0 = C.wL2 - a * a;
  float sg, cg;
  sincosf(g, &sg, &cg);
  const float s2 = sg * sg;
  const float half = 0.5f * eta0;
  p.hs2 = half * s2;
  p.hc = half * cg;
  p.hI = half * (1.f - 0.5f * s2);
  p.hq = 0.5f * p.hs2;
  p.hsin2g = half * 2.f * sg * cg;
  p.hsg = half * sg;
  p.s2h = 0.5f * s2;
  p.cgh = 0.5f * cg;
  p.eta0 = eta0;
  p.alpha = al;
  p.oma = 1.f - al;
  const float ja = fminf(fmaxf(rintf(a * 20.f), 0.f), 99.f);
  p.ja = (int)ja;
  p.a0 = ja * 0.05f;
  p.da = a - p.a0;
}

// Weideman's series for w(z), z = u + i a, a >= 0:
//   w = 1/(sqrt(pi) (L - iz)) + 2/(L - iz)^2 sum_{n=0}^{N-1} a_{n+1} Z^n,
//   Z = (L + iz)/(L - iz).
// With den = L - iz = (L + a) - iu:  Z = ((L^2 - a^2 - u^2) + i 2Lu)/|den|^2.
// The polynomial has real coefficients c_k = 2 a_{k+1}, so it is evaluated
// by the second-order recurrence for division by the real quadratic
// (x - Z)(x - conj Z) = x^2 - r x + s (r = 2 Re Z, s = |Z|^2):
//   b_{N-1} = c_{N-1}, b_k = c_k + r b_{k+1} - s b_{k+2},
//   p(Z) = b_1 Z + c_0 - s b_2,
// two real FMAs per coefficient instead of a complex multiply-add (four);
// in float32 its error matches complex Horner's over a in [0, 5], |u| <= 40
// (both are dominated by the series' own 6e-7 truncation error).
__device__ __forceinline__ void faddeeva(float u, const Pix& p, const Consts& C, float& H,
                                         float& F) {
  const float D = fmaf(u, u, p.denr2);
  const float rD = frcp(D);
  const float idr = p.denr * rD, idi = u * rD;  // 1/den
  const float Zr = fmaf(-u, u, p.c0) * rD;
  const float Zi = C.w2L * idi;
  const float r = 2.f * Zr;
  const float s = fmaf(Zr, Zr, Zi * Zi);
  // c_k = wc[k + 1]
  float b2 = C.wc[NW];
  float b1 = fmaf(r, b2, C.wc[NW - 1]);
#pragma unroll
  for (int k = NW - 3; k >= 1; --k) {
    const float b0 = fmaf(r, b1, fmaf(-s, b2, C.wc[k + 1]));
    b2 = b1;
    b1 = b0;
  }
  const float pr = fmaf(b1, Zr, fmaf(-s, b2, C.wc[1]));
  const float pi = b1 * Zi;
  const float qr = fmaf(pr, idr, fmaf(-pi, idi, INV_SQRT_PI));
  const float qi = fmaf(pr, idi, pi * idr);
  H = fmaf(idr, qr, -idi * qi);
  F = fmaf(idr, qi, idi * qr);
}

// H and F from the Taylor table of Sect. 3.2 (Eqs. 10-13): nodes at
// u = 0.05 i (i < 500), a = 0.05 j (j < 100), nearest node, first or second
// order; H even and F odd in u.  Beyond the last node's cell in |u| the
// asymptotic series w(z) ~ (i / sqrt(pi)) (1/z)(1 + 1/(2z^2) + 3/(4z^4) +
// 15/(8z^6)) is used.  The damping node and offset are per pixel (Pix).
constexpr int VT_NU = 500, VT_NA = 100;
template <int ORDER>
__device__ __forceinline__ void faddeeva_taylor(float u, const Pix& p, const Consts& C, float& H,
                                                float& F) {
  const float x = fabsf(u);
  float Ht, Ft;
  if (x < 24.975f) {
    const float fi = rintf(x * 20.f);
    const float u0 = fi * 0.05f;
    const float2 n = C.vtab[p.ja * VT_NU + (int)fi];
    const float h = n.x, f = n.y;
    const float al = fmaf(2.f * p.a0, h, fmaf(2.f * u0, f, -TWO_OVER_SQRT_PI));
    const float be = 2.f * fmaf(p.a0, f, -u0 * h);
    const float du = x - u0, da = p.da;
    Ht = fmaf(al, da, fmaf(be, du, h));
    Ft = fmaf(be, da, fmaf(-al, du, f));
    if (ORDER >= 2) {
      const float P = fmaf(p.a0, al, fmaf(u0, be, h));
      const float Q = fmaf(p.a0, be, fmaf(-u0, al, f));
      const float d2 = fmaf(da, da, -du * du), dd = 2.f * da * du;
      Ht = fmaf(P, d2, fmaf(Q, dd, Ht));
      Ft = fmaf(Q, d2, fmaf(-P, dd, Ft));
    }
  } else {
    const float a = p.a;
    const float r = frcp(fmaf(x, x, a * a));
    const float zr = x * r, zi = -a * r;  // 1/z
    const float z2r = fmaf(zr, zr, -zi * zi), z2i = 2.f * zr * zi;
    float sr = fmaf(z2r, 1.875f, 0.75f), si = z2i * 1.875f;
    float tr = fmaf(sr, z2r, fmaf(-si, z2i, 0.5f)), ti = fmaf(sr, z2i, si * z2r);
    sr = fmaf(tr, z2r, fmaf(-ti, z2i, 1.f));
    si = fmaf(tr, z2i, ti * z2r);
    const float wr = fmaf(sr, zr, -si * zi), wi = fmaf(sr, zi, si * zr);  // s / z
    Ht = -INV_SQRT_PI * wi;  // w = (i / sqrt(pi)) (s / z)
    Ft = INV_SQRT_PI * wr;
  }
  H = Ht;
  F = u < 0.f ? -Ft : Ft;
}

// H and F by the evaluation the launch uses: 0 Weideman's series,
// 1 or 2 the Taylor table at that order.
template <int V>
__device__ __forceinline__ void voigt_hf(float u, const Pix& p, const Consts& C, float& H,
                                         float& F) {
  if constexpr (V == 0)
    faddeeva(u, p, C, H, F);
  else
    faddeeva_taylor<V>(u, p, C, H, F);
}

// Contributions of one synthesis point to the per-row accumulators
// (all normalised by S1; magnetic Q, U in the psi = 0 frame):
//   c[0] I_mix = alpha I_m + (1 - alpha) I_0,  c[1] I_m - I_0,
//   c[2] Q0, c[3] U0, c[4] V,
//   c[5 + 4q + X], q in {B, gamma, v, Doppler width, a, eta0},
//   X in {I_mix, Q0, U0, V}: derivatives up to per-pixel factors
//   (B: 2 C_Z/DlD, gamma: 1 per radian, v: -2 (lambda0/c)/DlD, DlD: -2/DlD,
//   a: 2, eta0: 1; the factors 2 of Eqs. 8-9 are left to them).
template <bool DERIV, int V = 0>
__device__ __forceinline__ void point_contrib(float dl, const Pix& p, const Consts& C,
                                              float* c) {
  const float up = fmaf(dl, p.invD, -p.vsi);
  const float ub = up + p.zs, ur = up - p.zs;
  float Hp, Fp, Hb, Fb, Hr, Fr;
  voigt_hf<V>(up, p, C, Hp, Fp);
  voigt_hf<V>(ub, p, C, Hb, Fb);
  voigt_hf<V>(ur, p, C, Hr, Fr);

  const float sH = 0.5f * (Hb + Hr), dHl = Hp - sH, dHv = Hr - Hb;
  const float dFl = fmaf(-0.5f, Fb + Fr, Fp), dFv = Fr - Fb;
  // absorption-matrix elements, psi = 0 frame
  const float eI = fmaf(p.eta0, sH, fmaf(p.hs2, dHl, 1.f));
  const float eQ = p.hs2 * dHl, eV = p.hc * dHv;
  const float rQ = p.hs2 * dFl, rV = p.hc * dFv;
  // Unno-Rachkovsky
  const float eI2 = eI * eI;
  const float Pi = fmaf(eQ, rQ, eV * rV);
  const float R2 = fmaf(rQ, rQ, rV * rV);
  const float T = fmaf(-eV, eV, fmaf(-eQ, eQ, eI2)) + R2;
  const float Del = fmaf(eI2, T, -Pi * Pi);
  const float rDel = frcp(Del);
  const float NI = eI * (eI2 + R2);
  const float NQ = fmaf(eI2, eQ, rQ * Pi);
  const float NU = eI * fmaf(eQ, rV, -eV * rQ);
  const float NV = fmaf(eI2, eV, rV * Pi);
  const float Im = NI * rDel, Qh = -NQ * rDel, Uh = -NU * rDel, Vh = -NV * rDel;
  const float I0 = frcp(fmaf(p.eta0, Hp, 1.f));
  c[0] = fmaf(p.alpha, Im, p.oma * I0);
  c[1] = Im - I0;
  c[2] = Qh;
  c[3] = Uh;
  c[4] = Vh;
  if (!DERIV) return;

  // Eqs. 8-9, halved: al = a H + u F - 1/sqrt(pi) = (dH/da) / 2,
  // be = a F - u H = (dF/da) / 2, and dH/du = -dF/da, dF/du = dH/da.  Every
  // tangent below that carries them (B, v, Doppler width, damping) is half
  // its value; the factor 2 is applied with the per-parameter factors after
  // filtering (row_factors, assemble_sample).
  const float alp = fmaf(p.a, Hp, fmaf(up, Fp, -INV_SQRT_PI)), bep = fmaf(p.a, Fp, -up * Hp);
  const float alb = fmaf(p.a, Hb, fmaf(ub, Fb, -INV_SQRT_PI)), beb = fmaf(p.a, Fb, -ub * Hb);
  const float alr = fmaf(p.a, Hr, fmaf(ur, Fr, -INV_SQRT_PI)), ber = fmaf(p.a, Fr, -ur * Hr);
  // the sigma components enter through their sums and differences (below)
  const float Sbe = beb + ber, Dbe = beb - ber, Sal = alb + alr, Dal = alb - alr;
  const float cSbe = p.hc * Sbe, cDbe = p.hc * Dbe, cSal = p.hc * Sal, cDal = p.hc * Dal;

  // the central component's profile tangents times its element factor
  // eta0 sin^2(gamma) / 2, which every output's sensitivity to Hp and Fp carries
  const float alpS = p.hs2 * alp, bepS = p.hs2 * bep;

  // d Delta / d(eta_I, eta_Q, eta_V, rho_Q, rho_V), divided by Delta; the
  // eta_Q and eta_V ones are -2 N_Q and -2 N_V, i.e. 2 Q and 2 V after division
  const float eIr = eI * rDel, eIr2 = eIr + eIr, rQr = rQ * rDel, rVr = rV * rDel,
              Pir = Pi * rDel, eI2r = eI2 * rDel;
  const float DI = eIr2 * (T + eI2);
  const float DQ = Qh + Qh, DV = Vh + Vh;
  const float Dq = 2.f * fmaf(eI2, rQr, -Pir * eQ);
  const float Dw = 2.f * fmaf(eI2, rVr, -Pir * eV);

  // element tangents for gamma (per radian) and eta0
  const float gI = p.hsin2g * dHl, gV = -p.hsg * dHv, gq = p.hsin2g * dFl, gw = -p.hsg * dFv;
  const float nI = fmaf(p.s2h, dHl, sH), nQ = p.s2h * dHl, nV = p.cgh * dHv, nq = p.s2h * dFl,
              nw = p.cgh * dFv;

  // G[X][e] = d(output X)/d(element e), X = N_X/Delta with sign; the
  // I_mix row carries alpha
  float G[4][5];
  {
    const float ra = rDel * p.alpha, Ima = Im * p.alpha, eIr2a = eIr2 * p.alpha;
    G[0][0] = fmaf(-Ima, DI, fmaf(3.f, eI2, R2) * ra);
    G[0][1] = -Ima * DQ;
    G[0][2] = -Ima * DV;
    G[0][3] = fmaf(-Ima, Dq, eIr2a * rQ);
    G[0][4] = fmaf(-Ima, Dw, eIr2a * rV);
  }
  const float qv = rQr * rV;
  G[1][0] = -fmaf(Qh, DI, eIr2 * eQ);
  G[1][1] = -fmaf(Qh, DQ, fmaf(rQr, rQ, eI2r));
  G[1][2] = -fmaf(Qh, DV, qv);
  G[1][3] = -fmaf(Qh, Dq, fmaf(rQr, eQ, Pir));
  G[1][4] = -fmaf(Qh, Dw, rQr * eV);
  G[2][0] = -fmaf(Uh, DI, fmaf(eQ, rV, -eV * rQ) * rDel);
  G[2][1] = -fmaf(Uh, DQ, eIr * rV);
  G[2][2] = -fmaf(Uh, DV, -eIr * rQ);
  G[2][3] = -fmaf(Uh, Dq, -eIr * eV);
  G[2][4] = -fmaf(Uh, Dw, eIr * eQ);
  G[3][0] = -fmaf(Vh, DI, eIr2 * eV);
  G[3][1] = -fmaf(Vh, DQ, qv);
  G[3][2] = -fmaf(Vh, DV, fmaf(rVr, rV, eI2r));
  G[3][3] = -fmaf(Vh, Dq, rVr * eQ);
  G[3][4] = -fmaf(Vh, Dw, fmaf(rVr, eV, Pir));
  // field-free component: dI0/dHp = -eta0 I0^2, dI0/deta0 = -Hp I0^2
  const float I02o = I0 * I0 * p.oma, k0 = -p.eta0 * I02o;
  const float d0v = k0 * bep, d0a = k0 * alp;
  const float d0e = -Hp * I02o;

#pragma unroll
  for (int X = 0; X < 4; ++X) {
    const float GI = G[X][0], GQ = G[X][1], GV = G[X][2], Gq = G[X][3], Gw = G[X][4];
    // sensitivities to the six profile values: SH_p = hs2 GIQ, SF_p = hs2 Gq
    // (hs2 carried by alpS and bepS), SH_b,r = x1 -/+ hc GV,
    // SF_b,r = y1 -/+ hc Gw (hc carried by the c* sums and differences)
    const float GIQ = GI + GQ;
    const float x1 = fmaf(p.hI, GI, -p.hq * GQ);
    const float y1 = -p.hq * Gq;
    // u-tangent weights t_c = SH_c be_c - SF_c al_c: the central one, and
    // the sum and difference of the sigma ones
    const float tp = fmaf(GIQ, bepS, -Gq * alpS);
    const float tbr = fmaf(x1, Sbe, fmaf(-GV, cDbe, fmaf(-y1, Sal, Gw * cDal)));
    const float dB = fmaf(x1, Dbe, fmaf(-GV, cSbe, fmaf(-y1, Dal, Gw * cSal)));
    float dv = tp + tbr;
    // damping: sum over components of SH_c al_c + SF_c be_c
    float da = fmaf(GIQ, alpS, fmaf(Gq, bepS, fmaf(x1, Sal, fmaf(-GV, cDal, fmaf(y1, Sbe, -Gw * cDbe)))));
    const float dg = fmaf(GIQ, gI, fmaf(GV, gV, fmaf(Gq, gq, Gw * gw)));
    float de = fmaf(GI, nI, fmaf(GQ, nQ, fmaf(GV, nV, fmaf(Gq, nq, Gw * nw))));
    if (X == 0) {
      dv += d0v;
      da += d0a;
      de += d0e;
    }
    // Doppler width: sum over components of u_c t_c, with u_b,r = u_p +/- zs
    const float dD = fmaf(up, dv, p.zs * dB);
    c[5 + 0 + X] = dB;
    c[5 + 4 + X] = dg;
    c[5 + 8 + X] = dv;
    c[5 + 12 + X] = dD;
    c[5 + 16 + X] = da;
    c[5 + 20 + X] = de;
  }
}

// Accumulate the filtered contributions of every synthesis point.
template <int NOBS, bool DERIV, int V = 0>
__device__ __forceinline__ void synth_accumulate(const Point* __restrict__ pts, const Pix& p,
                                                 const Consts& C, float (&acc)[NOBS][NACC]) {
  constexpr int NC = DERIV ? NACC : 5;
#pragma unroll
  for (int i = 0; i < NOBS; ++i)
#pragma unroll
    for (int m = 0; m < NACC; ++m) acc[i][m] = 0.f;
  // wave-uniform records through the scalar cache, each loaded one point
  // ahead so that its latency hides behind the current point's arithmetic
  // (one wave per SIMD has nothing else to issue meanwhile)
  const int last = C.n_pts - 1;
  if (last < 0) return;  // no synthesis point carries a tap
  Point P = load_uniform(pts, 0);
  for (int k = 0; k <= last; ++k) {
    const Point Pn = load_uniform(pts, k < last ? k + 1 : last);
    float c[NACC];
    point_contrib<DERIV, V>(P.dl, p, C, c);
    const uint32_t mask = __float_as_uint(P.w[6]);
#pragma unroll
    for (int i = 0; i < NOBS; ++i) {
      if (mask & (1u << i)) {
        const float w = P.w[i];
#pragma unroll
        for (int m = 0; m < NC; ++m) acc[i][m] = fmaf(w, c[m], acc[i][m]);
      }
    }
    P = Pn;
  }
}

// f(std::integral_constant<int, I>{}) for I = 0 .. N-1: the index is a
// constant expression in f, so tables indexed by it fold at compile time
// whatever the unrolling heuristics decide.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Read-modify-write of the float4 slots [C0, C1) of a lane-interleaved LDS
// array (slot c of lane l at base[c * 64 + l]): each read is issued two
// slots ahead of its arithmetic, so that its latency hides behind the
// arithmetic of the slots before it (at one wave per SIMD nothing else
// would).  f(std::integral_constant<int, c>, h) updates slot c in place.
template <int C, int C1, class F>
__device__ __forceinline__ void lds_rmw4_from(float4* __restrict__ base, int lane, float4 a,
                                              float4 b, F& f) {
  if constexpr (C < C1) {
    float4 nb = b;
    if constexpr (C + 2 < C1) nb = base[(C + 2) * 64 + lane];
    float4 h = a;
    f(std::integral_constant<int, C>{}, h);
    base[C * 64 + lane] = h;
    lds_rmw4_from<C + 1, C1>(base, lane, b, nb, f);
  }
}
template <int C0, int C1, class F>
__device__ __forceinline__ void lds_rmw4(float4* __restrict__ base, int lane, F&& f) {
  static_assert(C0 < C1, "empty slot range");
  const float4 a = base[C0 * 64 + lane];
  float4 b = a;
  if constexpr (C0 + 1 < C1) b = base[(C0 + 1) * 64 + lane];
  lds_rmw4_from<C0, C1>(base, lane, a, b, f);
}

// The dense accumulation over windowed records (Consts::sw_k >= 0, so
// 1 <= sw_k <= n_pts - 1): five register slots instead of six rows.  At
// record sw_k the row held by slot 4 is parked in the lane's LDS slots
// (8 float4, lane-interleaved) and slot 4 takes the row that starts there;
// the parked row's taps on the records it still shares with that row (mask
// bit 5) are added in LDS.  Every row receives the same sequence of
// products as in synth_accumulate.
constexpr int PARK4 = (NACC + 3) / 4;  // float4 slots of a parked row

__device__ __forceinline__ float4 pack4(const float* a, int c) {
  return make_float4(a[4 * c], 4 * c + 1 < NACC ? a[4 * c + 1] : 0.f,
                     4 * c + 2 < NACC ? a[4 * c + 2] : 0.f, 4 * c + 3 < NACC ? a[4 * c + 3] : 0.f);
}

template <int V = 0>
__device__ __forceinline__ void synth_accumulate_win(const Point* __restrict__ pts, const Pix& p,
                                                     const Consts& C, float (&acc)[5][NACC],
                                                     float4* __restrict__ park, int lane) {
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int m = 0; m < NACC; ++m) acc[i][m] = 0.f;
  const int last = C.n_pts - 1, sw = C.sw_k;
  // two loops, before and after the switch, so that no accumulator is
  // redefined inside a loop
  auto point = [&](const Point& P, bool parked) {
    float c[NACC];
    point_contrib<true, V>(P.dl, p, C, c);
    const uint32_t mask = __float_as_uint(P.w[6]);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (mask & (1u << i)) {
        const float w = P.w[i];
#pragma unroll
        for (int m = 0; m < NACC; ++m) acc[i][m] = fmaf(w, c[m], acc[i][m]);
      }
    }
    if (parked && (mask & 32u)) {
      const float w = P.w[5];
      lds_rmw4<0, PARK4>(park, lane, [&](auto qq, float4& t) __attribute__((always_inline)) {
        constexpr int q = decltype(qq)::value;
        t.x = fmaf(w, c[4 * q], t.x);
        if constexpr (4 * q + 1 < NACC) t.y = fmaf(w, c[4 * q + 1], t.y);
        if constexpr (4 * q + 2 < NACC) t.z = fmaf(w, c[4 * q + 2], t.z);
        if constexpr (4 * q + 3 < NACC) t.w = fmaf(w, c[4 * q + 3], t.w);
      });
    }
  };
  Point P = load_uniform(pts, 0);
  for (int k = 0; k < sw; ++k) {
    const Point Pn = load_uniform(pts, k + 1);  // k + 1 <= sw <= last
    point(P, false);
    P = Pn;
  }
#pragma unroll
  for (int c = 0; c < PARK4; ++c) park[c * 64 + lane] = pack4(acc[4], c);
#pragma unroll
  for (int m = 0; m < NACC; ++m) acc[4][m] = 0.f;
  for (int k = sw; k <= last; ++k) {
    const Point Pn = load_uniform(pts, k < last ? k + 1 : last);
    point(P, true);
    P = Pn;
  }
}

// The parked row back in registers.
__device__ __forceinline__ void unpark(const float4* __restrict__ park, int lane, float* a) {
#pragma unroll
  for (int q = 0; q < PARK4; ++q) {
    const float4 t = park[q * 64 + lane];
    a[4 * q] = t.x;
    if (4 * q + 1 < NACC) a[4 * q + 1] = t.y;
    if (4 * q + 2 < NACC) a[4 * q + 2] = t.z;
    if (4 * q + 3 < NACC) a[4 * q + 3] = t.w;
  }
}

// The same accumulation shared by a pair of lanes (lane & 1 = odd): each
// lane takes every other synthesis point (two wave-uniform records per
// step, each lane selecting its own), then the pair adds its partial sums,
// so both lanes hold the full sums.  Used when a launch has at least two
// lanes per pixel: a pass then takes about half the time.
template <int NOBS, int V = 0, bool DERIV = true>
__device__ __forceinline__ void synth_accumulate_pair(const Point* __restrict__ pts,
                                                      const Pix& p, const Consts& C,
                                                      float (&acc)[NOBS][NACC], bool odd) {
  constexpr int NC = DERIV ? NACC : 5;
#pragma unroll
  for (int i = 0; i < NOBS; ++i)
#pragma unroll
    for (int m = 0; m < NACC; ++m) acc[i][m] = 0.f;
  for (int k = 0; k < C.n_pts; k += 2) {
    const Point P0 = load_uniform(pts, k);
    Point P1;
    if (k + 1 < C.n_pts) {
      P1 = load_uniform(pts, k + 1);
    } else {
      P1.dl = 0.f;
#pragma unroll
      for (int i = 0; i < 7; ++i) P1.w[i] = 0.f;  // taps and mask zero: contributes nothing
    }
    float c[NACC];
    point_contrib<DERIV, V>(odd ? P1.dl : P0.dl, p, C, c);
    const uint32_t mask = __float_as_uint(P0.w[6]) | __float_as_uint(P1.w[6]);
#pragma unroll
    for (int i = 0; i < NOBS; ++i) {
      if (mask & (1u << i)) {  // a record's taps are zero outside its own mask
        const float w = odd ? P1.w[i] : P0.w[i];
#pragma unroll
        for (int m = 0; m < NC; ++m) acc[i][m] = fmaf(w, c[m], acc[i][m]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NOBS; ++i)
#pragma unroll
    for (int m = 0; m < NC; ++m) acc[i][m] += __shfl_xor(acc[i][m], 1);
}

// Banded instruments (many observed samples, each seeing a short window of
// the synthesis grid that advances BAND_S points per sample, at most
// BAND_S * BAND_R points long).  The grid is cut into blocks of BAND_S
// consecutive points; block b feeds the rows b - BAND_R + 1 .. b, and row j
// is complete once block j + BAND_R - 1 has been added.  w[q][r] is the tap
// of point q of the block in row b - BAND_R + 1 + r (zero outside the band).
constexpr int BAND_S = 4;
constexpr int BAND_R = 4;
struct __attribute__((aligned(16))) Block {
  float dl[BAND_S];
  float w[BAND_S][BAND_R];
};

// Sliding-window accumulation over a banded instrument: only the BAND_R rows
// a block touches are held in registers; each completed row is handed to
// row(j, acc_j) in increasing j, then its registers are reused.  pre(j) is
// called when the block that completes row j starts, so that the caller can
// issue that row's loads early (one wave per SIMD leaves little else to
// hide their latency).
template <bool DERIV, class PreFn, class RowFn>
__device__ __forceinline__ void band_accumulate(const Block* __restrict__ blk, int n_obs,
                                                const Pix& p, const Consts& C, PreFn&& pre,
                                                RowFn&& row) {
  constexpr int NC = DERIV ? NACC : 5;
  float acc[BAND_R][NACC];
#pragma unroll
  for (int r = 0; r < BAND_R; ++r)
#pragma unroll
    for (int m = 0; m < NACC; ++m) acc[r][m] = 0.f;
  const int nb = n_obs + BAND_R - 1;
  for (int b = 0; b < nb; ++b) {
    const Block B = load_uniform(blk, b);  // wave-uniform: one scalar load of the record
    const int j = b - (BAND_R - 1);
    if (j >= 0) pre(j);
#pragma unroll
    for (int q = 0; q < BAND_S; ++q) {
      float c[NACC];
      point_contrib<DERIV>(B.dl[q], p, C, c);
#pragma unroll
      for (int r = 0; r < BAND_R; ++r) {
        const float w = B.w[q][r];
#pragma unroll
        for (int m = 0; m < NC; ++m) acc[r][m] = fmaf(w, c[m], acc[r][m]);
      }
    }
    if (j >= 0) row(j, acc[0]);
#pragma unroll
    for (int r = 0; r < BAND_R - 1; ++r)
#pragma unroll
      for (int m = 0; m < NC; ++m) acc[r][m] = acc[r + 1][m];
#pragma unroll
    for (int m = 0; m < NC; ++m) acc[BAND_R - 1][m] = 0.f;
  }
}

// Per-pixel factors that turn accumulated sums into Stokes values and
// Jacobian rows (API units).
struct RowFactors {
  float S0, S1, alpha, S1a, c2p, s2p;
  float fB, fg, fv, fD;  // per-parameter factors for B, gamma, v, DlD
};

__device__ __forceinline__ void row_factors(const float* M, const Pix& p, const Consts& C,
                                            RowFactors& f) {
  f.S0 = M[7];
  f.S1 = M[8];
  f.alpha = M[9];
  f.S1a = f.S1 * f.alpha;
  sincosf(2.f * M[2] * DEG, &f.s2p, &f.c2p);
  // B, v and Doppler width: twice the factor, since their accumulated
  // tangents are half-values (point_contrib)
  f.fB = 2.f * C.cz * p.invD;
  f.fg = DEG;
  f.fv = -2.f * C.lam_over_c * p.invD;
  f.fD = -2.f * p.invD;
}

// Stokes values (I, Q, U, V) of observed sample i and, with DERIV, the four
// Jacobian rows J[s][0..9].
template <bool DERIV>
__device__ __forceinline__ void assemble_sample(const float* acc, float row_sum,
                                                const RowFactors& f, float S[4],
                                                float J[4][NPAR]) {
  const float Q0 = f.S1a * acc[2], U0 = f.S1a * acc[3];
  S[0] = fmaf(f.S0, row_sum, f.S1 * acc[0]);
  S[1] = fmaf(f.c2p, Q0, -f.s2p * U0);
  S[2] = fmaf(f.s2p, Q0, f.c2p * U0);
  S[3] = f.S1a * acc[4];
  if (!DERIV) return;
  const float qf[6] = {f.fB, f.fg, f.fv, f.fD, 2.f, 1.f};  // damping: half-values too
  const int qidx[6] = {0, 1, 3, 4, 5, 6};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const float dI = acc[5 + 4 * q + 0] * f.S1 * qf[q];
    const float dQ0 = acc[5 + 4 * q + 1] * f.S1a * qf[q];
    const float dU0 = acc[5 + 4 * q + 2] * f.S1a * qf[q];
    const float dV = acc[5 + 4 * q + 3] * f.S1a * qf[q];
    J[0][qidx[q]] = dI;
    J[1][qidx[q]] = fmaf(f.c2p, dQ0, -f.s2p * dU0);
    J[2][qidx[q]] = fmaf(f.s2p, dQ0, f.c2p * dU0);
    J[3][qidx[q]] = dV;
  }
  // azimuth: dQ/dpsi = -2U, dU/dpsi = 2Q (per radian)
  J[0][2] = 0.f;
  J[1][2] = -2.f * DEG * S[2];
  J[2][2] = 2.f * DEG * S[1];
  J[3][2] = 0.f;
  // S0, S1, alpha
  J[0][7] = row_sum;
  J[1][7] = 0.f;
  J[2][7] = 0.f;
  J[3][7] = 0.f;
  const float aQ0 = f.alpha * acc[2], aU0 = f.alpha * acc[3];
  J[0][8] = acc[0];
  J[1][8] = fmaf(f.c2p, aQ0, -f.s2p * aU0);
  J[2][8] = fmaf(f.s2p, aQ0, f.c2p * aU0);
  J[3][8] = f.alpha * acc[4];
  const float sQ0 = f.S1 * acc[2], sU0 = f.S1 * acc[3];
  J[0][9] = f.S1 * acc[1];
  J[1][9] = fmaf(f.c2p, sQ0, -f.s2p * sU0);
  J[2][9] = fmaf(f.s2p, sQ0, f.c2p * sU0);
  J[3][9] = f.S1 * acc[4];
}

__host__ __device__ constexpr int pk(int p, int q) { return p * (p + 1) / 2 + q; }
// Jacobian entries that assemble_sample sets to zero by construction: the
// azimuth column of I and V, the S0 column of Q, U and V.  Products with
// them are left out of g and H (for finite entries that changes nothing).
__host__ __device__ constexpr bool jzero(int s, int p) {
  return (p == 2 && (s == 0 || s == 3)) || (p == 7 && s != 0);
}
// The same for packed entry e of H (row or column 2, row or column 7),
// written without a loop so that it folds in unrolled code.
__host__ __device__ constexpr bool hzero(int s, int e) {
  const bool in2 = (e >= 3 && e <= 5) || e == 8 || e == 12 || e == 17 || e == 23 || e == 30 ||
                   e == 38 || e == 47;
  const bool in7 = (e >= 28 && e <= 35) || e == 43 || e == 52;
  return ((s == 0 || s == 3) && in2) || (s != 0 && in7);
}
// row and column of packed entry e (inverse of pk)
__host__ __device__ constexpr int pk_row(int e) {
  int p = 0;
  while ((p + 1) * (p + 2) / 2 <= e) ++p;
  return p;
}
__host__ __device__ constexpr int pk_col(int e) { return e - pk_row(e) * (pk_row(e) + 1) / 2; }
// float4 slots holding the packed H (entries 0-54) and g (55-64); the
// first slot that holds an entry of g
constexpr int HG4 = (65 + 3) / 4, G4_FIRST = 55 / 4;
constexpr int H4 = (55 + 3) / 4;  // float4 slots holding the packed H alone
static_assert(pk_row(54) == 9 && pk_col(54) == 9 && pk_row(45) == 9 && pk_col(44) == 8, "pk");
constexpr bool hzero_matches() {
  for (int s = 0; s < 4; ++s)
    for (int e = 0; e < 55; ++e)
      if (hzero(s, e) != (jzero(s, pk_row(e)) || jzero(s, pk_col(e)))) return false;
  return true;
}
static_assert(hzero_matches(), "hzero lists the entries of H with a zero factor");

// ---------------------------------------------------------------------
// Damped solve in float64 (Eqs. 3-5 with the diagonal scaled by 1 + eps):
// equilibrate C = D^-1/2 H D^-1/2, Cholesky of C + eps I; frozen or
// leverage-free parameters are decoupled (unit row, zero right-hand side).
// Returns 0 on success, 1 if the factorisation broke down (the caller then
// runs the eigen fallback), 2 if nothing is free.
__device__ __forceinline__ int solve_cholesky(const float* H, const float* g, double eps,
                                              uint32_t free_mask, double* delta, double* sc,
                                              double* b) {
  double maxd = 0.0;
#pragma unroll
  for (int p = 0; p < NPAR; ++p)
    if ((free_mask >> p) & 1u) maxd = fmax(maxd, (double)H[pk(p, p)]);
  int nact = 0;
#pragma unroll
  for (int p = 0; p < NPAR; ++p) {
    const double d = (double)H[pk(p, p)];
    const bool act = ((free_mask >> p) & 1u) && maxd > 0.0 && d > 1e-30 * maxd;
    sc[p] = act ? 1.0 / sqrt(d) : 0.0;
    nact += act ? 1 : 0;
    delta[p] = 0.0;
  }
  if (nact == 0) return 2;
  double L[55];
#pragma unroll
  for (int p = 0; p < NPAR; ++p) {
#pragma unroll
    for (int q = 0; q < p; ++q) L[pk(p, q)] = sc[p] * (double)H[pk(p, q)] * sc[q];
    L[pk(p, p)] = (sc[p] != 0.0) ? 1.0 + eps : 1.0;
    b[p] = sc[p] * (double)g[p];
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NPAR; ++j) {
    double d = L[pk(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-L[pk(j, k)], L[pk(j, k)], d);
    ok = ok && (d > 0.0) && (d < 1.0e300);
    const double ljj = sqrt(fmax(d, 1e-300));
    const double rl = 1.0 / ljj;
    L[pk(j, j)] = ljj;
#pragma unroll
    for (int i = j + 1; i < NPAR; ++i) {
      double s = L[pk(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma(-L[pk(i, k)], L[pk(j, k)], s);
      L[pk(i, j)] = s * rl;
    }
  }
  if (!ok) return 1;
  double y[NPAR];
#pragma unroll
  for (int i = 0; i < NPAR; ++i) {
    double s = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = fma(-L[pk(i, k)], y[k], s);
    y[i] = s / L[pk(i, i)];
  }
#pragma unroll
  for (int i = NPAR - 1; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int k = i + 1; k < NPAR; ++k) s = fma(-L[pk(k, i)], y[k], s);
    y[i] = s / L[pk(i, i)];
  }
#pragma unroll
  for (int p = 0; p < NPAR; ++p) delta[p] = sc[p] * y[p];
  return 0;
}

// Eigen (= SVD, the matrix being symmetric) fallback: cyclic Jacobi on the
// equilibrated C + eps I, components with |lambda| below 1e-12 of the
// largest discarded.  It is rare (a few per million solves), so the whole
// wave computes it for one lane at a time, in an LDS record of WS_DOUBLES
// (A at sws[e], eigenvectors at sws[100 + e], the step written to
// sws[200 + p]): lanes 0..9 take rows or columns of each rotation, lanes
// 10..19 the eigenvector columns.  Off-diagonal elements at the rounding
// level of the matrix (1e-15 of the diagonal's norm) are left unrotated and
// a sweep that rotates nothing ends the iteration.  (Run by the lane alone
// on a workspace in global memory, strided across the grid's lanes, and
// always for its 60 sweeps, it took milliseconds per call.)
constexpr int WS_DOUBLES = 210;

// LDS of a pass, per wave, in float4 slots of 64 lanes: the banded pass's H
// and g (HG4), or the windowed dense pass's H (H4) and parked row (PARK4).
// The eigen-fallback record lies in the parked row's slots: it is used
// between passes only.
constexpr int PASS4 = (HG4 > H4 + PARK4) ? HG4 : H4 + PARK4;
static_assert(PARK4 * 64 * 16 >= WS_DOUBLES * 8, "the fallback record fits the parked row");
__device__ __forceinline__ double* ws_record(float4* sHa) {
  return reinterpret_cast<double*>(sHa + H4 * 64);
}

// Called by all 64 lanes of a one-wave workgroup for the system of lane
// L: H (packed, element stride hs) and g (stride gs) are read through
// generic pointers (LDS or global), eps is lane L's damping.
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __noinline__ void solve_eigen_wave(const float* H, int hs, const float* g, int gs,
                                              double eps, uint32_t free_mask, double* sws,
                                              int lane) {
  double sc[NPAR], b[NPAR];
  double maxd = 0.0;
  for (int p = 0; p < NPAR; ++p)
    if ((free_mask >> p) & 1u) maxd = fmax(maxd, (double)H[pk(p, p) * hs]);
  for (int p = 0; p < NPAR; ++p) {
    const double d = (double)H[pk(p, p) * hs];
    const bool act = ((free_mask >> p) & 1u) && maxd > 0.0 && d > 1e-30 * maxd;
    sc[p] = act ? 1.0 / sqrt(d) : 0.0;
    b[p] = sc[p] * (double)g[p * gs];
  }
  for (int e = lane; e < NPAR * NPAR; e += 64) {
    const int i = e / NPAR, j = e - i * NPAR;
    const int hi = i > j ? pk(i, j) : pk(j, i);
    double v = sc[i] * (double)H[hi * hs] * sc[j];
    if (i == j) v = (sc[i] != 0.0) ? 1.0 + eps : 1.0;
    sws[e] = v;
    sws[100 + e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < NPAR * NPAR; e += 64) {
      const double v = sws[e];
      if (e % (NPAR + 1) == 0) dia += v * v;
      else off += v * v;
    }
    off = wave_sum_f64(off);
    dia = wave_sum_f64(dia);
    if (!(off > 1e-32 * dia)) break;
    const double floor_ = 1e-15 * sqrt(dia);
    bool rotated = false;
    for (int p = 0; p < NPAR - 1; ++p)
      for (int q = p + 1; q < NPAR; ++q) {
        const double apq = sws[p * NPAR + q];
        if (!(fabs(apq) > floor_)) continue;  // the same decision on every lane
        rotated = true;
        const double th = (sws[q * NPAR + q] - sws[p * NPAR + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(fma(th, th, 1.0)));
        const double c = 1.0 / sqrt(fma(t, t, 1.0)), s = t * c;
        __syncthreads();  // every lane has read the pivot elements
        if (lane < NPAR) {  // columns p and q of A
          const int k = lane;
          const double akp = sws[k * NPAR + p], akq = sws[k * NPAR + q];
          sws[k * NPAR + p] = c * akp - s * akq;
          sws[k * NPAR + q] = s * akp + c * akq;
        } else if (lane < 2 * NPAR) {  // columns p and q of V
          const int k = lane - NPAR;
          const double vkp = sws[100 + k * NPAR + p], vkq = sws[100 + k * NPAR + q];
          sws[100 + k * NPAR + p] = c * vkp - s * vkq;
          sws[100 + k * NPAR + q] = s * vkp + c * vkq;
        }
        __syncthreads();
        if (lane < NPAR) {  // rows p and q of A
          const int k = lane;
          const double apk = sws[p * NPAR + k], aqk = sws[q * NPAR + k];
          sws[p * NPAR + k] = c * apk - s * aqk;
          sws[q * NPAR + k] = s * apk + c * aqk;
        }
        __syncthreads();
      }
    if (!rotated) break;
  }
  double lmax = 0.0;
  for (int j = 0; j < NPAR; ++j) lmax = fmax(lmax, fabs(sws[j * NPAR + j]));
  double pr[NPAR];
  for (int j = 0; j < NPAR; ++j) {
    const double lam = sws[j * NPAR + j];
    pr[j] = 0.0;
    if (!(fabs(lam) >= 1e-12 * lmax) || lam == 0.0) continue;
    for (int i = 0; i < NPAR; ++i) pr[j] = fma(sws[100 + i * NPAR + j], b[i], pr[j]);
    pr[j] /= lam;
  }
  __syncthreads();  // A and V are read
  if (lane < NPAR) {
    const int i = lane;
    double y = 0.0;
    for (int j = 0; j < NPAR; ++j) {
      const double lam = sws[j * NPAR + j];
      if (!(fabs(lam) >= 1e-12 * lmax) || lam == 0.0) continue;
      y = fma(sws[100 + i * NPAR + j], pr[j], y);
    }
    sws[200 + i] = sc[i] * y;
  }
  __syncthreads();
}

// Table 2 (rows read top-down).
__device__ __forceinline__ double eps_down(double e) {
  return e > 1e4 ? e * 0.01 : (e >= 1e-4 ? e * 0.1 : e * 0.5);
}
__device__ __forceinline__ double eps_up(double e) {
  return e < 1e-4 ? e * 100.0 : (e > 1e4 ? e * 10.0 : e * 2.0);
}

__device__ __forceinline__ double clampd(double x, double lo, double hi) {
  return fmin(fmax(x, lo), hi);
}

// Box projection after the step: (-B, gamma) == (B, 180 - gamma); gamma is
// even in itself and 360-periodic; psi is 180-periodic; then clip.
__device__ __forceinline__ void project(double* M) {
  if (M[0] < 0.0) {
    M[0] = -M[0];
    M[1] = 180.0 - M[1];
  }
  double g = M[1] - 360.0 * floor(M[1] * (1.0 / 360.0));
  if (g > 180.0) g = 360.0 - g;
  M[1] = clampd(g, 0.0, 180.0);
  double ps = M[2] - 180.0 * floor(M[2] * (1.0 / 180.0));
  M[2] = clampd(ps, 0.0, 180.0);
  M[0] = clampd(M[0], 0.0, 5000.0);
  M[3] = clampd(M[3], -20.0, 20.0);
  M[4] = clampd(M[4], 5.0, 150.0);
  M[5] = clampd(M[5], 0.0, 5.0);
  M[6] = clampd(M[6], 1e-3, 1e3);
  M[7] = clampd(M[7], -1.0, 3.0);
  M[8] = clampd(M[8], 0.0, 5.0);
  M[9] = clampd(M[9], 0.0, 1.0);
}

}  // namespace vfisv
