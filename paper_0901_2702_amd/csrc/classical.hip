// Classical initial guess of Sect. 5: the weak-field / magnetograph
// estimates of B and gamma (Jefferies & Mickey 1991), the azimuth from the
// linear polarisation (Auer et al. 1977) and the velocity from the line
// position, per pixel from its observed samples:
//   I_c = max_k I_k; v = c * cog(I_c - I_k) / lambda0;
//   B_par = -sum V_k I'_k / (C_Z sum I'_k^2)      (V = -C_Z B_par dI/dl);
//   B_perp^2 = 4 sum |Q + iU|_k |I''_k| / (C_Z^2 sum I''_k^2);
//   2 psi = atan2(sum U_k, sum Q_k)   (linear polarisation over the line);
// with I' and I'' finite differences across the (non-uniform) samples; the
// weak-field signals scale with the filling factor, taken at its default
// 0.6 (B_par / 0.6, B_perp / sqrt(0.6)); the other parameters come from the
// default model, S0 and S1 scaled to I_c.  A vanishing denominator gives 0.
// With a base model (the network's start) the two are combined as the
// paper's initialisation does: the azimuth always classical, B and gamma
// classical only below a polarisation level, everything else from the base.
// One pixel per lane; the loops run over the observed samples.  For six
// samples (the filtergram case) a lane loads its pixel's 24 values with six
// 16-byte loads up front and the loops unroll over registers; other sample
// counts read the values from memory as they go.
#include <hip/hip_runtime.h>

#include "classical.h"
#include "me_device.h"

namespace vfisv {

// NO > 0: exactly NO samples, the pixel's rows 16-byte aligned; NO == 0: any.
template <int NO>
__global__ __launch_bounds__(256) void classical_init_kernel(const ClassicalArgs A) {
  const int no = NO > 0 ? NO : A.n_obs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float* G = A.stokes + i * (int64_t)(4 * no);
    float R[NO > 0 ? 4 * NO : 1];
    if constexpr (NO > 0) {
      const float4* g4 = reinterpret_cast<const float4*>(G);
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        const float4 t = g4[j];
        R[4 * j] = t.x;
        R[4 * j + 1] = t.y;
        R[4 * j + 2] = t.z;
        R[4 * j + 3] = t.w;
      }
    }
    // sample k of Stokes parameter s (0 I, 1 Q, 2 U, 3 V)
    auto at = [&](int s, int k) -> float {
      if constexpr (NO > 0)
        return R[s * NO + k];
      else
        return G[s * no + k];
    };
    bool finite = true;
    float Ic = -INFINITY;
#pragma unroll
    for (int k = 0; k < no; ++k)
      finite = finite && isfinite(at(0, k)) && isfinite(at(1, k)) && isfinite(at(2, k)) &&
               isfinite(at(3, k));
#pragma unroll
    for (int k = 0; k < no; ++k) Ic = fmaxf(Ic, at(0, k));
    float sd = 0.f, sdx = 0.f, sVI = 0.f, sII = 0.f, sLI = 0.f, sI2 = 0.f, sU = 0.f, sQ = 0.f,
          pol = 0.f;
#pragma unroll
    for (int k = 0; k < no; ++k) {
      const float d = Ic - at(0, k);
      sd += d;
      sdx = fmaf(d, A.x[k], sdx);
      // first difference: central inside, one-sided at the ends
      const int a = k > 0 ? k - 1 : 0, b = k < no - 1 ? k + 1 : no - 1;
      const float Ip = (at(0, b) - at(0, a)) / (A.x[b] - A.x[a]);
      // second difference: three-point at the interior sample c nearest k
      const int c = k < 1 ? 1 : (k > no - 2 ? no - 2 : k);
      const float h0 = A.x[c] - A.x[c - 1], h1 = A.x[c + 1] - A.x[c];
      const float Ipp = 2.f * (h0 * at(0, c + 1) - (h0 + h1) * at(0, c) + h1 * at(0, c - 1)) /
                        (h0 * h1 * (h0 + h1));
      const float Qk = at(1, k), Uk = at(2, k), Vk = at(3, k);
      const float L = sqrtf(fmaf(Qk, Qk, Uk * Uk));
      sVI = fmaf(Vk, Ip, sVI);
      sII = fmaf(Ip, Ip, sII);
      sLI = fmaf(L, fabsf(Ipp), sLI);
      sI2 = fmaf(Ipp, Ipp, sI2);
      sU += Uk;
      sQ += Qk;
      pol = fmaxf(pol, sqrtf(fmaf(L, L, Vk * Vk)));
    }
    // base rows are read before params rows are written (they may alias)
    double Mb[NPAR];
    if (A.base) {
#pragma unroll
      for (int q = 0; q < NPAR; ++q) Mb[q] = A.base[i * NPAR + q];
    }
    double M[NPAR] = {1500.0, 90.0, 90.0, 0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6};
    const float level = (finite && Ic > 0.f) ? pol / Ic : __builtin_nanf("");
    if (finite && no >= 3) {
      const double lam_cog = sd != 0.f ? (double)sdx / (double)sd : 0.0;
      const double b_par = sII != 0.f ? -(double)sVI / ((double)A.cz * (double)sII) : 0.0;
      const double bp2 =
          sI2 != 0.f ? 4.0 * (double)sLI / ((double)A.cz * (double)A.cz * (double)sI2) : 0.0;
      const double bl = b_par / 0.6, bt = sqrt(fmax(bp2, 0.0)) / sqrt(0.6);
      M[0] = sqrt(bl * bl + bt * bt);
      M[1] = atan2(bt, bl) * (180.0 / 3.14159265358979323846);
      M[2] = 0.5 * atan2((double)sU, (double)sQ) * (180.0 / 3.14159265358979323846);
      M[3] = C_KMS * lam_cog / (double)A.lam0_mA;
      M[7] = 0.3 * (double)Ic;
      M[8] = 0.7 * (double)Ic;
    }
    if (A.base) {
      if (finite) {
        Mb[2] = M[2];
        if (level < A.pol_threshold) {  // false for a NaN level
          Mb[0] = M[0];
          Mb[1] = M[1];
        }
      }
#pragma unroll
      for (int q = 0; q < NPAR; ++q) M[q] = Mb[q];
    }
    project(M);
#pragma unroll
    for (int q = 0; q < NPAR; ++q) A.params[i * NPAR + q] = (float)M[q];
    if (A.pol) A.pol[i] = level;
  }
}

// Per-pixel weights of Sect. 4.3 (Eqs. 1, 14, 15): W = w^2 / sigma^2 with
// w_Q = w_U = w_V = 1 and w_I = 0.7778 |I_c(mu) - I_c| + 0.3, where I_c is
// the pixel's largest observed intensity and I_c(mu) the continuum
// centre-to-limb polynomial (Neckel & Labs 1994) at mu clamped to [0, 1].
// Non-finite mu or Stokes-I samples give NaN for the I weights.
template <int NO>
__global__ __launch_bounds__(256) void weights_kernel(const WeightsArgs A) {
  const int no = NO > 0 ? NO : A.n_obs;
  const float wq = (float)A.inv_var[1], wu = (float)A.inv_var[2], wv = (float)A.inv_var[3];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float* G = A.stokes + i * (int64_t)(4 * no);
    float Ic = -INFINITY;
    bool finite = true;
    if constexpr (NO == 6) {
      const float4 a = *reinterpret_cast<const float4*>(G);
      const float2 b = *reinterpret_cast<const float2*>(G + 4);
      const float v[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        finite = finite && isfinite(v[k]);
        Ic = fmaxf(Ic, v[k]);
      }
    } else {
      for (int k = 0; k < no; ++k) {
        finite = finite && isfinite(G[k]);
        Ic = fmaxf(Ic, G[k]);
      }
    }
    double m = (double)A.mu[i];
    finite = finite && isfinite(m);
    m = fmin(fmax(m, 0.0), 1.0);
    // Eq. 15 by Horner's rule
    const double icm =
        0.33644 +
        m * (1.30590 + m * (-1.79238 + m * (2.45050 + m * (-1.89979 + m * 0.59943))));
    const double wI = 0.7778 * fabs(icm - (double)Ic) + 0.3;
    const float WI = finite ? (float)(wI * wI * A.inv_var[0]) : __builtin_nanf("");
    float* out = A.W + i * (int64_t)(4 * no);
    if constexpr (NO == 6) {
      float4* o4 = reinterpret_cast<float4*>(out);
      o4[0] = make_float4(WI, WI, WI, WI);
      o4[1] = make_float4(WI, WI, wq, wq);
      o4[2] = make_float4(wq, wq, wq, wq);
      o4[3] = make_float4(wu, wu, wu, wu);
      o4[4] = make_float4(wu, wu, wv, wv);
      o4[5] = make_float4(wv, wv, wv, wv);
    } else {
      for (int k = 0; k < no; ++k) {
        out[k] = WI;
        out[no + k] = wq;
        out[2 * no + k] = wu;
        out[3 * no + k] = wv;
      }
    }
  }
}

hipError_t launch_weights(const WeightsArgs& a, int grid, hipStream_t s) {
  if (a.n_obs == 6 && reinterpret_cast<uintptr_t>(a.stokes) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(a.W) % 16 == 0)
    weights_kernel<6><<<grid, 256, 0, s>>>(a);
  else
    weights_kernel<0><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_classical(const ClassicalArgs& a, int grid, hipStream_t s) {
  if (a.n_obs == 6 && reinterpret_cast<uintptr_t>(a.stokes) % 16 == 0)
    classical_init_kernel<6><<<grid, 256, 0, s>>>(a);
  else
    classical_init_kernel<0><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace vfisv
