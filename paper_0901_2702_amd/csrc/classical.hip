// Classical initial guess of Sect. 5: the weak-field / magnetograph
// estimates of B and gamma (Jefferies & Mickey 1991), the azimuth from the
// linear polarisation (Auer et al. 1977) and the velocity from the line
// position, per pixel from its observed samples:
//   I_c = max_k I_k; v = c * cog(I_c - I_k) / lambda0;
//   B_par = -sum V_k I'_k / (C_Z sum I'_k^2)      (V = -C_Z B_par dI/dl);
//   B_perp^2 = 4 sum |Q + iU|_k |I''_k| / (C_Z^2 sum I''_k^2);
//   2 psi = atan2(sum U_k I''_k, sum Q_k I''_k);
// with I' and I'' finite differences across the (non-uniform) samples; the
// weak-field signals scale with the filling factor, taken at its default
// 0.6 (B_par / 0.6, B_perp / sqrt(0.6)); the other parameters come from the
// default model, S0 and S1 scaled to I_c.  A vanishing denominator gives 0.
// One pixel per lane; the loops run over the observed samples.
#include <hip/hip_runtime.h>

#include "classical.h"
#include "me_device.h"

namespace vfisv {

__global__ __launch_bounds__(256) void classical_init_kernel(const ClassicalArgs A) {
  const int no = A.n_obs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float* S = A.stokes + i * (int64_t)(4 * no);
    const float* I = S;
    const float* Q = S + no;
    const float* U = S + 2 * no;
    const float* V = S + 3 * no;
    bool finite = true;
    float Ic = -INFINITY;
    for (int k = 0; k < 4 * no; ++k) finite = finite && isfinite(S[k]);
    for (int k = 0; k < no; ++k) Ic = fmaxf(Ic, I[k]);
    float sd = 0.f, sdx = 0.f, sVI = 0.f, sII = 0.f, sLI = 0.f, sI2 = 0.f, sUI = 0.f, sQI = 0.f,
          pol = 0.f;
    for (int k = 0; k < no; ++k) {
      const float d = Ic - I[k];
      sd += d;
      sdx = fmaf(d, A.x[k], sdx);
      // first difference: central inside, one-sided at the ends
      const int a = k > 0 ? k - 1 : 0, b = k < no - 1 ? k + 1 : no - 1;
      const float Ip = (I[b] - I[a]) / (A.x[b] - A.x[a]);
      // second difference: three-point at the interior sample c nearest k
      const int c = k < 1 ? 1 : (k > no - 2 ? no - 2 : k);
      const float h0 = A.x[c] - A.x[c - 1], h1 = A.x[c + 1] - A.x[c];
      const float Ipp =
          2.f * (h0 * I[c + 1] - (h0 + h1) * I[c] + h1 * I[c - 1]) / (h0 * h1 * (h0 + h1));
      const float L = sqrtf(fmaf(Q[k], Q[k], U[k] * U[k]));
      sVI = fmaf(V[k], Ip, sVI);
      sII = fmaf(Ip, Ip, sII);
      sLI = fmaf(L, fabsf(Ipp), sLI);
      sI2 = fmaf(Ipp, Ipp, sI2);
      sUI = fmaf(U[k], Ipp, sUI);
      sQI = fmaf(Q[k], Ipp, sQI);
      pol = fmaxf(pol, sqrtf(fmaf(L, L, V[k] * V[k])));
    }
    double M[NPAR] = {1500.0, 90.0, 90.0, 0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6};
    if (finite && no >= 3) {
      const double lam_cog = sd != 0.f ? (double)sdx / (double)sd : 0.0;
      const double b_par = sII != 0.f ? -(double)sVI / ((double)A.cz * (double)sII) : 0.0;
      const double bp2 =
          sI2 != 0.f ? 4.0 * (double)sLI / ((double)A.cz * (double)A.cz * (double)sI2) : 0.0;
      const double bl = b_par / 0.6, bt = sqrt(fmax(bp2, 0.0)) / sqrt(0.6);
      M[0] = sqrt(bl * bl + bt * bt);
      M[1] = atan2(bt, bl) * (180.0 / 3.14159265358979323846);
      M[2] = 0.5 * atan2((double)sUI, (double)sQI) * (180.0 / 3.14159265358979323846);
      M[3] = C_KMS * lam_cog / (double)A.lam0_mA;
      M[7] = 0.3 * (double)Ic;
      M[8] = 0.7 * (double)Ic;
    }
    project(M);
#pragma unroll
    for (int q = 0; q < NPAR; ++q) A.params[i * NPAR + q] = (float)M[q];
    if (A.pol) A.pol[i] = (finite && Ic > 0.f) ? pol / Ic : __builtin_nanf("");
  }
}

hipError_t launch_classical(const ClassicalArgs& a, int grid, hipStream_t s) {
  classical_init_kernel<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace vfisv
