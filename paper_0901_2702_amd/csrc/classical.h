// Per-pixel preparatory kernels: the classical initial guess and the
// Stokes weights (declarations shared by classical.hip and the C-ABI layer).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vfisv {

struct ClassicalArgs {
  const float* stokes;  // [n][4][n_obs]
  const float* x;       // [n_obs] observed wavelength of each sample [mA]
  int n_obs;
  int64_t n;
  float cz;             // Eq. 7 constant [mA/G]
  float lam0_mA;
  float* params;        // [n][10]
  float* pol;           // [n] polarisation level, or NULL
  const float* base;    // [n][10] model to combine with, or NULL (classical only)
  float pol_threshold;  // with base: classical B and gamma below this level
};

hipError_t launch_classical(const ClassicalArgs& a, int grid, hipStream_t s);

struct WeightsArgs {
  const float* stokes;  // [n][4][n_obs]
  const float* mu;      // [n]
  int n_obs;
  int64_t n;
  double inv_var[4];    // 1 / sigma^2 per Stokes parameter
  float* W;             // [n][4][n_obs]
};

hipError_t launch_weights(const WeightsArgs& a, int grid, hipStream_t s);

}  // namespace vfisv
