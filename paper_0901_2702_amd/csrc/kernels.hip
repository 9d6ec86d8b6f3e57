// gfx950 kernels of the Milne-Eddington Levenberg-Marquardt inverter.
//
//  * lm_kernel: persistent, one pixel per lane.  Every loop turn each live
//    lane runs one synthesis pass with derivatives at its current model
//    (the starting model of a fresh pixel, else the trial of the last
//    damped step), decides acceptance on the float64 chi^2 (Eq. 1), keeps
//    the normal equations of the best model in LDS (Fig. 6: derivatives and
//    Hessian of the best model are reused after a failed step), updates the
//    damping by Table 2 and takes the next float64 damped step.  Lanes whose
//    pixel has finished take the next pixel index from a device counter, so
//    pixels with few iterations do not leave lanes idle while other pixels
//    in the wave still iterate.
//  * synth_kernel: the same synthesis pass for given models (values and
//    optional Jacobian), written out.
//  * solve_kernel: the damped solve alone, for given normal equations.
#include <hip/hip_runtime.h>

#include "me_device.h"
#include "kernels.h"

namespace vfisv {

__global__ void reset_work_kernel(unsigned long long* work, int all) {
  if (threadIdx.x < (all ? WORK_SLOTS : 1)) work[threadIdx.x] = 0ull;
}

__device__ __forceinline__ unsigned long long bcast_lane0(unsigned long long v) {
  const unsigned lo = __shfl((unsigned)(v & 0xffffffffull), 0);
  const unsigned hi = __shfl((unsigned)(v >> 32), 0);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffull), off);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), off);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

template <int NOBS>
__global__ __launch_bounds__(64) void lm_kernel(const LMArgs A) {
  constexpr int ROWS = 4 * NOBS;
  __shared__ float sHG[65 * 64];  // H (55, packed) and g (10) per lane
  const int lane = threadIdx.x;
  const int64_t glane = (int64_t)blockIdx.x * 64 + lane;

  const unsigned long long n_total = A.n_dev ? *A.n_dev : (unsigned long long)A.n;
  bool live = false, fresh = false, exhausted = false;
  int64_t pix = 0;
  float Mb[NPAR], Mc[NPAR];
  double chib = 0.0, eps = 0.0;
  int it = 0;
  unsigned long long n_pix = 0, n_trial = 0, n_acc = 0, n_pass = 0, n_fb = 0;

  for (;;) {
    // ---- refill lanes whose pixel finished --------------------------------
    {
      const bool need = !live && !exhausted;
      const unsigned long long nm = __ballot(need);
      if (nm) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&A.work[0], (unsigned long long)__popcll(nm));
        base = bcast_lane0(base);
        if (need) {
          const int rank = __popcll(nm & ((1ull << lane) - 1ull));
          const unsigned long long idx = base + (unsigned long long)rank;
          if (idx < n_total) {
            pix = A.idx ? (int64_t)A.idx[idx] : (int64_t)idx;
            const float* obs = A.stokes + pix * ROWS;
            const float* Wp = A.W_pp ? A.W + pix * ROWS : A.W;
            bool finite = true;
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
              finite = finite && isfinite(obs[r]) && isfinite(Wp[r]);
            if (!finite) {
#pragma unroll
              for (int q = 0; q < NPAR; ++q) A.params[pix * NPAR + q] = __builtin_nanf("");
              A.chi2[pix] = __builtin_nan("");
              A.iters[pix] = 0;
              if (A.status) A.status[pix] = 3;
              ++n_pix;
            } else {
              double M0[NPAR];
              if (A.init) {
#pragma unroll
                for (int q = 0; q < NPAR; ++q) M0[q] = (double)A.init[pix * NPAR + q];
              } else {
                const double d0[NPAR] = {1500.0, 90.0, 90.0, 0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6};
#pragma unroll
                for (int q = 0; q < NPAR; ++q) M0[q] = d0[q];
              }
              project(M0);
#pragma unroll
              for (int q = 0; q < NPAR; ++q) Mc[q] = (float)M0[q];
              live = true;
              fresh = true;
              eps = A.eps0;
              it = 0;
            }
          } else {
            exhausted = true;
          }
        }
      }
    }
    if (__ballot(live) == 0ull) {
      if (__ballot(!exhausted) == 0ull) break;
      continue;  // lanes that met non-finite input refill first
    }
    if (!live) continue;

    // ---- synthesis pass with derivatives at Mc ----------------------------
    ++n_pass;
    Pix px;
    pix_setup(Mc, A.C, px);
    float acc[NOBS][NACC];
    synth_accumulate<NOBS, true>(A.pts, px, A.C, acc);
    RowFactors rf;
    row_factors(Mc, px, A.C, rf);
    const float* obs = A.stokes + pix * ROWS;
    const float* Wp = A.W_pp ? A.W + pix * ROWS : A.W;

    double chi = 0.0;
#pragma unroll
    for (int i = 0; i < NOBS; ++i) {
      float S[4], J[4][NPAR];
      assemble_sample<false>(acc[i], A.C.row_sum[i], rf, S, J);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float r = obs[s * NOBS + i] - S[s];
        chi = fma((double)Wp[s * NOBS + i] * (double)r, (double)r, chi);
      }
    }
    chi *= A.inv_dof;
    const bool accept = fresh || (isfinite(chi) && chi < chib);
    if (accept) {
      float H[55], g[NPAR];
#pragma unroll
      for (int e = 0; e < 55; ++e) H[e] = 0.f;
#pragma unroll
      for (int e = 0; e < NPAR; ++e) g[e] = 0.f;
#pragma unroll
      for (int i = 0; i < NOBS; ++i) {
        float S[4], J[4][NPAR];
        assemble_sample<true>(acc[i], A.C.row_sum[i], rf, S, J);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float w = Wp[s * NOBS + i];
          const float r = obs[s * NOBS + i] - S[s];
#pragma unroll
          for (int p = 0; p < NPAR; ++p) {
            const float wj = w * J[s][p];
            g[p] = fmaf(wj, r, g[p]);
#pragma unroll
            for (int q = 0; q <= p; ++q) H[pk(p, q)] = fmaf(wj, J[s][q], H[pk(p, q)]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 55; ++e) sHG[e * 64 + lane] = H[e];
#pragma unroll
      for (int e = 0; e < NPAR; ++e) sHG[(55 + e) * 64 + lane] = g[e];
    }

    // ---- Levenberg-Marquardt bookkeeping (Sect. 4.2, Table 2) -------------
    int done = -1;
    if (fresh) {
      if (!isfinite(chi)) done = 3;
#pragma unroll
      for (int q = 0; q < NPAR; ++q) Mb[q] = Mc[q];
      chib = chi;
    } else {
      ++it;
      ++n_trial;
      if (accept) {
        const double dec = chib - chi;
#pragma unroll
        for (int q = 0; q < NPAR; ++q) Mb[q] = Mc[q];
        chib = chi;
        eps = eps_down(eps);
        ++n_acc;
        if (dec < A.rel_tol * (chi + dec)) done = 0;
      } else {
        eps = eps_up(eps);
        if (eps > A.eps_max) done = 2;
      }
    }
    fresh = false;
    if (done < 0 && it >= A.max_iter) done = 1;

    if (done >= 0) {
#pragma unroll
      for (int q = 0; q < NPAR; ++q) A.params[pix * NPAR + q] = Mb[q];
      A.chi2[pix] = chib;
      A.iters[pix] = it;
      if (A.status) A.status[pix] = done;
      ++n_pix;
      live = false;
    } else {
      // ---- damped float64 step from the best model ------------------------
      float H[55], g[NPAR];
#pragma unroll
      for (int e = 0; e < 55; ++e) H[e] = sHG[e * 64 + lane];
#pragma unroll
      for (int e = 0; e < NPAR; ++e) g[e] = sHG[(55 + e) * 64 + lane];
      double delta[NPAR], sc[NPAR], b[NPAR];
      const int code = solve_cholesky(H, g, eps, A.free_mask, delta, sc, b);
      if (code == 1) {
        ++n_fb;
        double* ws = A.ws + glane;
        solve_eigen_fallback(&sHG[lane], 64, &sHG[55 * 64 + lane], 64, eps, A.free_mask, ws,
                             A.ws_stride);
#pragma unroll
        for (int q = 0; q < NPAR; ++q) delta[q] = ws[(int64_t)(200 + q) * A.ws_stride];
      }
      double Mt[NPAR];
#pragma unroll
      for (int q = 0; q < NPAR; ++q) Mt[q] = (double)Mb[q] + delta[q];
      project(Mt);
#pragma unroll
      for (int q = 0; q < NPAR; ++q) Mc[q] = (float)Mt[q];
    }
  }

  // ---- work counters: one atomic per wave and counter ----------------------
  n_pix = wave_sum(n_pix);
  n_trial = wave_sum(n_trial);
  n_acc = wave_sum(n_acc);
  n_pass = wave_sum(n_pass);
  n_fb = wave_sum(n_fb);
  if (lane == 0) {
    atomicAdd(&A.work[1], n_pix);
    atomicAdd(&A.work[2], n_trial);
    atomicAdd(&A.work[3], n_acc);
    atomicAdd(&A.work[4], n_pass);
    atomicAdd(&A.work[5], n_fb);
    atomicAdd(&A.work[6], 1ull);
  }
}

template <int NOBS, bool DERIV>
__global__ __launch_bounds__(64) void synth_kernel(const SynthArgs A) {
  constexpr int ROWS = 4 * NOBS;
  for (int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x; i < A.n;
       i += (int64_t)gridDim.x * 64) {
    float M[NPAR];
#pragma unroll
    for (int q = 0; q < NPAR; ++q) M[q] = A.params[i * NPAR + q];
    Pix px;
    pix_setup(M, A.C, px);
    float acc[NOBS][NACC];
    synth_accumulate<NOBS, DERIV>(A.pts, px, A.C, acc);
    RowFactors rf;
    row_factors(M, px, A.C, rf);
#pragma unroll
    for (int o = 0; o < NOBS; ++o) {
      float S[4], J[4][NPAR];
      assemble_sample<DERIV>(acc[o], A.C.row_sum[o], rf, S, J);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t r = i * ROWS + s * NOBS + o;
        A.stokes[r] = A.noise ? S[s] + A.noise[r] : S[s];
        if (DERIV) {
#pragma unroll
          for (int p = 0; p < NPAR; ++p) A.jac[r * NPAR + p] = J[s][p];
        }
      }
    }
  }
}

__global__ __launch_bounds__(64) void solve_kernel(const SolveArgs A) {
  for (int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x; i < A.n;
       i += (int64_t)gridDim.x * 64) {
    float H[55], g[NPAR];
#pragma unroll
    for (int e = 0; e < 55; ++e) H[e] = A.H[i * 55 + e];
#pragma unroll
    for (int e = 0; e < NPAR; ++e) g[e] = A.g[i * NPAR + e];
    double delta[NPAR], sc[NPAR], b[NPAR];
    const double eps = A.eps[i];
    int code = solve_cholesky(H, g, eps, A.free_mask, delta, sc, b);
    if (code == 1) {
      double* ws = A.ws + (int64_t)blockIdx.x * 64 + threadIdx.x;
      solve_eigen_fallback(A.H + i * 55, 1, A.g + i * NPAR, 1, eps, A.free_mask, ws, A.ws_stride);
#pragma unroll
      for (int q = 0; q < NPAR; ++q) delta[q] = ws[(int64_t)(200 + q) * A.ws_stride];
    }
#pragma unroll
    for (int p = 0; p < NPAR; ++p) A.delta[i * NPAR + p] = delta[p];
    if (A.code) A.code[i] = code;
  }
}

// ---- launch helpers (host) --------------------------------------------------

hipError_t launch_reset(unsigned long long* work, bool all, hipStream_t s) {
  reset_work_kernel<<<1, 64, 0, s>>>(work, all ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_lm(const LMArgs& a, int grid, hipStream_t s) {
  lm_kernel<NOBS_HMI><<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_synth(const SynthArgs& a, bool deriv, int grid, hipStream_t s) {
  if (deriv) synth_kernel<NOBS_HMI, true><<<grid, 64, 0, s>>>(a);
  else synth_kernel<NOBS_HMI, false><<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int grid, hipStream_t s) {
  solve_kernel<<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t lm_blocks_per_cu(int* out) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, lm_kernel<NOBS_HMI>, 64, 0);
}

}  // namespace vfisv
