// Kernel argument blocks and launch helpers shared by kernels.hip and the
// C-ABI layer (capi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me_device.h"

namespace vfisv {

// work[] slots: 0 synthesis passes with derivatives, 1 pixels done,
// 2 trials, 3 accepts, 4 passes, 5 eigen fallbacks, 6 waves, 7 J^T W J
// builds, 8 Jacobians the fits need (starts and accepted models that do not
// end their fit); COUNTER_SLOTS counters in all; QUEUE_SLOT0 + NQ * batch +
// q: head of pixel queue q (one per XCD) of a batch
constexpr int NQ = 8;
constexpr int COUNTER_SLOTS = 9;
constexpr int QUEUE_SLOT0 = 16;
constexpr int MAX_BATCHES = 4;
constexpr int WORK_SLOTS = QUEUE_SLOT0 + NQ * MAX_BATCHES;

// Instrument layouts: six observed samples with taps anywhere on the grid
// (HMI-shaped), or a banded filter (Block records).
enum InstKind : int { KIND_DENSE6 = 0, KIND_BAND = 1 };
constexpr int HIST_MAX = 4096;  // iteration-histogram bins (kept after the work slots)

struct LMArgs {
  Consts C;
  const Point* pts;        // KIND_DENSE6
  const Point* pts5;       // KIND_DENSE6, windowed records (C.sw_k >= 0)
  const Point* ptsv;       // KIND_DENSE6, the rows in the windowed pass's slot
                           // order (values-only pass; = pts when C.sw_k < 0)
  const Block* blocks;     // KIND_BAND: C.n_obs + BAND_R - 1 blocks
  const float* row_sums;   // KIND_BAND: [n_obs] sums of the kept taps
  const float* stokes;
  const float* W;
  const float* init;
  float* params;
  double* chi2;
  int32_t* iters;
  int32_t* status;
  unsigned long long* work;
  int64_t n;                         // pixels, unless n_dev is given
  const unsigned long long* n_dev;   // device-side pixel count, or NULL
  const int32_t* idx;                // pixel ids to invert, or NULL (0..n-1)
  double eps0, eps_max, rel_tol, inv_dof;
  int max_iter;
  int W_pp;
  uint32_t free_mask;
  int chunk_log2;  // pixels per queue block = 2^chunk_log2
  int qbase;       // first of this batch's NQ queue-head slots in work[]
  int lpp_max;     // 2: dense pixels may use a pair of lanes when the grid has
                   // at least two lanes per pixel, else 1
  int fixed_iters;  // > 0: fixed-iteration scheme with restarts (else 0)
  int restarts;     // restarts allowed per pixel in that scheme
  unsigned long long seed;  // key of the restart perturbations
  double hess_reuse;        // keep J^T W J for steps from models below this chi^2
  long long lane_cap;       // lanes of the grid that are resident at once
  long long pair_max;       // lane pairs (lpp_max 2) when the batch has at most this
                            // many pixels
  const float4* stokes4;    // KIND_BAND: [n][n_obs] interleaved copy of stokes, or NULL
  int deriv_split;          // 0: every pass computes derivatives (fused); k in 1..64:
                            // values-only passes for the trials, a derivative pass
                            // once k/64 of a wave's live lanes wait for one
};

// Several batches (instrument + pixels + outputs) in one persistent launch:
// every wave works through the batches in order.
struct BatchArgs {
  LMArgs a[MAX_BATCHES];
  int kind[MAX_BATCHES];
  int n_batches;
};

struct SynthArgs {
  Consts C;
  const Point* pts;
  const Block* blocks;
  const float* row_sums;
  const float* params;
  const float* noise;
  float* stokes;
  float* jac;
  int64_t n;
};

struct SolveArgs {
  const float* H;
  const float* g;
  const double* eps;
  double* delta;
  int32_t* code;
  int64_t n;
  uint32_t free_mask;
};

hipError_t launch_reset(unsigned long long* work, bool all, hipStream_t s);
hipError_t launch_hist(const int32_t* iters, int64_t n, int n_bins, unsigned long long* out,
                       int max_blocks, hipStream_t s);
hipError_t launch_lm(const LMArgs& a, int kind, int voigt, int grid, hipStream_t s);
hipError_t launch_lm_batches(const BatchArgs& b, int grid, hipStream_t s);
hipError_t launch_synth(const SynthArgs& a, int kind, int voigt, bool deriv, int grid,
                        hipStream_t s);
hipError_t launch_solve(const SolveArgs& a, int grid, hipStream_t s);
// out[p][j] = (I, Q, U, V) of sample j of pixel p, from in = [n][4][n_obs]
hipError_t launch_interleave(const float* in, float4* out, int64_t n, int n_obs, hipStream_t s);
hipError_t lm_blocks_per_cu(int* out);
hipError_t band_blocks_per_cu(int* out);

}  // namespace vfisv
