// Library-internal definitions shared by the C-ABI translation units
// (capi.hip, mlp_capi.hip).  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "kernels.h"
#include "vfisv.h"

namespace vfisv {
// A named range around one C-ABI call, for tracers (roctx: rocprofv3
// --marker-trace shows the calls beside their kernels).  Host-side only:
// nothing is enqueued, so it is safe under graph capture.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace vfisv

struct vfisv_ctx {
  int device = 0;
  int num_cus = 0;
  int lm_blocks_per_cu = 1;
  int band_blocks_per_cu = 1;
  unsigned long long* d_work = nullptr;  // WORK_SLOTS counters
  int64_t max_lanes = 0;                 // lanes of the largest persistent grid
  float2* d_vtab = nullptr;              // Taylor table {H, F}, built on first use
  float wc[vfisv::NW + 1];
  float wL = 0.f;
  // scheduling picked by vfisv_autotune, per instrument layout (KIND_*)
  struct Tuned {
    bool valid = false;
    int grid_waves = 0;
    int chunk_log2 = 8;
    int deriv_split = VFISV_DERIV_SPLIT_DEFAULT;
  } tuned[2];
  // learned-start scratch (grown on demand)
  void* d_learn = nullptr;
  size_t learn_bytes = 0;
  // device address of the fixed scratch array of the allocation-free
  // learned path on this context's device (resolved at vfisv_create)
  void* noalloc_scratch = nullptr;
  // per-phase timing of the learned path (vfisv_learned_phase_timing):
  // events between its phases and the work counters after the short fit
  // ([0, 16)) and after the re-fit ([16, 32))
  bool phase_on = false;
  bool phase_valid = false;
  hipEvent_t phase_ev[6] = {};
  unsigned long long* d_phase_snap = nullptr;
  // interleaved observations of banded batches (grown on demand)
  void* d_obs4 = nullptr;
  size_t obs4_bytes = 0;
  std::string err;
};

struct vfisv_instrument {
  vfisv_ctx* ctx = nullptr;
  int device = 0;  // the context's device, kept so that destroying the
                   // instrument never reads the context
  int kind = vfisv::KIND_DENSE6;
  vfisv::Point* d_pts = nullptr;       // KIND_DENSE6
  vfisv::Point* d_pts5 = nullptr;      // KIND_DENSE6, windowed records (C.sw_k >= 0)
  vfisv::Point* d_ptsv = nullptr;      // KIND_DENSE6, rows in the windowed slot order
  vfisv::Block* d_blocks = nullptr;    // KIND_BAND
  float* d_row_sums = nullptr;         // KIND_BAND
  float* d_obs_x = nullptr;            // [n_obs] observed wavelength of each sample
  vfisv::Consts C;
  vfisv_instrument_info info;
};

namespace vfisv_capi {

// Make ctx's device current and clear the thread's last HIP error, which the
// launch checks read (an earlier call, of this library or not, may have left
// one there).
inline hipError_t use_device(const vfisv_ctx* ctx) {
  const hipError_t e = hipSetDevice(ctx->device);
  (void)hipGetLastError();
  return e;
}

int fail(vfisv_ctx* ctx, int code, const std::string& msg);
int hip_fail(vfisv_ctx* ctx, hipError_t e, const char* what);
int check_inst(vfisv_ctx* ctx, const vfisv_instrument* inst, const char* fn);
int grid_for(int64_t n, int64_t cap);
// Build the Taylor table of H and F on the device (once per context).
int ensure_vtab(vfisv_ctx* ctx);
// may_alloc = false: refuse (VFISV_E_UNSUPPORTED) options that would make
// the library allocate (the Taylor table before it exists).
int check_options(vfisv_ctx* ctx, const vfisv_instrument* inst, const vfisv_options* opt,
                  vfisv_options* out, double* inv_dof, bool may_alloc = true);
// Resolve the device address of the allocation-free path's scratch array on
// ctx's device (current on the calling thread); once per device.
int noalloc_scratch_setup(vfisv_ctx* ctx);

// Enqueue the persistent LM kernel.  With idx != NULL the pixels are
// idx[0 .. count), count read from n_dev on the device (n bounds the grid);
// reset_all clears every work counter, otherwise only the queue heads.
// lpp_max = 2 lets dense pixels use a pair of lanes each when the resident
// lanes give every pixel a pair, or at most a tenth of the pixels wait for
// a free pair (results then differ from the one-lane path by float32
// rounding of the synthesis sums).  may_alloc =
// false: a whole banded batch is read in the API layout instead of through
// the context's interleaved copy (same values, so the same results).
int enqueue_lm(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
               const unsigned long long* n_dev, const int32_t* idx, const float* stokes,
               const float* W, int W_pp, const float* init, const vfisv_options& o,
               double inv_dof, float* params, double* chi2, int32_t* iters, int32_t* status,
               hipStream_t s, bool reset_all, int lpp_max = 1, bool may_alloc = true);

}  // namespace vfisv_capi
