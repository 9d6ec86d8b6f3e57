// Learned initialiser: bfloat16 MFMA multilayer perceptron kernels
// (declarations shared by mlp.hip and the C-ABI layer).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vfisv {

typedef __bf16 bf16;

constexpr int MLP_H = 256;      // hidden width
constexpr int MLP_OUT = 32;     // 10 codes padded to one 32-wide MFMA k-step
constexpr int MLP_NCODE = 10;
constexpr int MLP_SPLITK = 16;  // batch chunks of the weight-gradient GEMMs

// Offsets (in floats) of the packed parameter vector:
//   W1 [K0][H], b1 [H], W2 [H][H], b2 [H], W3 [H][H], b3 [H], W4 [H][32], b4 [32]
// with K0 = n_in rounded up to a multiple of 32 (rows beyond n_in are 0).
struct MlpLayout {
  int n_in, K0;
  int64_t oW[4], ob[4], total;
  int in_dim[4], out_dim[4];
};

inline MlpLayout mlp_layout(int n_in) {
  MlpLayout L;
  L.n_in = n_in;
  L.K0 = (n_in + 31) / 32 * 32;
  const int ins[4] = {L.K0, MLP_H, MLP_H, MLP_H};
  const int outs[4] = {MLP_H, MLP_H, MLP_H, MLP_OUT};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    L.in_dim[l] = ins[l];
    L.out_dim[l] = outs[l];
    L.oW[l] = off;
    off += (int64_t)ins[l] * outs[l];
    L.ob[l] = off;
    off += outs[l];
  }
  L.total = off;
  return L;
}

// Device buffers of one network (owned by the C-ABI object).
struct MlpDev {
  MlpLayout L;
  float* master;      // [total] float32 parameters
  float* adam_m;      // [total]
  float* adam_v;      // [total]
  bf16* Wt[4];        // [out][in]  forward B operand
  bf16* Wk[4];        // [in][out]  backward (dX) B operand
  float* in_mean;     // [K0] (0 beyond n_in)
  float* in_istd;     // [K0] 1/std (0 beyond n_in)
  float* out_mean;    // [7]: v, DlD, a, eta0, S0, S1, alpha
  float* out_std;     // [7]
};

// Work buffers for a batch of M rows.
struct MlpWork {
  int64_t cap;        // rows
  bf16* X0;           // [cap][K0]
  bf16* X0t;          // [K0][cap]        (training)
  bf16* Y[3];         // [cap][H]
  bf16* Yt[3];        // [H][cap]         (training)
  float* Z[3];        // [cap][H] pre-activations (training)
  float* Y4;          // [cap][32]
  bf16* dZ[4];        // [cap][H or 32]   (training)
  bf16* dZt[4];       // [H or 32][cap]   (training)
  float* dW;          // [SPLITK][max layer size] partial weight gradients
  float* grad;        // [total] assembled gradient
  double* loss;       // [1]
};

hipError_t mlp_forward(const MlpDev& net, MlpWork& w, int64_t M, const float* stokes,
                       const int32_t* rows, bool train, hipStream_t s);
hipError_t mlp_decode(const MlpDev& net, const float* Y4, int64_t M, float* codes,
                      float* params, hipStream_t s);
// Fused inference (inputs -> decoded codes/params in one kernel); LDS bytes
// it needs for an input width K0.  The widest input it serves keeps its
// 64-row tile within the 160 KB of LDS of a workgroup.
constexpr int MLP_LDS_MAX = 160 * 1024;
constexpr int MLP_MAX_IN = 1248;  // K0 + 8 padded columns, 64 rows, bf16
hipError_t mlp_infer(const MlpDev& net, int64_t M, const float* stokes, float* codes,
                     float* params, hipStream_t s);
size_t mlp_infer_lds_bytes(int K0);
hipError_t mlp_backward(const MlpDev& net, MlpWork& w, int64_t M, const float* targets,
                        const int32_t* rows, hipStream_t s);
hipError_t mlp_adam(const MlpDev& net, const MlpWork& w, float lr, float beta1, float beta2,
                    float eps, int step, hipStream_t s);
hipError_t mlp_refresh_bf16(const MlpDev& net, hipStream_t s);
hipError_t zero_u64(unsigned long long* p, int n, hipStream_t s);
// dst[0, n) = src[0, n) by a kernel (capturable, unlike a memcpy node).
hipError_t copy_u64(unsigned long long* dst, const unsigned long long* src, int n, hipStream_t s);

// Training-set preparation and the control-set error (the training loop of
// vfisv_mlp_train).  col_moments adds, for columns col0 .. col0 + ncols - 1
// of the row-major X [n][ld], the sum and the sum of squares of each column
// into sums[2 c], sums[2 c + 1] (float64; sums must start at zero).
hipError_t col_moments(const float* X, int64_t n, int ld, int col0, int ncols, double* sums,
                       hipStream_t s);
// Standardised codes T [n][10] of the models P [n][10] (API units): the
// field vector (B cos g, B sin g cos 2 psi, B sin g sin 2 psi) / 3000, then
// (v .. alpha - out_mean) / out_std.
hipError_t encode_targets(const float* P, int64_t n, const float* out_mean, const float* out_std,
                          float* T, hipStream_t s);
// out[0] += sum over count values of (A - B)^2, in float64.
hipError_t sq_diff_sum(const float* A, const float* B, int64_t count, double* out, hipStream_t s);

// Learned-start helpers for the inversion.  Selection: pixels with finite
// chi^2 above tau, and with `unconverged` also those whose status (low 4
// bits) is neither CONVERGED nor NONFINITE.  Merge: the re-fit replaces the
// short fit where its chi^2 is lower, or always with keep_refit.
hipError_t fallback_select(const double* chi2, const int32_t* status, int64_t n, double tau,
                           bool unconverged, int32_t* list, unsigned long long* count,
                           hipStream_t s);
hipError_t fallback_merge(const int32_t* list, const unsigned long long* count, int64_t n,
                          const float* p_fb, const double* c_fb, const int32_t* i_fb,
                          const int32_t* s_fb, bool keep_refit, float* params, double* chi2,
                          int32_t* iters, int32_t* status, hipStream_t s);

}  // namespace vfisv
