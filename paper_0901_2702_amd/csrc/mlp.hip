// Learned initialiser on gfx950: a multilayer perceptron (K0 -> 256 -> 256 ->
// 256 -> 32 (10 used), GELU with the erf normal CDF) evaluated and trained with bfloat16 MFMA
// (v_mfma_f32_16x16x32_bf16, float32 accumulation) and Adam on float32
// master weights.
//
// The paper initialises B, gamma and v_los with small back-propagation
// networks trained on synthetic filtered noisy profiles, with early stopping
// on a control set (Sect. 5).  Here one network proposes all ten starting
// parameters, trained on profiles synthesised by the library's own forward
// model.
//
// Every GEMM is C = A . Bt^T with A [M][Kd] and Bt [N][Kd] both contiguous
// along Kd, so each lane fetches its 8-element MFMA fragments with one
// 16-byte load:  forward  X [B][K] . Wt [N][K]^T;  input gradient
// dZ [B][N] . W [K][N]^T;  weight gradient X^T [K][B] . dZ^T [N][B]^T (in the
// [in][out] order of the master weights, so that the Adam kernel reads it
// coalesced), split along the batch into MLP_SPLITK partial sums that the
// Adam kernel adds.
#include <hip/hip_runtime.h>

#include "me_device.h"
#include "mlp.h"

namespace vfisv {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// GELU(z) = z Phi(z) with the exact (erf) normal CDF Phi, evaluated
// branch-free from erfc(|z| / sqrt 2) by the rational-exponential
// approximation of Abramowitz & Stegun 7.1.26 (Hastings):
//   erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
//   t = 1 / (1 + p x),
// absolute error below 1.5e-7 -- under a thousandth of the bfloat16 step the
// activations are rounded to.  Phi(z) = 1 - erfc(x) / 2 for z >= 0 and
// erfc(x) / 2 for z < 0 (so the negative tail keeps its relative accuracy);
// the halves are folded into the coefficients.  The device library's erff
// branches on |x| (divergent lanes, two polynomials) and took twice the
// instructions of the network's epilogues.
struct PhiPdf {
  float Phi;  // Phi(z)
  float e;    // exp(-z^2 / 2)
};
__device__ __forceinline__ PhiPdf phi_pdf(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = frcp(fmaf(0.3275911f, x, 1.f));
  float p = fmaf(t, 0.5f * 1.061405429f, 0.5f * -1.453152027f);
  p = fmaf(t, p, 0.5f * 1.421413741f);
  p = fmaf(t, p, 0.5f * -0.284496736f);
  p = fmaf(t, p, 0.5f * 0.254829592f);
  // exp(-z^2 / 2) = 2^(-z^2 log2(e) / 2)
  const float e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);
  const float h = t * p * e;  // erfc(x) / 2
  return PhiPdf{z >= 0.f ? 1.f - h : h, e};
}
__device__ __forceinline__ float gelu(float z) { return z * phi_pdf(z).Phi; }
// d/dz [z Phi(z)] = Phi(z) + z phi(z), phi(z) = exp(-z^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_grad(float z) {
  const PhiPdf f = phi_pdf(z);
  return fmaf(z * 0.39894228040143268f, f.e, f.Phi);
}

// ---- GEMM ------------------------------------------------------------------
// One wave computes a 32 x 32 tile of C (2 x 2 MFMA tiles of 16 x 16) over
// the Kd range [z * k_chunk, min((z + 1) * k_chunk, Kd)); Kd and k_chunk are
// multiples of 32.  The fragments of KC k-steps are loaded before the first
// MFMA of the group, so that one memory latency serves KC k-steps (the
// 256-deep products of the hidden layers take one group).  MFMA 16x16x32
// lane layout: lane l feeds A row (l & 15) and B column (l & 15) with
// k = 8 (l >> 4) .. +7, and receives C rows 4 (l >> 4) .. +3 of column
// (l & 15); the epilogue gets those four rows at once.
constexpr int GT = 2;   // 16 x 16 MFMA tiles per wave along each of M and N
constexpr int GKC = 8;  // k-steps loaded per group
template <class Epi>
__global__ __launch_bounds__(64) void gemm_abt(const bf16* __restrict__ A, int64_t lda,
                                               const bf16* __restrict__ Bt, int64_t ldb,
                                               int64_t M, int N, int64_t Kd, int64_t k_chunk,
                                               Epi epi) {
  const int l = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.x * 16 * GT;
  const int n0 = blockIdx.y * 16 * GT;
  const int64_t kbeg = (int64_t)blockIdx.z * k_chunk;
  const int64_t kend = kbeg + k_chunk < Kd ? kbeg + k_chunk : Kd;
  const int lr = l & 15, lk = (l >> 4) * 8;
  f32x4 acc[GT][GT];
#pragma unroll
  for (int rb = 0; rb < GT; ++rb)
#pragma unroll
    for (int cb = 0; cb < GT; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 zero;
#pragma unroll
  for (int i = 0; i < 8; ++i) zero[i] = (bf16)0.f;
  const bf16* arow[GT];
  const bf16* bcol[GT];
  bool aok[GT], bok[GT];
#pragma unroll
  for (int t = 0; t < GT; ++t) {
    const int64_t row = m0 + t * 16 + lr;
    const int col = n0 + t * 16 + lr;
    aok[t] = row < M;
    bok[t] = col < N;
    arow[t] = A + (aok[t] ? row : 0) * lda + lk;
    bcol[t] = Bt + (int64_t)(bok[t] ? col : 0) * ldb + lk;
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += 32 * GKC) {
    bf16x8 a[GKC][GT], b[GKC][GT];
#pragma unroll
    for (int kc = 0; kc < GKC; ++kc) {
      const int64_t k = k0 + 32 * kc;
      const bool kin = k < kend;
#pragma unroll
      for (int t = 0; t < GT; ++t) {
        a[kc][t] = kin && aok[t] ? *(const bf16x8*)(arow[t] + k) : zero;
        b[kc][t] = kin && bok[t] ? *(const bf16x8*)(bcol[t] + k) : zero;
      }
    }
#pragma unroll
    for (int kc = 0; kc < GKC; ++kc) {
      if (k0 + 32 * kc >= kend) break;  // wave-uniform
#pragma unroll
      for (int rb = 0; rb < GT; ++rb)
#pragma unroll
        for (int cb = 0; cb < GT; ++cb)
          acc[rb][cb] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][rb], b[kc][cb], acc[rb][cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int rb = 0; rb < GT; ++rb)
#pragma unroll
    for (int cb = 0; cb < GT; ++cb) {
      const int64_t row0 = m0 + rb * 16 + (l >> 4) * 4;
      const int col = n0 + cb * 16 + lr;
      if (row0 < M && col < N) epi(row0, col, acc[rb][cb], blockIdx.z);
    }
}

// Epilogues receive the four rows row0 .. row0 + 3 (M is a multiple of 32,
// so all four exist) of one column.  Transposed copies store the four
// consecutive values with one 8-byte write.
__device__ __forceinline__ void store4_bf16(bf16* p, float v0, float v1, float v2, float v3) {
  typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
  bf16x4 v;
  v[0] = (bf16)v0;
  v[1] = (bf16)v1;
  v[2] = (bf16)v2;
  v[3] = (bf16)v3;
  *(bf16x4*)p = v;
}

struct EpiHidden {  // z = acc + b; y = gelu(z)
  const float* bias;
  bf16* Y;
  bf16* Yt;
  float* Z;
  int64_t ld, ldt;
  __device__ void operator()(int64_t row0, int col, f32x4 acc, int) const {
    float y[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc[j] + bias[col];
      if (Z) Z[(row0 + j) * ld + col] = z;
      y[j] = gelu(z);
      Y[(row0 + j) * ld + col] = (bf16)y[j];
    }
    if (Yt) store4_bf16(Yt + (int64_t)col * ldt + row0, y[0], y[1], y[2], y[3]);
  }
};

struct EpiOut {  // linear output layer
  const float* bias;
  float* Y4;
  __device__ void operator()(int64_t row0, int col, f32x4 acc, int) const {
#pragma unroll
    for (int j = 0; j < 4; ++j) Y4[(row0 + j) * MLP_OUT + col] = acc[j] + bias[col];
  }
};

struct EpiBwdX {  // dz_prev = (dZ . W^T) * gelu'(z_prev)
  const float* Zp;
  bf16* dZ;
  bf16* dZt;
  int64_t ld, ldt;
  __device__ void operator()(int64_t row0, int col, f32x4 acc, int) const {
    float d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      d[j] = acc[j] * gelu_grad(Zp[(row0 + j) * ld + col]);
      dZ[(row0 + j) * ld + col] = (bf16)d[j];
    }
    store4_bf16(dZt + (int64_t)col * ldt + row0, d[0], d[1], d[2], d[3]);
  }
};

struct EpiDW {  // partial weight gradient, [split][in][out]
  float* part;
  int64_t split_stride;
  int ldo;
  __device__ void operator()(int64_t row0, int col, f32x4 acc, int z) const {
#pragma unroll
    for (int j = 0; j < 4; ++j) part[(int64_t)z * split_stride + (row0 + j) * ldo + col] = acc[j];
  }
};

template <class Epi>
static hipError_t gemm(const bf16* A, int64_t lda, const bf16* Bt, int64_t ldb, int64_t M, int N,
                       int64_t Kd, int splits, const Epi& e, hipStream_t s) {
  const int64_t chunk = ((Kd + splits - 1) / splits + 31) / 32 * 32;
  dim3 grid((unsigned)((M + 16 * GT - 1) / (16 * GT)), (unsigned)((N + 16 * GT - 1) / (16 * GT)),
            (unsigned)splits);
  gemm_abt<Epi><<<grid, 64, 0, s>>>(A, lda, Bt, ldb, M, N, Kd, chunk, e);
  return hipGetLastError();
}

// ---- element-wise kernels --------------------------------------------------

__global__ void encode_kernel(const float* __restrict__ stokes, const int32_t* __restrict__ rows,
                              int64_t M, int n_in, int K0, const float* __restrict__ mean,
                              const float* __restrict__ istd, bf16* X0, bf16* X0t, int64_t cap) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * K0) return;
  const int64_t m = t / K0;
  const int k = (int)(t - m * K0);
  const int64_t src = rows ? (int64_t)rows[m] : m;
  const float x = k < n_in ? (stokes[src * n_in + k] - mean[k]) * istd[k] : 0.f;
  const bf16 xb = (bf16)x;
  X0[m * K0 + k] = xb;
  if (X0t) X0t[(int64_t)k * cap + m] = xb;
}

__global__ void loss_grad_kernel(const float* __restrict__ Y4, const float* __restrict__ T,
                                 const int32_t* __restrict__ rows, int64_t M, int64_t cap,
                                 bf16* dZ, bf16* dZt, double* loss) {
  __shared__ float red[256];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float d2 = 0.f;
  if (t < M * MLP_OUT) {
    const int64_t m = t / MLP_OUT;
    const int c = (int)(t - m * MLP_OUT);
    float d = 0.f;
    if (c < MLP_NCODE) {
      const int64_t src = rows ? (int64_t)rows[m] : m;
      d = Y4[m * MLP_OUT + c] - T[src * MLP_NCODE + c];
    }
    d2 = d * d;
    const bf16 g = (bf16)(2.f * d / (float)(M * MLP_NCODE));
    dZ[m * MLP_OUT + c] = g;
    dZt[(int64_t)c * cap + m] = g;
  }
  red[threadIdx.x] = d2;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, (double)red[0]);
}

// db[n] = sum over the batch of dZ^T[n][:].  One block of 256 threads per
// column; the batch dimension is contiguous, so each thread reads 8 values
// per load (M and cap are multiples of 32: 16-byte aligned rows), then a
// wave reduction and one LDS step combine the 256 partial sums.
// All four layers in one launch: block b takes column b - first[l] of the
// layer l whose columns it falls in.
struct BiasGradArgs {
  const bf16* dZt[4];
  float* grad_b[4];
  int first[5];  // first block of each layer; first[4] = total columns
};

__global__ __launch_bounds__(256) void bias_grad_kernel(const BiasGradArgs a, int64_t M,
                                                        int64_t cap) {
  __shared__ float red[4];
  int l = 0;
  while (l < 3 && (int)blockIdx.x >= a.first[l + 1]) ++l;
  const int n = (int)blockIdx.x - a.first[l];
  float* grad_b = a.grad_b[l];
  const bf16* row = a.dZt[l] + (int64_t)n * cap;
  float s = 0.f;
  for (int64_t m = (int64_t)threadIdx.x * 8; m < M; m += 256 * 8) {
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(row + m);
#pragma unroll
    for (int k = 0; k < 8; ++k) s += (float)v[k];
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) grad_b[n] = (red[0] + red[1]) + (red[2] + red[3]);
}

struct AdamArgs {
  float* master;
  float* m;
  float* v;
  float* grad;
  const float* part[4];
  bf16* Wt[4];
  bf16* Wk[4];
  int64_t oW[4], ob[4];
  int in_dim[4], out_dim[4];
  int64_t split_stride[4];
  int64_t total;
  float lr, beta1, beta2, eps, bc1, bc2;
  int update;  // 0: only assemble the gradient
};

__global__ void adam_kernel(const AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.total) return;
  int l = 0;
  while (l < 3 && i >= a.oW[l + 1]) ++l;
  float g;
  const bool is_w = i < a.ob[l];
  int k = 0, n = 0;
  if (is_w) {
    const int64_t e = i - a.oW[l];
    k = (int)(e / a.out_dim[l]);
    n = (int)(e - (int64_t)k * a.out_dim[l]);
    g = 0.f;
    for (int s = 0; s < MLP_SPLITK; ++s)
      g += a.part[l][(int64_t)s * a.split_stride[l] + e];
    a.grad[i] = g;
  } else {
    g = a.grad[i];  // written by bias_grad_kernel
  }
  if (!a.update) return;
  const float m = a.beta1 * a.m[i] + (1.f - a.beta1) * g;
  const float v = a.beta2 * a.v[i] + (1.f - a.beta2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  const float w = a.master[i] - a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
  a.master[i] = w;
  if (is_w) {
    a.Wt[l][(int64_t)n * a.in_dim[l] + k] = (bf16)w;
    a.Wk[l][(int64_t)k * a.out_dim[l] + n] = (bf16)w;
  }
}

struct RefreshArgs {
  const float* master;
  bf16* Wt[4];
  bf16* Wk[4];
  int64_t oW[4];
  int in_dim[4], out_dim[4];
};

__global__ void refresh_kernel(const RefreshArgs a, int l) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.in_dim[l] * a.out_dim[l]) return;
  const int k = (int)(e / a.out_dim[l]);
  const int n = (int)(e - (int64_t)k * a.out_dim[l]);
  const bf16 w = (bf16)a.master[a.oW[l] + e];
  a.Wt[l][(int64_t)n * a.in_dim[l] + k] = w;
  a.Wk[l][e] = w;
}

// Network outputs -> model parameters (the field vector is encoded as
// (B cos g, B sin g cos 2psi, B sin g sin 2psi) / 3000), then the box.
__device__ __forceinline__ void decode_row(const float* y_in, const float* __restrict__ out_mean,
                                           const float* __restrict__ out_std, float* codes,
                                           float* params) {
  float y[MLP_NCODE];
#pragma unroll
  for (int c = 0; c < MLP_NCODE; ++c) y[c] = y_in[c];
  if (codes) {
#pragma unroll
    for (int c = 0; c < MLP_NCODE; ++c) codes[c] = y[c];
  }
  if (!params) return;
  double P[NPAR];
  const double bt = sqrt((double)y[1] * y[1] + (double)y[2] * y[2]);
  P[0] = 3000.0 * sqrt((double)y[0] * y[0] + bt * bt);
  P[1] = atan2(bt, (double)y[0]) * (180.0 / 3.14159265358979323846);
  P[2] = 0.5 * atan2((double)y[2], (double)y[1]) * (180.0 / 3.14159265358979323846);
#pragma unroll
  for (int c = 3; c < MLP_NCODE; ++c) P[c] = (double)y[c] * out_std[c - 3] + out_mean[c - 3];
  project(P);
#pragma unroll
  for (int c = 0; c < NPAR; ++c) params[c] = (float)P[c];
}

__global__ void decode_kernel(const float* __restrict__ Y4, int64_t M,
                              const float* __restrict__ out_mean,
                              const float* __restrict__ out_std, float* codes, float* params) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  decode_row(Y4 + m * MLP_OUT, out_mean, out_std, codes ? codes + m * MLP_NCODE : nullptr,
             params ? params + m * NPAR : nullptr);
}

// ---- fused inference ---------------------------------------------------------
// One workgroup of four waves carries FT rows through the whole network:
// standardised inputs and hidden activations stay in one LDS tile
// (bfloat16, rows padded by 8 elements so that the 16 rows an MFMA operand
// reads fall in different banks; each layer finishes reading the tile before
// any wave overwrites it with the layer's outputs), weights are read as MFMA
// operands from L2, and the outputs are decoded in place.  Wave w owns
// hidden columns [64 w, 64 w + 64) and output rows [16 w, 16 w + 16).
// (128-row tiles would halve the weight reads but need 335 registers per
// lane, one wave per SIMD: measured 1.5x slower.)  The MFMA sequence per
// output element
// (same instruction, same k order, same epilogue) is that of gemm_abt, so
// the results equal those of the layer-by-layer path.
constexpr int FT = 64;
constexpr int LDH = MLP_H + 8;
// waves per inference workgroup; each owns IW_COLS of a hidden layer's 256
// columns for the tile's 64 rows (eight waves keep the registers per wave
// low enough for four waves per SIMD, which hide the weight loads' latency)
constexpr int IW = 8;
constexpr int IW_CB = MLP_H / (16 * IW);  // 16-column MFMA tiles per wave

struct MlpInferArgs {
  const float* stokes;
  int64_t M;
  int n_in, K0;
  const float* mean;
  const float* istd;
  const bf16* Wt[4];
  const float* bias[4];
  const float* out_mean;
  const float* out_std;
  float* codes;
  float* params;
};

template <int KS>
__device__ __forceinline__ void fused_hidden(bf16* buf, int ldin, int Kd, const bf16* W,
                                             const float* __restrict__ bias, int wave, int l) {
  const bf16* in = buf;
  const int K = KS > 0 ? KS : Kd;
  const int lr = l & 15, lk = (l >> 4) * 8;
  f32x4 acc[4][IW_CB];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < IW_CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16* wrow = W + (int64_t)(wave * 16 * IW_CB + lr) * K + lk;
  auto mfma_step = [&](const bf16x8 (&b)[IW_CB], int k) {
    bf16x8 a[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) a[rb] = *(const bf16x8*)(in + (rb * 16 + lr) * ldin + k + lk);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < IW_CB; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
  };
  if constexpr (KS > 0) {
    // the weights (read from L2 by every row tile) two k-steps ahead of
    // their MFMAs
    constexpr int NK = KS / 32, PF = 2;
    bf16x8 b[NK][IW_CB];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      if (s == 0) {
#pragma unroll
        for (int q = 0; q < PF && q < NK; ++q)
#pragma unroll
          for (int cb = 0; cb < IW_CB; ++cb)
            b[q][cb] = *(const bf16x8*)(wrow + (int64_t)cb * 16 * K + 32 * q);
      }
      if (s + PF < NK) {
#pragma unroll
        for (int cb = 0; cb < IW_CB; ++cb)
          b[s + PF][cb] = *(const bf16x8*)(wrow + (int64_t)cb * 16 * K + 32 * (s + PF));
      }
      mfma_step(b[s], 32 * s);
    }
  } else {
    for (int k = 0; k < K; k += 32) {
      bf16x8 b[IW_CB];
#pragma unroll
      for (int cb = 0; cb < IW_CB; ++cb) b[cb] = *(const bf16x8*)(wrow + (int64_t)cb * 16 * K + k);
      mfma_step(b, k);
    }
  }
  __syncthreads();  // every wave has read the layer's inputs
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < IW_CB; ++cb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + (l >> 4) * 4 + j;
        const int col = wave * 16 * IW_CB + cb * 16 + lr;
        buf[row * LDH + col] = (bf16)gelu(acc[rb][cb][j] + bias[col]);
      }
  __syncthreads();
}

__global__ __launch_bounds__(IW * 64) void mlp_infer_kernel(const MlpInferArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int ldx = a.K0 + 8;
  bf16* buf = (bf16*)smem;  // [FT][max(K0 + 8, LDH)]
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int64_t row0 = (int64_t)blockIdx.x * FT;
  for (int idx = tid; idx < FT * a.K0; idx += IW * 64) {
    const int r = idx / a.K0, k = idx - r * a.K0;
    const int64_t row = row0 + r;
    float x = 0.f;
    if (k < a.n_in && row < a.M) x = (a.stokes[row * a.n_in + k] - a.mean[k]) * a.istd[k];
    buf[r * ldx + k] = (bf16)x;
  }
  __syncthreads();
  fused_hidden<0>(buf, ldx, a.K0, a.Wt[0], a.bias[0], wave, l);
  fused_hidden<MLP_H>(buf, LDH, MLP_H, a.Wt[1], a.bias[1], wave, l);
  fused_hidden<MLP_H>(buf, LDH, MLP_H, a.Wt[2], a.bias[2], wave, l);
  float* y4 = (float*)smem;  // [FT][MLP_OUT + 1], over the tile once it is read
  {  // output layer: waves 0-3 take rows [16 wave, 16 wave + 16), 32 columns
    const int lr = l & 15, lk = (l >> 4) * 8;
    const bool mine = wave < FT / 16;  // wave-uniform
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    if (mine) {
#pragma unroll
      for (int k = 0; k < MLP_H; k += 32) {
        const bf16x8 av = *(const bf16x8*)(buf + (wave * 16 + lr) * LDH + k + lk);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const bf16x8 bv = *(const bf16x8*)(a.Wt[3] + (int64_t)(cb * 16 + lr) * MLP_H + k + lk);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[cb], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // the tile is read; its space takes the outputs
    if (mine) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = wave * 16 + (l >> 4) * 4 + j;
          const int col = cb * 16 + lr;
          y4[row * (MLP_OUT + 1) + col] = acc[cb][j] + a.bias[3][col];
        }
    }
  }
  __syncthreads();
  if (tid < FT) {
    const int64_t row = row0 + tid;
    if (row < a.M)
      decode_row(&y4[tid * (MLP_OUT + 1)], a.out_mean, a.out_std,
                 a.codes ? a.codes + row * MLP_NCODE : nullptr,
                 a.params ? a.params + row * NPAR : nullptr);
  }
}

// Networks with at most 32 inputs (the HMI filtergrams: one k-step in the
// first layer): a persistent grid of one 8-wave workgroup per CU whose waves
// keep their columns' weights of the two 256 x 256 layers in registers
// (128 per lane) and walk the 64-row tiles, so the weights are read from L2 once per
// workgroup instead of once per tile.  The tile and the per-element MFMA
// sequence (same instruction, same k order) are those of mlp_infer_kernel,
// with the hidden layers' operands swapped (the output transposed, so that
// a lane's four results are consecutive columns of one row: one 8-byte LDS
// write instead of four 2-byte ones; each element is the same dot product);
// the hidden layers' GELU comes from a table (below), so an activation may
// differ from mlp_infer_kernel's in its last bfloat16 bit where its value
// lies within 6e-7 of a rounding midpoint.  Output layer: wave w takes rows
// [16 (w / 2), 16 (w / 2) + 16) and columns [16 (w % 2), +16).
// GELU by linear interpolation in a table of GELU at z = -6 + i / 512
// (i < 6144, each entry {GELU(z_i), GELU(z_i+1) - GELU(z_i)}, built in LDS by
// each workgroup from gelu()): interpolation error below (1/512)^2 / 8 times
// max |GELU''| = 0.8, i.e. 4e-7, on top of gelu()'s 1.5e-7, against
// 2^-9 relative for the bfloat16 the result is stored in; above z = 6
// GELU(z) = z to 6e-9, below -6 the first entry (-6e-9) stands for ~0.
// About ten vector instructions instead of gelu()'s thirteen plus two
// transcendental ones, in the epilogue that bounds the resident kernel.
constexpr int GELU_TAB_N = 6144;
__device__ __forceinline__ float gelu_tab(const float2* __restrict__ tab, float z) {
  const float x = fminf(fmaxf(fmaf(z, 512.f, 3072.f), 0.f), (float)(GELU_TAB_N - 1));
  const float i = floorf(x);
  const float2 e = tab[(int)i];
  const float g = fmaf(x - i, e.y, e.x);
  return z >= 6.f ? z : g;
}

__device__ __forceinline__ void resident_hidden_epilogue(bf16* buf, const f32x4 (&acc)[4][IW_CB],
                                                         const float* __restrict__ bias,
                                                         const float2* __restrict__ tab, int wave,
                                                         int l) {
  typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
#pragma unroll
  for (int cb = 0; cb < IW_CB; ++cb) {
    const int col0 = wave * 16 * IW_CB + cb * 16 + (l >> 4) * 4;
    const float4 b4 = *reinterpret_cast<const float4*>(bias + col0);
    const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int row = rb * 16 + (l & 15);
      bf16x4 v;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (bf16)gelu_tab(tab, acc[rb][cb][j] + bb[j]);
      *reinterpret_cast<bf16x4*>(buf + row * LDH + col0) = v;
    }
  }
}

// The layer as D^T = W X^T: the weights are the A operand and the tile's
// rows the B operand, so that lane l receives four consecutive output
// columns of one row and stores them with one 8-byte write.
template <int NK>
__device__ __forceinline__ void resident_hidden(bf16* buf, int ldin, const bf16x8 (&w)[NK][IW_CB],
                                                const float* __restrict__ bias,
                                                const float2* __restrict__ tab, int wave, int l) {
  const int lr = l & 15, lk = (l >> 4) * 8;
  f32x4 acc[4][IW_CB];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < IW_CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NK; ++s) {
    bf16x8 av[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      av[rb] = *(const bf16x8*)(buf + (rb * 16 + lr) * ldin + 32 * s + lk);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < IW_CB; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[s][cb], av[rb], acc[rb][cb], 0, 0, 0);
  }
  __syncthreads();  // every wave has read the layer's inputs
  resident_hidden_epilogue(buf, acc, bias, tab, wave, l);
  __syncthreads();
}

static_assert(IW == 8 && IW_CB == 2, "the resident kernel's output split assumes 8 waves");
// LDS of the resident kernel: the 64-row tile (or the outputs over it), then
// the GELU table
constexpr size_t RESIDENT_TAB_OFFSET = sizeof(bf16) * FT * LDH;
constexpr size_t RESIDENT_LDS = RESIDENT_TAB_OFFSET + sizeof(float2) * GELU_TAB_N;
static_assert(sizeof(float) * FT * (MLP_OUT + 1) <= RESIDENT_TAB_OFFSET && RESIDENT_TAB_OFFSET % 16 == 0,
              "the outputs fit over the tile");

__global__ __launch_bounds__(IW * 64, 1) void mlp_infer_resident_kernel(const MlpInferArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int K0 = 32, NKH = MLP_H / 32;
  constexpr int ldx = K0 + 8;
  bf16* buf = (bf16*)smem;  // [FT][LDH]
  float* y4 = (float*)smem;  // [FT][MLP_OUT + 1], over the tile once it is read
  float2* tab = (float2*)(smem + RESIDENT_TAB_OFFSET);  // [GELU_TAB_N]
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int lr = l & 15, lk = (l >> 4) * 8;
  for (int i = tid; i < GELU_TAB_N; i += IW * 64) {
    const float z0 = -6.f + (float)i * (1.f / 512.f), z1 = -6.f + (float)(i + 1) * (1.f / 512.f);
    const float g0 = gelu(z0);
    tab[i] = make_float2(g0, gelu(z1) - g0);
  }
  // (the table is complete before the first epilogue: the first tile's
  // input barrier comes first)
  // this wave's columns of every layer, as MFMA B fragments
  // (hidden layers 1 and 2: 128 registers; the small first and output
  // layers are read through the caches at each tile)
  bf16x8 w1[NKH][IW_CB], w2[NKH][IW_CB];
#pragma unroll
  for (int cb = 0; cb < IW_CB; ++cb) {
    const int col = wave * 16 * IW_CB + cb * 16 + lr;
#pragma unroll
    for (int s = 0; s < NKH; ++s) {
      w1[s][cb] = *(const bf16x8*)(a.Wt[1] + (int64_t)col * MLP_H + 32 * s + lk);
      w2[s][cb] = *(const bf16x8*)(a.Wt[2] + (int64_t)col * MLP_H + 32 * s + lk);
    }
  }
  const int orb = wave >> 1, ocb = wave & 1;  // output-layer block of this wave
  const int64_t n_tiles = (a.M + FT - 1) / FT;
  // the inputs of the workgroup's next tile are loaded into registers while
  // the current one is computed (4 values per lane), so that their latency
  // is not exposed between the tiles
  constexpr int NXL = FT * K0 / (IW * 64);
  static_assert(NXL * IW * 64 == FT * K0, "whole input tiles");
  float xin[NXL];
  auto load_inputs = [&](int64_t t) {
#pragma unroll
    for (int q = 0; q < NXL; ++q) {
      const int idx = tid + q * IW * 64;
      const int r = idx / K0, k = idx - r * K0;
      const int64_t row = t * FT + r;
      xin[q] = (k < a.n_in && row < a.M) ? a.stokes[row * a.n_in + k] : 0.f;
    }
  };
  if (blockIdx.x < n_tiles) load_inputs(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t row0 = tile * FT;
#pragma unroll
    for (int q = 0; q < NXL; ++q) {
      const int idx = tid + q * IW * 64;
      const int r = idx / K0, k = idx - r * K0;
      buf[r * ldx + k] = (bf16)(k < a.n_in ? (xin[q] - a.mean[k]) * a.istd[k] : 0.f);
    }
    if (tile + gridDim.x < n_tiles) load_inputs(tile + gridDim.x);
    bf16x8 w0[1][IW_CB];
#pragma unroll
    for (int cb = 0; cb < IW_CB; ++cb)
      w0[0][cb] = *(const bf16x8*)(a.Wt[0] + (int64_t)(wave * 16 * IW_CB + cb * 16 + lr) * K0 + lk);
    __syncthreads();
    resident_hidden<1>(buf, ldx, w0, a.bias[0], tab, wave, l);
    resident_hidden<NKH>(buf, LDH, w1, a.bias[1], tab, wave, l);
    resident_hidden<NKH>(buf, LDH, w2, a.bias[2], tab, wave, l);
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NKH; ++s) {
      const bf16x8 av = *(const bf16x8*)(buf + (orb * 16 + lr) * LDH + 32 * s + lk);
      const bf16x8 wv = *(const bf16x8*)(a.Wt[3] + (int64_t)(ocb * 16 + lr) * MLP_H + 32 * s + lk);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, wv, acc, 0, 0, 0);
    }
    __syncthreads();  // the tile is read; its space takes the outputs
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = orb * 16 + (l >> 4) * 4 + j;
      y4[row * (MLP_OUT + 1) + ocb * 16 + lr] = acc[j] + a.bias[3][ocb * 16 + lr];
    }
    __syncthreads();
    if (tid < FT) {
      const int64_t row = row0 + tid;
      if (row < a.M)
        decode_row(&y4[tid * (MLP_OUT + 1)], a.out_mean, a.out_std,
                   a.codes ? a.codes + row * MLP_NCODE : nullptr,
                   a.params ? a.params + row * NPAR : nullptr);
    }
    __syncthreads();  // the outputs are read before the next tile's inputs
  }
}

static_assert(MLP_MAX_IN % 32 == 0 && FT * (MLP_MAX_IN + 8) * 2 <= MLP_LDS_MAX,
              "the widest input must fit a tile");

size_t mlp_infer_lds_bytes(int K0) {
  const int ldx = K0 + 8, ld = ldx > LDH ? ldx : LDH;
  const size_t tile = sizeof(bf16) * (size_t)FT * ld;
  const size_t outs = sizeof(float) * FT * (MLP_OUT + 1);
  return tile > outs ? tile : outs;
}

hipError_t mlp_infer(const MlpDev& net, int64_t M, const float* stokes, float* codes,
                     float* params, hipStream_t s) {
  const MlpLayout& L = net.L;
  MlpInferArgs a;
  a.stokes = stokes;
  a.M = M;
  a.n_in = L.n_in;
  a.K0 = L.K0;
  a.mean = net.in_mean;
  a.istd = net.in_istd;
  for (int l = 0; l < 4; ++l) {
    a.Wt[l] = net.Wt[l];
    a.bias[l] = net.master + L.ob[l];
  }
  a.out_mean = net.out_mean;
  a.out_std = net.out_std;
  a.codes = codes;
  a.params = params;
  // tiles of wide inputs exceed the 64 KB default of dynamic LDS and need
  // the kernel attribute (gfx950 has 160 KB per workgroup); set once per
  // process, before the first launch (not a stream operation)
  static const hipError_t attr = hipFuncSetAttribute(
      (const void*)mlp_infer_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, MLP_LDS_MAX);
  if (attr != hipSuccess) return attr;
  const size_t lds = mlp_infer_lds_bytes(L.K0);
  const int64_t tiles = (M + FT - 1) / FT;
  if (tiles < 1) return hipSuccess;
  if (L.K0 == 32) {
    // one workgroup per CU (the CU count of this device, queried once)
    static int cus[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (cus[dev] == 0) {
      int v = 0;
      e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      cus[dev] = v > 0 ? v : 1;
    }
    static const hipError_t rattr =
        hipFuncSetAttribute((const void*)mlp_infer_resident_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)RESIDENT_LDS);
    if (rattr != hipSuccess) return rattr;
    const int64_t grid = tiles < cus[dev] ? tiles : cus[dev];
    mlp_infer_resident_kernel<<<(unsigned)grid, IW * 64, RESIDENT_LDS, s>>>(a);
    return hipGetLastError();
  }
  mlp_infer_kernel<<<(unsigned)tiles, IW * 64, lds, s>>>(a);
  return hipGetLastError();
}

// Pixels whose fit is not acceptable go to the list.  Each block takes a
// contiguous chunk of SELECT_PER_THREAD * 256 pixels, ranks its selections
// with a block-wide scan in LDS and reserves its slots with one atomic, so
// the counter sees one update per 4096 pixels (same-address atomics
// serialise in L2).
constexpr int SELECT_PER_THREAD = 16;
__global__ __launch_bounds__(256) void fallback_select_kernel(const double* __restrict__ chi2,
                                                              const int32_t* __restrict__ status,
                                                              int64_t n, double tau,
                                                              int unconverged, int32_t* list,
                                                              unsigned long long* count) {
  __shared__ unsigned int scan[256];
  __shared__ unsigned long long base;
  const int t = threadIdx.x;
  const int64_t start = (int64_t)blockIdx.x * 256 * SELECT_PER_THREAD;
  unsigned int mask = 0u, c = 0u;
#pragma unroll
  for (int k = 0; k < SELECT_PER_THREAD; ++k) {
    const int64_t i = start + (int64_t)k * 256 + t;
    if (i < n) {
      const double v = chi2[i];
      bool sel = !(v <= tau) && !isnan(v);  // not acceptable (non-finite input stays as is)
      if (unconverged && !isnan(v)) {
        const int code = status[i] & 15;
        sel = sel || (code != 0 && code != 3);
      }
      if (sel) {
        mask |= 1u << k;
        ++c;
      }
    }
  }
  scan[t] = c;
  __syncthreads();
  // inclusive Hillis-Steele scan over the 256 counts
  for (int off = 1; off < 256; off <<= 1) {
    const unsigned int v = t >= off ? scan[t - off] : 0u;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  if (t == 255) base = scan[255] ? atomicAdd(count, (unsigned long long)scan[255]) : 0ull;
  __syncthreads();
  unsigned long long pos = base + scan[t] - c;
#pragma unroll
  for (int k = 0; k < SELECT_PER_THREAD; ++k)
    if (mask & (1u << k)) list[pos++] = (int32_t)(start + (int64_t)k * 256 + t);
}

__global__ void fallback_merge_kernel(const int32_t* __restrict__ list,
                                      const unsigned long long* __restrict__ count,
                                      const float* __restrict__ p_fb,
                                      const double* __restrict__ c_fb,
                                      const int32_t* __restrict__ i_fb,
                                      const int32_t* __restrict__ s_fb, int keep_refit,
                                      float* params, double* chi2, int32_t* iters,
                                      int32_t* status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((unsigned long long)t >= *count) return;
  const int64_t i = list[t];
  const bool better = keep_refit || c_fb[i] < chi2[i];
  if (better) {
#pragma unroll
    for (int q = 0; q < NPAR; ++q) params[i * NPAR + q] = p_fb[i * NPAR + q];
    chi2[i] = c_fb[i];
  }
  iters[i] += i_fb[i];
  if (status) status[i] = (better ? s_fb[i] : status[i]) | 16;
}

// ---- host-side sequences ---------------------------------------------------

static unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t mlp_forward(const MlpDev& net, MlpWork& w, int64_t M, const float* stokes,
                       const int32_t* rows, bool train, hipStream_t s) {
  const MlpLayout& L = net.L;
  encode_kernel<<<blocks_for(M * L.K0, 256), 256, 0, s>>>(
      stokes, rows, M, L.n_in, L.K0, net.in_mean, net.in_istd, w.X0, train ? w.X0t : nullptr,
      w.cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bf16* X = w.X0;
  int64_t ldx = L.K0;
  for (int l = 0; l < 3; ++l) {
    EpiHidden ep{net.master + L.ob[l], w.Y[l], train ? w.Yt[l] : nullptr,
                 train ? w.Z[l] : nullptr, MLP_H, w.cap};
    e = gemm(X, ldx, net.Wt[l], L.in_dim[l], M, MLP_H, L.in_dim[l], 1, ep, s);
    if (e != hipSuccess) return e;
    X = w.Y[l];
    ldx = MLP_H;
  }
  EpiOut eo{net.master + L.ob[3], w.Y4};
  return gemm(X, ldx, net.Wt[3], MLP_H, M, MLP_OUT, MLP_H, 1, eo, s);
}

hipError_t mlp_decode(const MlpDev& net, const float* Y4, int64_t M, float* codes, float* params,
                      hipStream_t s) {
  decode_kernel<<<blocks_for(M, 256), 256, 0, s>>>(Y4, M, net.out_mean, net.out_std, codes,
                                                   params);
  return hipGetLastError();
}

__global__ void copy_u64_kernel(unsigned long long* dst, const unsigned long long* src, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t copy_u64(unsigned long long* dst, const unsigned long long* src, int n, hipStream_t s) {
  copy_u64_kernel<<<1, 64, 0, s>>>(dst, src, n);
  return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

hipError_t zero_u64(unsigned long long* p, int n, hipStream_t s) {
  zero_u64_kernel<<<blocks_for(n, 64), 64, 0, s>>>(p, n);
  return hipGetLastError();
}

// ---- training-set preparation --------------------------------------------

// Each block takes MOM_ROWS consecutive rows.  With fewer than 256 columns
// thread t owns column t % ncols and every (256 / ncols)-th row from
// t / ncols, so that consecutive threads read consecutive elements; with
// more, thread t owns columns t, t + 256, ...  Sums stay in registers, then
// go to LDS and to the global float64 accumulators once per block.
constexpr int MOM_ROWS = 2048;

__global__ __launch_bounds__(256) void col_moments_kernel(const float* __restrict__ X, int64_t n,
                                                          int ld, int col0, int ncols,
                                                          double* sums) {
  extern __shared__ double acc[];  // [2 * ncols]
  const int t = threadIdx.x;
  for (int c = t; c < 2 * ncols; c += blockDim.x) acc[c] = 0.0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * MOM_ROWS;
  const int rows = (int)(n - r0 < MOM_ROWS ? n - r0 : MOM_ROWS);
  if (ncols < 256) {
    const int tpc = 256 / ncols;
    if (t < tpc * ncols) {
      const int c = t % ncols;
      double s1 = 0.0, s2 = 0.0;
      for (int r = t / ncols; r < rows; r += tpc) {
        const double x = (double)X[(r0 + r) * ld + col0 + c];
        s1 += x;
        s2 += x * x;
      }
      atomicAdd(&acc[2 * c], s1);
      atomicAdd(&acc[2 * c + 1], s2);
    }
  } else {
    for (int c = t; c < ncols; c += 256) {
      double s1 = 0.0, s2 = 0.0;
      for (int r = 0; r < rows; ++r) {
        const double x = (double)X[(r0 + r) * ld + col0 + c];
        s1 += x;
        s2 += x * x;
      }
      acc[2 * c] += s1;  // this thread alone owns column c
      acc[2 * c + 1] += s2;
    }
  }
  __syncthreads();
  for (int c = t; c < 2 * ncols; c += blockDim.x) atomicAdd(&sums[c], acc[c]);
}

hipError_t col_moments(const float* X, int64_t n, int ld, int col0, int ncols, double* sums,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  col_moments_kernel<<<blocks_for(n, MOM_ROWS), 256, sizeof(double) * 2 * ncols, s>>>(
      X, n, ld, col0, ncols, sums);
  return hipGetLastError();
}

__global__ void encode_targets_kernel(const float* __restrict__ P, int64_t n,
                                      const float* __restrict__ out_mean,
                                      const float* __restrict__ out_std, float* T) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const float* p = P + m * NPAR;
  float* t = T + m * MLP_NCODE;
  const float g = p[1] * (float)(3.14159265358979323846 / 180.0);
  const float p2 = p[2] * (float)(3.14159265358979323846 / 90.0);
  const float b = p[0] * (1.f / 3000.f);
  t[0] = b * cosf(g);
  t[1] = b * sinf(g) * cosf(p2);
  t[2] = b * sinf(g) * sinf(p2);
#pragma unroll
  for (int c = 3; c < MLP_NCODE; ++c) t[c] = (p[c] - out_mean[c - 3]) / out_std[c - 3];
}

hipError_t encode_targets(const float* P, int64_t n, const float* out_mean, const float* out_std,
                          float* T, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  encode_targets_kernel<<<blocks_for(n, 256), 256, 0, s>>>(P, n, out_mean, out_std, T);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void sq_diff_sum_kernel(const float* __restrict__ A,
                                                          const float* __restrict__ B,
                                                          int64_t count, double* out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)A[i] - (double)B[i];
    v += d * d;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

hipError_t sq_diff_sum(const float* A, const float* B, int64_t count, double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  sq_diff_sum_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(A, B, count, out);
  return hipGetLastError();
}

hipError_t mlp_backward(const MlpDev& net, MlpWork& w, int64_t M, const float* targets,
                        const int32_t* rows, hipStream_t s) {
  const MlpLayout& L = net.L;
  loss_grad_kernel<<<blocks_for(M * MLP_OUT, 256), 256, 0, s>>>(
      w.Y4, targets, rows, M, w.cap, w.dZ[3], w.dZt[3], w.loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int l = 3; l >= 0; --l) {
    const int out = L.out_dim[l], in = L.in_dim[l];
    const int64_t stride = (int64_t)out * in;
    int64_t off = 0;
    for (int q = 0; q < l; ++q) off += (int64_t)L.in_dim[q] * L.out_dim[q] * MLP_SPLITK;
    // weight gradient: dW[in][out] = X^T[in][B] . dZ^T[out][B]^T
    const bf16* Xt = l == 0 ? w.X0t : w.Yt[l - 1];
    EpiDW ed{w.dW + off, stride, out};
    e = gemm(Xt, w.cap, w.dZt[l], w.cap, in, out, M, MLP_SPLITK, ed, s);
    if (e != hipSuccess) return e;
    if (l > 0) {  // input gradient through W and the previous GELU
      EpiBwdX eb{w.Z[l - 1], w.dZ[l - 1], w.dZt[l - 1], MLP_H, w.cap};
      e = gemm(w.dZ[l], out, net.Wk[l], out, M, in, out, 1, eb, s);
      if (e != hipSuccess) return e;
    }
  }
  // bias gradients of every layer: column sums of dZ^T, one launch
  BiasGradArgs bg;
  int cols = 0;
  for (int l = 0; l < 4; ++l) {
    bg.dZt[l] = w.dZt[l];
    bg.grad_b[l] = w.grad + L.ob[l];
    bg.first[l] = cols;
    cols += L.out_dim[l];
  }
  bg.first[4] = cols;
  bias_grad_kernel<<<cols, 256, 0, s>>>(bg, M, w.cap);
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpDev& net, const MlpWork& w, float lr, float beta1, float beta2,
                    float eps, int step, hipStream_t s) {
  const MlpLayout& L = net.L;
  AdamArgs a;
  a.master = net.master;
  a.m = net.adam_m;
  a.v = net.adam_v;
  a.grad = w.grad;
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    a.part[l] = w.dW + off;
    off += (int64_t)L.in_dim[l] * L.out_dim[l] * MLP_SPLITK;
    a.Wt[l] = net.Wt[l];
    a.Wk[l] = net.Wk[l];
    a.oW[l] = L.oW[l];
    a.ob[l] = L.ob[l];
    a.in_dim[l] = L.in_dim[l];
    a.out_dim[l] = L.out_dim[l];
    a.split_stride[l] = (int64_t)L.in_dim[l] * L.out_dim[l];
  }
  a.total = L.total;
  a.lr = lr;
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  a.update = step > 0 ? 1 : 0;
  a.bc1 = step > 0 ? 1.f - powf(beta1, (float)step) : 1.f;
  a.bc2 = step > 0 ? 1.f - powf(beta2, (float)step) : 1.f;
  adam_kernel<<<blocks_for(L.total, 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t mlp_refresh_bf16(const MlpDev& net, hipStream_t s) {
  RefreshArgs r;
  r.master = net.master;
  for (int l = 0; l < 4; ++l) {
    r.Wt[l] = net.Wt[l];
    r.Wk[l] = net.Wk[l];
    r.oW[l] = net.L.oW[l];
    r.in_dim[l] = net.L.in_dim[l];
    r.out_dim[l] = net.L.out_dim[l];
  }
  for (int l = 0; l < 4; ++l) {
    const int64_t n = (int64_t)net.L.in_dim[l] * net.L.out_dim[l];
    refresh_kernel<<<blocks_for(n, 256), 256, 0, s>>>(r, l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fallback_select(const double* chi2, const int32_t* status, int64_t n, double tau,
                           bool unconverged, int32_t* list, unsigned long long* count,
                           hipStream_t s) {
  if (unconverged && !status) return hipErrorInvalidValue;
  fallback_select_kernel<<<blocks_for(n, 256 * SELECT_PER_THREAD), 256, 0, s>>>(
      chi2, status, n, tau, unconverged ? 1 : 0, list, count);
  return hipGetLastError();
}

hipError_t fallback_merge(const int32_t* list, const unsigned long long* count, int64_t n,
                          const float* p_fb, const double* c_fb, const int32_t* i_fb,
                          const int32_t* s_fb, bool keep_refit, float* params, double* chi2,
                          int32_t* iters, int32_t* status, hipStream_t s) {
  fallback_merge_kernel<<<blocks_for(n, 256), 256, 0, s>>>(
      list, count, p_fb, c_fb, i_fb, s_fb, keep_refit ? 1 : 0, params, chi2, iters, status);
  return hipGetLastError();
}

}  // namespace vfisv
