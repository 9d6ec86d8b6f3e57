// C ABI of the learned initialiser (network objects, inference, training
// steps, save/load) and of the learned-start inversion with plain-LM
// fallback.  Declared in include/vfisv.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "capi_internal.h"
#include "mlp.h"
#include "vfisv.h"

using namespace vfisv;
using namespace vfisv_capi;

struct vfisv_mlp {
  vfisv_ctx* ctx = nullptr;
  int device = 0;  // the context's device, kept so that destroying the
                   // network never reads the context
  MlpDev dev;
  MlpWork train;
  int step = 0;
  std::vector<float> in_mean, in_std, out_mean, out_std;  // host copies
};

namespace {

// polarisation level below which the weak-field B and gamma replace the
// network's in the combined start (Sect. 5)
constexpr float COMBINED_POL_THRESHOLD = 0.06f;
// version 1: normalisation and parameters; version 2 adds the optimiser
// state (Adam moments and step count) so that training resumes where it was
constexpr uint32_t FILE_VERSION = 2;
const char FILE_MAGIC[8] = {'V', 'F', 'I', 'S', 'V', 'M', 'L', 'P'};

template <class T>
hipError_t dalloc(T** p, int64_t count) {
  return hipMalloc((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

void free_work(MlpWork& w) {
  hipFree(w.X0);
  hipFree(w.X0t);
  for (int l = 0; l < 3; ++l) {
    hipFree(w.Y[l]);
    hipFree(w.Yt[l]);
    hipFree(w.Z[l]);
  }
  hipFree(w.Y4);
  for (int l = 0; l < 4; ++l) {
    hipFree(w.dZ[l]);
    hipFree(w.dZt[l]);
  }
  hipFree(w.dW);
  hipFree(w.grad);
  hipFree(w.loss);
  std::memset(&w, 0, sizeof w);
}

hipError_t alloc_work(MlpWork& w, const MlpLayout& L, int64_t cap, bool training) {
  free_work(w);
  w.cap = cap;
  hipError_t e = dalloc(&w.X0, cap * L.K0);
  for (int l = 0; l < 3 && e == hipSuccess; ++l) e = dalloc(&w.Y[l], cap * MLP_H);
  if (e == hipSuccess) e = dalloc(&w.Y4, cap * MLP_OUT);
  if (e == hipSuccess) e = dalloc(&w.loss, 1);
  if (training) {
    if (e == hipSuccess) e = dalloc(&w.X0t, cap * L.K0);
    for (int l = 0; l < 3 && e == hipSuccess; ++l) e = dalloc(&w.Yt[l], cap * MLP_H);
    for (int l = 0; l < 3 && e == hipSuccess; ++l) e = dalloc(&w.Z[l], cap * MLP_H);
    for (int l = 0; l < 4 && e == hipSuccess; ++l) {
      const int64_t width = l == 3 ? MLP_OUT : MLP_H;
      e = dalloc(&w.dZ[l], cap * width);
      if (e == hipSuccess) e = dalloc(&w.dZt[l], cap * width);
    }
    int64_t part = 0;
    for (int l = 0; l < 4; ++l) part += (int64_t)L.in_dim[l] * L.out_dim[l] * MLP_SPLITK;
    if (e == hipSuccess) e = dalloc(&w.dW, part);
    if (e == hipSuccess) e = dalloc(&w.grad, L.total);
  }
  if (e != hipSuccess) free_work(w);
  return e;
}

void free_dev(MlpDev& d) {
  hipFree(d.master);
  hipFree(d.adam_m);
  hipFree(d.adam_v);
  for (int l = 0; l < 4; ++l) {
    hipFree(d.Wt[l]);
    hipFree(d.Wk[l]);
  }
  hipFree(d.in_mean);
  hipFree(d.in_istd);
  hipFree(d.out_mean);
  hipFree(d.out_std);
}

int build(vfisv_ctx* ctx, int n_in, const float* in_mean, const float* in_std,
          const float* out_mean, const float* out_std, const float* params, uint64_t seed,
          vfisv_mlp** out) {
  if (n_in < 1 || n_in > MLP_MAX_IN)
    return fail(ctx, VFISV_E_INVALID, "mlp: n_in must be 1.." + std::to_string(MLP_MAX_IN));
  if (!in_mean || !in_std || !out_mean || !out_std)
    return fail(ctx, VFISV_E_INVALID, "mlp: NULL normalisation");
  for (int k = 0; k < n_in; ++k)
    if (!std::isfinite(in_mean[k]) || !(in_std[k] > 0.f) || !std::isfinite(in_std[k]))
      return fail(ctx, VFISV_E_INVALID, "mlp: input mean/std must be finite, std > 0");
  for (int k = 0; k < 7; ++k)
    if (!std::isfinite(out_mean[k]) || !(out_std[k] > 0.f) || !std::isfinite(out_std[k]))
      return fail(ctx, VFISV_E_INVALID, "mlp: output mean/std must be finite, std > 0");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  vfisv_mlp* m = new (std::nothrow) vfisv_mlp();
  if (!m) return fail(ctx, VFISV_E_NOMEM, "mlp: host allocation");
  m->ctx = ctx;
  m->device = ctx->device;
  std::memset(&m->dev, 0, sizeof m->dev);
  std::memset(&m->train, 0, sizeof m->train);
  MlpDev& d = m->dev;
  d.L = mlp_layout(n_in);
  const MlpLayout& L = d.L;
  m->in_mean.assign(in_mean, in_mean + n_in);
  m->in_std.assign(in_std, in_std + n_in);
  m->out_mean.assign(out_mean, out_mean + 7);
  m->out_std.assign(out_std, out_std + 7);

  std::vector<float> host(L.total, 0.f);
  if (params) {
    std::memcpy(host.data(), params, sizeof(float) * L.total);
  } else {  // He initialisation; padding rows/columns stay zero
    std::mt19937_64 rng(seed);
    for (int l = 0; l < 4; ++l) {
      const int fan_in = l == 0 ? n_in : L.in_dim[l];
      const int outs = l == 3 ? MLP_NCODE : L.out_dim[l];
      std::normal_distribution<double> nd(0.0, std::sqrt((l == 3 ? 1.0 : 2.0) / fan_in));
      for (int k = 0; k < fan_in; ++k)
        for (int n = 0; n < outs; ++n) host[L.oW[l] + (int64_t)k * L.out_dim[l] + n] = (float)nd(rng);
    }
  }
  std::vector<float> mean(L.K0, 0.f), istd(L.K0, 0.f);
  for (int k = 0; k < n_in; ++k) {
    mean[k] = in_mean[k];
    istd[k] = 1.f / in_std[k];
  }
  e = dalloc(&d.master, L.total);
  if (e == hipSuccess) e = dalloc(&d.adam_m, L.total);
  if (e == hipSuccess) e = dalloc(&d.adam_v, L.total);
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    e = dalloc(&d.Wt[l], (int64_t)L.in_dim[l] * L.out_dim[l]);
    if (e == hipSuccess) e = dalloc(&d.Wk[l], (int64_t)L.in_dim[l] * L.out_dim[l]);
  }
  if (e == hipSuccess) e = dalloc(&d.in_mean, L.K0);
  if (e == hipSuccess) e = dalloc(&d.in_istd, L.K0);
  if (e == hipSuccess) e = dalloc(&d.out_mean, 7);
  if (e == hipSuccess) e = dalloc(&d.out_std, 7);
  if (e != hipSuccess) {
    free_dev(d);
    delete m;
    return fail(ctx, VFISV_E_NOMEM, "mlp: device allocation");
  }
  e = hipMemcpy(d.master, host.data(), sizeof(float) * L.total, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(d.adam_m, 0, sizeof(float) * L.total);
  if (e == hipSuccess) e = hipMemset(d.adam_v, 0, sizeof(float) * L.total);
  if (e == hipSuccess) e = hipMemcpy(d.in_mean, mean.data(), 4 * L.K0, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.in_istd, istd.data(), 4 * L.K0, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.out_mean, out_mean, 4 * 7, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.out_std, out_std, 4 * 7, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = mlp_refresh_bf16(d, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_dev(d);
    delete m;
    return hip_fail(ctx, e, "mlp: upload");
  }
  *out = m;
  return VFISV_OK;
}

int ensure_train(vfisv_mlp* m, int64_t rows) {
  if (m->train.cap >= rows) return VFISV_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = alloc_work(m->train, m->dev.L, rows, true);
  if (e == hipSuccess) e = hipMemset(m->train.loss, 0, sizeof(double));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(m->ctx, VFISV_E_NOMEM, "mlp: training buffers");
  return VFISV_OK;
}

int check_mlp(vfisv_ctx* ctx, const vfisv_mlp* m, const char* fn) {
  if (!m) return fail(ctx, VFISV_E_INVALID, std::string(fn) + ": mlp is NULL");
  if (m->ctx != ctx) return fail(ctx, VFISV_E_INVALID, std::string(fn) + ": mlp of another context");
  return VFISV_OK;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Regularised incomplete gamma functions P(a, x) and Q(a, x) = 1 - P(a, x):
// the power series of P (Abramowitz & Stegun 6.5.29) below x = a + 1, above
// it Legendre's continued fraction for Q (A&S 6.5.31), evaluated by the
// modified Lentz method; the other one by difference, so that each is
// accurate where it is small.
void gamma_pq(double a, double x, double* P, double* Q) {
  if (!(x > 0.0)) {
    *P = 0.0;
    *Q = 1.0;
    return;
  }
  const double pre = std::exp(-x + a * std::log(x) - std::lgamma(a));
  if (x < a + 1.0) {
    double ap = a, term = 1.0 / a, sum = term;
    for (int k = 0; k < 1000000; ++k) {
      ap += 1.0;
      term *= x / ap;
      sum += term;
      if (std::fabs(term) < std::fabs(sum) * 1e-17) break;
    }
    *P = sum * pre;
    *Q = 1.0 - *P;
    return;
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 1000000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-16) break;
  }
  *Q = pre * h;
  *P = 1.0 - *Q;
}

// q-quantile of chi^2_dof / dof: the x with P(dof / 2, x dof / 2) = q, by
// bisection (the CDF is increasing); above the median on Q = 1 - q, so that
// upper quantiles keep their relative accuracy.
double chi2_reduced_quantile(int dof, double q) {
  const double a = 0.5 * dof;
  const bool upper = q > 0.5;
  const double target = upper ? 1.0 - q : q;
  auto below = [&](double x) {  // true while x lies below the quantile
    double P, Q;
    gamma_pq(a, x * a, &P, &Q);
    return upper ? Q > target : P < target;
  };
  double lo = 0.0, hi = 1.0 + 10.0 / std::sqrt((double)dof);
  while (below(hi)) hi *= 2.0;
  for (int it = 0; it < 400 && hi - lo > 1e-14 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid)) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

extern "C" {

int vfisv_mlp_create(vfisv_ctx* ctx, int n_in, const float* in_mean, const float* in_std,
                     const float* out_mean, const float* out_std, uint64_t seed,
                     vfisv_mlp** out) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_create: ctx is NULL");
  if (!out) return fail(ctx, VFISV_E_INVALID, "mlp_create: out is NULL");
  *out = nullptr;
  return build(ctx, n_in, in_mean, in_std, out_mean, out_std, nullptr, seed, out);
}

int vfisv_mlp_destroy(vfisv_mlp* m) {
  if (!m) return VFISV_OK;
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  free_work(m->train);
  free_dev(m->dev);
  delete m;
  return VFISV_OK;
}

int64_t vfisv_mlp_num_params(const vfisv_mlp* m) { return m ? m->dev.L.total : -1; }

int vfisv_mlp_num_inputs(const vfisv_mlp* m) { return m ? m->dev.L.n_in : -1; }

int vfisv_mlp_get_params(vfisv_mlp* m, float* host, int64_t n) {
  if (!m || !host) return VFISV_E_INVALID;
  if (n != m->dev.L.total) return fail(m->ctx, VFISV_E_INVALID, "mlp_get_params: size mismatch");
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host, m->dev.master, 4 * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(m->ctx, e, "mlp_get_params");
  return VFISV_OK;
}

int vfisv_mlp_set_params(vfisv_mlp* m, const float* host, int64_t n) {
  if (!m || !host) return VFISV_E_INVALID;
  if (n != m->dev.L.total) return fail(m->ctx, VFISV_E_INVALID, "mlp_set_params: size mismatch");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return fail(m->ctx, VFISV_E_INVALID, "mlp_set_params: non-finite");
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(m->dev.master, host, 4 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->dev.adam_m, 0, 4 * n);
  if (e == hipSuccess) e = hipMemset(m->dev.adam_v, 0, 4 * n);
  if (e == hipSuccess) e = mlp_refresh_bf16(m->dev, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(m->ctx, e, "mlp_set_params");
  m->step = 0;
  return VFISV_OK;
}

int vfisv_mlp_forward(vfisv_ctx* ctx, vfisv_mlp* m, int64_t n, const float* stokes, float* codes,
                      float* params, void* stream) {
  vfisv::TraceRange trace_("vfisv_mlp_forward");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_forward: ctx is NULL");
  int rc = check_mlp(ctx, m, "mlp_forward");
  if (rc) return rc;
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "mlp_forward: n < 0");
  if (n == 0) return VFISV_OK;
  if (!stokes || (!codes && !params)) return fail(ctx, VFISV_E_INVALID, "mlp_forward: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  // one fused launch: inputs -> decoded codes / starting models, no scratch
  e = mlp_infer(m->dev, n, stokes, codes, params, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "mlp_forward");
  return VFISV_OK;
}

int vfisv_mlp_gradient(vfisv_ctx* ctx, vfisv_mlp* m, int64_t n, const float* stokes,
                       const float* targets, float* grad, double* loss, void* stream) {
  vfisv::TraceRange trace_("vfisv_mlp_gradient");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_gradient: ctx is NULL");
  int rc = check_mlp(ctx, m, "mlp_gradient");
  if (rc) return rc;
  if (n <= 0 || n % 32 != 0 || n > (1 << 22))
    return fail(ctx, VFISV_E_INVALID, "mlp_gradient: n must be a positive multiple of 32");
  if (!stokes || !targets || !grad) return fail(ctx, VFISV_E_INVALID, "mlp_gradient: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  rc = ensure_train(m, n);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  MlpWork& w = m->train;
  e = zero_u64((unsigned long long*)w.loss, 1, s);
  if (e == hipSuccess) e = mlp_forward(m->dev, w, n, stokes, nullptr, true, s);
  if (e == hipSuccess) e = mlp_backward(m->dev, w, n, targets, nullptr, s);
  if (e == hipSuccess) e = mlp_adam(m->dev, w, 0.f, 0.f, 0.f, 0.f, 0, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, w.grad, 4 * m->dev.L.total, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, w.loss, 8, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "mlp_gradient");
  return VFISV_OK;
}

int vfisv_mlp_train_step(vfisv_ctx* ctx, vfisv_mlp* m, const float* stokes, const float* targets,
                         const int32_t* rows, int batch, float lr, void* stream) {
  vfisv::TraceRange trace_("vfisv_mlp_train_step");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_train_step: ctx is NULL");
  int rc = check_mlp(ctx, m, "mlp_train_step");
  if (rc) return rc;
  if (batch <= 0 || batch % 32 != 0 || batch > (1 << 20))
    return fail(ctx, VFISV_E_INVALID, "mlp_train_step: batch must be a positive multiple of 32");
  if (!stokes || !targets || !rows) return fail(ctx, VFISV_E_INVALID, "mlp_train_step: NULL buffer");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(ctx, VFISV_E_INVALID, "mlp_train_step: lr");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  rc = ensure_train(m, batch);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  MlpWork& w = m->train;
  e = mlp_forward(m->dev, w, batch, stokes, rows, true, s);
  if (e == hipSuccess) e = mlp_backward(m->dev, w, batch, targets, rows, s);
  if (e == hipSuccess) e = mlp_adam(m->dev, w, lr, 0.9f, 0.999f, 1e-8f, m->step + 1, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train_step");
  m->step += 1;
  return VFISV_OK;
}

int vfisv_mlp_take_loss(vfisv_mlp* m, double* sum_sq) {
  if (!m || !sum_sq) return VFISV_E_INVALID;
  *sum_sq = 0.0;
  if (m->train.cap == 0) return VFISV_OK;
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(sum_sq, m->train.loss, 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = zero_u64((unsigned long long*)m->train.loss, 1, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(m->ctx, e, "mlp_take_loss");
  return VFISV_OK;
}

int vfisv_mlp_stats(vfisv_ctx* ctx, int64_t n, int n_in, const float* stokes,
                    const float* params, float* in_mean, float* in_std, float* out_mean,
                    float* out_std, void* stream) {
  vfisv::TraceRange trace_("vfisv_mlp_stats");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_stats: ctx is NULL");
  if (n < 2) return fail(ctx, VFISV_E_INVALID, "mlp_stats: n must be >= 2");
  if (n_in < 1 || n_in > MLP_MAX_IN)
    return fail(ctx, VFISV_E_INVALID, "mlp_stats: n_in must be 1.." + std::to_string(MLP_MAX_IN));
  if (!stokes || !params || !in_mean || !in_std || !out_mean || !out_std)
    return fail(ctx, VFISV_E_INVALID, "mlp_stats: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int nsum = 2 * (n_in + 7);
  double* d = nullptr;
  e = dalloc(&d, nsum);
  if (e != hipSuccess) return fail(ctx, VFISV_E_NOMEM, "mlp_stats: scratch");
  std::vector<double> h((size_t)nsum);
  e = zero_u64((unsigned long long*)d, nsum, s);
  if (e == hipSuccess) e = col_moments(stokes, n, n_in, 0, n_in, d, s);
  if (e == hipSuccess) e = col_moments(params, n, NPAR, 3, 7, d + 2 * n_in, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, sizeof(double) * nsum, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(d);
  if (e != hipSuccess) return hip_fail(ctx, e, "mlp_stats");
  auto moments = [&](int c, float* mean, float* sd) {
    const double mu = h[2 * (size_t)c] / (double)n;
    const double var = h[2 * (size_t)c + 1] / (double)n - mu * mu;
    *mean = (float)mu;
    *sd = (float)std::fmax(std::sqrt(std::fmax(var, 0.0)), 1e-6);
  };
  for (int c = 0; c < n_in; ++c) moments(c, &in_mean[c], &in_std[c]);
  for (int c = 0; c < 7; ++c) moments(n_in + c, &out_mean[c], &out_std[c]);
  for (int c = 0; c < n_in; ++c)
    if (!std::isfinite(in_mean[c]) || !std::isfinite(in_std[c]))
      return fail(ctx, VFISV_E_INVALID, "mlp_stats: non-finite training profiles");
  for (int c = 0; c < 7; ++c)
    if (!std::isfinite(out_mean[c]) || !std::isfinite(out_std[c]))
      return fail(ctx, VFISV_E_INVALID, "mlp_stats: non-finite training models");
  return VFISV_OK;
}

}  // extern "C"

namespace {

// SplitMix64 (Steele, Lea and Flood 2014): output number c of the stream
// seeded with seed.
uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Fisher-Yates shuffle of 0 .. n-1; the draw for position i is an integer
// in [0, i] taken from the high bits of a 64x64-bit product.
void shuffle(int32_t* p, int64_t n, uint64_t key) {
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    const unsigned __int128 prod =
        (unsigned __int128)splitmix64(key, (uint64_t)i) * (unsigned __int128)(uint64_t)(i + 1);
    const int64_t j = (int64_t)(prod >> 64);
    const int32_t t = p[i];
    p[i] = p[j];
    p[j] = t;
  }
}

struct TrainScratch {
  float *T = nullptr, *Tc = nullptr, *codes = nullptr, *best = nullptr;
  int32_t* perm = nullptr;
  double* acc = nullptr;
  int32_t* host[2] = {nullptr, nullptr};
  ~TrainScratch() {
    hipFree(T);
    hipFree(Tc);
    hipFree(codes);
    hipFree(best);
    hipFree(perm);
    hipFree(acc);
    for (int k = 0; k < 2; ++k)
      if (host[k]) hipHostFree(host[k]);
  }
};

}  // namespace

extern "C" {

int vfisv_mlp_train(vfisv_ctx* ctx, vfisv_mlp* m, const vfisv_train_spec* sp,
                    vfisv_train_report* report, double* train_mse, double* control_mse,
                    void* stream) {
  vfisv::TraceRange trace_("vfisv_mlp_train");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_train: ctx is NULL");
  int rc = check_mlp(ctx, m, "mlp_train");
  if (rc) return rc;
  if (!sp) return fail(ctx, VFISV_E_INVALID, "mlp_train: spec is NULL");
  if (!sp->stokes || !sp->params || !sp->ctrl_stokes || !sp->ctrl_params)
    return fail(ctx, VFISV_E_INVALID, "mlp_train: NULL buffer");
  if (sp->batch <= 0 || sp->batch % 32 != 0 || sp->batch > (1 << 20))
    return fail(ctx, VFISV_E_INVALID, "mlp_train: batch must be a positive multiple of 32");
  if (sp->n < sp->batch || sp->n > INT32_MAX)
    return fail(ctx, VFISV_E_INVALID, "mlp_train: n must be in batch .. 2^31 - 1");
  if (sp->n_ctrl < 1) return fail(ctx, VFISV_E_INVALID, "mlp_train: n_ctrl must be >= 1");
  if (sp->epochs < 1) return fail(ctx, VFISV_E_INVALID, "mlp_train: epochs must be >= 1");
  if (!(sp->lr > 0.f) || !std::isfinite(sp->lr) || !(sp->min_lr_frac > 0.f) ||
      !(sp->min_lr_frac <= 1.f))
    return fail(ctx, VFISV_E_INVALID, "mlp_train: lr > 0 and min_lr_frac in (0, 1] needed");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  rc = ensure_train(m, sp->batch);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const MlpLayout& L = m->dev.L;
  const int64_t n = sp->n, nc = sp->n_ctrl;
  TrainScratch w;
  e = dalloc(&w.T, n * MLP_NCODE);
  if (e == hipSuccess) e = dalloc(&w.Tc, nc * MLP_NCODE);
  if (e == hipSuccess) e = dalloc(&w.codes, nc * MLP_NCODE);
  if (e == hipSuccess) e = dalloc(&w.best, L.total);
  if (e == hipSuccess) e = dalloc(&w.perm, n);
  if (e == hipSuccess) e = dalloc(&w.acc, 1);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipHostMalloc((void**)&w.host[k], sizeof(int32_t) * (size_t)n, hipHostMallocDefault);
  if (e != hipSuccess) return fail(ctx, VFISV_E_NOMEM, "mlp_train: scratch");
  e = encode_targets(sp->params, n, m->dev.out_mean, m->dev.out_std, w.T, s);
  if (e == hipSuccess) e = encode_targets(sp->ctrl_params, nc, m->dev.out_mean, m->dev.out_std, w.Tc, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train: targets");
  // any loss left from earlier steps is not this run's
  double dummy = 0.0;
  rc = vfisv_mlp_take_loss(m, &dummy);
  if (rc) return rc;

  const int64_t steps_per_epoch = n / sp->batch;
  const int64_t total = (int64_t)sp->epochs * steps_per_epoch;
  const double pi = 3.14159265358979323846;
  double best = INFINITY;
  int best_ep = -1, ep = 0, cur = 0;
  int64_t step = 0;
  shuffle(w.host[cur], n, sp->seed);
  for (; ep < sp->epochs; ++ep) {
    e = hipMemcpyAsync(w.perm, w.host[cur], sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train: order upload");
    for (int64_t b = 0; b < steps_per_epoch; ++b, ++step) {
      const double frac = total > 1 ? (double)step / (double)(total - 1) : 0.0;
      const double f = sp->min_lr_frac + (1.0 - sp->min_lr_frac) * 0.5 * (1.0 + std::cos(pi * frac));
      const int32_t* rows = w.perm + b * sp->batch;
      e = mlp_forward(m->dev, m->train, sp->batch, sp->stokes, rows, true, s);
      if (e == hipSuccess) e = mlp_backward(m->dev, m->train, sp->batch, w.T, rows, s);
      if (e == hipSuccess)
        e = mlp_adam(m->dev, m->train, (float)(sp->lr * f), 0.9f, 0.999f, 1e-8f, m->step + 1, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train: step");
      m->step += 1;
    }
    // the next epoch's order is drawn on the host while this one runs
    if (ep + 1 < sp->epochs) shuffle(w.host[1 - cur], n, sp->seed + (uint64_t)(ep + 1));
    double sum_sq = 0.0;
    rc = vfisv_mlp_take_loss(m, &sum_sq);
    if (rc) return rc;
    e = zero_u64((unsigned long long*)w.acc, 1, s);
    if (e == hipSuccess) e = mlp_infer(m->dev, nc, sp->ctrl_stokes, w.codes, nullptr, s);
    if (e == hipSuccess) e = sq_diff_sum(w.codes, w.Tc, nc * MLP_NCODE, w.acc, s);
    double csum = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&csum, w.acc, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train: control error");
    const double tr = sum_sq / ((double)steps_per_epoch * sp->batch * MLP_NCODE);
    const double ce = csum / ((double)nc * MLP_NCODE);
    if (train_mse) train_mse[ep] = tr;
    if (control_mse) control_mse[ep] = ce;
    if (ce < best) {
      best = ce;
      best_ep = ep;
      e = hipMemcpyAsync(w.best, m->dev.master, sizeof(float) * (size_t)L.total,
                         hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train: keep best");
    } else if (!(ce <= best * 1.02) && ep - best_ep >= 3) {
      ++ep;  // the control error is rising: stop
      break;
    }
    cur = 1 - cur;
  }
  if (best_ep >= 0) {
    e = hipMemcpyAsync(m->dev.master, w.best, sizeof(float) * (size_t)L.total,
                       hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = mlp_refresh_bf16(m->dev, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "mlp_train: restore best");
  if (report) {
    report->epochs_run = ep;
    report->best_epoch = best_ep;
    report->best_control_mse = best;
    report->steps = step;
  }
  return VFISV_OK;
}

int vfisv_mlp_save(vfisv_mlp* m, const char* path) {
  if (!m || !path) return VFISV_E_INVALID;
  const MlpLayout& L = m->dev.L;
  const size_t nt = (size_t)L.total;
  std::vector<float> params(nt), am(nt), av(nt);
  int rc = vfisv_mlp_get_params(m, params.data(), L.total);
  if (rc) return rc;
  hipError_t e = hipMemcpy(am.data(), m->dev.adam_m, 4 * nt, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(av.data(), m->dev.adam_v, 4 * nt, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(m->ctx, e, "mlp_save: optimiser state");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(m->ctx, VFISV_E_INVALID, std::string("mlp_save: cannot open ") + path);
  const uint32_t n_in = (uint32_t)L.n_in;
  const uint64_t total = (uint64_t)L.total;
  const int64_t step = m->step;
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &n_in, 4);
  h = fnv1a(h, &total, 8);
  h = fnv1a(h, m->in_mean.data(), 4 * n_in);
  h = fnv1a(h, m->in_std.data(), 4 * n_in);
  h = fnv1a(h, m->out_mean.data(), 28);
  h = fnv1a(h, m->out_std.data(), 28);
  h = fnv1a(h, params.data(), 4 * total);
  h = fnv1a(h, &step, 8);
  h = fnv1a(h, am.data(), 4 * total);
  h = fnv1a(h, av.data(), 4 * total);
  bool ok = std::fwrite(FILE_MAGIC, 1, 8, f) == 8 && std::fwrite(&FILE_VERSION, 4, 1, f) == 1 &&
            std::fwrite(&n_in, 4, 1, f) == 1 && std::fwrite(&total, 8, 1, f) == 1 &&
            std::fwrite(m->in_mean.data(), 4, n_in, f) == n_in &&
            std::fwrite(m->in_std.data(), 4, n_in, f) == n_in &&
            std::fwrite(m->out_mean.data(), 4, 7, f) == 7 &&
            std::fwrite(m->out_std.data(), 4, 7, f) == 7 &&
            std::fwrite(params.data(), 4, total, f) == total && std::fwrite(&step, 8, 1, f) == 1 &&
            std::fwrite(am.data(), 4, total, f) == total &&
            std::fwrite(av.data(), 4, total, f) == total && std::fwrite(&h, 8, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(m->ctx, VFISV_E_INVALID, "mlp_save: write failed");
  return VFISV_OK;
}

int vfisv_mlp_load(vfisv_ctx* ctx, const char* path, vfisv_mlp** out) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "mlp_load: ctx is NULL");
  if (!path || !out) return fail(ctx, VFISV_E_INVALID, "mlp_load: NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(ctx, VFISV_E_INVALID, std::string("mlp_load: cannot open ") + path);
  char magic[8];
  uint32_t ver = 0, n_in = 0;
  uint64_t total = 0, h_file = 0;
  int64_t step = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, FILE_MAGIC, 8) == 0 &&
            std::fread(&ver, 4, 1, f) == 1 && (ver == 1 || ver == FILE_VERSION) &&
            std::fread(&n_in, 4, 1, f) == 1 && n_in >= 1 && n_in <= MLP_MAX_IN &&
            std::fread(&total, 8, 1, f) == 1 && (int64_t)total == mlp_layout((int)n_in).total;
  std::vector<float> im, is, om(7), os(7), params, am, av;
  if (ok) {
    im.resize(n_in);
    is.resize(n_in);
    params.resize(total);
    ok = std::fread(im.data(), 4, n_in, f) == n_in && std::fread(is.data(), 4, n_in, f) == n_in &&
         std::fread(om.data(), 4, 7, f) == 7 && std::fread(os.data(), 4, 7, f) == 7 &&
         std::fread(params.data(), 4, total, f) == total;
  }
  if (ok && ver >= 2) {
    am.resize(total);
    av.resize(total);
    ok = std::fread(&step, 8, 1, f) == 1 && step >= 0 &&
         std::fread(am.data(), 4, total, f) == total &&
         std::fread(av.data(), 4, total, f) == total;
  }
  ok = ok && std::fread(&h_file, 8, 1, f) == 1;
  std::fclose(f);
  if (!ok) return fail(ctx, VFISV_E_INVALID, "mlp_load: not a network file of a known version");
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &n_in, 4);
  h = fnv1a(h, &total, 8);
  h = fnv1a(h, im.data(), 4 * n_in);
  h = fnv1a(h, is.data(), 4 * n_in);
  h = fnv1a(h, om.data(), 28);
  h = fnv1a(h, os.data(), 28);
  h = fnv1a(h, params.data(), 4 * total);
  if (ver >= 2) {
    h = fnv1a(h, &step, 8);
    h = fnv1a(h, am.data(), 4 * total);
    h = fnv1a(h, av.data(), 4 * total);
  }
  if (h != h_file) return fail(ctx, VFISV_E_INVALID, "mlp_load: checksum mismatch");
  int rc = build(ctx, (int)n_in, im.data(), is.data(), om.data(), os.data(), params.data(), 0, out);
  if (rc || ver < 2) return rc;
  // the optimiser state: training continues with the same moments and step
  vfisv_mlp* m = *out;
  hipError_t e = hipMemcpy(m->dev.adam_m, am.data(), 4 * (size_t)total, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->dev.adam_v, av.data(), 4 * (size_t)total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    vfisv_mlp_destroy(m);
    *out = nullptr;
    return hip_fail(ctx, e, "mlp_load: optimiser state");
  }
  m->step = (int)step;
  return VFISV_OK;
}

int vfisv_mlp_get_norm(const vfisv_mlp* m, float* in_mean, float* in_std, float* out_mean,
                       float* out_std) {
  if (!m || !in_mean || !in_std || !out_mean || !out_std) return VFISV_E_INVALID;
  std::memcpy(in_mean, m->in_mean.data(), sizeof(float) * m->in_mean.size());
  std::memcpy(in_std, m->in_std.data(), sizeof(float) * m->in_std.size());
  std::memcpy(out_mean, m->out_mean.data(), sizeof(float) * 7);
  std::memcpy(out_std, m->out_std.data(), sizeof(float) * 7);
  return VFISV_OK;
}

}  // extern "C"

namespace {

// Scratch of one learned-path call over n pixels, carved from one buffer:
// init [n][10] f32 | list [n] i32 | count u64 | p_fb [n][10] f32 |
// c_fb [n] f64 | i_fb [n] i32 | s_fb [n] i32 | s_short [n] i32 (the short
// fit's status when the caller passes none), each part 256-byte aligned.
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
struct LearnedScratch {
  size_t o_init = 0, o_list = 0, o_cnt = 0, o_pfb = 0, o_cfb = 0, o_ifb = 0, o_sfb = 0,
         o_sst = 0, bytes = 0;
  constexpr explicit LearnedScratch(int64_t n) {
    auto al = align256;
    o_init = 0;
    o_list = o_init + al(sizeof(float) * NPAR * n);
    o_cnt = o_list + al(sizeof(int32_t) * n);
    o_pfb = o_cnt + 256;
    o_cfb = o_pfb + al(sizeof(float) * NPAR * n);
    o_ifb = o_cfb + al(sizeof(double) * n);
    o_sfb = o_ifb + al(sizeof(int32_t) * n);
    o_sst = o_sfb + al(sizeof(int32_t) * n);
    bytes = o_sst + al(sizeof(int32_t) * n);
  }
};

// The fixed scratch of vfisv_invert_learned_noalloc: one copy per GPU the
// library runs on, held until the process ends.  Host code never uses this
// name as an address (on the host it only stands for the symbol): the
// device address comes from hipGetSymbolAddress, once per device, in
// noalloc_scratch_setup below.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static_assert(LearnedScratch(VFISV_NOALLOC_MAX_PIXELS).bytes <= NOALLOC_SCRATCH_BYTES,
              "the fixed scratch serves the documented largest batch");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace vfisv_capi {

int noalloc_scratch_setup(vfisv_ctx* ctx) {
  static std::mutex mu;
  static std::vector<void*> per_device;  // device address of scratch, by device
  std::lock_guard<std::mutex> lock(mu);
  if ((int)per_device.size() <= ctx->device) per_device.resize((size_t)ctx->device + 1, nullptr);
  if (!per_device[(size_t)ctx->device]) {
    void* p = nullptr;
    // the caller has made ctx->device current
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                      "vfisv_create: address of the allocation-free scratch");
    per_device[(size_t)ctx->device] = p;
  }
  ctx->noalloc_scratch = per_device[(size_t)ctx->device];
  return VFISV_OK;
}

}  // namespace vfisv_capi


namespace {

// The learned-start inversion.  noalloc: the scratch is the fixed device
// array (at most NOALLOC_SCRATCH_BYTES) and nothing is allocated; otherwise
// the context's scratch, grown on demand.
int invert_learned_impl(vfisv_ctx* ctx, const vfisv_instrument* inst, vfisv_mlp* m, int64_t n,
                        const float* stokes, const float* W, int W_per_pixel,
                        const vfisv_options* opt, int learned_max_iter, double chi2_accept,
                        float* params, double* chi2, int32_t* iters, int32_t* status,
                        void* stream, bool noalloc) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "invert_learned: ctx is NULL");
  int rc = check_inst(ctx, inst, "invert_learned");
  if (rc) return rc;
  rc = check_mlp(ctx, m, "invert_learned");
  if (rc) return rc;
  if (m->dev.L.n_in != 4 * inst->C.n_obs)
    return fail(ctx, VFISV_E_INVALID, "invert_learned: network inputs != 4 * n_obs");
  vfisv_options o;
  double inv_dof;
  rc = check_options(ctx, inst, opt, &o, &inv_dof, !noalloc);
  if (rc) return rc;
  if (o.fixed_iters != 0)
    return fail(ctx, VFISV_E_UNSUPPORTED, "invert_learned: the fixed-iteration scheme is not served here");
  // from the network's start most trials are accepted (about half, against
  // a third from the default model), so the fused pass is the default here
  if (o.deriv_split < 0) o.deriv_split = 0;
  if (learned_max_iter < 0) return fail(ctx, VFISV_E_INVALID, "invert_learned: learned_max_iter < 0");
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "invert_learned: n < 0");
  if (n == 0) return VFISV_OK;
  if (n > INT32_MAX) return fail(ctx, VFISV_E_INVALID, "invert_learned: n must be < 2^31");
  if (noalloc && n > VFISV_NOALLOC_MAX_PIXELS)
    return fail(ctx, VFISV_E_INVALID,
                "invert_learned_noalloc: n = " + std::to_string(n) + " exceeds the " +
                    std::to_string(VFISV_NOALLOC_MAX_PIXELS) +
                    " pixels its fixed scratch serves; split the batch");
  if (!stokes || !W || !params || !chi2 || !iters)
    return fail(ctx, VFISV_E_INVALID, "invert_learned: NULL buffer");
  const double tau =
      chi2_accept > 0.0 ? chi2_accept : chi2_reduced_quantile((int)std::lround(1.0 / inv_dof), 0.99);
  const bool refit_unconverged = (o.fallback_rule & VFISV_REFIT_UNCONVERGED) != 0;
  const bool refit_default = (o.fallback_rule & VFISV_REFIT_FROM_DEFAULT) != 0;
  const bool keep_refit = (o.fallback_rule & VFISV_REFIT_KEEP_REFIT) != 0;
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");

  const LearnedScratch sl(n);
  char* base = nullptr;
  if (noalloc) {
    if (!ctx->noalloc_scratch || sl.bytes > NOALLOC_SCRATCH_BYTES)
      return fail(ctx, VFISV_E_INVALID, "invert_learned_noalloc: scratch unavailable");
    base = (char*)ctx->noalloc_scratch;
  } else {
    if (ctx->learn_bytes < sl.bytes) {
      e = hipDeviceSynchronize();
      if (ctx->d_learn) hipFree(ctx->d_learn);
      ctx->d_learn = nullptr;
      ctx->learn_bytes = 0;
      if (e == hipSuccess) e = hipMalloc(&ctx->d_learn, sl.bytes);
      if (e != hipSuccess) return fail(ctx, VFISV_E_NOMEM, "invert_learned: scratch allocation");
      ctx->learn_bytes = sl.bytes;
    }
    base = (char*)ctx->d_learn;
  }
  float* init = (float*)(base + sl.o_init);
  int32_t* list = (int32_t*)(base + sl.o_list);
  unsigned long long* count = (unsigned long long*)(base + sl.o_cnt);
  float* p_fb = (float*)(base + sl.o_pfb);
  double* c_fb = (double*)(base + sl.o_cfb);
  int32_t* i_fb = (int32_t*)(base + sl.o_ifb);
  int32_t* s_fb = (int32_t*)(base + sl.o_sfb);
  int32_t* s_short = status ? status : (int32_t*)(base + sl.o_sst);
  hipStream_t s = (hipStream_t)stream;
  // per-phase events (measurement), not inside a graph capture
  bool timing = ctx->phase_on;
  if (timing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cs);
    timing = e == hipSuccess && cs == hipStreamCaptureStatusNone;
  }
  auto mark = [&](int k) -> hipError_t {
    return timing ? hipEventRecord(ctx->phase_ev[k], s) : hipSuccess;
  };

  // 1. network proposal of the starting model
  e = mark(0);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: phase event");
  rc = vfisv_mlp_forward(ctx, m, n, stokes, nullptr, init, stream);
  if (rc) return rc;
  e = mark(1);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: phase event");
  // 2. short LM from the proposal
  vfisv_options ol = o;
  ol.max_iter = learned_max_iter;
  rc = enqueue_lm(ctx, inst, n, nullptr, nullptr, stokes, W, W_per_pixel, init, ol, inv_dof,
                  params, chi2, iters, s_short, s, true, 1, !noalloc);
  if (rc) return rc;
  e = mark(2);
  if (e == hipSuccess && timing) e = copy_u64(ctx->d_phase_snap, ctx->d_work, 16, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: phase record");
  // 3. pixels whose fit is not acceptable go to plain LM from the combined
  // start of Sect. 5 (the proposal with the classical azimuth, and the
  // weak-field B and gamma where the polarisation is weak), written over the
  // proposals once the short LM has read them
  e = zero_u64(count, 1, s);
  if (e == hipSuccess)
    e = fallback_select(chi2, s_short, n, tau, refit_unconverged, list, count, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: fallback selection");
  const bool combined = inst->C.n_obs >= 3 && !refit_default;
  if (combined) {
    rc = vfisv_init_combined(ctx, inst, n, stokes, init, COMBINED_POL_THRESHOLD, init, nullptr,
                             stream);
    if (rc) return rc;
  }
  e = mark(3);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: phase event");
  rc = enqueue_lm(ctx, inst, n, count, list, stokes, W, W_per_pixel, combined ? init : nullptr, o,
                  inv_dof, p_fb, c_fb, i_fb, s_fb, s, false, 2, !noalloc);
  if (rc) return rc;
  e = mark(4);
  if (e == hipSuccess && timing) e = copy_u64(ctx->d_phase_snap + 16, ctx->d_work, 16, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: phase record");
  // 4. keep the better of the two fits; flag the pixel
  e = fallback_merge(list, count, n, p_fb, c_fb, i_fb, s_fb, keep_refit, params, chi2, iters,
                     status, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: merge");
  e = mark(5);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_learned: phase event");
  if (timing) ctx->phase_valid = true;
  return VFISV_OK;
}


}  // namespace

extern "C" {

int vfisv_invert_learned(vfisv_ctx* ctx, const vfisv_instrument* inst, vfisv_mlp* m, int64_t n,
                         const float* stokes, const float* W, int W_per_pixel,
                         const vfisv_options* opt, int learned_max_iter, double chi2_accept,
                         float* params, double* chi2, int32_t* iters, int32_t* status,
                         void* stream) {
  vfisv::TraceRange trace_("vfisv_invert_learned");
  return invert_learned_impl(ctx, inst, m, n, stokes, W, W_per_pixel, opt, learned_max_iter,
                             chi2_accept, params, chi2, iters, status, stream, false);
}

int vfisv_learned_phase_timing(vfisv_ctx* ctx, int on) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "learned_phase_timing: ctx is NULL");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (!on) {
    if (ctx->phase_on) hipDeviceSynchronize();
    for (hipEvent_t& ev : ctx->phase_ev)
      if (ev) {
        hipEventDestroy(ev);
        ev = nullptr;
      }
    if (ctx->d_phase_snap) hipFree(ctx->d_phase_snap);
    ctx->d_phase_snap = nullptr;
    ctx->phase_on = ctx->phase_valid = false;
    return VFISV_OK;
  }
  if (ctx->phase_on) return VFISV_OK;
  for (hipEvent_t& ev : ctx->phase_ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_phase_snap, 32 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    vfisv_learned_phase_timing(ctx, 0);
    return hip_fail(ctx, e, "learned_phase_timing: events");
  }
  ctx->phase_on = true;
  ctx->phase_valid = false;
  return VFISV_OK;
}

int vfisv_learned_phases_get(vfisv_ctx* ctx, vfisv_learned_phases* out) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "learned_phases_get: ctx is NULL");
  if (!out) return fail(ctx, VFISV_E_INVALID, "learned_phases_get: out is NULL");
  if (!ctx->phase_on || !ctx->phase_valid)
    return fail(ctx, VFISV_E_INVALID, "learned_phases_get: no timed learned-path call");
  hipError_t e = use_device(ctx);
  if (e == hipSuccess) e = hipEventSynchronize(ctx->phase_ev[5]);
  for (int k = 0; k < 5 && e == hipSuccess; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ctx->phase_ev[k], ctx->phase_ev[k + 1]);
    out->ms[k] = ms;
  }
  unsigned long long w[32];
  if (e == hipSuccess) e = hipMemcpy(w, ctx->d_phase_snap, sizeof w, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "learned_phases_get");
  auto fill = [](vfisv_counters& c, const unsigned long long* a, const unsigned long long* b) {
    // counters of a, less those of b (b == nullptr: none)
    auto d = [&](int i) { return (int64_t)(a[i] - (b ? b[i] : 0ull)); };
    c.pixels = d(1);
    c.trials = d(2);
    c.accepts = d(3);
    c.passes = d(4);
    c.svd_fallbacks = d(5);
    c.grid_waves = d(6);
    c.hessians = d(7);
    c.derivative_passes = d(0);
    c.jacobians = d(8);
  };
  fill(out->short_fit, w, nullptr);
  fill(out->refit, w + 16, w);
  return VFISV_OK;
}

int vfisv_chi2_quantile(int dof, double q, double* out) {
  if (!out || dof < 1 || dof > 1000000 || !(q > 0.0 && q < 1.0)) return VFISV_E_INVALID;
  *out = chi2_reduced_quantile(dof, q);
  return VFISV_OK;
}

int vfisv_invert_learned_noalloc(vfisv_ctx* ctx, const vfisv_instrument* inst, vfisv_mlp* m,
                                 int64_t n, const float* stokes, const float* W, int W_per_pixel,
                                 const vfisv_options* opt, int learned_max_iter,
                                 double chi2_accept, float* params, double* chi2, int32_t* iters,
                                 int32_t* status, void* stream) {
  vfisv::TraceRange trace_("vfisv_invert_learned_noalloc");
  return invert_learned_impl(ctx, inst, m, n, stokes, W, W_per_pixel, opt, learned_max_iter,
                             chi2_accept, params, chi2, iters, status, stream, true);
}

}  // extern "C"
