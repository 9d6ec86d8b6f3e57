// C ABI of libvfisv.so (declared in include/vfisv.h): argument checking,
// instrument preparation, device buffers owned by the library, and kernel
// launches.  No torch types cross this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "capi_internal.h"
#include "classical.h"
#include "kernels.h"
#include "vfisv.h"

using namespace vfisv;

static thread_local std::string g_create_err;

namespace vfisv_capi {

int fail(vfisv_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_create_err = msg;
  return code;
}

int hip_fail(vfisv_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, VFISV_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int check_inst(vfisv_ctx* ctx, const vfisv_instrument* inst, const char* fn) {
  if (!inst) return fail(ctx, VFISV_E_INVALID, std::string(fn) + ": instrument is NULL");
  if (inst->ctx != ctx)
    return fail(ctx, VFISV_E_INVALID, std::string(fn) + ": instrument of another context");
  return VFISV_OK;
}

int grid_for(int64_t n, int64_t cap) {
  const int64_t waves = (n + 63) / 64;
  return (int)(waves < cap ? (waves < 1 ? 1 : waves) : cap);
}

int check_options(vfisv_ctx* ctx, const vfisv_instrument* inst, const vfisv_options* opt,
                  vfisv_options* out, double* inv_dof, bool may_alloc) {
  vfisv_options o;
  vfisv_options_default(&o);
  if (opt) o = *opt;
  if (o.max_iter < 0) return fail(ctx, VFISV_E_INVALID, "options: max_iter < 0");
  if (!(o.eps0 > 0.0) || !(o.eps_max > 0.0) || !(o.rel_tol >= 0.0) || !std::isfinite(o.eps0) ||
      !std::isfinite(o.rel_tol))
    return fail(ctx, VFISV_E_INVALID, "options: eps0, eps_max must be > 0 and rel_tol >= 0");
  if (o.grid_waves < 0) return fail(ctx, VFISV_E_INVALID, "options: grid_waves < 0");
  if (o.chunk_log2 < -1 || o.chunk_log2 > 20)
    return fail(ctx, VFISV_E_INVALID, "options: chunk_log2 outside -1..20");
  if (o.lanes_per_pixel != 1 && o.lanes_per_pixel != 2)
    return fail(ctx, VFISV_E_INVALID, "options: lanes_per_pixel must be 1 or 2");
  if (o.voigt < 0 || o.voigt > 2) return fail(ctx, VFISV_E_INVALID, "options: voigt must be 0, 1 or 2");
  if (o.fixed_iters < 0 || o.fixed_iters > 100000)
    return fail(ctx, VFISV_E_INVALID, "options: fixed_iters outside 0..100000");
  if (o.restarts < 0 || o.restarts > 4095)
    return fail(ctx, VFISV_E_INVALID, "options: restarts outside 0..4095");
  if (!(o.hess_reuse >= 0.0)) return fail(ctx, VFISV_E_INVALID, "options: hess_reuse must be >= 0");
  if (o.deriv_split < -1 || o.deriv_split > 64)
    return fail(ctx, VFISV_E_INVALID, "options: deriv_split outside -1..64");
  if (o.fallback_rule & ~7u)
    return fail(ctx, VFISV_E_INVALID, "options: fallback_rule takes the VFISV_REFIT_* bits only");
  if (o.voigt != 0 && inst->kind != KIND_DENSE6)
    return fail(ctx, VFISV_E_UNSUPPORTED, "options: the Taylor table serves HMI-shaped instruments");
  if (o.voigt != 0 && !may_alloc && !ctx->d_vtab)
    return fail(ctx, VFISV_E_UNSUPPORTED,
                "options: the Taylor table is built on first use, which allocates; build it "
                "with an earlier call that may allocate");
  if (o.voigt != 0) {
    const int rc = ensure_vtab(ctx);
    if (rc) return rc;
  }
  o.free_mask &= 0x3FFu;
  int nfree = 0;
  for (int p = 0; p < NPAR; ++p) nfree += (o.free_mask >> p) & 1u;
  const int dof = 4 * inst->C.n_obs - nfree;
  if (dof <= 0)
    return fail(ctx, VFISV_E_INVALID, "options: 4*n_obs - free parameters must be > 0");
  *out = o;
  *inv_dof = 1.0 / (double)dof;
  return VFISV_OK;
}

static void fill_lm_args(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                         const unsigned long long* n_dev, const int32_t* idx,
                         const float* stokes, const float* W, int W_pp, const float* init,
                         const vfisv_options& o, double inv_dof, float* params, double* chi2,
                         int32_t* iters, int32_t* status, LMArgs& a) {
  a.C = inst->C;
  a.C.vtab = ctx->d_vtab;
  a.pts = inst->d_pts;
  a.pts5 = inst->d_pts5;
  a.ptsv = inst->d_ptsv ? inst->d_ptsv : inst->d_pts;
  a.blocks = inst->d_blocks;
  a.row_sums = inst->d_row_sums;
  a.qbase = QUEUE_SLOT0;
  a.lpp_max = 1;
  a.lane_cap = 0;
  a.pair_max = 0;
  a.stokes = stokes;
  a.stokes4 = nullptr;
  a.W = W;
  a.init = init;
  a.params = params;
  a.chi2 = chi2;
  a.iters = iters;
  a.status = status;
  a.work = ctx->d_work;
  a.n = n;
  a.n_dev = n_dev;
  a.idx = idx;
  a.eps0 = o.eps0;
  a.eps_max = o.eps_max;
  a.rel_tol = o.rel_tol;
  a.inv_dof = inv_dof;
  a.max_iter = o.max_iter;
  a.W_pp = W_pp ? 1 : 0;
  a.free_mask = o.free_mask & 0x3FFu;
  const vfisv_ctx::Tuned& t = ctx->tuned[inst->kind];
  a.chunk_log2 = o.chunk_log2 >= 0 ? o.chunk_log2 : (t.valid ? t.chunk_log2 : 8);
  a.fixed_iters = o.fixed_iters;
  a.restarts = o.restarts;
  a.seed = (unsigned long long)o.restart_seed;
  a.hess_reuse = o.hess_reuse;
  a.deriv_split = o.deriv_split >= 0 ? o.deriv_split
                                     : (t.valid ? t.deriv_split : VFISV_DERIV_SPLIT_DEFAULT);
}

static int lm_grid(vfisv_ctx* ctx, int64_t n, int bpc, const vfisv_options& o, int kind) {
  int64_t cap = (int64_t)ctx->num_cus * bpc;
  if (o.grid_waves > 0) cap = o.grid_waves;
  else if (kind >= 0 && ctx->tuned[kind].valid) cap = ctx->tuned[kind].grid_waves;
  if (cap > ctx->max_lanes / 64) cap = ctx->max_lanes / 64;
  return grid_for(n, cap);
}

// The context's buffer for interleaved observations, grown to at least
// `bytes` (hipFree waits for the work that may still read the old one).
static int grow_obs4(vfisv_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->obs4_bytes) return VFISV_OK;
  if (ctx->d_obs4) hipFree(ctx->d_obs4);
  ctx->d_obs4 = nullptr;
  ctx->obs4_bytes = 0;
  hipError_t e = hipMalloc(&ctx->d_obs4, bytes);
  if (e != hipSuccess) {
    ctx->d_obs4 = nullptr;
    return hip_fail(ctx, e, "invert: interleaved observations");
  }
  ctx->obs4_bytes = bytes;
  return VFISV_OK;
}

int enqueue_lm(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
               const unsigned long long* n_dev, const int32_t* idx, const float* stokes,
               const float* W, int W_pp, const float* init, const vfisv_options& o,
               double inv_dof, float* params, double* chi2, int32_t* iters, int32_t* status,
               hipStream_t s, bool reset_all, int lpp_max, bool may_alloc) {
  LMArgs a;
  fill_lm_args(ctx, inst, n, n_dev, idx, stokes, W, W_pp, init, o, inv_dof, params, chi2, iters,
               status, a);
  if (o.lanes_per_pixel > lpp_max) lpp_max = o.lanes_per_pixel;
  if (inst->kind != KIND_DENSE6) lpp_max = 1;
  a.lpp_max = lpp_max;
  // with lane pairs the grid is sized for two lanes per pixel (the kernel
  // falls back to one lane per pixel when they do not fit)
  const int bpc = inst->kind == KIND_DENSE6 ? ctx->lm_blocks_per_cu : ctx->band_blocks_per_cu;
  const int grid = lm_grid(ctx, lpp_max == 2 && !n_dev ? 2 * n : n, bpc, o, inst->kind);
  const int64_t resident = (int64_t)ctx->num_cus * bpc;
  a.lane_cap = (long long)(grid < resident ? grid : resident) * 64;
  // Pairs while at most a tenth of the pixels wait for a free pair: the
  // waiting pixels start as the first pairs finish, so a launch whose
  // pixels all need about the same number of passes (the learned path's
  // refit: 1M HMI pixels, up to 50 trials) takes 0.6x the one-lane time
  // when all pixels fit in pairs, 0.83x with 6.6% of them waiting (34,936
  // pixels on 65,536 lanes) and 1.4x with 29% waiting (42,324 pixels).
  a.pair_max = a.lane_cap / 2 + a.lane_cap / 20;
  if (inst->kind == KIND_BAND && !idx && !n_dev && n > 0 && may_alloc) {
    // a whole banded batch: the pass reads an interleaved copy
    const int no = inst->C.n_obs;
    const int rc = grow_obs4(ctx, sizeof(float4) * (size_t)n * (size_t)no);
    if (rc) return rc;
    float4* o4 = (float4*)ctx->d_obs4;
    hipError_t e0 = launch_interleave(stokes, o4, n, no, s);
    if (e0 != hipSuccess) return hip_fail(ctx, e0, "invert: interleave");
    a.stokes4 = o4;
  }
  hipError_t e = launch_reset(ctx->d_work, reset_all, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert: counter reset");
  e = launch_lm(a, inst->kind, o.voigt, grid, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert launch");
  return VFISV_OK;
}

}  // namespace vfisv_capi

using namespace vfisv_capi;

// Weideman (1994) coefficients: with L = sqrt(N / sqrt(2)) and
// f(t) = exp(-t^2) (L^2 + t^2), a_n is the n-th Fourier cosine coefficient of
// f(L tan(theta / 2)) over theta in [-pi, pi], computed here by the
// trapezoidal rule on 2M points (spectrally accurate for this smooth
// periodic function).
static void weideman_coefficients(int N, double* L_out, double* a /* [N + 1] */) {
  const double L = std::sqrt(N / std::sqrt(2.0));
  const int M = 8 * N;
  const double pi = 3.14159265358979323846;
  for (int n = 0; n <= N; ++n) {
    double s = 0.0;
    for (int k = -M + 1; k <= M; ++k) {
      const double th = k * pi / M;
      double F = 0.0;
      if (k != M) {
        const double t = L * std::tan(0.5 * th);
        F = std::exp(-t * t) * (L * L + t * t);
      }
      s += F * std::cos(n * th);
    }
    a[n] = s / (2.0 * M);
  }
  *L_out = L;
}

namespace vfisv_capi {

// The Taylor table's nodes {H, F}(u = 0.05 i, a = 0.05 j), i < 500, j < 100,
// from Weideman's series with 32 terms in double precision (within 4e-14 of
// w(z) over the table's range), rounded to float.
int ensure_vtab(vfisv_ctx* ctx) {
  if (ctx->d_vtab) return VFISV_OK;
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  double L, a[33];
  weideman_coefficients(32, &L, a);
  const double inv_sqrt_pi = 0.56418958354775628695;
  std::vector<float2> tab((size_t)VT_NU * VT_NA);
  for (int j = 0; j < VT_NA; ++j)
    for (int i = 0; i < VT_NU; ++i) {
      const std::complex<double> z(0.05 * i, 0.05 * j);
      const std::complex<double> den = L - std::complex<double>(0.0, 1.0) * z;
      const std::complex<double> Z = (L + std::complex<double>(0.0, 1.0) * z) / den;
      std::complex<double> p = a[32];
      for (int n = 31; n >= 1; --n) p = p * Z + a[n];
      const std::complex<double> w = 2.0 * p / (den * den) + inv_sqrt_pi / den;
      tab[(size_t)j * VT_NU + i] = make_float2((float)w.real(), (float)w.imag());
    }
  float2* d = nullptr;
  e = hipMalloc(&d, sizeof(float2) * tab.size());
  if (e != hipSuccess) return fail(ctx, VFISV_E_NOMEM, "Taylor table allocation");
  e = hipMemcpy(d, tab.data(), sizeof(float2) * tab.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(d);
    return hip_fail(ctx, e, "Taylor table copy");
  }
  ctx->d_vtab = d;
  return VFISV_OK;
}

}  // namespace vfisv_capi

extern "C" {

const char* vfisv_version(void) { return "vfisv-gfx950 0.2.0"; }

const char* vfisv_last_error(const vfisv_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}


int vfisv_create(vfisv_ctx** out, int device) {
  if (!out) return fail(nullptr, VFISV_E_INVALID, "vfisv_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev)
    return fail(nullptr, VFISV_E_INVALID, "vfisv_create: no HIP device " + std::to_string(device));
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  vfisv_ctx* c = new (std::nothrow) vfisv_ctx();
  if (!c) return fail(nullptr, VFISV_E_NOMEM, "vfisv_create: host allocation");
  c->device = device;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "hipGetDeviceProperties");
  }
  c->num_cus = prop.multiProcessorCount;
  int bpc = 0;
  e = lm_blocks_per_cu(&bpc);
  if (e != hipSuccess || bpc < 1) bpc = 1;
  c->lm_blocks_per_cu = bpc;
  bpc = 0;
  e = band_blocks_per_cu(&bpc);
  if (e != hipSuccess || bpc < 1) bpc = 1;
  c->band_blocks_per_cu = bpc;
  // the largest persistent grid: 8 waves per CU
  c->max_lanes = (int64_t)c->num_cus * 8 * 64;
  e = hipMalloc(&c->d_work, sizeof(unsigned long long) * (WORK_SLOTS + HIST_MAX));
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, VFISV_E_NOMEM, "vfisv_create: counter allocation");
  }
  e = launch_reset(c->d_work, true, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hipFree(c->d_work);
    delete c;
    return hip_fail(nullptr, e, "vfisv_create: counter reset");
  }
  if (noalloc_scratch_setup(c) != VFISV_OK) {
    g_create_err = c->err;
    hipFree(c->d_work);
    delete c;
    return VFISV_E_DEVICE;
  }
  double L, a[NW + 1];
  weideman_coefficients(NW, &L, a);
  c->wL = (float)L;
  c->wc[0] = 0.f;
  for (int n = 1; n <= NW; ++n) c->wc[n] = (float)(2.0 * a[n]);
  *out = c;
  return VFISV_OK;
}

int vfisv_destroy(vfisv_ctx* ctx) {
  if (!ctx) return VFISV_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  hipFree(ctx->d_work);
  if (ctx->d_learn) hipFree(ctx->d_learn);
  if (ctx->d_obs4) hipFree(ctx->d_obs4);
  if (ctx->d_vtab) hipFree(ctx->d_vtab);
  vfisv_learned_phase_timing(ctx, 0);
  delete ctx;
  return VFISV_OK;
}

void vfisv_options_default(vfisv_options* o) {
  if (!o) return;
  o->max_iter = 50;
  o->eps0 = 1e-3;
  o->eps_max = 1e8;
  o->rel_tol = 1e-5;
  o->free_mask = 0x3FFu;
  o->grid_waves = 0;
  o->chunk_log2 = -1;
  o->lanes_per_pixel = 1;
  o->voigt = 0;
  o->fixed_iters = 0;
  o->restarts = 0;
  o->restart_seed = 0;
  o->hess_reuse = 0.0;
  o->fallback_rule = 0u;
  o->deriv_split = -1;
}

int vfisv_instrument_create(vfisv_ctx* ctx, const vfisv_instrument_desc* d,
                            vfisv_instrument** out) {
  vfisv::TraceRange trace_("vfisv_instrument_create");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "instrument_create: ctx is NULL");
  if (!d || !out) return fail(ctx, VFISV_E_INVALID, "instrument_create: NULL argument");
  *out = nullptr;
  if (!d->fine_offset_mA || !d->filter)
    return fail(ctx, VFISV_E_INVALID, "instrument_create: NULL table");
  if (d->n_fine < 1 || d->n_fine > 4096)
    return fail(ctx, VFISV_E_INVALID, "instrument_create: n_fine must be in 1..4096");
  if (d->n_obs < 1) return fail(ctx, VFISV_E_INVALID, "instrument_create: n_obs must be >= 1");
  if (!(d->lambda0_A > 0.0) || !std::isfinite(d->lambda0_A) || !std::isfinite(d->geff))
    return fail(ctx, VFISV_E_INVALID, "instrument_create: bad lambda0 or geff");
  if (!(d->tap_threshold >= 0.0 && d->tap_threshold < 1.0))
    return fail(ctx, VFISV_E_INVALID, "instrument_create: tap_threshold must be in [0, 1)");
  for (int k = 0; k < d->n_fine; ++k)
    if (!std::isfinite(d->fine_offset_mA[k]))
      return fail(ctx, VFISV_E_INVALID, "instrument_create: non-finite fine offset");
  const int nf = d->n_fine, no = d->n_obs;
  for (int64_t i = 0; i < (int64_t)nf * no; ++i)
    if (!std::isfinite(d->filter[i]) || d->filter[i] < 0.0)
      return fail(ctx, VFISV_E_INVALID, "instrument_create: filter taps must be finite and >= 0");
  if (no > 4096) return fail(ctx, VFISV_E_INVALID, "instrument_create: n_obs must be <= 4096");

  vfisv_instrument* inst = new (std::nothrow) vfisv_instrument();
  if (!inst) return fail(ctx, VFISV_E_NOMEM, "instrument_create: host allocation");
  inst->ctx = ctx;
  inst->device = ctx->device;
  std::memset(&inst->C, 0, sizeof(Consts));
  inst->C.sw_k = -1;
  double max_drop = 0.0;
  std::vector<double> kept((size_t)no * nf);
  std::vector<float> row_sum((size_t)no);
  for (int i = 0; i < no; ++i) {
    double rmax = 0.0, rsum = 0.0, drop = 0.0, ksum = 0.0;
    for (int k = 0; k < nf; ++k) {
      rmax = std::fmax(rmax, d->filter[(size_t)i * nf + k]);
      rsum += d->filter[(size_t)i * nf + k];
    }
    for (int k = 0; k < nf; ++k) {
      const double w = d->filter[(size_t)i * nf + k];
      const bool keep = w > 0.0 && w >= d->tap_threshold * rmax && (float)w != 0.0f;
      kept[(size_t)i * nf + k] = keep ? w : 0.0;
      if (!keep) drop += w;
      ksum += keep ? (double)(float)w : 0.0;
    }
    if (rsum > 0.0) max_drop = std::fmax(max_drop, drop / rsum);
    row_sum[(size_t)i] = (float)ksum;
  }
  std::vector<Point> pts, pts5, ptsv;
  std::vector<Block> blocks;
  int n_taps = 0, n_active = 0;
  if (no == NOBS_HMI) {
    // dense: one record per synthesis point with a non-zero tap
    for (int i = 0; i < no; ++i) inst->C.row_sum[i] = row_sum[(size_t)i];
    for (int k = 0; k < nf; ++k) {
      Point p;
      std::memset(&p, 0, sizeof p);
      p.dl = (float)d->fine_offset_mA[k];
      uint32_t mask = 0;
      for (int i = 0; i < no; ++i) {
        p.w[i] = (float)kept[(size_t)i * nf + k];
        if (p.w[i] != 0.f) {
          mask |= 1u << i;
          ++n_taps;
        }
      }
      std::memcpy(&p.w[6], &mask, 4);
      if (mask) pts.push_back(p);
    }
    n_active = (int)pts.size();
    // Windowed records: row a (the first to end) and row b (the last to
    // start) share register slot 4 when they overlap on at most OV_MAX
    // records; the other four rows take slots 0-3 in order.
    std::vector<int> fr(no, -1), lr(no, -1);
    for (int k = 0; k < (int)pts.size(); ++k)
      for (int i = 0; i < no; ++i)
        if (pts[(size_t)k].w[i] != 0.f) {
          if (fr[(size_t)i] < 0) fr[(size_t)i] = k;
          lr[(size_t)i] = k;
        }
    int ra = -1, rb = -1;
    bool all_rows = true;
    for (int i = 0; i < no; ++i) {
      if (fr[(size_t)i] < 0) all_rows = false;
      if (ra < 0 || lr[(size_t)i] < lr[(size_t)ra]) ra = i;
    }
    for (int i = 0; i < no; ++i)
      if (i != ra && (rb < 0 || fr[(size_t)i] > fr[(size_t)rb])) rb = i;
    if (all_rows && ra >= 0 && rb >= 0 && fr[(size_t)ra] < fr[(size_t)rb] &&
        lr[(size_t)ra] - fr[(size_t)rb] + 1 <= OV_MAX) {
      const int sw = fr[(size_t)rb];
      int slot = 0;
      for (int i = 0; i < no; ++i)
        if (i != ra && i != rb) inst->C.slot_row[slot++] = i;
      inst->C.slot_row[4] = rb;
      inst->C.slot_row[5] = ra;
      for (int q = 0; q < 6; ++q) inst->C.slot_rs[q] = row_sum[(size_t)inst->C.slot_row[q]];
      pts5.resize(pts.size());
      for (int k = 0; k < (int)pts.size(); ++k) {
        const Point& P = pts[(size_t)k];
        Point& Q = pts5[(size_t)k];
        std::memset(&Q, 0, sizeof Q);
        Q.dl = P.dl;
        for (int q = 0; q < 4; ++q) Q.w[q] = P.w[inst->C.slot_row[q]];
        Q.w[4] = k < sw ? P.w[ra] : P.w[rb];
        Q.w[5] = k < sw ? 0.f : P.w[ra];
        uint32_t m = 0;
        for (int q = 0; q < 6; ++q)
          if (Q.w[q] != 0.f) m |= 1u << q;
        std::memcpy(&Q.w[6], &m, 4);
      }
      inst->C.sw_k = sw;
      // the values-only pass: all six rows in the slot order above
      ptsv.resize(pts.size());
      for (int k = 0; k < (int)pts.size(); ++k) {
        const Point& P = pts[(size_t)k];
        Point& Q = ptsv[(size_t)k];
        std::memset(&Q, 0, sizeof Q);
        Q.dl = P.dl;
        uint32_t m = 0;
        for (int q = 0; q < 6; ++q) {
          Q.w[q] = P.w[inst->C.slot_row[q]];
          if (Q.w[q] != 0.f) m |= 1u << q;
        }
        std::memcpy(&Q.w[6], &m, 4);
      }
    }
  } else {
    // banded: row i's kept taps must lie in points a0 + 4 i .. a0 + 4 i + 15
    int64_t a0 = INT64_MAX;
    std::vector<int> first((size_t)no, -1), last((size_t)no, -1);
    for (int i = 0; i < no; ++i) {
      for (int k = 0; k < nf; ++k)
        if (kept[(size_t)i * nf + k] != 0.0) {
          if (first[(size_t)i] < 0) first[(size_t)i] = k;
          last[(size_t)i] = k;
        }
      if (first[(size_t)i] >= 0) a0 = std::min<int64_t>(a0, first[(size_t)i] - (int64_t)BAND_S * i);
    }
    bool band = a0 != INT64_MAX;
    for (int i = 0; band && i < no; ++i)
      if (first[(size_t)i] >= 0 && last[(size_t)i] - (a0 + (int64_t)BAND_S * i) > BAND_S * BAND_R - 1)
        band = false;
    if (!band) {
      delete inst;
      return fail(ctx, VFISV_E_UNSUPPORTED,
                  "instrument_create: the filter must have 6 rows, or be banded with each row "
                  "within 16 consecutive synthesis points advancing 4 points per row");
    }
    const int nb = no + BAND_R - 1;
    blocks.resize((size_t)nb);
    std::vector<char> used((size_t)nf, 0);
    for (int b2 = 0; b2 < nb; ++b2) {
      Block& B = blocks[(size_t)b2];
      for (int q = 0; q < BAND_S; ++q) {
        const int64_t k = a0 + (int64_t)BAND_S * b2 + q;
        const bool in = k >= 0 && k < nf;
        B.dl[q] = in ? (float)d->fine_offset_mA[k] : 0.f;
        for (int r = 0; r < BAND_R; ++r) {
          const int j = b2 - (BAND_R - 1) + r;
          const double w = (in && j >= 0 && j < no) ? kept[(size_t)j * nf + (size_t)k] : 0.0;
          B.w[q][r] = (float)w;
          if (B.w[q][r] != 0.f) {
            ++n_taps;
            used[(size_t)k] = 1;
          }
        }
      }
    }
    for (int k = 0; k < nf; ++k) n_active += used[(size_t)k];
    inst->kind = KIND_BAND;
  }
  const double lam0_mA = d->lambda0_A * 1000.0;
  inst->C.lam_over_c = (float)(lam0_mA / C_KMS);
  const double cz = 4.66685e-10 * d->geff * d->lambda0_A * d->lambda0_A;  // Eq. 7
  inst->C.cz = (float)cz;
  inst->C.n_pts = (int)pts.size();
  inst->C.n_obs = no;
  for (int n = 0; n <= NW; ++n) inst->C.wc[n] = ctx->wc[n];
  inst->C.wL = ctx->wL;
  inst->C.wL2 = ctx->wL * ctx->wL;
  inst->C.w2L = 2.f * ctx->wL;
  inst->info.n_active_fine = n_active;
  inst->info.n_taps = n_taps;
  inst->info.max_dropped_rel = max_drop;
  inst->info.cz_mA_per_G = cz;
  inst->info.lm_register_rows =
      inst->kind == KIND_BAND ? BAND_R : (inst->C.sw_k >= 0 ? 5 : NOBS_HMI);

  hipError_t e = use_device(ctx);
  if (e != hipSuccess) {
    delete inst;
    return hip_fail(ctx, e, "hipSetDevice");
  }
  // observed wavelength of each sample: the centroid of its filter row
  std::vector<float> obs_x((size_t)no);
  for (int i = 0; i < no; ++i) {
    double sw = 0.0, swx = 0.0;
    for (int k = 0; k < nf; ++k) {
      sw += d->filter[(size_t)i * nf + k];
      swx += d->filter[(size_t)i * nf + k] * d->fine_offset_mA[k];
    }
    obs_x[(size_t)i] = sw > 0.0 ? (float)(swx / sw) : 0.f;
  }
  e = hipMalloc(&inst->d_obs_x, sizeof(float) * (size_t)no);
  if (e == hipSuccess)
    e = hipMemcpy(inst->d_obs_x, obs_x.data(), sizeof(float) * (size_t)no, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (inst->d_obs_x) hipFree(inst->d_obs_x);
    delete inst;
    return hip_fail(ctx, e, "instrument_create: sample table");
  }
  if (inst->kind == KIND_DENSE6) {
    const size_t bytes = sizeof(Point) * (pts.empty() ? 1 : pts.size());
    e = hipMalloc(&inst->d_pts, bytes);
    if (e == hipSuccess && !pts.empty())
      e = hipMemcpy(inst->d_pts, pts.data(), sizeof(Point) * pts.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !pts5.empty()) {
      e = hipMalloc(&inst->d_pts5, sizeof(Point) * pts5.size());
      if (e == hipSuccess)
        e = hipMemcpy(inst->d_pts5, pts5.data(), sizeof(Point) * pts5.size(),
                      hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !ptsv.empty()) {
      e = hipMalloc(&inst->d_ptsv, sizeof(Point) * ptsv.size());
      if (e == hipSuccess)
        e = hipMemcpy(inst->d_ptsv, ptsv.data(), sizeof(Point) * ptsv.size(),
                      hipMemcpyHostToDevice);
    }
  } else {
    e = hipMalloc(&inst->d_blocks, sizeof(Block) * blocks.size());
    if (e == hipSuccess) e = hipMalloc(&inst->d_row_sums, sizeof(float) * (size_t)no);
    if (e == hipSuccess)
      e = hipMemcpy(inst->d_blocks, blocks.data(), sizeof(Block) * blocks.size(),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(inst->d_row_sums, row_sum.data(), sizeof(float) * (size_t)no,
                    hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (inst->d_pts) hipFree(inst->d_pts);
    if (inst->d_pts5) hipFree(inst->d_pts5);
  if (inst->d_ptsv) hipFree(inst->d_ptsv);
    if (inst->d_ptsv) hipFree(inst->d_ptsv);
    if (inst->d_blocks) hipFree(inst->d_blocks);
    if (inst->d_row_sums) hipFree(inst->d_row_sums);
    hipFree(inst->d_obs_x);
    delete inst;
    return hip_fail(ctx, e, "instrument_create: device tables");
  }
  *out = inst;
  return VFISV_OK;
}

int vfisv_instrument_info_get(const vfisv_instrument* inst, vfisv_instrument_info* info) {
  if (!inst || !info) return VFISV_E_INVALID;
  *info = inst->info;
  return VFISV_OK;
}

int vfisv_instrument_destroy(vfisv_instrument* inst) {
  if (!inst) return VFISV_OK;
  hipSetDevice(inst->device);
  hipDeviceSynchronize();
  if (inst->d_pts) hipFree(inst->d_pts);
  if (inst->d_pts5) hipFree(inst->d_pts5);
  if (inst->d_ptsv) hipFree(inst->d_ptsv);
  if (inst->d_blocks) hipFree(inst->d_blocks);
  if (inst->d_row_sums) hipFree(inst->d_row_sums);
  if (inst->d_obs_x) hipFree(inst->d_obs_x);
  delete inst;
  return VFISV_OK;
}

int vfisv_synthesize(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                     const float* params, const float* noise, float* stokes, float* jac,
                     void* stream) {
  return vfisv_synthesize_voigt(ctx, inst, n, params, noise, stokes, jac, 0, stream);
}

int vfisv_synthesize_voigt(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                           const float* params, const float* noise, float* stokes, float* jac,
                           int voigt, void* stream) {
  vfisv::TraceRange trace_("vfisv_synthesize_voigt");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "synthesize: ctx is NULL");
  int rc = check_inst(ctx, inst, "synthesize");
  if (rc) return rc;
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "synthesize: n < 0");
  if (voigt < 0 || voigt > 2) return fail(ctx, VFISV_E_INVALID, "synthesize: voigt must be 0..2");
  if (voigt != 0 && inst->kind != KIND_DENSE6)
    return fail(ctx, VFISV_E_UNSUPPORTED, "synthesize: the Taylor table serves HMI-shaped instruments");
  if (n == 0) return VFISV_OK;
  if (!params || !stokes) return fail(ctx, VFISV_E_INVALID, "synthesize: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (voigt != 0) {
    rc = ensure_vtab(ctx);
    if (rc) return rc;
  }
  SynthArgs a;
  a.C = inst->C;
  a.C.vtab = ctx->d_vtab;
  a.pts = inst->d_pts;
  a.blocks = inst->d_blocks;
  a.row_sums = inst->d_row_sums;
  a.params = params;
  a.noise = noise;
  a.stokes = stokes;
  a.jac = jac;
  a.n = n;
  const int grid = grid_for(n, (int64_t)ctx->num_cus * 16);
  e = launch_synth(a, inst->kind, voigt, jac != nullptr, grid, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "synthesize launch");
  return VFISV_OK;
}

int vfisv_invert(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n, const float* stokes,
                 const float* W, int W_per_pixel, const float* init, const vfisv_options* opt,
                 float* params, double* chi2, int32_t* iters, int32_t* status, void* stream) {
  vfisv::TraceRange trace_("vfisv_invert");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "invert: ctx is NULL");
  int rc = check_inst(ctx, inst, "invert");
  if (rc) return rc;
  vfisv_options o;
  double inv_dof;
  rc = check_options(ctx, inst, opt, &o, &inv_dof);
  if (rc) return rc;
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "invert: n < 0");
  if (n == 0) return VFISV_OK;
  if (n > INT32_MAX) return fail(ctx, VFISV_E_INVALID, "invert: n must be < 2^31");
  if (!stokes || !W || !params || !chi2 || !iters)
    return fail(ctx, VFISV_E_INVALID, "invert: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return enqueue_lm(ctx, inst, n, nullptr, nullptr, stokes, W, W_per_pixel, init, o, inv_dof,
                    params, chi2, iters, status, (hipStream_t)stream, true);
}

int vfisv_invert_batches(vfisv_ctx* ctx, const vfisv_batch* batches, int n_batches,
                         const vfisv_options* opt, void* stream) {
  vfisv::TraceRange trace_("vfisv_invert_batches");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "invert_batches: ctx is NULL");
  if (!batches) return fail(ctx, VFISV_E_INVALID, "invert_batches: batches is NULL");
  if (n_batches < 1 || n_batches > MAX_BATCHES)
    return fail(ctx, VFISV_E_INVALID, "invert_batches: n_batches must be in 1..4");
  BatchArgs B;
  std::memset(&B, 0, sizeof B);
  B.n_batches = n_batches;
  int64_t total = 0;
  vfisv_options o;
  for (int i = 0; i < n_batches; ++i) {
    const vfisv_batch& b = batches[i];
    int rc = check_inst(ctx, b.inst, "invert_batches");
    if (rc) return rc;
    double inv_dof;
    rc = check_options(ctx, b.inst, opt, &o, &inv_dof);
    if (rc) return rc;
    if (b.n < 0 || b.n > INT32_MAX)
      return fail(ctx, VFISV_E_INVALID, "invert_batches: n must be in 0 .. 2^31 - 1");
    if (o.voigt != 0)
      return fail(ctx, VFISV_E_UNSUPPORTED, "invert_batches: the Taylor table is not served here");
    if (o.fixed_iters != 0)
      return fail(ctx, VFISV_E_UNSUPPORTED, "invert_batches: the fixed-iteration scheme is not served here");
    if (b.n > 0 && (!b.stokes || !b.W || !b.params || !b.chi2 || !b.iters))
      return fail(ctx, VFISV_E_INVALID, "invert_batches: NULL buffer");
    fill_lm_args(ctx, b.inst, b.n, nullptr, nullptr, b.stokes, b.W, b.W_per_pixel, b.init, o,
                 inv_dof, b.params, b.chi2, b.iters, b.status, B.a[i]);
    B.a[i].qbase = QUEUE_SLOT0 + NQ * i;
    B.kind[i] = b.inst->kind;
    total += b.n;
  }
  if (total == 0) return VFISV_OK;
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const int grid = lm_grid(ctx, total, ctx->band_blocks_per_cu, o, -1);
  hipStream_t s = (hipStream_t)stream;
  // banded batches read interleaved copies, side by side in one buffer
  size_t need = 0;
  for (int i = 0; i < n_batches; ++i)
    if (B.kind[i] == KIND_BAND) need += (size_t)batches[i].n * (size_t)batches[i].inst->C.n_obs;
  if (need > 0) {
    const int rc = grow_obs4(ctx, sizeof(float4) * need);
    if (rc) return rc;
    float4* o4 = (float4*)ctx->d_obs4;
    for (int i = 0; i < n_batches; ++i) {
      if (B.kind[i] != KIND_BAND || batches[i].n == 0) continue;
      const int no = batches[i].inst->C.n_obs;
      e = launch_interleave(batches[i].stokes, o4, batches[i].n, no, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "invert_batches: interleave");
      B.a[i].stokes4 = o4;
      o4 += (size_t)batches[i].n * (size_t)no;
    }
  }
  e = launch_reset(ctx->d_work, true, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_batches: counter reset");
  e = launch_lm_batches(B, grid, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "invert_batches launch");
  return VFISV_OK;
}

int vfisv_autotune(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                   const float* stokes, const float* W, int W_per_pixel, const vfisv_options* opt,
                   int64_t sample, vfisv_tuning* out, void* stream) {
  vfisv::TraceRange trace_("vfisv_autotune");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "autotune: ctx is NULL");
  int rc = check_inst(ctx, inst, "autotune");
  if (rc) return rc;
  vfisv_options o;
  double inv_dof;
  rc = check_options(ctx, inst, opt, &o, &inv_dof);
  if (rc) return rc;
  if (n < 1 || n > INT32_MAX) return fail(ctx, VFISV_E_INVALID, "autotune: n must be in 1..2^31-1");
  if (!stokes || !W) return fail(ctx, VFISV_E_INVALID, "autotune: NULL buffer");
  if (sample <= 0) sample = 131072;
  const int64_t m = sample < n ? sample : n;
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  float* params = nullptr;
  double* chi2 = nullptr;
  int32_t* iters = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  e = hipMalloc(&params, sizeof(float) * NPAR * (size_t)m);
  if (e == hipSuccess) e = hipMalloc(&chi2, sizeof(double) * (size_t)m);
  if (e == hipSuccess) e = hipMalloc(&iters, sizeof(int32_t) * (size_t)m);
  if (e == hipSuccess) e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  // candidates: the derivative-pass split (fused, or a derivative pass once
  // k/64 of a wave's lanes wait) at the default schedule, then the
  // persistent grid (waves per CU, up to what is resident) x queue block
  // size at the best split
  const int bpc_default = inst->kind == KIND_DENSE6 ? ctx->lm_blocks_per_cu
                                                    : ctx->band_blocks_per_cu;
  const int splits[] = {0, 2, 4, 8, 16, 32};
  const int waves_per_cu[] = {1, 2, 3, 4, 6, 8};
  const int chunks[] = {4, 8, 12};
  vfisv_tuning best;
  std::memset(&best, 0, sizeof best);
  best.best_ms = 1e300;
  best.default_ms = -1.0;
  int cand = 0;
  auto time_one = [&](const vfisv_options& oc, float* ms) {
    *ms = 1e30f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      e = hipEventRecord(ev0, s);
      if (e != hipSuccess) break;
      rc = enqueue_lm(ctx, inst, m, nullptr, nullptr, stokes, W, W_per_pixel, nullptr, oc,
                      inv_dof, params, chi2, iters, nullptr, s, true);
      if (rc) break;
      e = hipEventRecord(ev1, s);
      if (e == hipSuccess) e = hipEventSynchronize(ev1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, ev0, ev1);
      if (e == hipSuccess && t < *ms) *ms = t;
    }
    ++cand;
  };
  const int64_t gw_default = (int64_t)ctx->num_cus * bpc_default;
  // A sample of m of the n pixels runs on a grid scaled by m / n, so that
  // each lane inverts as many pixels as in the whole launch (up to 8 per
  // lane, which bounds a candidate's time): the share of the launch that is
  // its tail (where latency, not throughput, counts) then matches, and the
  // choice made on the sample holds for the batch.
  // (one factor for every candidate, so that their ratios are kept)
  const double scale =
      std::min(1.0, std::max((double)m / (double)n, (double)m / (512.0 * (double)gw_default)));
  auto sample_grid = [&](int64_t gw) {
    return (int)std::max<int64_t>(8, std::llround((double)gw * scale));
  };
  int best_split = VFISV_DERIV_SPLIT_DEFAULT;
  float best_split_ms = 1e30f;
  for (int si = 0; e == hipSuccess && !rc && si < 6; ++si) {
    vfisv_options oc = o;
    oc.grid_waves = sample_grid(std::min<int64_t>(gw_default, ctx->max_lanes / 64));
    oc.chunk_log2 = 8;
    oc.deriv_split = o.fixed_iters > 0 ? 0 : splits[si];
    float ms;
    time_one(oc, &ms);
    if (rc || e != hipSuccess) break;
    if (splits[si] == VFISV_DERIV_SPLIT_DEFAULT) best.default_ms = ms;
    if (ms < best_split_ms) {
      best_split_ms = ms;
      best_split = oc.deriv_split;
    }
    if (o.fixed_iters > 0) break;  // the fixed-iteration scheme always fuses
  }
  if (e == hipSuccess && !rc) {  // the default schedule at the best split
    best.best_ms = best_split_ms;
    best.grid_waves = (int)std::min<int64_t>(gw_default, ctx->max_lanes / 64);
    best.chunk_log2 = 8;
    best.deriv_split = best_split;
  }
  for (int wi = 0; e == hipSuccess && !rc && wi < 6; ++wi) {
    const int64_t gw = (int64_t)ctx->num_cus * waves_per_cu[wi];
    // a persistent grid larger than what is resident only adds waves that
    // start when the work is gone
    if (gw > ctx->max_lanes / 64 || waves_per_cu[wi] > bpc_default) continue;
    for (int ci = 0; e == hipSuccess && ci < 3; ++ci) {
      vfisv_options oc = o;
      oc.grid_waves = sample_grid(gw);
      oc.chunk_log2 = chunks[ci];
      oc.deriv_split = best_split;
      float ms;
      time_one(oc, &ms);
      if (rc) break;
      if (e == hipSuccess && ms < best.best_ms) {
        best.best_ms = ms;
        best.grid_waves = (int)gw;
        best.chunk_log2 = chunks[ci];
        best.deriv_split = best_split;
      }
    }
  }
  if (ev0) hipEventDestroy(ev0);
  if (ev1) hipEventDestroy(ev1);
  if (params) hipFree(params);
  if (chi2) hipFree(chi2);
  if (iters) hipFree(iters);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
  best.candidates = cand;
  best.sample = m;
  vfisv_ctx::Tuned& t = ctx->tuned[inst->kind];
  t.valid = true;
  t.grid_waves = best.grid_waves;
  t.chunk_log2 = best.chunk_log2;
  t.deriv_split = best.deriv_split;
  if (out) *out = best;
  return VFISV_OK;
}

namespace {

int init_start(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n, const float* stokes,
               const float* base, float pol_threshold, float* params, float* pol,
               void* stream, const char* what) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, std::string(what) + ": ctx is NULL");
  int rc = check_inst(ctx, inst, what);
  if (rc) return rc;
  if (n < 0) return fail(ctx, VFISV_E_INVALID, std::string(what) + ": n < 0");
  if (inst->C.n_obs < 3)
    return fail(ctx, VFISV_E_UNSUPPORTED, std::string(what) + ": needs at least 3 observed samples");
  if (!(pol_threshold >= 0.f))
    return fail(ctx, VFISV_E_INVALID, std::string(what) + ": pol_threshold must be >= 0");
  if (n == 0) return VFISV_OK;
  if (!stokes || !params) return fail(ctx, VFISV_E_INVALID, std::string(what) + ": NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  ClassicalArgs a;
  a.stokes = stokes;
  a.x = inst->d_obs_x;
  a.n_obs = inst->C.n_obs;
  a.n = n;
  a.cz = inst->C.cz;
  a.lam0_mA = inst->C.lam_over_c * (float)C_KMS;
  a.params = params;
  a.pol = pol;
  a.base = base;
  a.pol_threshold = pol_threshold;
  const int64_t blocks = (n + 255) / 256;
  const int64_t cap = (int64_t)ctx->num_cus * 16;
  e = launch_classical(a, (int)(blocks < cap ? blocks : cap), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  return VFISV_OK;
}

}  // namespace

int vfisv_init_classical(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                         const float* stokes, float* params, float* pol, void* stream) {
  vfisv::TraceRange trace_("vfisv_init_classical");
  return init_start(ctx, inst, n, stokes, nullptr, 0.f, params, pol, stream, "init_classical");
}

int vfisv_init_combined(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                        const float* stokes, const float* base, float pol_threshold,
                        float* params, float* pol, void* stream) {
  vfisv::TraceRange trace_("vfisv_init_combined");
  if (n > 0 && !base && ctx) return fail(ctx, VFISV_E_INVALID, "init_combined: base is NULL");
  return init_start(ctx, inst, n, stokes, base, pol_threshold, params, pol, stream,
                    "init_combined");
}

int vfisv_stokes_weights(vfisv_ctx* ctx, const vfisv_instrument* inst, int64_t n,
                         const float* stokes, const float* mu, const float* sigma, float* W,
                         void* stream) {
  vfisv::TraceRange trace_("vfisv_stokes_weights");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "stokes_weights: ctx is NULL");
  int rc = check_inst(ctx, inst, "stokes_weights");
  if (rc) return rc;
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "stokes_weights: n < 0");
  if (!sigma) return fail(ctx, VFISV_E_INVALID, "stokes_weights: sigma is NULL");
  WeightsArgs a;
  for (int s = 0; s < 4; ++s) {
    if (!(sigma[s] > 0.f) || !std::isfinite(sigma[s]))
      return fail(ctx, VFISV_E_INVALID, "stokes_weights: sigma must be finite and > 0");
    a.inv_var[s] = 1.0 / ((double)sigma[s] * (double)sigma[s]);
  }
  if (n == 0) return VFISV_OK;
  if (!stokes || !mu || !W) return fail(ctx, VFISV_E_INVALID, "stokes_weights: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  a.stokes = stokes;
  a.mu = mu;
  a.n_obs = inst->C.n_obs;
  a.n = n;
  a.W = W;
  const int64_t blocks = (n + 255) / 256;
  const int64_t cap = (int64_t)ctx->num_cus * 16;
  e = launch_weights(a, (int)(blocks < cap ? blocks : cap), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "stokes_weights launch");
  return VFISV_OK;
}

int vfisv_get_counters(vfisv_ctx* ctx, vfisv_counters* out) {
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "get_counters: ctx is NULL");
  if (!out) return fail(ctx, VFISV_E_INVALID, "get_counters: out is NULL");
  hipError_t e = use_device(ctx);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  unsigned long long w[WORK_SLOTS];
  if (e == hipSuccess) e = hipMemcpy(w, ctx->d_work, sizeof w, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "get_counters");
  out->pixels = (int64_t)w[1];
  out->trials = (int64_t)w[2];
  out->accepts = (int64_t)w[3];
  out->passes = (int64_t)w[4];
  out->svd_fallbacks = (int64_t)w[5];
  out->grid_waves = (int64_t)w[6];
  out->hessians = (int64_t)w[7];
  out->derivative_passes = (int64_t)w[0];
  out->jacobians = (int64_t)w[8];
  return VFISV_OK;
}

int vfisv_iter_histogram(vfisv_ctx* ctx, int64_t n, const int32_t* iters, int n_bins,
                         int64_t* hist, void* stream) {
  vfisv::TraceRange trace_("vfisv_iter_histogram");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "iter_histogram: ctx is NULL");
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "iter_histogram: n < 0");
  if (n_bins < 1 || n_bins > HIST_MAX)
    return fail(ctx, VFISV_E_INVALID, "iter_histogram: n_bins outside 1..4096");
  if (!hist || (n > 0 && !iters)) return fail(ctx, VFISV_E_INVALID, "iter_histogram: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* bins = ctx->d_work + WORK_SLOTS;
  e = launch_hist(iters, n, n_bins, bins, ctx->num_cus * 8, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "iter_histogram launch");
  std::vector<unsigned long long> h((size_t)n_bins);
  e = hipMemcpyAsync(h.data(), bins, sizeof(unsigned long long) * n_bins, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "iter_histogram copy");
  for (int b = 0; b < n_bins; ++b) hist[b] = (int64_t)h[(size_t)b];
  return VFISV_OK;
}

int vfisv_solve(vfisv_ctx* ctx, int64_t n, const float* H, const float* g, const double* eps,
                uint32_t free_mask, double* delta, int32_t* code, void* stream) {
  vfisv::TraceRange trace_("vfisv_solve");
  if (!ctx) return fail(nullptr, VFISV_E_INVALID, "solve: ctx is NULL");
  if (n < 0) return fail(ctx, VFISV_E_INVALID, "solve: n < 0");
  if (n == 0) return VFISV_OK;
  if (!H || !g || !eps || !delta) return fail(ctx, VFISV_E_INVALID, "solve: NULL buffer");
  hipError_t e = use_device(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  SolveArgs a;
  a.H = H;
  a.g = g;
  a.eps = eps;
  a.delta = delta;
  a.code = code;
  a.n = n;
  a.free_mask = free_mask & 0x3FFu;
  const int grid = grid_for(n, ctx->max_lanes / 64);
  e = launch_solve(a, grid, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "solve launch");
  return VFISV_OK;
}

}  // extern "C"
