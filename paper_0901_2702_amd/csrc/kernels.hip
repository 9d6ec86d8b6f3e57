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
  const int t = threadIdx.x;
  if (t < WORK_SLOTS && (all || t >= QUEUE_SLOT0)) work[t] = 0ull;
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

// SplitMix64 (Steele, Lea and Flood 2014) as a counter-based generator:
// output number c of the stream seeded with seed.  Restart k of a pixel draws
// parameter q from output (pixel << 16 | k << 4 | q), top 53 bits.
__device__ __forceinline__ double restart_uniform(unsigned long long seed, int64_t pix, int k,
                                                  int q) {
  const unsigned long long c = ((unsigned long long)pix << 16) |
                               ((unsigned long long)(k & 0xFFF) << 4) | (unsigned long long)q;
  unsigned long long z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Scale of restart perturbations: half-widths of the synthetic priors.
__device__ __forceinline__ double restart_half(int q) {
  constexpr double h[NPAR] = {1500.0, 90.0, 90.0, 3.0, 15.0, 0.25, 14.5, 0.2, 0.2, 0.4};
  return h[q];
}

struct WaveCounters {
  unsigned long long pix = 0, trial = 0, acc = 0, pass = 0, fb = 0, hess = 0, jpass = 0,
                     jneed = 0;
};

// One synthesis pass with derivatives at Mc for the pixel's observations:
// returns the reduced chi^2 (Eq. 1) in float64 and, when the trial is
// accepted (fresh start, or finite and below chib), leaves the float32
// normal equations H (55, packed) and g (10) of Mc in this lane's LDS
// column.  NOBS = 6: dense HMI-shaped filter, all 174 row accumulators held
// until chi^2 decides whether H and g are built.  NOBS = 0: banded filter,
// rows folded into chi^2, H and g as they complete (H and g are built for
// every trial, since the rows are gone once chi^2 is known).
// keep_h: the step starts from a model near the minimum (Sect. 4.4): only g
// is rebuilt and stored, H stays as it is in LDS.
// One pass of the dense layout over windowed records: the same chi^2 and
// normal equations as lm_pass, from five register slots and the row parked
// in LDS.  After the pass every row is folded into chi^2, g (registers) and
// H (the lane's LDS slots, 14 float4, read and written once per row), for
// every lane: some lane of the wave accepts in practically every pass, so
// the wave would run the fold anyway, and with H out of the registers the
// fold needs no more of them than the point loop.  Accepted lanes then copy
// H and g to the parking area.
template <int NOBS, int V>
__device__ __forceinline__ double lm_pass_win(const LMArgs& A, const Pix& px, const RowFactors& rf,
                                              int64_t pix, bool fresh, double chib, bool keep_h,
                                              float* sHG, float4* sHa, int lane, bool& accept) {
  constexpr int ROWS = 4 * NOBS;
  const float* obs = A.stokes + pix * ROWS;
  const float* Wp = A.W_pp ? A.W + pix * ROWS : A.W;
  float4* park = sHa + H4 * 64;
  float acc[5][NACC];
  synth_accumulate_win<V>(A.pts5, px, A.C, acc, park, lane);
  double chi = 0.0;
  float g[NPAR];
#pragma unroll
  for (int e = 0; e < NPAR; ++e) g[e] = 0.f;
  if (!keep_h) {
#pragma unroll
    for (int c = 0; c < H4; ++c) sHa[c * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  auto fold = [&](const float* a, int q) {
    const int i = A.C.slot_row[q];
    float S[4], J[4][NPAR], WJ[4][NPAR];
    assemble_sample<true>(a, A.C.slot_rs[q], rf, S, J);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float w = Wp[s * NOBS + i];
      const float r = obs[s * NOBS + i] - S[s];
      chi = fma((double)w * (double)r, (double)r, chi);
#pragma unroll
      for (int p = 0; p < NPAR; ++p) {
        WJ[s][p] = w * J[s][p];
        if (!jzero(s, p)) g[p] = fmaf(WJ[s][p], r, g[p]);
      }
    }
    if (!keep_h) {
      lds_rmw4<0, H4>(sHa, lane, [&](auto cc, float4& h) __attribute__((always_inline)) {
        float* hv = &h.x;
        static_for<4>([&](auto kk) __attribute__((always_inline)) {
          constexpr int k = decltype(kk)::value, e = 4 * decltype(cc)::value + k;
          if constexpr (e < 55) {
            constexpr int p = pk_row(e), q2 = pk_col(e);
            static_for<4>([&](auto ss) __attribute__((always_inline)) {
              constexpr int s = decltype(ss)::value;
              if constexpr (!hzero(s, e)) hv[k] = fmaf(WJ[s][p], J[s][q2], hv[k]);
            });
          }
        });
      });
    }
  };
#pragma unroll
  for (int q = 0; q < 5; ++q) fold(acc[q], q);
  {
    float a[NACC];
    unpark(park, lane, a);
    fold(a, 5);
  }
  chi *= A.inv_dof;
  accept = fresh || (isfinite(chi) && chi < chib);
  if (accept) {
    if (!keep_h) {
#pragma unroll
      for (int c = 0; c < H4; ++c) {
        const float4 h = sHa[c * 64 + lane];
        const float hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (4 * c + k < 55) sHG[(4 * c + k) * 64 + lane] = hv[k];
      }
    }
#pragma unroll
    for (int e = 0; e < NPAR; ++e) sHG[(55 + e) * 64 + lane] = g[e];
  }
  return chi;
}

template <int NOBS, int LPP, int V>
__device__ __forceinline__ double lm_pass(const LMArgs& A, const float* Mc, int64_t pix,
                                          bool fresh, double chib, bool keep_h, float* sHG,
                                          float4* sHa, int lane, bool& accept) {
  Pix px;
  pix_setup(Mc, A.C, px);
  RowFactors rf;
  row_factors(Mc, px, A.C, rf);
  double chi = 0.0;
  if constexpr (NOBS > 0 && LPP == 1) {
    if (A.C.sw_k >= 0) return lm_pass_win<NOBS, V>(A, px, rf, pix, fresh, chib, keep_h, sHG, sHa,
                                                   lane, accept);
  }
  if constexpr (NOBS > 0) {
    constexpr int ROWS = 4 * NOBS;
    const float* obs = A.stokes + pix * ROWS;
    const float* Wp = A.W_pp ? A.W + pix * ROWS : A.W;
    float acc[NOBS][NACC];
    if constexpr (LPP == 2)
      synth_accumulate_pair<NOBS, V>(A.pts, px, A.C, acc, lane & 1);
    else
      synth_accumulate<NOBS, true, V>(A.pts, px, A.C, acc);
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
    accept = fresh || (isfinite(chi) && chi < chib);
    if (accept && !keep_h) {
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
            if (jzero(s, p)) continue;
            g[p] = fmaf(wj, r, g[p]);
#pragma unroll
            for (int q = 0; q <= p; ++q)
              if (!jzero(s, q)) H[pk(p, q)] = fmaf(wj, J[s][q], H[pk(p, q)]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 55; ++e) sHG[e * 64 + lane] = H[e];
#pragma unroll
      for (int e = 0; e < NPAR; ++e) sHG[(55 + e) * 64 + lane] = g[e];
    } else if (accept) {  // H kept: the gradient alone
      float g[NPAR];
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
          for (int p = 0; p < NPAR; ++p)
            if (!jzero(s, p)) g[p] = fmaf(w * J[s][p], r, g[p]);
        }
      }
#pragma unroll
      for (int e = 0; e < NPAR; ++e) sHG[(55 + e) * 64 + lane] = g[e];
    }
  } else {
    const int no = A.C.n_obs;
    const float* obs = A.stokes + pix * (int64_t)(4 * no);
    const float* Wp = A.W_pp ? A.W + pix * (int64_t)(4 * no) : A.W;
    // H (packed, entries 0-54) and g (55-64) are accumulated in the lane's
    // slots of LDS (17 float4, lane-interleaved), read and written once per
    // completed row, so that the registers hold the band window and the
    // synthesis point
#pragma unroll
    for (int c = 0; c < HG4; ++c)
      if (c >= G4_FIRST || !keep_h) sHa[c * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    float ob[4], wb[4], rs = 0.f;
    band_accumulate<true>(
        A.blocks, no, px, A.C,
        [&](int j) {
          rs = A.row_sums[j];
          if (A.stokes4) {  // one 16-byte load; a line serves 8 consecutive rows
            const float4 o4 = A.stokes4[pix * (int64_t)no + j];
            ob[0] = o4.x;
            ob[1] = o4.y;
            ob[2] = o4.z;
            ob[3] = o4.w;
          } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) ob[s] = obs[s * no + j];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) wb[s] = Wp[s * no + j];
        },
        [&](int, const float* a) {
          float S[4], J[4][NPAR], WJ[4][NPAR], R[4];
          assemble_sample<true>(a, rs, rf, S, J);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const float w = wb[s];
            R[s] = ob[s] - S[s];
            chi = fma((double)w * (double)R[s], (double)R[s], chi);
#pragma unroll
            for (int p = 0; p < NPAR; ++p) WJ[s][p] = w * J[s][p];
          }
          // slot c: entries of H (unless H is kept) and of g
          auto upd = [&](auto cc, float4& h, auto with_h) __attribute__((always_inline)) {
            float* hv = &h.x;
            static_for<4>([&](auto kk) __attribute__((always_inline)) {
              constexpr int k = decltype(kk)::value, e = 4 * decltype(cc)::value + k;
              if constexpr (e < 55 && decltype(with_h)::value) {
                constexpr int p = pk_row(e), q2 = pk_col(e);
                static_for<4>([&](auto ss) __attribute__((always_inline)) {
                  constexpr int s = decltype(ss)::value;
                  if constexpr (!hzero(s, e)) hv[k] = fmaf(WJ[s][p], J[s][q2], hv[k]);
                });
              } else if constexpr (e >= 55 && e < 65) {
                static_for<4>([&](auto ss) __attribute__((always_inline)) {
                  constexpr int s = decltype(ss)::value;
                  if constexpr (!jzero(s, e - 55)) hv[k] = fmaf(WJ[s][e - 55], R[s], hv[k]);
                });
              }
            });
          };
          if (!keep_h)
            lds_rmw4<0, HG4>(sHa, lane, [&](auto cc, float4& h) __attribute__((always_inline)) {
              upd(cc, h, std::true_type{});
            });
          else
            lds_rmw4<G4_FIRST, HG4>(sHa, lane, [&](auto cc, float4& h) __attribute__((always_inline)) {
              upd(cc, h, std::false_type{});
            });
        });
    chi *= A.inv_dof;
    accept = fresh || (isfinite(chi) && chi < chib);
    if (accept) {
#pragma unroll
      for (int c = 0; c < HG4; ++c) {
        if (c < G4_FIRST && keep_h) continue;
        const float4 h = sHa[c * 64 + lane];
        const float hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int e = 4 * c + k;
          if ((e < 55 && !keep_h) || (e >= 55 && e < 65)) sHG[e * 64 + lane] = hv[k];
        }
      }
    }
  }
  return chi;
}

// One synthesis pass without derivatives at Mc: the reduced chi^2 (Eq. 1)
// in float64 of a trial.  Every row receives the same products in the same
// order as in lm_pass, and the rows enter chi^2 in lm_pass's order (the
// windowed pass folds its register slots first and the parked row last;
// ptsv holds the rows in that order), so a model gets the same chi^2 from
// either pass.
template <int NOBS, int LPP, int V>
__device__ __forceinline__ double lm_pass_values(const LMArgs& A, const float* Mc, int64_t pix,
                                                 int lane) {
  Pix px;
  pix_setup(Mc, A.C, px);
  RowFactors rf;
  row_factors(Mc, px, A.C, rf);
  double chi = 0.0;
  if constexpr (NOBS > 0) {
    constexpr int ROWS = 4 * NOBS;
    const float* obs = A.stokes + pix * ROWS;
    const float* Wp = A.W_pp ? A.W + pix * ROWS : A.W;
    const bool win = LPP == 1 && A.C.sw_k >= 0;
    float acc[NOBS][NACC];
    if constexpr (LPP == 2)
      synth_accumulate_pair<NOBS, V, false>(A.pts, px, A.C, acc, lane & 1);
    else
      synth_accumulate<NOBS, false, V>(win ? A.ptsv : A.pts, px, A.C, acc);
#pragma unroll
    for (int q = 0; q < NOBS; ++q) {
      const int i = win ? A.C.slot_row[q] : q;
      float S[4], J[4][NPAR];
      assemble_sample<false>(acc[q], win ? A.C.slot_rs[q] : A.C.row_sum[q], rf, S, J);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float r = obs[s * NOBS + i] - S[s];
        chi = fma((double)Wp[s * NOBS + i] * (double)r, (double)r, chi);
      }
    }
  } else {
    const int no = A.C.n_obs;
    const float* obs = A.stokes + pix * (int64_t)(4 * no);
    const float* Wp = A.W_pp ? A.W + pix * (int64_t)(4 * no) : A.W;
    float ob[4], wb[4], rs = 0.f;
    band_accumulate<false>(
        A.blocks, no, px, A.C,
        [&](int j) {
          rs = A.row_sums[j];
          if (A.stokes4) {
            const float4 o4 = A.stokes4[pix * (int64_t)no + j];
            ob[0] = o4.x;
            ob[1] = o4.y;
            ob[2] = o4.z;
            ob[3] = o4.w;
          } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) ob[s] = obs[s * no + j];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) wb[s] = Wp[s * no + j];
        },
        [&](int, const float* a) {
          float S[4], J[4][NPAR];
          assemble_sample<false>(a, rs, rf, S, J);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const float r = ob[s] - S[s];
            chi = fma((double)wb[s] * (double)r, (double)r, chi);
          }
        });
  }
  return chi * A.inv_dof;
}

// The persistent LM loop of one wave over one batch: lanes take pixels
// from the batch's queues, fit them, and return when the queues are empty
// and every lane has finished.
// LPP = 2 (dense only): a pair of lanes carries one pixel; the even lane is
// the pair's leader (it takes queue positions, writes the results and counts
// the work), the odd lane mirrors its state: both see the same inputs and
// the same pair sums, so they take the same decisions.
// PAPER: the fixed-iteration scheme of Sect. 4.2 (A.fixed_iters trials per
// pixel, restarts from a perturbed best model, the best model seen is the
// result); otherwise exits on convergence, stall or A.max_iter.
template <int NOBS, int LPP, int V = 0, bool PAPER = false, bool SPLIT = false>
__device__ __forceinline__ void lm_loop(const LMArgs& A, float* sHG, float4* sHa, double* sws,
                                        int lane,
                                        int64_t glane,
                                        WaveCounters& wc) {
  static_assert(LPP == 1 || (LPP == 2 && NOBS > 0), "lane pairs serve the dense layout");
  const bool leader = LPP == 1 || (lane & 1) == 0;
  const int mate = lane & ~(LPP - 1);
  const unsigned long long n_total = A.n_dev ? *A.n_dev : (unsigned long long)A.n;
  const int rows = NOBS > 0 ? 4 * NOBS : 4 * A.C.n_obs;
  // Pixel queues: queue q owns the blocks b of 2^chunk_log2 consecutive
  // positions with b % NQ == q; its k-th position is
  // ((k / chunk) * NQ + q) * chunk + k % chunk.  A wave takes positions
  // from the queue of its XCD first (workgroups are dispatched to the XCDs
  // round-robin), so the lines of the pixels one XCD works on stay in that
  // XCD's L2, then from the others.
  const int home = blockIdx.x % NQ;
  const int sh = A.chunk_log2;
  const unsigned long long ch = 1ull << sh;
  const unsigned long long full = n_total >> (sh + 3), rem = n_total & ((ch << 3) - 1ull);
  unsigned dry = 0u;  // queues this wave has seen empty (wave-uniform)
  bool live = false, fresh = false, exhausted = false;
  int64_t pix = 0;
  float Mb[NPAR], Mc[NPAR];
  double chib = 0.0, eps = 0.0;
  int it = 0;
  // fixed-iteration scheme: best model seen, first chi^2, failed trials in
  // a row, restarts used, restart due / being evaluated
  float Mg[NPAR];
  double chig = 0.0, chi_first = 0.0;
  int bad = 0, kr = 0;
  bool pending = false, restart_eval = false;
  // the damped solve needs the eigen fallback: done with the whole wave at
  // the top of the next turn, where every lane is active
  bool need_fb = false;
  // derivative pass due (Fig. 6: derivatives only at accepted models): an
  // accepted trial of a values-only pass waits for the next derivative pass
  // of its wave; kh_wait: that pass keeps J^T W J (Sect. 4.4)
  bool need_j = false, kh_wait = false;
  const int limit = PAPER ? A.fixed_iters : A.max_iter;
  // SPLIT: trials in values-only passes, derivatives in their own pass (not
  // in the fixed-iteration scheme, whose restarts are fresh starts)
  static_assert(!(SPLIT && PAPER), "the fixed-iteration scheme fuses its passes");

  for (;;) {
    // ---- refill lanes whose pixel finished --------------------------------
    unsigned long long nm = __ballot(!live && !exhausted && leader);
    for (int j = 0; j < NQ && nm != 0ull; ++j) {
      const int q = (home + j) % NQ;
      if (dry & (1u << q)) continue;
      const unsigned long long r0 = rem > (unsigned long long)q * ch ? rem - q * ch : 0ull;
      const unsigned long long cnt = full * ch + (r0 < ch ? r0 : ch);
      const unsigned long long m = (unsigned long long)__popcll(nm);
      unsigned long long k0 = 0;
      if (lane == 0) k0 = atomicAdd(&A.work[A.qbase + q], m);
      k0 = bcast_lane0(k0);
      const unsigned long long got = k0 < cnt ? (cnt - k0 < m ? cnt - k0 : m) : 0ull;
      if (got < m) dry |= 1u << q;
      if (got == 0ull) continue;
      const bool need = (nm >> lane) & 1ull;
      const unsigned long long rank = (unsigned long long)__popcll(nm & ((1ull << lane) - 1ull));
      const bool take = need && rank < got;
      unsigned long long k = k0 + rank;
      bool mine = take;
      if constexpr (LPP == 2) {  // the odd lane follows its leader
        mine = __shfl(take ? 1 : 0, mate) != 0;
        const unsigned lo = __shfl((unsigned)(k & 0xffffffffull), mate);
        const unsigned hi = __shfl((unsigned)(k >> 32), mate);
        k = ((unsigned long long)hi << 32) | lo;
      }
      if (mine) {
        const unsigned long long pos =
            ((((k >> sh) << 3) + (unsigned long long)q) << sh) + (k & (ch - 1ull));
        pix = A.idx ? (int64_t)A.idx[pos] : (int64_t)pos;
        // (the observations and weights are not read here: a non-finite one
        // makes the first pass's chi^2 non-finite, and only then are they
        // examined, so that a refill does not wait on their loads)
        {
          double M0[NPAR];
          if (A.init) {
#pragma unroll
            for (int q2 = 0; q2 < NPAR; ++q2) M0[q2] = (double)A.init[pix * NPAR + q2];
          } else {
            const double d0[NPAR] = {1500.0, 90.0, 90.0, 0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6};
#pragma unroll
            for (int q2 = 0; q2 < NPAR; ++q2) M0[q2] = d0[q2];
          }
          project(M0);
#pragma unroll
          for (int q2 = 0; q2 < NPAR; ++q2) Mc[q2] = (float)M0[q2];
          live = true;
          fresh = true;
          eps = A.eps0;
          it = 0;
          bad = 0;
          kr = 0;
          pending = false;
          restart_eval = false;
        }
      }
      nm &= ~__ballot(take);
    }
    if (nm != 0ull && dry == (1u << NQ) - 1u) exhausted = exhausted || ((nm >> lane) & 1ull);
    if constexpr (LPP == 2) exhausted = __shfl(exhausted ? 1 : 0, mate) != 0;

    // ---- eigen/SVD fallbacks of the last steps, one lane at a time --------
    for (unsigned long long fbm = __ballot(need_fb); fbm != 0ull; fbm &= fbm - 1ull) {
      const int L = __ffsll((unsigned long long)fbm) - 1;
      solve_eigen_wave(&sHG[L], 64, &sHG[55 * 64 + L], 64, __shfl(eps, L), A.free_mask, sws,
                       lane);
      if (lane == L) {
        if (leader) ++wc.fb;
        double Mt[NPAR];
#pragma unroll
        for (int q = 0; q < NPAR; ++q) Mt[q] = (double)Mb[q] + sws[200 + q];
        project(Mt);
#pragma unroll
        for (int q = 0; q < NPAR; ++q) Mc[q] = (float)Mt[q];
        need_fb = false;
      }
      __syncthreads();  // lane L has read the step before the record is reused
    }
    const unsigned long long live_m = __ballot(live);
    if (live_m == 0ull) {
      if (__ballot(!exhausted) == 0ull) break;
      continue;  // (defensive: after a refill every lane is live or exhausted)
    }
    // ---- the wave's pass: with derivatives (fresh starts, accepted models
    // waiting for their Jacobian, and the other lanes' trials with their
    // Jacobian computed ahead), or, while few lanes wait, values only for
    // the trials ---------------------------------------------------------------
    const bool wait = need_j || fresh;
    bool jpass = true;
    if constexpr (SPLIT) {
      const int nw = __popcll(__ballot(live && wait)), nl = __popcll(live_m);
      jpass = nw == nl || nw * 64 >= A.deriv_split * nl;
    }
    if (!live || (!jpass && wait)) continue;

    if (leader) {
      ++wc.pass;
      if (jpass) ++wc.jpass;
    }
    bool accept = false;
    // Sect. 4.4: a step from a model already near the minimum keeps H
    const bool keep_h = need_j ? kh_wait : (!fresh && chib < A.hess_reuse);
    double chi;
    bool hess_counted = false;
    if (!SPLIT || jpass) {
      chi = lm_pass<NOBS, LPP, V>(A, Mc, pix, wait, chib, keep_h, sHG, sHa, lane, accept);
      hess_counted = leader && accept && !keep_h;
      if (hess_counted) ++wc.hess;
    } else {
      chi = lm_pass_values<NOBS, LPP, V>(A, Mc, pix, lane);
      accept = isfinite(chi) && chi < chib;
    }

    // ---- Levenberg-Marquardt bookkeeping (Sect. 4.2, Table 2) -------------
    int done = -1;
    bool bad_input = false;
    // the pass's model is a start or an accepted trial: the fit needs its
    // Jacobian unless it ends here
    const bool new_best = !need_j && (fresh || accept);
    if (need_j) {
      // the Jacobian, J^T W J and gradient of the accepted model Mb = Mc are
      // now in LDS; its chi^2 is the one the trial pass found
      need_j = false;
    } else if (fresh) {
      if (!isfinite(chi) && !restart_eval) {
        done = 3;
        // a non-finite observation or weight, rather than a start whose
        // synthesis is not finite: the pixel is not fitted at all (no
        // model, no iterations) and its pass is not counted as work
        const float* obs = A.stokes + pix * rows;
        const float* Wp = A.W_pp ? A.W + pix * rows : A.W;
        for (int r = 0; r < rows; ++r) bad_input = bad_input || !isfinite(obs[r]) || !isfinite(Wp[r]);
        if (bad_input && leader) {
          --wc.pass;
          if (jpass) --wc.jpass;
          if (hess_counted) --wc.hess;
        }
      }
#pragma unroll
      for (int q = 0; q < NPAR; ++q) Mb[q] = Mc[q];
      chib = chi;
      if constexpr (PAPER) {
        if (restart_eval) {  // the restart's evaluation is a trial
          ++it;
          if (leader) ++wc.trial;
          if (isfinite(chi) && chi < chig) {
#pragma unroll
            for (int q = 0; q < NPAR; ++q) Mg[q] = Mc[q];
            chig = chi;
          }
          bad = 0;
          restart_eval = false;
        } else {
          chi_first = chi;
          chig = chi;
#pragma unroll
          for (int q = 0; q < NPAR; ++q) Mg[q] = Mc[q];
        }
      }
    } else {
      ++it;
      if (leader) ++wc.trial;
      if (accept) {
        const double dec = chib - chi;
        // values-only pass: the derivatives of the new best model are due
        // (unless the fit ends here)
        need_j = !jpass;
        kh_wait = chib < A.hess_reuse;
#pragma unroll
        for (int q = 0; q < NPAR; ++q) Mb[q] = Mc[q];
        chib = chi;
        eps = eps_down(eps);
        if (leader) ++wc.acc;
        if constexpr (PAPER) {
          bad = 0;
          if (chi < chig) {
#pragma unroll
            for (int q = 0; q < NPAR; ++q) Mg[q] = Mc[q];
            chig = chi;
          }
        } else {
          if (dec < A.rel_tol * (chi + dec)) done = 0;
        }
      } else {
        eps = eps_up(eps);
        if constexpr (PAPER) ++bad;
        else if (eps > A.eps_max) done = 2;
      }
      if constexpr (PAPER) {
        // restart triggers: (a) after 10 trials chi^2 not down tenfold from
        // its first value, (b) 5 failed trials in a row, or a stall
        const bool stalled = eps > A.eps_max;
        if (kr < A.restarts && ((it == 10 && !(chig <= chi_first / 10.0)) || bad >= 5 || stalled))
          pending = true;
        else if (stalled)
          done = 2;
      }
    }
    fresh = false;
    if (done < 0 && it >= limit) done = 1;
    if (done >= 0) need_j = false;
    if (leader && new_best && done < 0) ++wc.jneed;

    if (done >= 0) {
      if (leader) {
        if (bad_input) {
#pragma unroll
          for (int q = 0; q < NPAR; ++q) A.params[pix * NPAR + q] = __builtin_nanf("");
          A.chi2[pix] = __builtin_nan("");
          A.iters[pix] = 0;
          if (A.status) A.status[pix] = 3;
        } else {
#pragma unroll
          for (int q = 0; q < NPAR; ++q) A.params[pix * NPAR + q] = PAPER ? Mg[q] : Mb[q];
          A.chi2[pix] = PAPER ? chig : chib;
          A.iters[pix] = it;
          if (A.status) A.status[pix] = PAPER ? (done | (kr << 8)) : done;
        }
        ++wc.pix;
      }
      live = false;
    } else if (PAPER && pending) {
      // ---- restart: the best model's free parameters, perturbed -----------
      ++kr;
      double Mt[NPAR];
#pragma unroll
      for (int q = 0; q < NPAR; ++q) {
        const double u = restart_uniform(A.seed, pix, kr, q);
        Mt[q] = ((A.free_mask >> q) & 1u)
                    ? (double)Mg[q] + (2.0 * u - 1.0) * 0.1 * kr * restart_half(q)
                    : (double)Mg[q];
      }
      project(Mt);
#pragma unroll
      for (int q = 0; q < NPAR; ++q) Mc[q] = (float)Mt[q];
      fresh = true;
      restart_eval = true;
      pending = false;
    } else if (need_j) {
      // waits for its wave's next derivative pass (no step without the
      // normal equations of Mb)
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
        need_fb = true;  // the step is taken at the top of the next turn
      } else {
        double Mt[NPAR];
#pragma unroll
        for (int q = 0; q < NPAR; ++q) Mt[q] = (double)Mb[q] + delta[q];
        project(Mt);
#pragma unroll
        for (int q = 0; q < NPAR; ++q) Mc[q] = (float)Mt[q];
      }
    }
  }
}

// ---- work counters: one atomic per wave and counter ----------------------
__device__ __forceinline__ void flush_counters(unsigned long long* work, WaveCounters wc,
                                               int lane) {
  const unsigned long long p = wave_sum(wc.pix), t = wave_sum(wc.trial), a = wave_sum(wc.acc),
                           s = wave_sum(wc.pass), f = wave_sum(wc.fb),
                           h = wave_sum(wc.hess), j = wave_sum(wc.jpass),
                           jn = wave_sum(wc.jneed);
  if (lane == 0) {
    atomicAdd(&work[0], j);
    atomicAdd(&work[8], jn);
    atomicAdd(&work[1], p);
    atomicAdd(&work[2], t);
    atomicAdd(&work[3], a);
    atomicAdd(&work[4], s);
    atomicAdd(&work[5], f);
    atomicAdd(&work[6], 1ull);
    atomicAdd(&work[7], h);
  }
}

// V: Voigt evaluation (0 Weideman's series, 1/2 Taylor table; dense only).
// SPLIT: values-only trial passes with derivative passes on demand (a
// separate kernel, so that the fused one keeps its own register allocation).
template <int NOBS, int V, bool PAPER, bool SPLIT = false>
__global__ __launch_bounds__(64) void lm_kernel(const LMArgs A) {
  __shared__ float sHG[65 * 64];  // H (55, packed) and g (10) per lane
  __shared__ float4 sHa[PASS4 * 64];  // the pass's accumulators in LDS
  double* sws = ws_record(sHa);       // the wave's eigen-fallback record
  const int lane = threadIdx.x;
  const int64_t glane = (int64_t)blockIdx.x * 64 + lane;
  WaveCounters wc;
  if constexpr (NOBS > 0) {
    const unsigned long long n_total = A.n_dev ? *A.n_dev : (unsigned long long)A.n;
    // pairs only for batches small enough (host's choice, pair_max)
    if (A.lpp_max >= 2 && n_total <= (unsigned long long)A.pair_max)
      lm_loop<NOBS, 2, V, PAPER, SPLIT>(A, sHG, sHa, sws, lane, glane, wc);
    else
      lm_loop<NOBS, 1, V, PAPER, SPLIT>(A, sHG, sHa, sws, lane, glane, wc);
  } else {
    lm_loop<NOBS, 1, V, PAPER, SPLIT>(A, sHG, sHa, sws, lane, glane, wc);
  }
  flush_counters(A.work, wc, lane);
}

// Several batches in one launch: each wave finishes its share of batch i
// (until that batch's queues are empty) before it turns to batch i + 1, so
// waves are uniform in instrument and the last batch fills the tail left by
// the earlier ones.
template <bool SPLIT>
__global__ __launch_bounds__(64) void lm_batches_kernel(const BatchArgs B) {
  __shared__ float sHG[65 * 64];
  __shared__ float4 sHa[PASS4 * 64];
  double* sws = ws_record(sHa);
  const int lane = threadIdx.x;
  const int64_t glane = (int64_t)blockIdx.x * 64 + lane;
  WaveCounters wc;
  for (int i = 0; i < B.n_batches; ++i) {
    if (B.kind[i] == KIND_DENSE6)
      lm_loop<NOBS_HMI, 1, 0, false, SPLIT>(B.a[i], sHG, sHa, sws, lane, glane, wc);
    else
      lm_loop<0, 1, 0, false, SPLIT>(B.a[i], sHG, sHa, sws, lane, glane, wc);
  }
  flush_counters(B.a[0].work, wc, lane);
}

template <int NOBS, bool DERIV, int V>
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
    synth_accumulate<NOBS, DERIV, V>(A.pts, px, A.C, acc);
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

// Synthesis through a banded instrument: rows are written as they complete.
template <bool DERIV>
__global__ __launch_bounds__(64) void synth_band_kernel(const SynthArgs A) {
  const int no = A.C.n_obs;
  for (int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x; i < A.n;
       i += (int64_t)gridDim.x * 64) {
    float M[NPAR];
#pragma unroll
    for (int q = 0; q < NPAR; ++q) M[q] = A.params[i * NPAR + q];
    Pix px;
    pix_setup(M, A.C, px);
    RowFactors rf;
    row_factors(M, px, A.C, rf);
    band_accumulate<DERIV>(A.blocks, no, px, A.C, [](int) {}, [&](int j, const float* a) {
      float S[4], J[4][NPAR];
      assemble_sample<DERIV>(a, A.row_sums[j], rf, S, J);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t r = i * (int64_t)(4 * no) + s * no + j;
        A.stokes[r] = A.noise ? S[s] + A.noise[r] : S[s];
        if (DERIV) {
#pragma unroll
          for (int p = 0; p < NPAR; ++p) A.jac[r * NPAR + p] = J[s][p];
        }
      }
    });
  }
}

__global__ __launch_bounds__(64) void solve_kernel(const SolveArgs A) {
  __shared__ double sws[WS_DOUBLES];  // the wave's eigen-fallback record
  const int lane = threadIdx.x;
  // a wave-uniform loop, so that every lane takes part in the fallbacks
  for (int64_t base = (int64_t)blockIdx.x * 64; base < A.n; base += (int64_t)gridDim.x * 64) {
    const int64_t i = base + lane;
    const bool valid = i < A.n;
    double delta[NPAR];
    int code = 0;
    double eps = 0.0;
    if (valid) {
      float H[55], g[NPAR];
#pragma unroll
      for (int e = 0; e < 55; ++e) H[e] = A.H[i * 55 + e];
#pragma unroll
      for (int e = 0; e < NPAR; ++e) g[e] = A.g[i * NPAR + e];
      double sc[NPAR], b[NPAR];
      eps = A.eps[i];
      code = solve_cholesky(H, g, eps, A.free_mask, delta, sc, b);
    }
    for (unsigned long long fbm = __ballot(valid && code == 1); fbm != 0ull; fbm &= fbm - 1ull) {
      const int L = __ffsll((unsigned long long)fbm) - 1;
      const int64_t iL = base + L;
      solve_eigen_wave(A.H + iL * 55, 1, A.g + iL * NPAR, 1, __shfl(eps, L), A.free_mask, sws,
                       lane);
      if (lane == L) {
#pragma unroll
        for (int q = 0; q < NPAR; ++q) delta[q] = sws[200 + q];
      }
      __syncthreads();  // lane L has read the step before the record is reused
    }
    if (valid) {
#pragma unroll
      for (int p = 0; p < NPAR; ++p) A.delta[i * NPAR + p] = delta[p];
      if (A.code) A.code[i] = code;
    }
  }
}

// ---- launch helpers (host) --------------------------------------------------

// Histogram of iteration counts: per-block LDS counts, flushed with one
// atomic per non-empty bin and block.  Values >= n_bins - 1 land in the last
// bin, negative values in bin 0.
__global__ __launch_bounds__(256) void hist_kernel(const int32_t* __restrict__ iters, int64_t n,
                                                   int n_bins, unsigned long long* out) {
  __shared__ unsigned int h[HIST_MAX];
  for (int b = threadIdx.x; b < n_bins; b += 256) h[b] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int v = iters[i];
    atomicAdd(&h[v < 0 ? 0 : (v >= n_bins ? n_bins - 1 : v)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < n_bins; b += 256)
    if (h[b]) atomicAdd(&out[b], (unsigned long long)h[b]);
}

__global__ void zero_bins_kernel(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0ull;
}

hipError_t launch_hist(const int32_t* iters, int64_t n, int n_bins, unsigned long long* out,
                       int max_blocks, hipStream_t s) {
  zero_bins_kernel<<<(n_bins + 255) / 256, 256, 0, s>>>(out, n_bins);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  const int64_t want = (n + 255) / 256;
  const int blocks = (int)(want < max_blocks ? want : max_blocks);
  hist_kernel<<<blocks, 256, 0, s>>>(iters, n, n_bins, out);
  return hipGetLastError();
}

hipError_t launch_reset(unsigned long long* work, bool all, hipStream_t s) {
  reset_work_kernel<<<1, 64, 0, s>>>(work, all ? 1 : 0);
  return hipGetLastError();
}

template <bool PAPER>
static void launch_lm_mode(const LMArgs& a, int kind, int voigt, int grid, hipStream_t s) {
  // the split pass serves Weideman's series outside the fixed-iteration scheme
  const bool split = !PAPER && voigt == 0 && a.deriv_split > 0;
  if (kind != KIND_DENSE6) {
    if (split) lm_kernel<0, 0, false, true><<<grid, 64, 0, s>>>(a);
    else lm_kernel<0, 0, PAPER><<<grid, 64, 0, s>>>(a);
  } else if (voigt == 1) {
    lm_kernel<NOBS_HMI, 1, PAPER><<<grid, 64, 0, s>>>(a);
  } else if (voigt == 2) {
    lm_kernel<NOBS_HMI, 2, PAPER><<<grid, 64, 0, s>>>(a);
  } else {
    if (split) lm_kernel<NOBS_HMI, 0, false, true><<<grid, 64, 0, s>>>(a);
    else lm_kernel<NOBS_HMI, 0, PAPER><<<grid, 64, 0, s>>>(a);
  }
}

hipError_t launch_lm(const LMArgs& a, int kind, int voigt, int grid, hipStream_t s) {
  if (a.fixed_iters > 0) launch_lm_mode<true>(a, kind, voigt, grid, s);
  else launch_lm_mode<false>(a, kind, voigt, grid, s);
  return hipGetLastError();
}

hipError_t launch_lm_batches(const BatchArgs& b, int grid, hipStream_t s) {
  bool split = false;
  for (int i = 0; i < b.n_batches; ++i) split = split || b.a[i].deriv_split > 0;
  if (split) lm_batches_kernel<true><<<grid, 64, 0, s>>>(b);
  else lm_batches_kernel<false><<<grid, 64, 0, s>>>(b);
  return hipGetLastError();
}

hipError_t launch_synth(const SynthArgs& a, int kind, int voigt, bool deriv, int grid,
                        hipStream_t s) {
  if (kind == KIND_DENSE6) {
    if (voigt == 1) {
      if (deriv) synth_kernel<NOBS_HMI, true, 1><<<grid, 64, 0, s>>>(a);
      else synth_kernel<NOBS_HMI, false, 1><<<grid, 64, 0, s>>>(a);
    } else if (voigt == 2) {
      if (deriv) synth_kernel<NOBS_HMI, true, 2><<<grid, 64, 0, s>>>(a);
      else synth_kernel<NOBS_HMI, false, 2><<<grid, 64, 0, s>>>(a);
    } else {
      if (deriv) synth_kernel<NOBS_HMI, true, 0><<<grid, 64, 0, s>>>(a);
      else synth_kernel<NOBS_HMI, false, 0><<<grid, 64, 0, s>>>(a);
    }
  } else {
    if (deriv) synth_band_kernel<true><<<grid, 64, 0, s>>>(a);
    else synth_band_kernel<false><<<grid, 64, 0, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int grid, hipStream_t s) {
  solve_kernel<<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

// The banded pass reads a row's four Stokes values together; in the API
// layout [n][4][n_obs] they lie in four cache lines that are each reused
// over 32 rows, longer than an XCD's L2 keeps them with every lane of the
// XCD streaming its own pixel, so the pass re-fetched them many times over.
__global__ __launch_bounds__(256) void interleave_kernel(const float* __restrict__ in,
                                                         float4* __restrict__ out, int64_t n,
                                                         int n_obs) {
  const int64_t total = n * (int64_t)n_obs;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t p = t / n_obs;
    const int64_t j = t - p * n_obs;
    const float* src = in + p * 4 * (int64_t)n_obs + j;
    out[t] = make_float4(src[0], src[n_obs], src[2 * (int64_t)n_obs], src[3 * (int64_t)n_obs]);
  }
}

hipError_t launch_interleave(const float* in, float4* out, int64_t n, int n_obs, hipStream_t s) {
  const int64_t total = n * (int64_t)n_obs;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  interleave_kernel<<<grid, 256, 0, s>>>(in, out, n, n_obs);
  return hipGetLastError();
}

hipError_t lm_blocks_per_cu(int* out) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, lm_kernel<NOBS_HMI, 0, false>, 64, 0);
}

hipError_t band_blocks_per_cu(int* out) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, lm_batches_kernel<false>, 64, 0);
}

}  // namespace vfisv
