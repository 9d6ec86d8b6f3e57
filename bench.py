"""Benchmark: inverted pixels/s of the Milne-Eddington LM inversion on one MI355X.

One step = one vfisv_invert over the whole batch (every pixel fitted from its
starting model to its exit), inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: 512 x 512 HMI-shaped pixels (Fe I 6173.3356 A, 6 Gaussian filters,
101-point synthesis grid), parameters drawn from the cfg0 priors (seed 1001),
N(0, 1e-3) noise, W = 1e6, plain Levenberg-Marquardt from the default model,
max 50 iterations.  Observations are synthesised on the device by the
library's own forward model from the seeded parameters and noise.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks used for the roofline fraction.
PEAK_FP32_TFLOPS = 157.3

# Algorithmic float32 work per unit, counted from the formula sequence of the
# synthesis ("Work per unit"): per synthesis point, per filter tap,
# per observed sample / Stokes row, plus the float64 solve.
FLOP_POINT_VALUES = 431      # 3 Faddeeva (124 each), absorption matrix, UR, mixing
FLOP_POINT_JAC_EXTRA = 379   # Eqs. 8-9, element and parameter tangents
FLOP_TAP_VALUES = 8          # 4 normalised Stokes values per tap
FLOP_TAP_JAC = 58            # 29 accumulators per tap
FLOP_SAMPLE_VALUES = 25      # assemble 4 values + 4 weighted squared residuals
FLOP_SAMPLE_JAC = 115 + 4 * 140  # assemble 4 Jacobian rows + normal equations
FLOP_SOLVE_FP64 = 1100       # equilibration, 10x10 Cholesky, substitutions, projection


def work_model(n_pts, n_taps, n_obs):
    f_trial = n_pts * FLOP_POINT_VALUES + n_taps * FLOP_TAP_VALUES + n_obs * FLOP_SAMPLE_VALUES
    f_jac = (n_pts * (FLOP_POINT_VALUES + FLOP_POINT_JAC_EXTRA) + n_taps * FLOP_TAP_JAC
             + n_obs * (FLOP_SAMPLE_VALUES + FLOP_SAMPLE_JAC))
    return f_trial, f_jac, FLOP_SOLVE_FP64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512 * 512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the inversion is per-pixel independent and "
              "this build runs on a single MI355X (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0901_2702_amd as vf
    import workloads as wl

    spec = wl.hmi_instrument()
    n = args.n
    seed = wl.CONFIGS["cfg1"]["seed"]
    P = wl.draw_params(n, seed)
    noise = wl.draw_noise(n, spec.n_obs, seed)
    W = wl.weights(spec.n_obs)

    ctx = vf.Context(0)
    dev = ctx.device
    inst = vf.Instrument.from_spec(ctx, spec)
    stream = torch.cuda.current_stream(dev)
    P_d = torch.tensor(P.astype(np.float32), device=dev)
    obs = vf.synthesize(ctx, inst, P_d, noise=torch.tensor(noise.astype(np.float32), device=dev))
    W_d = torch.tensor(W, device=dev)
    out = dict(params=torch.empty((n, 10), device=dev, dtype=torch.float32),
               chi2=torch.empty(n, device=dev, dtype=torch.float64),
               iters=torch.empty(n, device=dev, dtype=torch.int32),
               status=torch.empty(n, device=dev, dtype=torch.int32))
    opts = vf.Options()

    for _ in range(args.warmup):
        vf.invert(ctx, inst, obs, W_d, opts=opts, out=out)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        vf.invert(ctx, inst, obs, W_d, opts=opts, out=out)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kern_ms = float(np.mean(ev_ms))
    ms_per_step = wall * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3)

    c = ctx.counters()
    st = out["status"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    chi = out["chi2"].cpu().numpy()
    f_trial, f_jac, f_solve = work_model(inst.info["n_active_fine"], inst.info["n_taps"],
                                         spec.n_obs)
    alg_flops = (c["trials"] * (f_trial + f_solve) + (c["pixels"] + c["accepts"]) * f_jac)
    exec_flops = c["passes"] * f_jac + c["trials"] * f_solve
    achieved = alg_flops / (kern_ms * 1e-3) / 1e12

    result = {
        "metric": "inverted pixels/s on 1 MI355X, learned-init LM vs plain LM at matched chi^2",
        "value": round(value, 1),
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "512x512 HMI-shaped pixels (cfg0 priors, seed 1001, noise 1e-3), "
                        "plain LM from the default model, max 50 iterations",
            "init": "default model (plain LM); learned init not yet in this build",
            "pixels": n,
            "n_obs": spec.n_obs,
            "synthesis_points": inst.info["n_active_fine"],
            "filter_taps": inst.info["n_taps"],
            "grid_waves": c["grid_waves"],
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": None,
            "kernel": "lm_kernel",
            "kernel_ms": round(kern_ms, 4),
            "executed_tflops": round(exec_flops / (kern_ms * 1e-3) / 1e12, 3),
        },
        "work": {
            "trials": c["trials"], "accepts": c["accepts"], "passes": c["passes"],
            "svd_fallbacks": c["svd_fallbacks"], "mean_iters": float(it.mean()),
            "status_counts": np.bincount(st, minlength=4).tolist(),
            "chi2_median": float(np.median(chi)),
            "flop_per_trial": f_trial, "flop_per_jacobian_pass": f_jac,
            "flop64_per_solve": f_solve,
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        m = min(args.cpu_sample, n)
        oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
        obs_cpu = (oracle.forward_batch(oi, P[:m]) + noise[:m]).astype(np.float32)
        t1 = time.perf_counter()
        ref = oracle.invert(oi, obs_cpu, W)
        dt = time.perf_counter() - t1
        result["cpu_baseline"] = {
            "value": round(m / dt, 2), "unit": "pixels/s", "cores": ref["threads"],
            "kind": "oracle",
            "sample": "first %d of the %d pixels (same parameters and noise, observations "
                      "synthesised by the FP64 oracle), plain LM, max 50 iterations" % (m, n),
            "seconds": round(dt, 3),
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
