"""The full-disk configuration at its real size (13,176,792 pixels, clustered
quiet/active regions) in the launch configuration the benchmark times.

The whole disk is synthesised on the device; a seeded sample of 600 pixels
(300 quiet, 300 active) instead gets observations synthesised by the FP64
oracle, so that for those pixels the oracle and the GPU see identical float32
inputs.  Checked: properties that hold at any size (status and iteration
ranges, the box, work counters, the exact iteration histogram), the GPU's
chi^2 re-evaluated by the oracle at the GPU's own result, and the oracle's
own inversion of the sample (statistically, per class)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

vf = pytest.importorskip("paper_0901_2702_amd")

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[full-disk] " + msg, file=sys.stderr, flush=True)


def test_full_disk_plain_lm():
    ctx = vf.Context(0)
    dev = ctx.device
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    seed = wl.CONFIGS["full_disk"]["seed"]
    P, active, mask = wl.full_disk(seed=seed)
    n = P.shape[0]
    assert n == 13_176_792
    _say("generated %d pixels, %.4f active" % (n, active.mean()))
    noise = wl.draw_noise(n, spec.n_obs, seed).astype(np.float32)
    obs = vf.synthesize(ctx, inst, torch.tensor(P.astype(np.float32), device=dev),
                        noise=torch.tensor(noise, device=dev))
    rng = np.random.default_rng(4242)
    smp = np.sort(np.concatenate([rng.choice(np.flatnonzero(~active), 300, replace=False),
                                  rng.choice(np.flatnonzero(active), 300, replace=False)]))
    obs_s = (oracle.forward_batch(oi, P[smp]) + noise[smp].astype(np.float64)).astype(np.float32)
    obs[torch.tensor(smp, device=dev)] = torch.tensor(obs_s, device=dev)
    W = wl.weights(spec.n_obs)
    _say("inverting")
    out = vf.invert(ctx, inst, obs, torch.tensor(W, device=dev))
    c = ctx.counters()
    _say("counters %s" % c)

    # ---- properties at full size -------------------------------------------
    st = out["status"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    params = out["params"].cpu().numpy()
    chi2 = out["chi2"].cpu().numpy()
    assert np.isin(st, (0, 1, 2)).all()
    assert iters.min() >= 1 and iters.max() <= 50
    assert np.isfinite(params).all() and np.isfinite(chi2).all() and (chi2 >= 0).all()
    assert c["pixels"] == n and c["trials"] == int(iters.sum())
    assert 0 <= c["passes"] - c["trials"] - n <= c["accepts"]
    assert np.array_equal(vf.iter_histogram(ctx, out["iters"], 51),
                          np.bincount(iters, minlength=51))
    assert (params[:, 0] >= 0).all() and (params[:, 0] <= 5000).all()
    assert (params[:, 1] >= 0).all() and (params[:, 1] <= 180).all()
    assert (params[:, 2] >= 0).all() and (params[:, 2] <= 180).all()  # 180 == 0
    assert (params[:, 9] >= 0).all() and (params[:, 9] <= 1).all()

    # ---- the sample: chi^2 of the GPU's result, evaluated by the oracle --------
    gp, gc = params[smp].astype(np.float64), chi2[smp]
    ev = oracle.invert(oi, obs_s, W, init=gp, opts=oracle.Options(max_iter=0))
    rel = np.abs(gc - ev["chi2"]) / ev["chi2"]
    assert np.median(rel) < 2e-5 and rel.max() < 1e-3, (np.median(rel), rel.max())

    # ---- the sample: the oracle's own inversion from the default start --------
    ref = oracle.invert(oi, obs_s, W)
    for name, cls in (("quiet", ~active[smp]), ("active", active[smp])):
        a, b = np.median(gc[cls]), np.median(ref["chi2"][cls])
        _say("%s: median chi2 gpu %.4f oracle %.4f; mean iters gpu(sample) %.2f "
             "oracle %.2f gpu(all %s) %.2f" % (name, a, b, iters[smp][cls].mean(),
                                               ref["iters"][cls].mean(), name,
                                               iters[active if name == "active" else ~active]
                                               .mean()))
        assert abs(a - b) / b < 0.1, (name, a, b)
        assert abs(np.mean(gc[cls] < 2.0) - np.mean(ref["chi2"][cls] < 2.0)) < 0.08, name
        ia, ib = iters[smp][cls].mean(), ref["iters"][cls].mean()
        assert abs(ia - ib) / ib < 0.12, (name, ia, ib)
        # the sample is representative of its class over the whole disk
        ic = iters[active if name == "active" else ~active].mean()
        assert abs(ia - ic) / ic < 0.12, (name, ia, ic)
