"""Per-parameter parity with the FP64 oracle at the library's default options
on the 512 x 512 HMI set (262,144 pixels, seed 1001; Sect. 2 Eq. 1 and the
LM of Sect. 4.2), in the launch configuration of a whole-batch inversion.

The GPU inverts all 262,144 pixels from the default model; the oracle
inverts every 32nd of them (8,192) from the same float32 observations (which
the oracle synthesises), weights and start.  LM stops where the relative
chi^2 decrease falls below 1e-5, so two correct fits of one pixel may stop at
different points of the same valley; the bar is therefore stated on the
pixels that both sides fitted to convergence, and on those of them that
reached the same minimum (chi^2 within 1e-4 relative):

* chi^2 within 1e-4 relative for at least 97% of the pixels converged on
  both sides;
* on the same-minimum pixels, B within 1 G, v within 1 m/s, and (where the
  oracle's B exceeds 50 G; the angles are undetermined without a field)
  gamma and psi within 0.1 deg, each for at least 98.5% of the pixels.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")

STRIDE = 32


def test_default_options_per_parameter_parity():
    ctx = vf.Context(0)
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    n = wl.CONFIGS["hmi_512x512"]["n"]
    seed = wl.CONFIGS["hmi_512x512"]["seed"]
    assert n == 262144
    P = wl.draw_params(n, seed)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    print("[gpu] product parity: oracle synthesis of %d pixels" % n, flush=True)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, 6, seed)).astype(np.float32)
    W = wl.weights(6)
    dev = ctx.device
    print("[gpu] product parity: GPU inversion", flush=True)
    out = vf.invert(ctx, inst, torch.tensor(obs, device=dev), torch.tensor(W, device=dev))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy()[::STRIDE] for k, v in out.items()}
    print("[gpu] product parity: oracle inversion of %d pixels" % (n // STRIDE), flush=True)
    ref = oracle.invert(oi, obs[::STRIDE], W)
    both = ((g["status"] & 15) == 0) & (ref["status"] == 0)
    dchi = np.abs(g["chi2"] - ref["chi2"]) / ref["chi2"]
    same = both & (dchi < 1e-4)
    frac_chi = float(np.mean(dchi[both] < 1e-4))
    d = np.abs(g["params"].astype(np.float64) - ref["params"])
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    field = ref["params"][:, 0] > 50.0
    fr = {"B": np.mean(d[same, 0] < 1.0), "v": np.mean(d[same, 3] < 1e-3),
          "gamma": np.mean(d[same & field, 1] < 0.1), "psi": np.mean(d[same & field, 2] < 0.1)}
    print("[gpu] product parity: converged both %.3f, same minimum %.3f, chi2 within 1e-4 %.4f; "
          "within tolerance B %.4f gamma %.4f psi %.4f v %.4f"
          % (both.mean(), same.mean(), frac_chi, fr["B"], fr["gamma"], fr["psi"], fr["v"]),
          flush=True)
    assert both.sum() > 1000
    assert frac_chi >= 0.97
    for k, f in fr.items():
        assert f >= 0.985, k
    # every output of the whole batch is finite and inside the box
    p = out["params"].cpu().numpy()
    assert np.all(np.isfinite(p))
    assert np.all((p[:, 0] >= 0) & (p[:, 0] <= 5000) & (p[:, 9] >= 0) & (p[:, 9] <= 1))
