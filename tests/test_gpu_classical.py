"""Classical initial guess on the GPU against the FP64 oracle (Sect. 5:
weak-field B and gamma, linear-polarisation azimuth, line position), for the
HMI-shaped and the fine-spectrum instruments, on oracle-made observations."""
import numpy as np
import pytest
import torch

import oracle
from oracle import classical
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")


@pytest.fixture(scope="module")
def ctx():
    print("[gpu-classical] creating context", flush=True)
    return vf.Context(0)


@pytest.mark.parametrize("which", ["hmi", "fine"])
def test_classical_start_matches_the_oracle(ctx, which):
    spec = wl.hmi_instrument() if which == "hmi" else wl.fine_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 4096 if which == "hmi" else 512
    P = wl.draw_params(n, 61)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 61)).astype(np.float32)
    obs[:8] = oracle.forward_batch(oi, P[:8])  # a few noiseless pixels
    x = classical.sample_offsets(spec.filter, spec.fine_offset_mA)
    cz = oracle.zeeman_constant(spec.lambda0_A, spec.geff)
    ref, pol_ref = classical.classical_init(obs, x, spec.lambda0_A, cz, wl.default_model(),
                                            oracle.project)
    g, pol = vf.init_classical(ctx, inst, torch.tensor(obs, device=ctx.device))
    g, pol = g.cpu().numpy().astype(np.float64), pol.cpu().numpy()
    d = np.abs(g - ref)
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    rel_b = d[:, 0] / np.maximum(ref[:, 0], 1.0)
    print("[gpu-classical] %s: B rel p99.9 %.2e, gamma p99.9 %.2e, psi p99.9 %.2e, v max %.2e"
          % (which, np.quantile(rel_b, 0.999), np.quantile(d[:, 1], 0.999),
             np.quantile(d[:, 2], 0.999), d[:, 3].max()), flush=True)
    assert np.quantile(rel_b, 0.999) < 1e-3 and np.quantile(d[:, 1], 0.999) < 0.02
    assert np.quantile(d[:, 2], 0.999) < 0.02
    assert d[:, 3].max() < 1e-3 and np.max(d[:, 7:9] / ref[:, 7:9]) < 1e-6
    np.testing.assert_array_equal(g[:, [4, 5, 6, 9]], ref[:, [4, 5, 6, 9]].astype(np.float32))
    np.testing.assert_allclose(pol, pol_ref, rtol=1e-4, atol=1e-9)
    # non-finite samples: default model, polarisation level NaN
    bad = obs[:4].copy()
    bad[1, 3, 2] = np.nan
    gb, pb = vf.init_classical(ctx, inst, torch.tensor(bad, device=ctx.device))
    np.testing.assert_array_equal(gb.cpu().numpy()[1], wl.default_model().astype(np.float32))
    assert np.isnan(pb.cpu().numpy()[1]) and np.isfinite(pb.cpu().numpy()[[0, 2, 3]]).all()
