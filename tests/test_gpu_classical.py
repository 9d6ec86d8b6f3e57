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
    # a buffer that is not 16-byte aligned takes the generic kernel
    flat = torch.zeros(obs.size + 1, device=ctx.device)
    flat[1:] = torch.tensor(obs.ravel(), device=ctx.device)
    gm, pm = vf.init_classical(ctx, inst, flat[1:].view(obs.shape))
    gm = gm.cpu().numpy().astype(np.float64)
    dm = np.abs(gm - g)
    dm[:, 2] = np.minimum(dm[:, 2], 180.0 - dm[:, 2])
    assert np.quantile(dm[:, 0] / np.maximum(g[:, 0], 1.0), 0.999) < 1e-5
    assert np.quantile(dm[:, 1:3], 0.999) < 1e-3 and dm[:, 3].max() < 1e-5
    np.testing.assert_array_equal(pm.cpu().numpy(), pol)
    # non-finite samples: default model, polarisation level NaN
    bad = obs[:4].copy()
    bad[1, 3, 2] = np.nan
    gb, pb = vf.init_classical(ctx, inst, torch.tensor(bad, device=ctx.device))
    np.testing.assert_array_equal(gb.cpu().numpy()[1], wl.default_model().astype(np.float32))
    assert np.isnan(pb.cpu().numpy()[1]) and np.isfinite(pb.cpu().numpy()[[0, 2, 3]]).all()


def test_combined_start_matches_the_oracle(ctx):
    """Network-style base models combined with the classical azimuth and,
    below 6 % polarisation, the classical B and gamma; in place and out of
    place give the same bits."""
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 4096
    P = wl.draw_params(n, 62)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 62)).astype(np.float32)
    obs[5, 0, 1] = np.inf                      # keeps the base model
    obs[6] = -np.abs(obs[6])                   # no continuum: level NaN
    base = wl.draw_params(n, 63).astype(np.float32)
    x = classical.sample_offsets(spec.filter, spec.fine_offset_mA)
    cz = oracle.zeeman_constant(spec.lambda0_A, spec.geff)
    thr = 0.06
    ref, pol_ref = classical.combined_init(obs, base.astype(np.float64), thr, x, spec.lambda0_A,
                                           cz, wl.default_model(), oracle.project)
    dev = ctx.device
    tb = torch.tensor(base, device=dev)
    g, pol = vf.init_combined(ctx, inst, torch.tensor(obs, device=dev), tb, thr)
    g2, _ = vf.init_combined(ctx, inst, torch.tensor(obs, device=dev), tb.clone(), thr,
                             out=None)
    inplace = tb.clone()
    vf.init_combined(ctx, inst, torch.tensor(obs, device=dev), inplace, thr, out=inplace)
    assert torch.equal(g, g2) and torch.equal(g, inplace)
    g, pol = g.cpu().numpy().astype(np.float64), pol.cpu().numpy()
    assert np.isnan(pol[5]) and np.isnan(pol[6])
    # the selection is taken on the GPU's own float32 level; pixels whose
    # FP64 level lies within rounding of the threshold are left out
    low_gpu = pol < thr
    sure = ~np.isclose(pol_ref, thr, rtol=1e-4, atol=0) | np.isnan(pol_ref)
    assert np.array_equal(low_gpu[sure], (pol_ref < thr)[sure])
    assert 0.1 < low_gpu.mean() < 0.9
    d = np.abs(g - ref)[sure]
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    rel_b = d[:, 0] / np.maximum(ref[sure, 0], 1.0)
    print("[gpu-classical] combined: %.3f below threshold; B rel p99.9 %.2e, psi p99.9 %.2e"
          % (low_gpu.mean(), np.quantile(rel_b, 0.999), np.quantile(d[:, 2], 0.999)), flush=True)
    assert np.quantile(rel_b, 0.999) < 1e-3 and np.quantile(d[:, 1], 0.999) < 0.02
    assert np.quantile(d[:, 2], 0.999) < 0.02
    # everything else is the base, bit for bit after the box
    np.testing.assert_array_equal(g[:, 3:], ref[:, 3:].astype(np.float32))
    np.testing.assert_array_equal(g[~low_gpu & sure, :2],
                                  ref[~low_gpu & sure, :2].astype(np.float32))
    np.testing.assert_array_equal(g[5], ref[5].astype(np.float32))
