"""Per-pixel Stokes weights (Sect. 4.3, Eqs. 14-15) on the GPU against the
FP64 oracle, for the six-sample and the fine-spectrum layouts, and an
inversion that takes them."""
import numpy as np
import pytest
import torch

import oracle
from oracle import weights
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")


@pytest.fixture(scope="module")
def ctx():
    print("[gpu-weights] creating context", flush=True)
    return vf.Context(0)


@pytest.mark.parametrize("which", ["hmi", "fine"])
def test_weights_match_the_oracle(ctx, which):
    spec = wl.hmi_instrument() if which == "hmi" else wl.fine_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    n = 3000
    rng = np.random.default_rng(91)
    obs = rng.normal(0.0, 1e-3, (n, 4, spec.n_obs)).astype(np.float32)
    # continua from umbra to brighter than the quiet Sun
    obs[:, 0, :] += rng.uniform(0.1, 1.2, (n, 1)).astype(np.float32)
    mu = rng.uniform(-0.3, 1.3, n).astype(np.float32)   # clamped outside [0, 1]
    mu[7] = np.nan
    obs[8, 0, 3] = np.inf
    sigma = [1e-3, 2e-3, 2e-3, 3e-3]
    # the library takes sigma as float32
    sig32 = np.asarray(sigma, np.float32).astype(np.float64)
    ref = weights.stokes_weights(obs, np.clip(mu.astype(np.float64), 0.0, 1.0), sig32)
    dev = ctx.device
    W = vf.stokes_weights(ctx, inst, torch.tensor(obs, device=dev), torch.tensor(mu, device=dev),
                          sigma).cpu().numpy()
    assert W.shape == (n, 4, spec.n_obs)
    bad = np.zeros(n, bool)
    bad[[7, 8]] = True
    assert np.isnan(W[bad, 0]).all() and np.isfinite(W[~bad]).all()
    np.testing.assert_allclose(W[~bad], ref[~bad], rtol=2e-7, atol=0)
    np.testing.assert_array_equal(W[bad, 1:], ref[bad, 1:].astype(np.float32))
    # an unaligned output buffer takes the generic kernel, same values
    flat = torch.empty(W.size + 1, device=dev)
    vf.stokes_weights(ctx, inst, torch.tensor(obs, device=dev), torch.tensor(mu, device=dev),
                      sigma, out=flat[1:].view(W.shape))
    np.testing.assert_array_equal(flat[1:].view(W.shape).cpu().numpy()[~bad], W[~bad])


def test_inversion_with_eq14_weights(ctx):
    """The weights go straight into the inversion as per-pixel W: the GPU's
    chi^2 at its result, re-evaluated by the oracle with the oracle's
    weights, agrees; a NaN weight reports a non-finite chi^2."""
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 512
    P = wl.draw_params(n, 92)
    P[:, 7:9] *= np.linspace(0.2, 1.0, n)[:, None]  # spots to quiet Sun
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 92)).astype(np.float32)
    mu = np.linspace(0.05, 1.0, n).astype(np.float32)
    mu[3] = np.nan
    dev = ctx.device
    to = torch.tensor(obs, device=dev)
    W = vf.stokes_weights(ctx, inst, to, torch.tensor(mu, device=dev))
    out = vf.invert(ctx, inst, to, W)
    st = out["status"].cpu().numpy()
    assert st[3] == oracle.NONFINITE
    ok = np.arange(n) != 3
    Wr = weights.stokes_weights(obs, mu.astype(np.float64), [1e-3] * 4).astype(np.float32)
    gp = out["params"].cpu().numpy().astype(np.float64)
    ev = oracle.invert(oi, obs[ok], Wr[ok], init=gp[ok], opts=oracle.Options(max_iter=0))
    rel = np.abs(out["chi2"].cpu().numpy()[ok] - ev["chi2"]) / ev["chi2"]
    print("[gpu-weights] chi2 re-evaluated: median rel %.2e, max %.2e"
          % (np.median(rel), rel.max()), flush=True)
    assert np.median(rel) < 2e-5 and rel.max() < 1e-3
