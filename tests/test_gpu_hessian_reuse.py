"""Hessian reuse near the minimum (Sect. 4.4, Fig. 6) on the GPU against the
FP64 oracle: an accepted step from a model whose chi^2 is below
Options.hess_reuse keeps the previous J^T W J and rebuilds only the
gradient."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")

BIG = 1e300


@pytest.fixture(scope="module")
def setup():
    print("[gpu-hess] creating context", flush=True)
    ctx = vf.Context(0)
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 1024
    P = wl.draw_params(n, 71)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 71)).astype(np.float32)
    W = wl.weights(spec.n_obs)
    dev = ctx.device
    return ctx, inst, oi, P, obs, W, torch.tensor(obs, device=dev), torch.tensor(W, device=dev)


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_untriggered_reuse_changes_nothing(setup):
    ctx, inst, oi, P, obs, W, to, tW = setup
    a = _np(vf.invert(ctx, inst, to, tW))
    ca = ctx.counters()
    b = _np(vf.invert(ctx, inst, to, tW, opts=vf.Options(hess_reuse=1e-30)))
    cb = ctx.counters()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # every start and every accepted model that does not end its fit builds
    # its Hessian (a derivative pass that tried a trial ahead also builds it
    # for an accepted trial that ends the fit); the fused pass builds one for
    # every start and every accepted trial
    assert ca["jacobians"] <= ca["hessians"] == cb["hessians"] <= ca["pixels"] + ca["accepts"]
    f = _np(vf.invert(ctx, inst, to, tW, opts=vf.Options(deriv_split=0)))
    cf = ctx.counters()
    assert np.array_equal(f["chi2"], a["chi2"])
    assert cf["hessians"] == cf["pixels"] + cf["accepts"]


def test_counts_with_reuse_everywhere(setup):
    """Above every chi^2 only the starts (and, in the fixed-iteration
    scheme, the restarts) build a Hessian."""
    ctx, inst, oi, P, obs, W, to, tW = setup
    vf.invert(ctx, inst, to, tW, opts=vf.Options(hess_reuse=BIG))
    c = ctx.counters()
    assert c["hessians"] == c["pixels"] == len(P) and c["accepts"] > 0
    out = _np(vf.invert(ctx, inst, to, tW,
                        opts=vf.Options(hess_reuse=BIG, fixed_iters=30, restarts=2,
                                        restart_seed=4)))
    c = ctx.counters()
    assert c["hessians"] == len(P) + int((out["status"] >> 8).sum())


def test_linear_model_reuse_is_exact(setup):
    """Only S0 and S1 free: the profiles are linear in them, J^T W J never
    changes, and keeping it gives the plain fit bit for bit; both agree with
    the oracle's least-squares minimum."""
    ctx, inst, oi, P, obs, W, to, tW = setup
    mask = (1 << 7) | (1 << 8)
    init = P.copy()
    init[:, 7:9] = [0.45, 0.3]
    ti = torch.tensor(init.astype(np.float32), device=ctx.device)
    a = _np(vf.invert(ctx, inst, to, tW, init=ti, opts=vf.Options(free_mask=mask)))
    b = _np(vf.invert(ctx, inst, to, tW, init=ti,
                      opts=vf.Options(free_mask=mask, hess_reuse=BIG)))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ref = oracle.invert(oi, obs, W, init=init.astype(np.float32).astype(np.float64),
                        opts=oracle.Options(free_mask=mask, hess_reuse=BIG))
    rel = np.abs(b["chi2"] - ref["chi2"]) / ref["chi2"]
    print("[gpu-hess] linear: chi2 rel median %.2e p99 %.2e" % (np.median(rel),
                                                               np.quantile(rel, 0.99)), flush=True)
    assert np.quantile(rel, 0.99) < 2e-4
    np.testing.assert_allclose(b["params"][:, 7:9], ref["params"][:, 7:9], rtol=0, atol=2e-4)


def test_first_steps_with_a_kept_hessian(setup):
    """Three trials from the default start with the first Hessian kept:
    the GPU takes the oracle's steps (start H, fresh gradients)."""
    ctx, inst, oi, P, obs, W, to, tW = setup
    opts = dict(max_iter=3, hess_reuse=BIG)
    out = _np(vf.invert(ctx, inst, to, tW, opts=vf.Options(**opts)))
    ref = oracle.invert(oi, obs, W, opts=oracle.Options(**opts))
    same = np.isclose(out["params"][:, 0], ref["params"][:, 0], rtol=1e-3, atol=0.5)
    print("[gpu-hess] 3 kept-H steps: %.3f of pixels on the oracle's path" % same.mean(),
          flush=True)
    assert same.mean() > 0.9
    np.testing.assert_allclose(out["params"][same][:, [0, 3, 6, 9]],
                               ref["params"][same][:, [0, 3, 6, 9]], rtol=5e-3, atol=2e-3)


def test_reuse_statistics_match_the_oracle(setup):
    """From the default start with reuse below chi^2 = 2 (the noise level is
    1): the GPU and the oracle reach statistically the same fits with the
    same share of kept Hessians."""
    ctx, inst, oi, P, obs, W, to, tW = setup
    out = _np(vf.invert(ctx, inst, to, tW, opts=vf.Options(hess_reuse=2.0)))
    c = ctx.counters()
    ref = oracle.invert(oi, obs, W, opts=oracle.Options(hess_reuse=2.0))
    a, b = np.median(out["chi2"]), np.median(ref["chi2"])
    ia, ib = out["iters"].mean(), ref["iters"].mean()
    kept_g = 1.0 - c["hessians"] / (c["pixels"] + c["accepts"])
    rc = ref["counters"]
    kept_r = 1.0 - rc["hessians"] / rc["derivs"]
    print("[gpu-hess] tau 2: median chi2 %.4f / %.4f, iters %.2f / %.2f, kept %.3f / %.3f"
          % (a, b, ia, ib, kept_g, kept_r), flush=True)
    assert abs(a - b) / b < 0.05
    assert abs(ia - ib) / ib < 0.1
    assert kept_r > 0.05 and abs(kept_g - kept_r) < 0.05


@pytest.fixture(scope="module")
def fine_setup(setup):
    ctx = setup[0]
    spec = wl.fine_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 192
    P = wl.draw_params(n, 73)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 73)).astype(np.float32)
    W = wl.weights(spec.n_obs)
    dev = ctx.device
    return ctx, inst, oi, P, obs, W, torch.tensor(obs, device=dev), torch.tensor(W, device=dev)


def test_banded_reuse_linear_model_and_first_steps(fine_setup):
    """The banded layout accumulates g alone when the Hessian is kept: with
    only S0 and S1 free the kept Hessian gives the plain fit bit for bit and
    the oracle's minimum; three trials with the start's Hessian follow the
    oracle's path."""
    ctx, inst, oi, P, obs, W, to, tW = fine_setup
    print("[gpu-hess] banded layout, %d pixels" % len(P), flush=True)
    mask = (1 << 7) | (1 << 8)
    init = P.copy()
    init[:, 7:9] = [0.45, 0.3]
    ti = torch.tensor(init.astype(np.float32), device=ctx.device)
    a = _np(vf.invert(ctx, inst, to, tW, init=ti, opts=vf.Options(free_mask=mask)))
    b = _np(vf.invert(ctx, inst, to, tW, init=ti,
                      opts=vf.Options(free_mask=mask, hess_reuse=BIG)))
    c = ctx.counters()
    assert c["hessians"] == c["pixels"] == len(P) and c["accepts"] > 0
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ref = oracle.invert(oi, obs, W, init=init.astype(np.float32).astype(np.float64),
                        opts=oracle.Options(free_mask=mask, hess_reuse=BIG))
    rel = np.abs(b["chi2"] - ref["chi2"]) / ref["chi2"]
    assert np.quantile(rel, 0.99) < 2e-4
    np.testing.assert_allclose(b["params"][:, 7:9], ref["params"][:, 7:9], rtol=0, atol=2e-4)
    opts = dict(max_iter=3, hess_reuse=BIG)
    out = _np(vf.invert(ctx, inst, to, tW, opts=vf.Options(**opts)))
    ref = oracle.invert(oi, obs, W, opts=oracle.Options(**opts))
    same = np.isclose(out["params"][:, 0], ref["params"][:, 0], rtol=1e-3, atol=0.5)
    print("[gpu-hess] banded, 3 kept-H steps: %.3f on the oracle's path" % same.mean(),
          flush=True)
    assert same.mean() > 0.9
