"""Fine-spectrum path (banded instrument): 112 observed samples at 21.5 mA
seen through a 15-tap Gaussian instrumental profile on a 464-point grid
(the Hinode-like sampling of Sect. 4.1 on the 6302.5 A line of Sect. 3.1),
and several batches in one launch.  GPU results are compared with the FP64
oracle on oracle-made inputs."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")


@pytest.fixture(scope="module")
def ctx():
    print("[gpu-fine] creating context", flush=True)
    return vf.Context(0)


def _pair(ctx, spec):
    return spec, vf.Instrument.from_spec(ctx, spec), oracle.Instrument(
        spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)


@pytest.fixture(scope="module")
def fine(ctx):
    return _pair(ctx, wl.fine_instrument())


@pytest.fixture(scope="module")
def hmi(ctx):
    return _pair(ctx, wl.hmi_instrument())


def _dev(ctx, a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=ctx.device)


def _observations(oi, spec, n, seed):
    P = wl.draw_params(n, seed)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, seed)).astype(np.float32)
    return P, obs


def test_fine_instrument_layout(ctx, fine):
    spec, inst, oi = fine
    info = inst.info
    # rows j use points 4 j + 1 .. 4 j + 15 of the 464-point grid
    assert info["n_taps"] == 112 * 15
    assert info["n_active_fine"] == 4 * 111 + 15
    assert abs(info["cz_mA_per_G"] - 4.66685e-10 * 2.5 * 6302.4936 ** 2) < 1e-9
    # a filter that is neither 6 rows nor banded is refused
    bad = spec.filter.copy()
    bad[50, :] = 0.0
    bad[50, 100:130] = 1.0 / 30.0
    with pytest.raises(Exception):
        vf.Instrument(ctx, spec.lambda0_A, spec.geff, spec.fine_offset_mA, bad)


def test_fine_synthesis_parity(ctx, fine):
    spec, inst, oi = fine
    P = wl.draw_params(768, 15).astype(np.float32)
    P[:32, 0] = 0.0
    P[32:64, 9] = 0.0
    print("[gpu-fine] synthesis parity on %d models" % len(P), flush=True)
    S, J = vf.synthesize(ctx, inst, _dev(ctx, P), jac=True)
    S, J = S.cpu().numpy(), J.cpu().numpy()
    assert S.shape == (768, 4, 112) and J.shape == (768, 4, 112, 10)
    Pd = P.astype(np.float64)
    Sr = np.empty(S.shape)
    Jr = np.empty(J.shape)
    for k in range(len(P)):
        Sr[k], Jr[k] = oracle.forward(oi, Pd[k], jac=True)
    assert np.max(np.abs(S - Sr)) < 2e-6
    assert np.all(S[:32, 1:] == 0.0) and np.all(S[32:64, 1:] == 0.0)
    colmax = np.abs(Jr).max(axis=(1, 2), keepdims=True)
    typical = np.median(np.abs(Jr[64:]).max(axis=(1, 2)), axis=0)
    tol = 2e-4 * colmax + 3e-5 * typical
    bad = np.abs(J - Jr) > tol
    assert not bad.any(), "Jacobian outside tolerance at %s" % (np.argwhere(bad)[:5],)


def test_fine_first_iterations_follow_the_oracle(ctx, fine):
    """max_iter = 0 evaluates chi^2 (438 degrees of freedom) at the start;
    one step reproduces the oracle's damped step on most pixels."""
    spec, inst, oi = fine
    P, obs = _observations(oi, spec, 128, 16)
    W = wl.weights(spec.n_obs)
    out0 = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), opts=vf.Options(max_iter=0))
    ref0 = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=0))
    np.testing.assert_allclose(out0["chi2"].cpu().numpy(), ref0["chi2"], rtol=2e-4)
    out1 = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), opts=vf.Options(max_iter=1))
    ref1 = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=1))
    gp, rp = out1["params"].cpu().numpy(), ref1["params"]
    scale = np.array([1500, 90, 90, 3, 35, 0.25, 15, 0.3, 0.7, 0.6])
    close = (np.abs(gp - rp) / scale < 1e-3).all(axis=1)
    assert close.mean() > 0.9, close.mean()
    np.testing.assert_array_equal(out1["iters"].cpu().numpy(), ref1["iters"])


def test_fine_default_start_statistics(ctx, fine):
    spec, inst, oi = fine
    n = 256
    P, obs = _observations(oi, spec, n, 17)
    W = wl.weights(spec.n_obs)
    out = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W))
    ref = oracle.invert(oi, obs, W)
    gc, gi = out["chi2"].cpu().numpy(), out["iters"].cpu().numpy()
    a, b = np.median(gc), np.median(ref["chi2"])
    print("[gpu-fine] median chi2 %.4f vs %.4f, iters %.2f vs %.2f"
          % (a, b, gi.mean(), ref["iters"].mean()), flush=True)
    assert abs(a - b) / b < 0.05, (a, b)
    assert abs(np.mean(gc < 1.5) - np.mean(ref["chi2"] < 1.5)) < 0.06
    assert abs(gi.mean() - ref["iters"].mean()) / ref["iters"].mean() < 0.12
    c = ctx.counters()
    assert c["pixels"] == n and c["trials"] == gi.sum() and 0 <= c["passes"] - c["trials"] - n <= c["accepts"]


def test_batches_equal_separate_launches(ctx, fine, hmi):
    fs, finst, foi = fine
    hs, hinst, hoi = hmi
    _, fobs = _observations(foi, fs, 300, 18)
    _, hobs = _observations(hoi, hs, 2000, 19)
    fW, hW = _dev(ctx, wl.weights(fs.n_obs)), _dev(ctx, wl.weights(hs.n_obs))
    fo, ho = _dev(ctx, fobs), _dev(ctx, hobs)
    ref_f = {k: v.cpu().numpy() for k, v in vf.invert(ctx, finst, fo, fW).items()}
    ref_h = {k: v.cpu().numpy() for k, v in vf.invert(ctx, hinst, ho, hW).items()}
    empty = torch.empty((0, 4, 6), device=ctx.device)
    for order in (("f", "h"), ("h", "f"), ("f", "e", "h")):
        bs = []
        for o in order:
            if o == "f":
                bs.append(dict(inst=finst, stokes=fo, W=fW))
            elif o == "h":
                bs.append(dict(inst=hinst, stokes=ho, W=hW))
            else:
                bs.append(dict(inst=hinst, stokes=empty, W=hW))
        outs = vf.invert_batches(ctx, bs)
        c = ctx.counters()
        assert c["pixels"] == 2300, (order, c)
        for o, out in zip(order, outs):
            ref = ref_f if o == "f" else ref_h if o == "h" else None
            if ref is None:
                continue
            for k in ref:
                assert np.array_equal(out[k].cpu().numpy(), ref[k]), (order, o, k)
