"""Non-finite observations and weights (a NaN, +inf or -inf sample, an
infinite or NaN per-pixel weight): the pixel is not fitted -- parameters and
chi^2 NaN, no iterations, status NONFINITE -- and costs no counted work.

The library finds such pixels from the non-finite chi^2 of their first pass
and only then reads their inputs, so these tests check that the outcome is
the one of a check made before any work: every other pixel's result equals
its result in the same batch without the bad pixels, bit for bit, and the
work counters equal that batch's, plus the bad pixels in `pixels`; for the
fused pass, the dense and banded layouts, lane pairs and several batches in
one launch."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")

WORK = ("trials", "accepts", "jacobians")


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] nonfinite: creating context", flush=True)
    return vf.Context(0)


def _obs(spec, n, seed):
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    P = wl.draw_params(n, seed)
    return (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, seed)).astype(np.float32)


def _spoil(obs, W):
    """Bad inputs at fixed pixels: returns their indices."""
    obs[5, 0, 1] = np.nan
    obs[17, 2, obs.shape[2] - 1] = np.inf
    obs[40, 1, 0] = -np.inf
    W[61, 3, 2] = np.inf
    W[77, 0, 0] = np.nan
    return np.array([5, 17, 40, 61, 77])


def _run(ctx, inst, obs, W, **kw):
    dev = ctx.device
    out = vf.invert(ctx, inst, torch.tensor(obs, device=dev), torch.tensor(W, device=dev),
                    opts=vf.Options(**kw))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, ctx.counters()


CASES = {
    "hmi_fused": dict(spec=wl.hmi_instrument, n=3000, opts=dict(deriv_split=0)),
    "hmi_split": dict(spec=wl.hmi_instrument, n=3000, opts=dict(deriv_split=8)),
    "hmi_pairs": dict(spec=wl.hmi_instrument, n=1000, opts=dict(lanes_per_pixel=2, deriv_split=0)),
    "fine_fused": dict(spec=wl.fine_instrument, n=400, opts=dict(deriv_split=0)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_bad_inputs_are_not_fitted_and_cost_nothing(ctx, case):
    c = CASES[case]
    spec = c["spec"]()
    inst = vf.Instrument.from_spec(ctx, spec)
    n = c["n"]
    obs = _obs(spec, n, 91)
    W = np.ascontiguousarray(np.broadcast_to(wl.weights(spec.n_obs), (n, 4, spec.n_obs)))
    bad = _spoil(obs, W)
    good = np.setdiff1d(np.arange(n), bad)
    print("[gpu] nonfinite %s: batch with bad pixels" % case, flush=True)
    out, cnt = _run(ctx, inst, obs, W, **c["opts"])
    print("[gpu] nonfinite %s: clean batch" % case, flush=True)
    ref, cref = _run(ctx, inst, obs[good], W[good], **c["opts"])
    assert np.all(out["status"][bad] == vf.NONFINITE)
    assert np.all(np.isnan(out["params"][bad])) and np.all(np.isnan(out["chi2"][bad]))
    assert np.all(out["iters"][bad] == 0)
    for k in ("params", "chi2", "iters", "status"):
        assert np.array_equal(out[k][good], ref[k]), (case, k)
    assert cnt["pixels"] == cref["pixels"] + len(bad)
    for k in WORK:
        assert cnt[k] == cref[k], (case, k)
    # fused: one pass per trial and start, J^T W J at every start and accepted
    # trial (with the split pass these depend on which lanes share a wave)
    if c["opts"].get("deriv_split") == 0:
        for k in ("passes", "derivative_passes", "hessians"):
            assert cnt[k] == cref[k], (case, k)


def test_bad_inputs_in_batches(ctx):
    hspec, fspec = wl.hmi_instrument(), wl.fine_instrument()
    hi, fi = vf.Instrument.from_spec(ctx, hspec), vf.Instrument.from_spec(ctx, fspec)
    dev = ctx.device
    oh, of = _obs(hspec, 1200, 92), _obs(fspec, 300, 93)
    Wh = np.ascontiguousarray(np.broadcast_to(wl.weights(6), (1200, 4, 6)))
    Wf = np.ascontiguousarray(np.broadcast_to(wl.weights(fspec.n_obs), (300, 4, fspec.n_obs)))
    bh, bf = _spoil(oh, Wh), _spoil(of, Wf)
    print("[gpu] nonfinite batches", flush=True)
    outs = vf.invert_batches(ctx, [dict(inst=fi, stokes=torch.tensor(of, device=dev),
                                        W=torch.tensor(Wf, device=dev)),
                                   dict(inst=hi, stokes=torch.tensor(oh, device=dev),
                                        W=torch.tensor(Wh, device=dev))],
                             opts=vf.Options(deriv_split=0))
    torch.cuda.synchronize()
    for out, bad, n in ((outs[0], bf, 300), (outs[1], bh, 1200)):
        st = out["status"].cpu().numpy()
        assert np.all(st[bad] == vf.NONFINITE)
        assert np.all(np.isnan(out["params"].cpu().numpy()[bad]))
        assert np.all(out["iters"].cpu().numpy()[bad] == 0)
        good = np.setdiff1d(np.arange(n), bad)
        assert np.all((st[good] & 15) <= 2)
