"""Derivatives only after a successful trial (Fig. 6), as a scheduling choice:
with deriv_split > 0 the trials run values-only passes and an accepted model
waits for a derivative pass of its wave.  A model's chi^2 is the same from
either pass, and its Jacobian, J^T W J and gradient the same whichever pass
builds them, so every per-pixel result is the same bits as with the fused
pass (deriv_split 0) for every layout of the pass: the HMI filter's five
register slots, the six-row pass of a wider filter, lane pairs, the banded
fine-spectrum pass, several batches in one launch, per-pixel weights and the
kept Hessian of Sect. 4.4.  The work counters show what changes: the same
trials and accepts, fewer derivative passes (and fewer J^T W J builds: the
fused pass builds one for the accepted trial that ends a fit)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")

SPLITS = (1, 8, 16, 32, 64)


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] split: creating context", flush=True)
    return vf.Context(0)


def _obs(spec, n, seed):
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    P = wl.draw_params(n, seed)
    return (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, seed)).astype(np.float32)


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b, tag):
    for k in ("params", "chi2", "iters", "status"):
        x, y = a[k], b[k]
        eq = (x == y) | (np.isnan(x) & np.isnan(y)) if x.dtype.kind == "f" else x == y
        assert np.all(eq), (tag, k, int(np.sum(~eq)))


CASES = {
    "hmi": dict(spec=lambda: wl.hmi_instrument(), n=6000, rows=5),
    "wide": dict(spec=lambda: wl.hmi_instrument(fwhm_mA=100.0), n=3000, rows=6),
    "pairs": dict(spec=lambda: wl.hmi_instrument(), n=1500, rows=5, opts=dict(lanes_per_pixel=2)),
    "fine": dict(spec=lambda: wl.fine_instrument(), n=1200, rows=4),
    "hess_reuse": dict(spec=lambda: wl.hmi_instrument(), n=3000, rows=5,
                       opts=dict(hess_reuse=2.0)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_split_pass_gives_the_fused_results(ctx, case):
    c = CASES[case]
    spec = c["spec"]()
    inst = vf.Instrument.from_spec(ctx, spec)
    assert inst.info["lm_register_rows"] == c["rows"]
    n = c["n"]
    obs = _obs(spec, n, 71)
    dev = ctx.device
    o = torch.tensor(obs, device=dev)
    W = torch.tensor(wl.weights(spec.n_obs), device=dev)
    kw = c.get("opts", {})
    print("[gpu] split %s: fused" % case, flush=True)
    ref = _np(vf.invert(ctx, inst, o, W, opts=vf.Options(deriv_split=0, **kw)))
    c0 = ctx.counters()
    assert c0["derivative_passes"] == c0["passes"]
    for k in SPLITS:
        out = _np(vf.invert(ctx, inst, o, W, opts=vf.Options(deriv_split=k, **kw)))
        ck = ctx.counters()
        print("[gpu] split %s k=%d: passes %d (derivative %d) vs fused %d" % (
            case, k, ck["passes"], ck["derivative_passes"], c0["passes"]), flush=True)
        _same(ref, out, (case, k))
        for key in ("pixels", "trials", "accepts", "jacobians"):
            assert ck[key] == c0[key], (case, k, key)
        # J^T W J is built once per derivative pass at an accepted model: the
        # fused pass also builds it for the accepted trial that ends a fit
        assert ck["hessians"] <= c0["hessians"], (case, k)
        # fewer derivative passes, never fewer than the Jacobians the fits need
        assert ck["jacobians"] <= ck["derivative_passes"] < c0["derivative_passes"], (case, k)
        # every trial is one pass, every pixel starts with a derivative pass,
        # and an accepted model of a values-only pass needs one more
        assert ck["passes"] >= ck["trials"] + n


def test_split_in_batches_and_with_per_pixel_weights(ctx):
    hspec, fspec = wl.hmi_instrument(), wl.fine_instrument()
    hi, fi = vf.Instrument.from_spec(ctx, hspec), vf.Instrument.from_spec(ctx, fspec)
    dev = ctx.device
    oh = torch.tensor(_obs(hspec, 2000, 72), device=dev)
    of = torch.tensor(_obs(fspec, 600, 73), device=dev)
    rng = np.random.default_rng(74)
    Wh = torch.tensor((wl.weights(6)[None] * rng.uniform(0.5, 1.5, (2000, 4, 6)))
                      .astype(np.float32), device=dev)
    Wf = torch.tensor(wl.weights(fspec.n_obs), device=dev)
    outs = []
    for k in (0, 16):
        print("[gpu] split batches k=%d" % k, flush=True)
        b = vf.invert_batches(ctx, [dict(inst=fi, stokes=of, W=Wf), dict(inst=hi, stokes=oh, W=Wh)],
                              opts=vf.Options(deriv_split=k))
        outs.append([_np(x) for x in b])
    for a, b, tag in zip(outs[0], outs[1], ("fine", "hmi")):
        _same(a, b, tag)
    alone = _np(vf.invert(ctx, hi, oh, Wh, opts=vf.Options(deriv_split=16)))
    _same(alone, outs[1][1], "hmi alone")


def test_autotuner_covers_the_split(ctx):
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    dev = ctx.device
    o = torch.tensor(_obs(spec, 20000, 75), device=dev)
    W = torch.tensor(wl.weights(6), device=dev)
    t = vf.autotune(ctx, inst, o, W, sample=20000)
    print("[gpu] autotune: %s" % t, flush=True)
    assert 0 <= t["deriv_split"] <= 64 and t["best_ms"] <= t["default_ms"] * 1.02
    ref = _np(vf.invert(ctx, inst, o, W, opts=vf.Options(deriv_split=0)))
    out = _np(vf.invert(ctx, inst, o, W))  # the tuned choice
    _same(ref, out, "tuned")
