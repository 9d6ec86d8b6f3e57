"""Graph capture of the inversion: the launches of vfisv_invert and of the
learned path (network, short LM, selection, refit, merge) are stream-ordered
kernels with no allocation, memset node or host synchronisation once the
scratch has grown, so they can be captured in a HIP graph and replayed.
Each replay is checked bit for bit against the eager call, with eager work
and synchronisations between replays."""
import numpy as np
import pytest
import torch

import workloads as wl

vf = pytest.importorskip("paper_0901_2702_amd")
from paper_0901_2702_amd import learned  # noqa: E402


@pytest.fixture(scope="module")
def setup():
    ctx = vf.Context(0)
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    n = 6000
    P = wl.draw_params(n, 81)
    noise = wl.draw_noise(n, spec.n_obs, 81)
    dev = ctx.device
    obs = vf.synthesize(ctx, inst, torch.tensor(P.astype(np.float32), device=dev),
                        noise=torch.tensor(noise.astype(np.float32), device=dev))
    W = torch.tensor(wl.weights(spec.n_obs), device=dev)
    return ctx, inst, obs, W


def _alloc(n, dev):
    return dict(params=torch.empty((n, 10), device=dev, dtype=torch.float32),
                chi2=torch.empty(n, device=dev, dtype=torch.float64),
                iters=torch.empty(n, device=dev, dtype=torch.int32),
                status=torch.empty(n, device=dev, dtype=torch.int32))


def _check_replays(fn, out, ref, replays=3):
    fn()  # warm-up: grows any library scratch outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for r in range(replays):
        for v in out.values():
            v.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (r, k)


@pytest.mark.gpu
def test_plain_inversion_replays_exactly(setup):
    ctx, inst, obs, W = setup
    n = obs.shape[0]
    ref = vf.invert(ctx, inst, obs, W)
    torch.cuda.synchronize()
    out = _alloc(n, ctx.device)
    _check_replays(lambda: vf.invert(ctx, inst, obs, W, out=out), out, ref)


@pytest.mark.gpu
def test_learned_inversion_replays_exactly(setup):
    ctx, inst, obs, W = setup
    n = obs.shape[0]
    x = obs.view(n, -1)
    mean = x.mean(dim=0).cpu().numpy()
    std = x.std(dim=0).clamp_min(1e-6).cpu().numpy()
    # an untrained network: poor starts, so the refit launch has work
    net = learned.Mlp(ctx, x.shape[1], mean, std, np.zeros(7), np.ones(7), seed=5)
    ref = learned.invert_learned(ctx, inst, net, x, W)
    torch.cuda.synchronize()
    assert int(((ref["status"] & vf.FALLBACK_USED) != 0).sum()) > 0
    out = _alloc(n, ctx.device)
    _check_replays(lambda: learned.invert_learned(ctx, inst, net, x, W, out=out), out, ref)
