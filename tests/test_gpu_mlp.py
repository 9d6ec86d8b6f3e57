"""GPU parity of the learned initialiser (bfloat16 MFMA network) against the
FP64 numpy oracle with bfloat16 emulation, and its training / inversion
behaviour."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")
from paper_0901_2702_amd import learned  # noqa: E402

H = 256


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return vf.Context(0)


def _unpack(flat, n_in):
    K0 = (n_in + 31) // 32 * 32
    shapes = [(K0, H), (H,), (H, H), (H,), (H, H), (H,), (H, 32), (32,)]
    out, off = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(flat[off:off + k].reshape(sh).astype(np.float64))
        off += k
    assert off == flat.size
    P = {"W1": out[0][:n_in], "b1": out[1], "W2": out[2], "b2": out[3], "W3": out[4],
         "b3": out[5], "W4": out[6][:, :10], "b4": out[7][:10]}
    return P


def _random_net(ctx, n_in, seed):
    rng = np.random.default_rng(seed)
    in_mean = rng.normal(size=n_in) * 0.1
    in_std = rng.uniform(0.5, 2.0, n_in)
    net = learned.Mlp(ctx, n_in, in_mean, in_std, np.zeros(7), np.ones(7), seed=seed)
    flat = net.get_params()
    flat = flat + (rng.normal(size=flat.size) * 0.02).astype(np.float32)
    # keep padding rows/columns zero
    P = _unpack(flat, n_in)
    K0 = (n_in + 31) // 32 * 32
    W1 = np.zeros((K0, H)); W1[:n_in] = P["W1"]
    W4 = np.zeros((H, 32)); W4[:, :10] = P["W4"]
    b4 = np.zeros(32); b4[:10] = P["b4"]
    flat = np.concatenate([W1.ravel(), P["b1"], P["W2"].ravel(), P["b2"], P["W3"].ravel(),
                           P["b3"], W4.ravel(), b4]).astype(np.float32)
    net.set_params(flat)
    return net, flat, in_mean, in_std


def _abs_forward(P, cache):
    """|a3| |W4| + |b4| with the oracle's bfloat16 activations and weights:
    the sum of the magnitudes that make up each output, the scale of one
    bfloat16 rounding step taken differently by the two sides."""
    return np.abs(cache["a3"]) @ np.abs(omlp.to_bf16(P["W4"])) + np.abs(P["b4"])


def _abs_backward(P, cache, t):
    """The backward pass of the oracle with every factor replaced by its
    magnitude: for each gradient element, the sum of the magnitudes of the
    products that make it up (through every upstream path)."""
    r = omlp.to_bf16
    y = cache["y"]
    B, n_out = y.shape
    dz = np.abs(r(2.0 * (y - t) / (B * n_out)))
    G = {"W4": np.abs(cache["a3"]).T @ dz, "b4": dz.sum(axis=0)}
    da = dz @ np.abs(r(P["W4"])).T
    for l in (3, 2, 1):
        dz = da * np.abs(omlp.gelu_grad(cache["z%d" % l]))
        G["W%d" % l] = np.abs(cache["a%d" % (l - 1)]).T @ dz
        G["b%d" % l] = dz.sum(axis=0)
        if l > 1:
            da = dz @ np.abs(r(P["W%d" % l])).T
    return G


# A bfloat16 value holds 8 significant bits: where a pre-activation computed
# by the GPU (float32 MFMA sums) and by the oracle (float64) straddles a
# rounding midpoint, the two sides store activations one bfloat16 step
# (<= 2^-7 relative) apart.  Every output and gradient element is a sum of
# products of such values, so its difference is at most one such step of the
# sum of the magnitudes of its products (_abs_forward / _abs_backward) when
# every term differs by a step; such differences are rare (a pre-activation
# must fall within float32 rounding of a midpoint), so the measured worst
# case is ~1e-3 of that sum and the median ~1e-6 (float32 accumulation).
BF16_BOUND = 2.0 ** -7


@pytest.mark.parametrize("n_in", [24, 448, 1248])
def test_forward_matches_oracle(ctx, n_in):
    net, flat, mean, std = _random_net(ctx, n_in, 1)
    x = (np.random.default_rng(2).normal(size=(1000, n_in)) * std + mean).astype(np.float32)
    codes, params = net.forward(torch.tensor(x, device=ctx.device))
    codes = codes.cpu().numpy()
    P = _unpack(flat, n_in)
    xs = ((x - mean.astype(np.float32)) * (1.0 / std.astype(np.float32))).astype(np.float32)
    ref, cache = omlp.forward(P, xs, emulate_bf16=True)
    bound = _abs_forward(P, cache)
    err = np.abs(codes - ref)
    ratio = err / bound
    print("[gpu] forward max err %.3g, max err / magnitude sum %.3g, p99 %.3g, median %.3g"
          % (err.max(), ratio.max(), np.quantile(ratio, 0.99), np.median(ratio)))
    assert np.all(err <= BF16_BOUND * bound)
    assert np.median(ratio) < 1e-5
    # decoded starting models: all ten parameters follow the decoding of the
    # GPU's own codes (Sect. 5 network outputs -> model) and the box
    p = params.cpu().numpy().astype(np.float64)
    dec = omlp.decode_outputs(codes.astype(np.float64), np.zeros(7), np.ones(7))
    dec = np.array([oracle.project(m) for m in dec])
    d = np.abs(p - dec)
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])  # psi is 180-periodic
    scale = np.maximum(np.abs(dec), 1.0)
    print("[gpu] decode max rel err per parameter %s" % np.array2string(
        (d / scale).max(axis=0), precision=2))
    assert np.all(d[:, [1, 2]] < 1e-3)                       # degrees
    assert np.all(d[:, [0, 3, 4, 5, 6, 7, 8, 9]] <= 1e-6 * scale[:, [0, 3, 4, 5, 6, 7, 8, 9]])


@pytest.mark.parametrize("n_in", [24, 448])
def test_gradient_matches_oracle(ctx, n_in):
    """vfisv_mlp_gradient element by element against the oracle's backward
    pass with the GPU's bfloat16 roundings (BF16_BOUND of the magnitude sum
    of every element)."""
    net, flat, mean, std = _random_net(ctx, n_in, 3)
    rng = np.random.default_rng(4)
    x = (rng.normal(size=(512, n_in)) * std + mean).astype(np.float32)
    t = rng.normal(size=(512, 10)).astype(np.float32)
    g, loss = net.gradient(torch.tensor(x, device=ctx.device), torch.tensor(t, device=ctx.device))
    G = _unpack(g.cpu().numpy(), n_in)
    P = _unpack(flat, n_in)
    xs = ((x - mean.astype(np.float32)) * (1.0 / std.astype(np.float32))).astype(np.float32)
    y, cache = omlp.forward(P, xs, emulate_bf16=True)
    R = omlp.backward(P, cache, t.astype(np.float64), emulate_bf16=True)
    A = _abs_backward(P, cache, t.astype(np.float64))
    assert loss.item() == pytest.approx(np.sum((y - t) ** 2), rel=1e-4)
    for k in R:
        err = np.abs(G[k] - R[k])
        ratio = err / np.maximum(A[k], 1e-300)
        print("[gpu] grad %s: max err / magnitude sum %.3g, p99 %.3g, median %.3g"
              % (k, ratio.max(), np.quantile(ratio, 0.99), np.median(ratio)))
        assert np.all(err <= BF16_BOUND * A[k] + 1e-12 * np.abs(R[k]).max()), k
        assert np.median(ratio) < 1e-4, k
    # the padding of the first and last layers receives no gradient
    gf = g.cpu().numpy()
    K0 = (n_in + 31) // 32 * 32
    assert np.all(gf[n_in * H:K0 * H] == 0.0)


def test_adam_steps_match_the_oracle(ctx):
    """Five Adam steps of vfisv_mlp_train_step on one batch against the
    oracle's adam_step applied, step by step, to the GPU's gradient at the
    same weights: every float32 weight within float32 rounding of the
    float64 update (the update itself is lr * m-hat / (sqrt(v-hat) + eps),
    at most ~lr per step)."""
    n_in = 24
    net, flat, mean, std = _random_net(ctx, n_in, 9)
    rng = np.random.default_rng(10)
    B = 512
    dev = ctx.device
    x = torch.tensor((rng.normal(size=(B, n_in)) * std + mean).astype(np.float32), device=dev)
    t = torch.tensor(rng.normal(size=(B, 10)).astype(np.float32), device=dev)
    rows = torch.arange(B, dtype=torch.int32, device=dev)
    lr = 1e-3
    m = {"w": np.zeros(flat.size)}
    v = {"w": np.zeros(flat.size)}
    w_prev = net.get_params().astype(np.float64)
    for step in range(1, 6):
        g, _ = net.gradient(x, t)
        g = g.cpu().numpy().astype(np.float64)
        net.train_step(x, t, rows, lr)
        w_gpu = net.get_params().astype(np.float64)
        ref = omlp.adam_step({"w": w_prev}, {"w": g}, m, v, step, lr)["w"]
        err = np.abs(w_gpu - ref)
        moved = np.abs(w_gpu - w_prev)
        print("[gpu] adam step %d: max |dw| %.3g, max err %.3g" % (step, moved.max(), err.max()),
              flush=True)
        assert moved.max() > 0.5 * lr  # the step is taken
        # float32 weight rounding + float32 moments (relative 1e-6 of the step)
        assert np.all(err <= 2.0 ** -23 * np.abs(ref) + 1e-5 * lr), step
        w_prev = w_gpu


def test_input_width_limit(ctx):
    """The fused inference keeps a 64-row tile of the inputs in LDS: 1248
    inputs are the widest it serves (test_forward_matches_oracle covers
    them); a wider network is refused at creation."""
    with pytest.raises(vf.VfisvError):
        learned.Mlp(ctx, 1249, np.zeros(1249), np.ones(1249), np.zeros(7), np.ones(7))


def _fnv1a(h, b):
    for x in b:
        h ^= x
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_save_load_round_trip(ctx):
    """The file keeps normalisation, parameters and the optimiser state: a
    loaded network's next training step equals the saved one's bit for bit;
    a version-1 file (written here from the documented layout) loads with
    the optimiser state at zero; a flipped byte is refused."""
    import struct
    net, flat, mean, std = _random_net(ctx, 24, 5)
    dev = ctx.device
    rng = np.random.default_rng(6)
    x = torch.tensor((rng.normal(size=(256, 24)) * std + mean).astype(np.float32), device=dev)
    t = torch.tensor(rng.normal(size=(256, 10)).astype(np.float32), device=dev)
    rows = torch.arange(256, dtype=torch.int32, device=dev)
    for _ in range(3):
        net.train_step(x, t, rows, 1e-3)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        net2 = learned.Mlp.load(ctx, path)
        np.testing.assert_array_equal(net2.get_params(), net.get_params())
        for a, b in zip(net2.get_norm(), net.get_norm()):
            np.testing.assert_array_equal(a, b)
        xx = torch.randn(300, 24, device=dev)
        np.testing.assert_array_equal(net.forward(xx)[0].cpu().numpy(),
                                      net2.forward(xx)[0].cpu().numpy())
        net.train_step(x, t, rows, 1e-3)
        net2.train_step(x, t, rows, 1e-3)
        np.testing.assert_array_equal(net2.get_params(), net.get_params())
        # version 1: no optimiser state
        p = net.get_params()
        im, is_, om, os_ = net.get_norm()
        body = (struct.pack("<I", 24) + struct.pack("<Q", p.size) + im.tobytes() + is_.tobytes()
                + om.tobytes() + os_.tobytes() + p.tobytes())
        h = _fnv1a(1469598103934665603, body)
        path1 = os.path.join(d, "v1.bin")
        with open(path1, "wb") as f:
            f.write(b"VFISVMLP" + struct.pack("<I", 1) + body + struct.pack("<Q", h))
        net3 = learned.Mlp.load(ctx, path1)
        fresh = learned.Mlp(ctx, 24, im, is_, om, os_)
        fresh.set_params(p)  # zero optimiser state
        net3.train_step(x, t, rows, 1e-3)
        fresh.train_step(x, t, rows, 1e-3)
        np.testing.assert_array_equal(net3.get_params(), fresh.get_params())
        with open(path, "r+b") as f:
            f.seek(100)
            b = f.read(1)
            f.seek(100)
            f.write(bytes([b[0] ^ 0xFF]))
        with pytest.raises(vf.VfisvError):
            learned.Mlp.load(ctx, path)


@pytest.fixture(scope="module")
def small_trained(ctx):
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    print("[gpu] synthesising a small training set", flush=True)
    S, P = learned.make_training_set(ctx, inst, 262144, 11, wl.draw_params, wl.draw_noise)
    Sc, Pc = learned.make_training_set(ctx, inst, 16384, 12, wl.draw_params, wl.draw_noise)
    net, info = learned.train(ctx, inst, S, P, Sc, Pc, epochs=6, batch=2048, lr=2e-3,
                              log=lambda m: print("[gpu] " + m, flush=True))
    return spec, inst, net, info


def test_training_lowers_the_control_error(small_trained):
    spec, inst, net, info = small_trained
    h = info["history"]
    # standardised codes: predicting the mean gives a control error of ~1
    assert h[-1][2] < 0.8 * h[0][2]
    assert info["best_control_mse"] < 0.25


def test_learned_start_needs_fewer_iterations(ctx, small_trained):
    spec, inst, net, info = small_trained
    n = 8192
    P = wl.draw_params(n, 13)
    noise = wl.draw_noise(n, 6, 13)
    obs = vf.synthesize(ctx, inst, torch.tensor(P.astype(np.float32), device=ctx.device),
                        noise=torch.tensor(noise.astype(np.float32), device=ctx.device))
    W = torch.tensor(wl.weights(6), device=ctx.device)
    plain = vf.invert(ctx, inst, obs, W)
    lrn = learned.invert_learned(ctx, inst, net, obs.view(n, 24), W)
    pc, lc = plain["chi2"].cpu().numpy(), lrn["chi2"].cpu().numpy()
    pi, li = plain["iters"].cpu().numpy(), lrn["iters"].cpu().numpy()
    fb = (lrn["status"].cpu().numpy() & vf.FALLBACK_USED) != 0
    print("[gpu] plain: median chi2 %.4f, mean iters %.2f; learned: median chi2 %.4f, mean "
          "iters %.2f, fallback %.3f" % (np.median(pc), pi.mean(), np.median(lc), li.mean(),
                                         fb.mean()))
    assert li.mean() < 0.8 * pi.mean()
    assert np.median(lc) <= np.median(pc) * 1.01
    assert np.mean(lc > 1.01 * pc) < 0.2


def test_fine_learned_start_with_448_inputs(ctx):
    """The network's first layer takes the 448 samples of a fine spectrum;
    trained on fine pixels it shortens the LM on held-out fine pixels."""
    spec = wl.fine_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    S, P = learned.make_training_set(ctx, inst, 196608, 21, wl.draw_params, wl.draw_noise,
                                     chunk=65536)
    Sc, Pc = learned.make_training_set(ctx, inst, 16384, 22, wl.draw_params, wl.draw_noise)
    assert S.shape == (196608, 448)
    net, info = learned.train(ctx, inst, S, P, Sc, Pc, epochs=6, batch=2048, lr=2e-3,
                              log=lambda m: print("[gpu-fine] " + m, flush=True))
    assert info["best_control_mse"] < 0.3
    n = 2048
    Ph = wl.draw_params(n, 23)
    noise = wl.draw_noise(n, spec.n_obs, 23)
    obs = vf.synthesize(ctx, inst, torch.tensor(Ph.astype(np.float32), device=ctx.device),
                        noise=torch.tensor(noise.astype(np.float32), device=ctx.device))
    W = torch.tensor(wl.weights(spec.n_obs), device=ctx.device)
    plain = vf.invert(ctx, inst, obs, W)
    lrn = learned.invert_learned(ctx, inst, net, obs.view(n, 448), W)
    pc, lc = plain["chi2"].cpu().numpy(), lrn["chi2"].cpu().numpy()
    pi, li = plain["iters"].cpu().numpy(), lrn["iters"].cpu().numpy()
    fb = (lrn["status"].cpu().numpy() & vf.FALLBACK_USED) != 0
    print("[gpu-fine] plain: median chi2 %.4f, mean iters %.2f; learned: median chi2 %.4f, "
          "mean iters %.2f, fallback %.3f" % (np.median(pc), pi.mean(), np.median(lc),
                                              li.mean(), fb.mean()), flush=True)
    assert li.mean() < 0.8 * pi.mean()
    assert np.median(lc) <= np.median(pc) * 1.01


def test_learned_path_structure(ctx, small_trained):
    """The learned path is: the network's start, at most learned_max_iter
    LM trials, then for the pixels above the chi^2 threshold a plain LM from
    the combined start of Sect. 5 (network start, classical azimuth, weak
    field below 6 % polarisation), keeping the better fit.  Rebuilt here
    from the separate entry points, it gives the same bits."""
    spec, inst, net, info = small_trained
    n = 8192
    P = wl.draw_params(n, 14)
    noise = wl.draw_noise(n, 6, 14)
    dev = ctx.device
    obs = vf.synthesize(ctx, inst, torch.tensor(P.astype(np.float32), device=dev),
                        noise=torch.tensor(noise.astype(np.float32), device=dev))
    W = torch.tensor(wl.weights(6), device=dev)
    tau = 2.08
    lrn = {k: v.cpu().numpy() for k, v in learned.invert_learned(
        ctx, inst, net, obs.view(n, 24), W, learned_max_iter=15, chi2_accept=tau).items()}
    _, start = net.forward(obs.view(n, 24), codes=False)
    short = {k: v.cpu().numpy() for k, v in vf.invert(
        ctx, inst, obs, W, init=start, opts=vf.Options(max_iter=15)).items()}
    sel = np.flatnonzero(short["chi2"] > tau)
    print("[gpu] learned path: %d of %d refitted" % (len(sel), n), flush=True)
    assert 0 < len(sel) < n // 2
    comb, _ = vf.init_combined(ctx, inst, obs, start, 0.06)
    ts = torch.tensor(sel, device=dev)
    refit = {k: v.cpu().numpy() for k, v in vf.invert(
        ctx, inst, obs[ts].contiguous(), W, init=comb[ts].contiguous(),
        opts=vf.Options(lanes_per_pixel=2)).items()}
    keep = np.ones(n, bool)
    keep[sel] = False
    for k in ("params", "chi2", "iters"):
        assert np.array_equal(lrn[k][keep], short[k][keep]), k
    assert np.array_equal(lrn["status"][keep], short["status"][keep])
    better = refit["chi2"] < short["chi2"][sel]
    np.testing.assert_array_equal(lrn["chi2"][sel], np.where(better, refit["chi2"],
                                                             short["chi2"][sel]))
    np.testing.assert_array_equal(lrn["params"][sel], np.where(better[:, None], refit["params"],
                                                               short["params"][sel]))
    np.testing.assert_array_equal(lrn["iters"][sel], short["iters"][sel] + refit["iters"])
    assert np.all(lrn["status"][sel] & vf.FALLBACK_USED)


def test_native_training_run(ctx):
    """vfisv_mlp_stats against numpy; vfisv_mlp_train keeps the best epoch
    (its control error re-evaluated here from the oracle's target coding),
    and the same seed gives the same weights, another seed others."""
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    S, P = learned.make_training_set(ctx, inst, 32768, 31, wl.draw_params, wl.draw_noise)
    Sc, Pc = learned.make_training_set(ctx, inst, 4096, 32, wl.draw_params, wl.draw_noise)
    stats = learned.training_stats(ctx, S, P)
    Sh = S.cpu().numpy().astype(np.float64)
    P32 = P.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(stats[0], Sh.mean(axis=0), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(stats[1], Sh.std(axis=0), rtol=1e-4)
    np.testing.assert_allclose(stats[2], P32[:, 3:].mean(axis=0), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(stats[3], P32[:, 3:].std(axis=0), rtol=1e-4)
    kw = dict(epochs=4, batch=1024, lr=2e-3)
    nets = [learned.Mlp(ctx, 24, *stats, seed=4) for _ in range(3)]
    infos = [learned.train_network(ctx, nets[k], S, P, Sc, Pc, seed=9 if k < 2 else 10, **kw)
             for k in range(3)]
    p0, p1, p2 = (net.get_params() for net in nets)
    assert np.array_equal(p0, p1) and not np.array_equal(p0, p2)
    info = infos[0]
    ctrl = [h[2] for h in info["history"]]
    print("[gpu] native training: control mse %s, best epoch %d" % (ctrl, info["best_epoch"]),
          flush=True)
    assert info["steps"] == 4 * (32768 // 1024) and len(ctrl) == 4
    assert info["best_epoch"] == int(np.argmin(ctrl)) and info["best_control_mse"] == min(ctrl)
    assert ctrl[-1] < ctrl[0]
    codes, _ = nets[0].forward(Sc, codes=True, params=False)
    T = omlp.encode_targets(Pc.astype(np.float32).astype(np.float64), stats[2].astype(np.float64),
                            stats[3].astype(np.float64))
    mse = np.mean((codes.cpu().numpy().astype(np.float64) - T) ** 2)
    assert abs(mse - info["best_control_mse"]) < 1e-4 * mse, (mse, info["best_control_mse"])
