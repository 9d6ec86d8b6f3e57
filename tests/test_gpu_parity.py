"""GPU parity: libvfisv.so (through the C ABI) against the FP64 oracle.

Tolerances (each derived from the float32 arithmetic of the step it bounds):
* synthesis values: |S_gpu - S_ref| <= 2e-6 (float32 Faddeeva series, ~6e-7
  relative, through the Unno-Rachkovsky quotients);
* Jacobian: |J_gpu - J_ref| <= 2e-4 * column max + 3e-5 * typical column
  scale (columns that vanish as B -> 0 are float32 cancellation noise);
* damped solve (float64 on identical float32 inputs): 1e-10 relative;
* inversion: chi^2 within 2e-4 relative where both sides converged to the
  same minimum; B within 1 G, angles within 0.1 deg, v within 1 m/s on
  pixels whose FP64 1-sigma error makes the minimum well determined.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return vf.Context(0)


@pytest.fixture(scope="module")
def hmi(ctx):
    spec = wl.hmi_instrument()
    return spec, vf.Instrument.from_spec(ctx, spec), oracle.Instrument(
        spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)


def _dev(ctx, a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=ctx.device)


def _edge_params():
    base = np.array([1200.0, 50.0, 30.0, 0.5, 30.0, 0.2, 10.0, 0.3, 0.7, 0.8])
    rows = [base.copy()]
    edges = {0: (0.0, 5000.0, 1e-3), 1: (0.0, 90.0, 180.0), 2: (0.0, 179.99),
             3: (-20.0, 20.0), 4: (5.0, 150.0), 5: (0.0, 5.0), 6: (1e-3, 100.0),
             7: (-1.0, 3.0), 8: (0.0, 5.0), 9: (0.0, 1.0)}
    for p, vals in edges.items():
        for v in vals:
            m = base.copy()
            m[p] = v
            rows.append(m)
    return np.array(rows)


def test_synthesis_parity(ctx, hmi):
    spec, inst, oi = hmi
    P = np.concatenate([wl.draw_params(4096, 5), _edge_params()]).astype(np.float32)
    print("[gpu] synthesis parity on %d models" % len(P), flush=True)
    S, J = vf.synthesize(ctx, inst, _dev(ctx, P), jac=True)
    S, J = S.cpu().numpy(), J.cpu().numpy()
    Pd = P.astype(np.float64)
    Sr = np.empty(S.shape)
    Jr = np.empty(J.shape)
    for k in range(len(P)):
        Sr[k], Jr[k] = oracle.forward(oi, Pd[k], jac=True)
    assert np.max(np.abs(S - Sr)) < 2e-6
    colmax = np.abs(Jr).max(axis=(1, 2), keepdims=True)
    typical = np.median(np.abs(Jr[:4096]).max(axis=(1, 2)), axis=0)
    tol = 2e-4 * colmax + 3e-5 * typical
    bad = np.abs(J - Jr) > tol
    assert not bad.any(), "Jacobian outside tolerance at %s" % (np.argwhere(bad)[:5],)


def test_synthesis_exact_structure(ctx, hmi):
    spec, inst, oi = hmi
    P = wl.draw_params(256, 6).astype(np.float32)
    P[:64, 0] = 0.0      # B = 0
    P[64:128, 9] = 0.0   # alpha = 0
    P[128:192, 1] = 0.0  # gamma = 0
    S = vf.synthesize(ctx, inst, _dev(ctx, P)).cpu().numpy()
    assert np.all(S[:128, 1:] == 0.0)
    assert np.all(S[128:192, 1:3] == 0.0)
    noise = np.random.default_rng(0).normal(0, 1e-3, S.shape).astype(np.float32)
    Sn = vf.synthesize(ctx, inst, _dev(ctx, P), noise=_dev(ctx, noise)).cpu().numpy()
    np.testing.assert_array_equal(Sn, S + noise)


def _spd_batch(rng, n):
    Hs, gs, es = [], [], []
    for k in range(n):
        A = rng.normal(size=(24, 10)) * 10.0 ** rng.uniform(-2, 2, 10)
        H = A.T @ A
        g = A.T @ rng.normal(size=24)
        Hs.append(H[np.tril_indices(10)])
        gs.append(g)
        es.append(10.0 ** rng.uniform(-6, 3))
    return (np.array(Hs, np.float32), np.array(gs, np.float32), np.array(es))


def _unpack(h):
    H = np.zeros((10, 10))
    H[np.tril_indices(10)] = h
    return H + np.tril(H, -1).T


def test_solve_parity(ctx):
    rng = np.random.default_rng(0)
    H, g, eps = _spd_batch(rng, 300)
    # indefinite systems without damping: the Cholesky breaks down and the
    # eigen/SVD fallback solves them
    for k in range(20):
        Q, _ = np.linalg.qr(rng.normal(size=(10, 10)))
        lam = np.concatenate([[-0.3], rng.uniform(0.1, 1.0, 9)]) * 10.0 ** rng.uniform(-2, 4)
        Hs = Q @ np.diag(lam) @ Q.T
        H[k] = Hs[np.tril_indices(10)]
        g[k] = rng.normal(size=10).astype(np.float32)
        eps[k] = 0.0
    for mask in (0x3FF, 0x3FF & ~(1 << 7) & ~(1 << 2)):
        d, c = vf.solve(ctx, _dev(ctx, H), _dev(ctx, g), _dev(ctx, eps, torch.float64), mask)
        d, c = d.cpu().numpy(), c.cpu().numpy()
        for k in range(len(H)):
            ref, code = oracle.solve(_unpack(H[k].astype(np.float64)), g[k].astype(np.float64),
                                     eps[k], mask)
            assert c[k] == code, k
            assert np.max(np.abs(d[k] - ref)) <= 1e-9 * np.max(np.abs(ref)), k
        if mask == 0x3FF:
            # (an indefinite matrix may have a negative diagonal entry, which
            # freezes that parameter and can leave a definite system)
            assert (c[:20] == 1).sum() >= 15 and (c[20:] == 0).all()


def _observations(oi, spec, n, seed):
    P = wl.draw_params(n, seed)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, seed)).astype(np.float32)
    return P, obs


def test_first_iterations_follow_the_oracle(ctx, hmi):
    """max_iter = 0 returns the start; one step reproduces the oracle's
    first damped step and accept/reject decision."""
    spec, inst, oi = hmi
    P, obs = _observations(oi, spec, 256, 21)
    W = wl.weights(spec.n_obs)
    out0 = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), opts=vf.Options(max_iter=0))
    ref0 = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=0))
    np.testing.assert_allclose(out0["params"].cpu().numpy(), ref0["params"], rtol=1e-7)
    np.testing.assert_allclose(out0["chi2"].cpu().numpy(), ref0["chi2"], rtol=2e-4)
    assert (out0["iters"].cpu().numpy() == 0).all()
    assert (out0["status"].cpu().numpy() == vf.MAX_ITER).all()

    out1 = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), opts=vf.Options(max_iter=1))
    ref1 = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=1))
    p1 = out1["params"].cpu().numpy()
    same = np.isclose(p1[:, 0], ref1["params"][:, 0], rtol=1e-3, atol=0.5)
    assert same.mean() > 0.97
    cols = [0, 3, 6, 9]
    d = np.abs(p1 - ref1["params"])[same][:, cols]
    bound = 2e-3 * np.abs(ref1["params"][same][:, cols]) + 1e-3
    assert np.mean(d <= bound) > 0.995
    # the first damped step (Eq. 5, eps = 1e-3) magnifies the float32 error
    # of the Jacobian by the damped normal matrix's conditioning: every
    # element stays within 5x the oracle's own step spread under Jacobian
    # errors of 1e-4 relative (the Jacobian parity level)
    sens = _first_step_spread(oi, obs, W, 1e-4)[same][:, cols]
    assert np.all(d <= bound + 5.0 * sens)
    assert (out1["iters"].cpu().numpy() == 1).all()


def _first_step_spread(oi, obs, W, rel, reps=6, seed=0):
    """Standard deviation of the oracle's first damped step from the default
    model when its Jacobian carries relative errors of size rel."""
    rng = np.random.default_rng(seed)
    S, J = oracle.forward(oi, oracle.default_init(), jac=True)
    Jf = J.reshape(-1, 10)
    w = W.reshape(-1).astype(np.float64)
    out = np.zeros((len(obs), 10))
    for i in range(len(obs)):
        r = (obs[i].astype(np.float64) - S).reshape(-1)
        steps = []
        for _ in range(reps):
            Jp = Jf * (1.0 + rel * rng.standard_normal(Jf.shape))
            steps.append(oracle.solve(Jp.T @ (w[:, None] * Jp), Jp.T @ (w * r), 1e-3)[0])
        out[i] = np.std(steps, axis=0)
    return out


def _sigma(oi, M, W):
    _, J = oracle.forward(oi, M, jac=True)
    J = J.reshape(-1, 10)
    H = J.T @ (W.reshape(-1, 1).astype(np.float64) * J)
    try:
        C = np.linalg.inv(H)
    except np.linalg.LinAlgError:
        return np.full(10, np.inf)
    d = np.diag(C)
    return np.where(d > 0, np.sqrt(np.abs(d)), np.inf)


def test_inversion_near_truth_same_minimum(ctx, hmi):
    """Start both sides near the truth so that the minimum is the same; the
    oracle iterates to its float64 convergence, the GPU to its float32
    noise floor (where it stops as converged or stalled)."""
    spec, inst, oi = hmi
    n = 1024
    P, obs = _observations(oi, spec, n, 31)
    rng = np.random.default_rng(32)
    init = P + rng.normal(size=P.shape) * np.array([30, 2, 2, 0.05, 1, 0.02, 0.5, 0.01, 0.01, 0.02])
    init = np.array([oracle.project(m) for m in init]).astype(np.float32)
    W = wl.weights(spec.n_obs)
    print("[gpu] near-truth inversion of %d pixels" % n, flush=True)
    out = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), init=_dev(ctx, init),
                    opts=vf.Options(max_iter=300, rel_tol=1e-7))
    ref = oracle.invert(oi, obs, W, init=init.astype(np.float64),
                        opts=oracle.Options(max_iter=300, rel_tol=1e-9))
    gp, gc, gs = (out[k].cpu().numpy() for k in ("params", "chi2", "status"))
    at_min = (ref["status"] == vf.CONVERGED) & (gs != vf.MAX_ITER)
    assert at_min.mean() > 0.75
    rel = np.abs(gc - ref["chi2"]) / ref["chi2"]
    f1, f2 = np.mean(rel[at_min] < 1e-4), np.mean(rel[at_min] < 2e-2)
    print("[gpu] at minimum %d: chi2 within 1e-4 %.4f, within 2e-2 %.4f" % (at_min.sum(), f1, f2))
    # measured: 0.961 within 1e-4 and 0.9988 within 2e-2 of 863 pixels at the
    # minimum (the GPU's per-pixel results do not depend on the schedule)
    assert f1 > 0.955 and f2 > 0.998
    sig = np.array([_sigma(oi, ref["params"][k], W) for k in range(n)])
    d = np.abs(gp - ref["params"])
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    # the tolerance is required where the FP64 1-sigma error is below 10x it
    for p, tol in ((0, 1.0), (1, 0.1), (2, 0.1), (3, 1e-3)):
        wd = at_min & (sig[:, p] < 10 * tol)
        frac = np.mean(d[wd, p] < tol)
        print("[gpu] param %d: %d well-determined, %.4f within %g" % (p, wd.sum(), frac, tol))
        assert wd.sum() > 100 and frac > 0.99


@pytest.mark.parametrize("shape,rows", [("hmi", 5), ("reversed", 5), ("narrow", 5), ("wide", 6)])
def test_register_windows_follow_the_oracle(ctx, shape, rows):
    """The dense pass keeps five rows in registers when the first row to end
    and the last to start share at most four synthesis points (HMI: three;
    rows in reverse order; narrow filters: none shared), six otherwise (wider
    filters, 13 shared points); each layout follows the oracle from near the
    truth."""
    kw = {"hmi": {}, "reversed": {"centres_mA": (172.0, 103.2, 34.4, -34.4, -103.2, -172.0)},
          "narrow": {"fwhm_mA": 30.0}, "wide": {"fwhm_mA": 100.0}}[shape]
    spec = wl.hmi_instrument(**kw)
    inst = vf.Instrument.from_spec(ctx, spec)
    assert inst.info["lm_register_rows"] == rows
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 384
    P, obs = _observations(oi, spec, n, 61)
    rng = np.random.default_rng(62)
    init = P + rng.normal(size=P.shape) * np.array([30, 2, 2, 0.05, 1, 0.02, 0.5, 0.01, 0.01, 0.02])
    init = np.array([oracle.project(m) for m in init]).astype(np.float32)
    W = wl.weights(spec.n_obs)
    print("[gpu] register window %s: %d pixels" % (shape, n), flush=True)
    out = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), init=_dev(ctx, init),
                    opts=vf.Options(max_iter=300, rel_tol=1e-7))
    ref = oracle.invert(oi, obs, W, init=init.astype(np.float64),
                        opts=oracle.Options(max_iter=300, rel_tol=1e-9))
    gc, gs = out["chi2"].cpu().numpy(), out["status"].cpu().numpy()
    # wider filters blur the profiles: the oracle itself converges less often
    conv = ref["status"] == vf.CONVERGED
    at_min = conv & (gs != vf.MAX_ITER)
    assert conv.mean() > 0.6 and at_min.mean() > 0.85 * conv.mean()
    rel = np.abs(gc - ref["chi2"]) / ref["chi2"]
    assert np.mean(rel[at_min] < 1e-4) > 0.9 and np.mean(rel[at_min] < 2e-2) > 0.98
    # one step from the default model: the oracle's accept decision
    out1 = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W), opts=vf.Options(max_iter=1))
    ref1 = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=1))
    moved_g = np.any(out1["params"].cpu().numpy() != np.float32(oracle.default_init()), axis=1)
    moved_r = np.any(ref1["params"] != oracle.default_init(), axis=1)
    assert np.mean(moved_g == moved_r) > 0.97


def test_default_start_statistics(ctx, hmi):
    """Plain LM from the default model: GPU and oracle reach statistically
    the same fits (individual trajectories may split on float32 rounding)."""
    spec, inst, oi = hmi
    n = 4096
    P, obs = _observations(oi, spec, n, 1000)
    W = wl.weights(spec.n_obs)
    out = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, W))
    ref = oracle.invert(oi, obs, W)
    gc = out["chi2"].cpu().numpy()
    gi = out["iters"].cpu().numpy()
    # About half of the trajectories split on float32 rounding, and a split
    # fit ends higher or lower than the oracle's alike (measured 22-24% each
    # way): no side may end higher more often than the other.  The chi^2
    # distribution rises steeply between its 45th and 60th percentiles
    # (1.3 -> 2.2), so the median moves by several percent when a dozen
    # split fits change sides; 4,096 pixels keep that within the 5% bar.
    # Also compared: the share of fits at the noise level and the work.
    rel = (gc - ref["chi2"]) / ref["chi2"]
    higher, lower = np.mean(rel > 1e-4), np.mean(rel < -1e-4)
    print("[gpu] split fits: GPU higher %.3f, lower %.3f" % (higher, lower), flush=True)
    assert abs(higher - lower) < 0.05, (higher, lower)
    a, b = np.median(gc), np.median(ref["chi2"])
    assert abs(a - b) / b < 0.05, (a, b)
    assert abs(np.mean(gc < 2.0) - np.mean(ref["chi2"] < 2.0)) < 0.05
    assert abs(gi.mean() - ref["iters"].mean()) / ref["iters"].mean() < 0.1
    assert 1.0 - higher - lower > 0.4


def test_edge_cases(ctx, hmi):
    spec, inst, oi = hmi
    W = wl.weights(spec.n_obs)
    Wd = _dev(ctx, W)
    P, obs = _observations(oi, spec, 65, 41)
    # n = 0: nothing enqueued
    e = torch.empty((0, 4, 6), device=ctx.device)
    vf.invert(ctx, inst, e, Wd)
    obs[3, 2, 1] = np.nan
    out = vf.invert(ctx, inst, _dev(ctx, obs), Wd)
    st = out["status"].cpu().numpy()
    assert st[3] == vf.NONFINITE and np.isnan(out["params"][3].cpu().numpy()).all()
    assert np.isnan(out["chi2"][3].item()) and out["iters"][3].item() == 0
    assert (st[np.arange(65) != 3] <= 2).all()
    # per-pixel weights equal to the shared ones, an explicit default start
    Wpp = np.broadcast_to(W, (65, 4, 6)).copy()
    out2 = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, Wpp),
                     init=_dev(ctx, np.tile(wl.default_model(), (65, 1))))
    for k in ("params", "chi2", "iters", "status"):
        a, b = out[k].cpu().numpy(), out2[k].cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True), k
    # one pixel
    o1 = vf.invert(ctx, inst, _dev(ctx, obs[:1]), Wd)
    np.testing.assert_array_equal(o1["params"].cpu().numpy(), out["params"][:1].cpu().numpy())
    # fixed parameters stay at their starting values
    mask = 0x3FF & ~(1 << 7) & ~(1 << 8) & ~(1 << 5)
    o3 = vf.invert(ctx, inst, _dev(ctx, obs), Wd, opts=vf.Options(free_mask=mask))
    p3 = o3["params"].cpu().numpy()
    ok = np.arange(65) != 3
    assert np.all(p3[ok, 7] == np.float32(0.3)) and np.all(p3[ok, 8] == np.float32(0.7))
    assert np.all(p3[ok, 5] == np.float32(0.25))
    ref = oracle.lm_pixel(oi, obs[0], W, opts=oracle.Options(free_mask=mask, max_iter=0))
    o4 = vf.invert(ctx, inst, _dev(ctx, obs[:1]), Wd, opts=vf.Options(free_mask=mask, max_iter=0))
    assert o4["chi2"].item() == pytest.approx(ref["chi2"], rel=2e-4)


def test_scheduling_does_not_change_results(ctx, hmi):
    spec, inst, oi = hmi
    P, obs = _observations(oi, spec, 3000, 51)
    W = _dev(ctx, wl.weights(spec.n_obs))
    o = _dev(ctx, obs)
    ref = vf.invert(ctx, inst, o, W)
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    c = ctx.counters()
    assert c["pixels"] == 3000 and c["trials"] == ref["iters"].sum()
    assert 0 <= c["passes"] - c["trials"] - 3000 <= c["accepts"]
    for gw, cl, ds in ((1, 8, 0), (3, 0, 8), (17, 3, 64), (500, 8, 1), (0, 20, 32), (0, 6, -1)):
        out = vf.invert(ctx, inst, o, W, opts=vf.Options(grid_waves=gw, chunk_log2=cl,
                                                         deriv_split=ds))
        c = ctx.counters()
        assert c["grid_waves"] == min(gw or 10 ** 9, (3000 + 63) // 64)
        assert c["pixels"] == 3000 and 0 <= c["passes"] - c["trials"] - 3000 <= c["accepts"]
        for k in ref:
            assert np.array_equal(out[k].cpu().numpy(), ref[k]), (gw, cl, k)


@pytest.mark.gpu
def test_iter_histogram_is_exact(ctx, hmi):
    """Integer work: the device histogram equals numpy's count exactly."""
    import torch
    rng = np.random.default_rng(77)
    for n, n_bins in ((0, 5), (1, 1), (1000, 51), (300_001, 51), (70_000, 4096), (5000, 7)):
        it = rng.integers(0, 80, size=n).astype(np.int32)
        h = vf.iter_histogram(ctx, torch.tensor(it, device=ctx.device), n_bins)
        want = np.bincount(np.minimum(it, n_bins - 1), minlength=n_bins)
        assert h.dtype == np.int64 and np.array_equal(h, want), (n, n_bins)
    with pytest.raises(Exception):
        vf.iter_histogram(ctx, torch.zeros(3, dtype=torch.int32, device=ctx.device), 0)
    with pytest.raises(Exception):
        vf.iter_histogram(ctx, torch.zeros(3, dtype=torch.int32, device=ctx.device), 4097)
    # on an inversion's own output
    spec, inst, oi = hmi
    P, obs = _observations(oi, spec, 2000, 61)
    out = vf.invert(ctx, inst, _dev(ctx, obs), _dev(ctx, wl.weights(spec.n_obs)))
    it = out["iters"].cpu().numpy()
    h = vf.iter_histogram(ctx, out["iters"], 51)
    assert np.array_equal(h, np.bincount(it, minlength=51)) and h.sum() == 2000
    assert (h * np.arange(51)).sum() == ctx.counters()["trials"]


def test_autotune_picks_a_candidate_and_keeps_results(ctx, hmi):
    spec, inst, oi = hmi
    P, obs = _observations(oi, spec, 20000, 91)
    o = _dev(ctx, obs)
    W = _dev(ctx, wl.weights(spec.n_obs))
    ref = {k: v.cpu().numpy() for k, v in vf.invert(ctx, inst, o, W).items()}
    t = vf.autotune(ctx, inst, o, W, sample=8192)
    cus = torch.cuda.get_device_properties(ctx.device).multi_processor_count
    print("[gpu] autotune %s" % t, flush=True)
    assert t["sample"] == 8192 and t["candidates"] >= 12
    assert t["grid_waves"] % cus == 0 and t["chunk_log2"] in (4, 8, 12)
    assert 0 < t["best_ms"] <= t["default_ms"]
    out = vf.invert(ctx, inst, o, W)
    assert ctx.counters()["grid_waves"] == min(t["grid_waves"], (20000 + 63) // 64)
    for k in ref:
        assert np.array_equal(out[k].cpu().numpy(), ref[k]), k


def test_lane_pairs_follow_the_oracle(ctx, hmi):
    """lanes_per_pixel = 2: each pixel's synthesis is split over two lanes;
    the fit must still follow the oracle as the one-lane path does."""
    spec, inst, oi = hmi
    n = 1024
    P, obs = _observations(oi, spec, n, 1000)
    W = wl.weights(spec.n_obs)
    o, Wd = _dev(ctx, obs), _dev(ctx, W)
    op0 = vf.Options(max_iter=0, lanes_per_pixel=2)
    out0 = vf.invert(ctx, inst, o, Wd, opts=op0)
    assert ctx.counters()["grid_waves"] == 2 * n // 64
    ref0 = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=0))
    np.testing.assert_allclose(out0["chi2"].cpu().numpy(), ref0["chi2"], rtol=2e-4)
    out = vf.invert(ctx, inst, o, Wd, opts=vf.Options(lanes_per_pixel=2))
    c = ctx.counters()
    gc, gi = out["chi2"].cpu().numpy(), out["iters"].cpu().numpy()
    assert c["pixels"] == n and c["trials"] == gi.sum() and 0 <= c["passes"] - c["trials"] - n <= c["accepts"]
    assert np.isin(out["status"].cpu().numpy(), (0, 1, 2)).all()
    ref = oracle.invert(oi, obs, W)
    a, b = np.median(gc), np.median(ref["chi2"])
    assert abs(a - b) / b < 0.05, (a, b)
    assert abs(np.mean(gc < 2.0) - np.mean(ref["chi2"] < 2.0)) < 0.05
    assert abs(gi.mean() - ref["iters"].mean()) / ref["iters"].mean() < 0.1
    # against the one-lane path on the same pixels
    one = vf.invert(ctx, inst, o, Wd)
    oc = one["chi2"].cpu().numpy()
    assert np.mean(np.abs(gc - oc) / oc < 1e-4) > 0.4
    with pytest.raises(Exception):
        vf.invert(ctx, inst, o, Wd, opts=vf.Options(lanes_per_pixel=3))


def test_lane_pairs_waiting_for_a_free_pair(ctx, hmi):
    """Pairs while at most a tenth of the pixels wait: on a 16-wave grid
    (512 pairs) 560 pixels take pairs, 48 of them once an earlier pair has
    finished, and every pixel's result equals the one it gets when all
    pairs run at once (18 waves), bit for bit; 600 pixels (more than a
    tenth waiting) take one lane each and equal the one-lane path."""
    spec, inst, oi = hmi
    P, obs = _observations(oi, spec, 600, 1100)
    W = _dev(ctx, wl.weights(spec.n_obs))

    def run(n, **kw):
        out = vf.invert(ctx, inst, _dev(ctx, obs[:n]), W, opts=vf.Options(**kw))
        return {k: v.cpu().numpy() for k, v in out.items()}, ctx.counters()

    print("[gpu] pairs: all resident", flush=True)
    ref, cref = run(560, lanes_per_pixel=2)
    assert cref["grid_waves"] == 18
    print("[gpu] pairs: 48 waiting", flush=True)
    got, cgot = run(560, lanes_per_pixel=2, grid_waves=16)
    assert cgot["grid_waves"] == 16
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    for k in ("pixels", "trials", "accepts", "passes", "hessians"):
        assert cgot[k] == cref[k], k
    one, _ = run(560)
    assert np.mean(one["chi2"] != ref["chi2"]) > 0.5  # pairs did run
    print("[gpu] pairs: 600 pixels on 16 waves", flush=True)
    big, _ = run(600, lanes_per_pixel=2, grid_waves=16)
    one, _ = run(600)
    for k in one:
        assert np.array_equal(big[k], one[k]), k


@pytest.mark.parametrize("order", [1, 2])
def test_taylor_table_follows_the_oracle(ctx, hmi, order):
    """Voigt by the Taylor table (Sect. 3.2, Eqs. 10-13): synthesis, start
    chi^2 and the fit statistics against the oracle using the same table.
    Where float32 and float64 round |u| to different nearest nodes (a cell
    boundary, rare) the two sides use different expansions, so the largest
    difference is bounded by the expansion's own error, the rest by float32
    rounding."""
    spec, inst, oi = hmi
    ot = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter,
                           voigt=order)
    P = wl.draw_params(1024, 31).astype(np.float32)
    S = vf.synthesize(ctx, inst, _dev(ctx, P), voigt=order).cpu().numpy()
    Sr = oracle.forward_batch(ot, P.astype(np.float64))
    d = np.abs(S - Sr)
    assert np.quantile(d, 0.999) < 2e-6 and d.max() < (1e-3 if order == 1 else 1e-4), d.max()
    # the table against the exact evaluation, on the GPU itself
    S0 = vf.synthesize(ctx, inst, _dev(ctx, P)).cpu().numpy()
    assert np.abs(S - S0).max() < (2e-3 if order == 1 else 1e-4)
    n = 512
    Pn, obs = _observations(ot, spec, n, 32)
    W = wl.weights(spec.n_obs)
    o, Wd = _dev(ctx, obs), _dev(ctx, W)
    out0 = vf.invert(ctx, inst, o, Wd, opts=vf.Options(max_iter=0, voigt=order))
    ref0 = oracle.invert(ot, obs, W, opts=oracle.Options(max_iter=0))
    rel = np.abs(out0["chi2"].cpu().numpy() - ref0["chi2"]) / ref0["chi2"]
    assert np.median(rel) < 2e-5 and np.quantile(rel, 0.99) < 2e-4
    out = vf.invert(ctx, inst, o, Wd, opts=vf.Options(voigt=order))
    ref = oracle.invert(ot, obs, W)
    gc, gi = out["chi2"].cpu().numpy(), out["iters"].cpu().numpy()
    a, b = np.median(gc), np.median(ref["chi2"])
    assert abs(a - b) / b < 0.05, (a, b)
    assert abs(gi.mean() - ref["iters"].mean()) / ref["iters"].mean() < 0.12
    with pytest.raises(Exception):
        vf.invert(ctx, inst, o, Wd, opts=vf.Options(voigt=3))


def test_fixed_iterations_with_restarts_follow_the_oracle(ctx, hmi):
    """The fixed-iteration scheme with restarts (Sect. 4.2)."""
    spec, inst, oi = hmi
    n = 256
    P, obs = _observations(oi, spec, n, 51)
    W = wl.weights(spec.n_obs)
    o, Wd = _dev(ctx, obs), _dev(ctx, W)
    # restart timing, integer-exact: with nothing free every trial fails
    for fixed in (5, 6, 11, 17, 40):
        out = vf.invert(ctx, inst, o, Wd, opts=vf.Options(fixed_iters=fixed, restarts=3,
                                                          restart_seed=3, free_mask=0))
        ref = oracle.invert(oi, obs, W, opts=oracle.Options(fixed_iters=fixed, restarts=3, seed=3,
                                                           free_mask=0))
        np.testing.assert_array_equal(out["status"].cpu().numpy(), ref["status"])
        np.testing.assert_array_equal(out["iters"].cpu().numpy(), ref["iters"])
        c = ctx.counters()
        assert c["trials"] == ref["iters"].sum() and 0 <= c["passes"] - c["trials"] - n <= c["accepts"]
    # without restarts: LM without its convergence exit, bit for bit
    a = vf.invert(ctx, inst, o, Wd, opts=vf.Options(fixed_iters=30))
    b = vf.invert(ctx, inst, o, Wd, opts=vf.Options(max_iter=30, rel_tol=0.0))
    for k in ("params", "chi2", "iters", "status"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k
    # with restarts from starts near the truth: the oracle's statistics
    rng = np.random.default_rng(52)
    near = (P + rng.normal(size=P.shape) * [100, 10, 10, 0.3, 3, 0.05, 2, 0.03, 0.03, 0.05])
    near = np.array([oracle.project(m) for m in near]).astype(np.float32)
    opt = vf.Options(fixed_iters=30, restarts=3, restart_seed=5)
    g1 = vf.invert(ctx, inst, o, Wd, init=_dev(ctx, near), opts=opt)
    g2 = vf.invert(ctx, inst, o, Wd, init=_dev(ctx, near), opts=opt)
    for k in g1:
        assert np.array_equal(g1[k].cpu().numpy(), g2[k].cpu().numpy()), k
    ref = oracle.invert(oi, obs, W, init=near.astype(np.float64),
                        opts=oracle.Options(fixed_iters=30, restarts=3, seed=5))
    gc, gs = g1["chi2"].cpu().numpy(), g1["status"].cpu().numpy()
    gi = g1["iters"].cpu().numpy()
    assert ((gi == 30) | ((gs & 255) == 2)).all()
    a, b = np.median(gc), np.median(ref["chi2"])
    print("[gpu] fixed 30 + restarts: median chi2 %.4f vs %.4f, restarts used %.2f vs %.2f"
          % (a, b, (gs >> 8).mean(), (ref["status"] >> 8).mean()), flush=True)
    assert abs(a - b) / b < 0.05
    # a restart also fires after five failed trials in a row, and at its
    # float32 chi^2 noise floor the GPU meets that sooner than the float64
    # oracle: 0.28-0.41 more restarts per pixel over six sets of 256 pixels
    excess = (gs >> 8).mean() - (ref["status"] >> 8).mean()
    assert -0.1 < excess < 0.5
    assert np.mean(np.abs(gc - ref["chi2"]) / ref["chi2"] < 1e-3) > 0.5
    # another seed moves the restarted pixels only
    g3 = vf.invert(ctx, inst, o, Wd, init=_dev(ctx, near),
                   opts=vf.Options(fixed_iters=30, restarts=3, restart_seed=6))
    restarted = (gs >> 8) > 0
    assert not np.array_equal(g3["params"].cpu().numpy()[restarted],
                              g1["params"].cpu().numpy()[restarted])
