"""Pins of the oracle's fixed-iteration mode with restarts (Sect. 4.2: a
fixed number of iterations; restarts from a randomly perturbed best model
when (a) chi^2 has not fallen tenfold after 10 iterations or (b) 5 iterations
in a row brought no improvement)."""
import numpy as np
import pytest

import oracle
import workloads as wl


@pytest.fixture(scope="module")
def hmi():
    spec = wl.hmi_instrument()
    return spec, oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)


def test_splitmix64_published_first_output():
    # the first output of SplitMix64 seeded with 0 is 0xE220A8397B1DCDAF
    assert oracle.splitmix64(0, 0) == 0xE220A8397B1DCDAF


def test_restart_draws_are_uniform_and_keyed():
    u = np.array([oracle.restart_uniform(11, pix, k, p)
                  for pix in range(200) for k in range(1, 4) for p in range(10)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02 and abs(u.var() - 1 / 12) < 0.01
    assert np.histogram(u, bins=10, range=(0, 1))[0].min() > 0.07 * u.size
    assert oracle.restart_uniform(11, 5, 1, 0) != oracle.restart_uniform(12, 5, 1, 0)
    assert oracle.restart_uniform(11, 5, 1, 0) != oracle.restart_uniform(11, 5, 2, 0)


def test_fixed_mode_without_restarts_is_lm_without_the_exit(hmi):
    spec, oi = hmi
    P = wl.draw_params(48, 41)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(48, 6, 41)).astype(np.float32)
    W = wl.weights(6)
    a = oracle.invert(oi, obs, W, opts=oracle.Options(fixed_iters=30))
    b = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=30, rel_tol=0.0))
    for k in ("params", "chi2", "iters", "status"):
        assert np.array_equal(a[k], b[k]), k
    assert ((a["iters"] == 30) | ((a["status"] & 255) == 2)).all()


def test_trigger_timing_with_nothing_free(hmi):
    """With no free parameter every trial repeats the model and fails:
    trials 1-5 fail, trial 6 is restart 1 (trigger b); at trial 10 chi^2 has
    not fallen tenfold, so trial 11 is restart 2 (trigger a); trials 12-16
    fail, trial 17 is restart 3; then the limit of 3 holds, and once the
    damping (doubling from 1e-3, then x10 above 1e4 per Table 2) passes 1e8
    after 28 failed trials the pixel stalls, at trial 31."""
    spec, oi = hmi
    P = wl.draw_params(8, 42)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(8, 6, 42)).astype(np.float32)
    W = wl.weights(6)
    for fixed, want in ((5, 0), (6, 1), (10, 1), (11, 2), (16, 2), (17, 3), (30, 3), (40, 3)):
        r = oracle.invert(oi, obs, W, opts=oracle.Options(fixed_iters=fixed, restarts=3, seed=3,
                                                          free_mask=0))
        assert (r["status"] >> 8 == want).all(), (fixed, r["status"] >> 8)
        stall = fixed > 31
        assert (r["iters"] == (31 if stall else fixed)).all()
        assert ((r["status"] & 255) == (2 if stall else 1)).all()
        # nothing moves: frozen parameters are not perturbed either
        np.testing.assert_array_equal(r["params"], np.tile(oracle.default_init(), (8, 1)))


def test_restarts_are_seeded_and_never_lose_the_best(hmi):
    spec, oi = hmi
    n = 64
    P = wl.draw_params(n, 43)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, 6, 43)).astype(np.float32)
    W = wl.weights(6)
    start = oracle.invert(oi, obs, W, opts=oracle.Options(max_iter=0))["chi2"]
    o = oracle.Options(fixed_iters=30, restarts=4, seed=9)
    a, b = oracle.invert(oi, obs, W, opts=o), oracle.invert(oi, obs, W, opts=o)
    assert np.array_equal(a["params"], b["params"])
    assert (a["chi2"] <= start).all() and (a["iters"] == 30).all()
    assert ((a["status"] >> 8) <= 4).all() and (a["status"] >> 8).max() >= 1
    c = oracle.invert(oi, obs, W, opts=oracle.Options(fixed_iters=30, restarts=4, seed=10))
    restarted = (a["status"] >> 8) > 0
    assert not np.array_equal(a["params"][restarted], c["params"][restarted])
