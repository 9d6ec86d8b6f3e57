"""Pins of the learned-path oracle (oracle/learned.py; Sect. 5: network
initial guess, with a plain LM fit again where the guess serves badly).

* tau: the 0.99 quantile of chi^2_dof / dof against the closed form of the
  chi-square distribution for even dof (a Poisson sum), solved here by
  bisection, not by the oracle's library routine;
* the fallback as first stated (re-fit every pixel that did not converge or
  ends above tau, from the default model, keeping the re-fit), run from the
  default model itself, must reproduce plain LM with the full trial budget
  on every pixel: a dropped re-fit, a wrong start, budget or choice fails;
* the library's reading keeps the lower chi^2 of the two fits, re-fits
  exactly the pixels above tau, starts them from the combined start, adds
  the trials of both fits and flags them; an infinite tau re-fits nothing;
  non-finite input is not re-fitted;
* the network start: known codes decode to known models (the field-vector
  code of each axis and sign, the standardised parameters at 0 and 1).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import learned
from oracle import mlp
import workloads as wl


def _chi2_cdf_even(x, k):
    """P(chi^2_k <= x) for even k: 1 - exp(-x/2) sum_{j < k/2} (x/2)^j / j!."""
    h = 0.5 * x
    term, s = 1.0, 1.0
    for j in range(1, k // 2):
        term *= h / j
        s += term
    return 1.0 - math.exp(-h) * s


def _quantile_even(k, q=0.99):
    lo, hi = 0.0, 10.0 * k + 100.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _chi2_cdf_even(mid, k) < q:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi) / k


@pytest.mark.parametrize("dof", [2, 14, 100, 438])
def test_tau_is_the_chi2_quantile(dof):
    ref = _quantile_even(dof)
    assert learned.reduced_chi2_quantile(dof) == pytest.approx(ref, rel=1e-11)


def test_tau_for_the_hmi_and_fine_instruments():
    # 24 - 10 and 448 - 10 degrees of freedom
    assert learned.reduced_chi2_quantile(14) == pytest.approx(2.0815, abs=5e-5)
    assert learned.reduced_chi2_quantile(438) == pytest.approx(1.1639, abs=5e-5)


@pytest.fixture(scope="module")
def hmi_set():
    spec = wl.hmi_instrument()
    inst = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 96
    P = wl.draw_params(n, 77)
    obs = (oracle.forward_batch(inst, P) + wl.draw_noise(n, 6, 77)).astype(np.float32)
    return inst, P, obs, wl.weights(6)


def test_rule_as_stated_from_the_default_model_is_plain_lm(hmi_set):
    inst, P, obs, W = hmi_set
    n = obs.shape[0]
    starts = np.tile(oracle.default_init(), (n, 1))
    out = learned.learned_invert(inst, obs, W, starts, rule=learned.AS_STATED)
    plain = oracle.invert(inst, obs, W)
    short = out["short"]
    refit = out["refit"]
    # the re-fit set: every pixel that did not converge or ends above tau
    expect = ((short["status"] & 15) != oracle.CONVERGED) | (short["chi2"] > out["tau"])
    np.testing.assert_array_equal(refit, expect)
    assert 0 < refit.sum() < n
    np.testing.assert_array_equal(out["params"], plain["params"])
    np.testing.assert_array_equal(out["chi2"], plain["chi2"])
    np.testing.assert_array_equal(out["status"] & 15, plain["status"])
    np.testing.assert_array_equal((out["status"] & learned.FALLBACK) != 0, refit)
    np.testing.assert_array_equal(out["iters"][~refit], plain["iters"][~refit])
    np.testing.assert_array_equal(out["iters"][refit], short["iters"][refit] + plain["iters"][refit])


def _poor_starts(P, seed):
    """Starting models near the truth for half the pixels and at the far
    corner of the priors for the rest, so that some short fits end above tau."""
    rng = np.random.default_rng(seed)
    S = np.array(P, dtype=np.float64)
    S[:, 0] *= rng.uniform(0.9, 1.1, len(S))
    far = rng.random(len(S)) < 0.5
    S[far] = [4500.0, 170.0, 10.0, 15.0, 120.0, 3.0, 500.0, 2.0, 0.2, 0.05]
    return S


def test_library_reading_keeps_the_better_fit(hmi_set):
    inst, P, obs, W = hmi_set
    starts = _poor_starts(P, 5)
    out = learned.learned_invert(inst, obs, W, starts)
    short, refit = out["short"], out["refit"]
    np.testing.assert_array_equal(refit, short["chi2"] > out["tau"])
    assert 0 < refit.sum() < len(P)
    # re-fit from the combined start of Sect. 5 with the full budget
    idx = np.flatnonzero(refit)
    comb = learned.combined_starts(inst, obs[idx], starts[idx])
    r = oracle.invert(inst, obs[idx], W, init=comb)
    best = np.minimum(r["chi2"], short["chi2"][idx])
    np.testing.assert_array_equal(out["chi2"][idx], best)
    take = r["chi2"] < short["chi2"][idx]
    np.testing.assert_array_equal(out["params"][idx[take]], r["params"][take])
    np.testing.assert_array_equal(out["params"][idx[~take]], short["params"][idx[~take]])
    np.testing.assert_array_equal(out["iters"][idx], short["iters"][idx] + r["iters"])
    assert np.all(out["status"][idx] & learned.FALLBACK)
    keep = ~refit
    for k in ("params", "chi2", "iters", "status"):
        np.testing.assert_array_equal(out[k][keep], short[k][keep])
    # never worse than the short fit
    assert np.all(out["chi2"] <= short["chi2"])
    # the short fit has at most 15 trials
    assert short["iters"].max() <= 15


def test_infinite_threshold_refits_nothing(hmi_set):
    inst, P, obs, W = hmi_set
    starts = _poor_starts(P, 6)
    out = learned.learned_invert(inst, obs, W, starts, tau=np.inf)
    assert not out["refit"].any()
    assert not np.any(out["status"] & learned.FALLBACK)
    short = oracle.invert(inst, obs, W, init=starts, opts=oracle.Options(max_iter=15))
    np.testing.assert_array_equal(out["chi2"], short["chi2"])


def test_nonfinite_input_is_not_refitted(hmi_set):
    inst, P, obs, W = hmi_set
    o = np.array(obs[:8])
    o[3, 1, 2] = np.nan
    out = learned.learned_invert(inst, o, W, _poor_starts(P[:8], 7), tau=1e-300)
    assert out["status"][3] == oracle.NONFINITE and not out["refit"][3]
    others = np.delete(np.arange(8), 3)
    assert out["refit"][others].all()


def test_known_codes_decode_to_known_models():
    mean = np.array([0.5, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6])
    std = np.array([1.7, 8.7, 0.14, 8.4, 0.12, 0.12, 0.23])
    third = 1.0 / 3.0
    Y = np.zeros((7, 10))
    Y[0, 0] = third                 # along the line of sight: gamma 0
    Y[1, 0] = -third                # against it: gamma 180
    Y[2, 1] = third                 # transverse, Q-like: gamma 90, psi 0
    Y[3, 2] = third                 # transverse, U-like: psi 45
    Y[4, 1] = -third                # transverse, -Q: psi 90
    Y[5, 2] = -third                # -U: psi 135
    Y[6, 0] = Y[6, 1] = third       # gamma 45 (B sin g = B cos g), psi 0
    Y[6, 3:] = 1.0
    D = mlp.decode_outputs(Y, mean, std)
    expect_b = [1000.0] * 6 + [1000.0 * math.sqrt(2.0)]
    expect_g = [0.0, 180.0, 90.0, 90.0, 90.0, 90.0, 45.0]
    expect_p = [0.0, 0.0, 0.0, 45.0, 90.0, 135.0, 0.0]
    np.testing.assert_allclose(D[:, 0], expect_b, rtol=1e-14)
    np.testing.assert_allclose(D[:, 1], expect_g, atol=1e-12)
    np.testing.assert_allclose(D[2:, 2], expect_p[2:], atol=1e-12)
    np.testing.assert_allclose(D[:6, 3:], np.tile(mean, (6, 1)), rtol=0, atol=1e-15)
    np.testing.assert_allclose(D[6, 3:], mean + std, rtol=1e-15)


def test_known_models_encode_to_known_codes():
    mean = np.zeros(7)
    std = np.ones(7)
    P = np.array([[3000.0, 90.0, 45.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0],
                  [1500.0, 60.0, 0.0, 0, 0, 0, 0, 0, 0, 0],
                  [0.0, 33.0, 71.0, 0, 0, 0, 0, 0, 0, 0]])
    T = mlp.encode_targets(P, mean, std)
    np.testing.assert_allclose(T[0, :3], [0.0, 0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(T[0, 3:], [1, 2, 3, 4, 5, 6, 7], rtol=0)
    np.testing.assert_allclose(T[1, :3], [0.25, 0.5 * math.sqrt(3.0) / 2.0, 0.0], atol=1e-15)
    np.testing.assert_array_equal(T[2, :3], [0.0, 0.0, 0.0])


def test_network_start_of_a_linear_network():
    """A network whose hidden layers pass the standardised inputs through
    GELU and whose output layer is zero decodes its biases: the start is
    the model those codes name, whatever the inputs."""
    n_in = 24
    K0 = 32
    flat = np.zeros(K0 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 32 + 32, np.float32)
    b4 = np.zeros(32, np.float32)
    b4[:10] = [0.0, 0.5, 0.0, 0.0, 1.0, -1.0, 0.0, 0.5, 0.0, 0.0]
    flat[-32:] = b4
    std = np.array([1.7, 8.7, 0.14, 8.4, 0.12, 0.12, 0.23])
    out_mean = np.array([0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6])
    x = np.random.default_rng(3).normal(size=(5, n_in))
    M, y = learned.network_starts(flat, n_in, np.zeros(n_in), np.ones(n_in), out_mean, std, x)
    assert np.all(y == y[0])
    np.testing.assert_allclose(M[:, 0], 1500.0, rtol=1e-12)
    np.testing.assert_allclose(M[:, 1], 90.0, atol=1e-12)
    np.testing.assert_allclose(M[:, 4], 35.0 + 8.7, rtol=1e-12)
    np.testing.assert_allclose(M[:, 5], 0.25 - 0.14, rtol=1e-12)
    np.testing.assert_allclose(M[:, 7], 0.3 + 0.5 * 0.12, rtol=1e-12)
