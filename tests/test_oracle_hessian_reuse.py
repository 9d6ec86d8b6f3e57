"""Pins of the oracle's Hessian reuse (Sect. 4.4, Fig. 6: near the minimum
the curvature of the chi^2 surface barely changes, so an accepted step keeps
the previous J^T W J and only the gradient is rebuilt).  The paper gives no
threshold; `hess_reuse` is the chi^2 below which the model a step starts
from counts as near the minimum."""
import numpy as np
import pytest

import oracle
import workloads as wl

BIG = 1e300


@pytest.fixture(scope="module")
def hmi():
    spec = wl.hmi_instrument()
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    P = wl.draw_params(24, 51)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(24, 6, 51)).astype(np.float32)
    return oi, P, obs, wl.weights(6)


def test_off_is_the_plain_lm(hmi):
    oi, P, obs, W = hmi
    for k in range(8):
        a = oracle.lm_pixel(oi, obs[k], W)
        b = oracle.lm_pixel(oi, obs[k], W, opts=oracle.Options(hess_reuse=0.0))
        assert np.array_equal(a["params"], b["params"]) and a["chi2"] == b["chi2"]
        # every synthesis with derivatives builds the Hessian
        assert b["counters"]["hessians"] == b["counters"]["derivs"]


def test_threshold_compares_the_model_the_step_starts_from(hmi):
    """With the threshold at the start's chi^2 exactly, the first accepted
    step (from the start, not below it) rebuilds H and every later one
    (from models below it) keeps it: 2 builds.  Just above, none after the
    initial one."""
    oi, P, obs, W = hmi
    for k in range(8):
        c0 = oracle.lm_pixel(oi, obs[k], W, opts=oracle.Options(max_iter=0))["chi2"]
        at = oracle.lm_pixel(oi, obs[k], W, opts=oracle.Options(hess_reuse=c0))
        acc = at["counters"]["derivs"] - 1
        assert acc >= 2
        assert at["counters"]["hessians"] == 2, (k, at["counters"])
        above = oracle.lm_pixel(oi, obs[k], W, opts=oracle.Options(hess_reuse=np.nextafter(c0, 1e9)))
        assert above["counters"]["hessians"] == 1


def test_exact_when_the_model_is_linear(hmi):
    """With only S0 and S1 free the profiles are linear in the free
    parameters, J and so J^T W J do not change: keeping the first Hessian
    gives the plain fit bit for bit, with one Hessian built."""
    oi, P, obs, W = hmi
    mask = (1 << 7) | (1 << 8)
    for k in range(8):
        M0 = P[k].copy()
        M0[7:9] = [0.45, 0.3]
        a = oracle.lm_pixel(oi, obs[k], W, M0=M0, opts=oracle.Options(free_mask=mask))
        b = oracle.lm_pixel(oi, obs[k], W, M0=M0,
                            opts=oracle.Options(free_mask=mask, hess_reuse=BIG))
        assert np.array_equal(a["params"], b["params"]) and a["chi2"] == b["chi2"]
        assert a["iters"] == b["iters"] and b["counters"]["hessians"] == 1
        assert a["counters"]["hessians"] == a["counters"]["derivs"] > 1


def test_same_minimum_where_the_fit_ends():
    """The gradient stays exact, so a fit that stops on its own (converged
    or stalled) stops at the stationary point the plain fit finds: noiseless
    profiles from a start near the truth, the Hessian kept once chi^2 is
    below 1e-3."""
    spec = wl.hmi_instrument()
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    P = wl.draw_params(12, 52)
    P[:, 0] = np.maximum(P[:, 0], 400.0)
    obs = oracle.forward_batch(oi, P).astype(np.float32)
    W = wl.weights(6)
    M0 = P * (1.0 + 0.03 * np.random.default_rng(3).standard_normal(P.shape))
    M0[:, 2] = P[:, 2] + 2.0
    ended = 0
    for k in range(len(P)):
        r = oracle.lm_pixel(oi, obs[k], W, M0=oracle.project(M0[k]),
                            opts=oracle.Options(hess_reuse=1e-3, max_iter=400, rel_tol=1e-9))
        assert r["counters"]["hessians"] < r["counters"]["derivs"]
        if r["status"] != oracle.MAX_ITER:
            ended += 1
            assert r["chi2"] < 1e-9, (k, r["chi2"])
    assert ended >= len(P) // 2


def test_restarts_rebuild_the_hessian(hmi):
    """In the fixed-iteration scheme a restart evaluates a new model from
    scratch: its Hessian is built even when reuse is on."""
    oi, P, obs, W = hmi
    for k in range(8):
        r = oracle.lm_pixel(oi, obs[k], W, pixel=k,
                            opts=oracle.Options(fixed_iters=40, restarts=3, hess_reuse=BIG, seed=9))
        used = r["status"] >> 8
        assert r["counters"]["hessians"] == 1 + used
