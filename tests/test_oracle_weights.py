"""Pins of the oracle's per-pixel Stokes weights (Sect. 4.3, Eqs. 14-15)."""
import numpy as np
import pytest

from oracle import weights


def test_centre_to_limb_curve():
    """Eq. 15 is normalised to the disk centre (its coefficients sum to
    1.0001), falls monotonically towards the limb, and keeps about a third
    of the centre intensity at the limb."""
    mu = np.linspace(0.0, 1.0, 2001)
    I = weights.icont_mu(mu)
    assert I[-1] == pytest.approx(1.0001, abs=1e-12)
    assert I[0] == pytest.approx(0.33644, abs=1e-12)
    assert np.all(np.diff(I) > 0)
    # outside [0, 1] mu is clamped
    assert weights.icont_mu(1.5) == I[-1] and weights.icont_mu(-0.2) == I[0]


def test_quiet_sun_and_umbra_weights():
    """The paper's stated behaviour: w_I = 0.3 where the pixel is as bright
    as the quiet Sun at its mu, w_I close to 1 in a sunspot umbra."""
    for mu in (0.1, 0.5, 0.9, 1.0):
        assert weights.w_stokes_i(weights.icont_mu(mu), mu) == pytest.approx(0.3, abs=1e-15)
    umbra = weights.w_stokes_i(np.array([0.1, 0.2, 0.3]), 1.0)
    assert np.all((umbra > 0.8) & (umbra < 1.05))
    # brighter and darker than the quiet Sun by the same amount: same weight
    q = weights.icont_mu(0.7)
    assert weights.w_stokes_i(q + 0.2, 0.7) == pytest.approx(weights.w_stokes_i(q - 0.2, 0.7))


def test_weight_array_layout():
    """W = w^2 / sigma^2: Stokes I from Eq. 14 with the pixel's largest
    observed intensity as its continuum; Q, U, V weight one; the same at
    every sample."""
    rng = np.random.default_rng(0)
    n, n_obs = 5, 6
    obs = rng.uniform(0.2, 0.9, (n, 4, n_obs))
    obs[0, 0, :] = weights.icont_mu(0.8) * np.linspace(0.5, 1.0, n_obs)  # max = quiet Sun
    mu = np.array([0.8, 1.0, 0.5, 0.2, 0.0])
    sigma = [1e-3, 2e-3, 2e-3, 4e-3]
    W = weights.stokes_weights(obs, mu, sigma)
    assert W.shape == (n, 4, n_obs)
    assert np.allclose(W[0, 0], 0.09 / 1e-6, rtol=1e-12)
    np.testing.assert_allclose(W[:, 1:3], 1.0 / 4e-6, rtol=1e-12)
    np.testing.assert_allclose(W[:, 3], 1.0 / 16e-6, rtol=1e-12)
    assert np.all(W[:, 0] == W[:, 0, :1])
    # a darker continuum (a spot) raises the weight of I
    spot = obs.copy()
    spot[1, 0] *= 0.3
    assert weights.stokes_weights(spot, mu, sigma)[1, 0, 0] > W[1, 0, 0]
