"""FP64 oracle of the per-pixel Stokes weights -- TEST INFRASTRUCTURE.

Sect. 4.3 (Eqs. 1, 14, 15): chi^2 weights each residual by w_ij^2 / sigma_i^2.
The empirical recipe keeps w_Q = w_U = w_V = 1 and gives Stokes I the weight
    w_I = 0.7778 |I_cont(mu) - I_cont(x, y)| + 0.3                    (Eq. 14)
with the continuum centre-to-limb curve (Neckel & Labs 1994, near 6173 A)
    I_cont(mu) = 0.33644 + 1.30590 mu - 1.79238 mu^2 + 2.45050 mu^3
                 - 1.89979 mu^4 + 0.59943 mu^5                        (Eq. 15)
Readings: I_cont(x, y) is the pixel's largest observed intensity, in units of
the disk-centre quiet-Sun continuum (the unit of I_cont(mu)); mu is clamped
to [0, 1]; sigma is one noise level per Stokes parameter, the same at every
wavelength.  The result is W = w^2 / sigma^2 per pixel, Stokes parameter and
sample, the layout the inversion takes for per-pixel weights.
"""
import numpy as np

EQ15 = (0.33644, 1.30590, -1.79238, 2.45050, -1.89979, 0.59943)


def icont_mu(mu):
    """Eq. 15, evaluated as the printed sum of powers."""
    m = np.clip(np.asarray(mu, dtype=np.float64), 0.0, 1.0)
    return sum(c * m ** k for k, c in enumerate(EQ15))


def w_stokes_i(icont_pixel, mu):
    """Eq. 14."""
    return 0.7778 * np.abs(icont_mu(mu) - np.asarray(icont_pixel, dtype=np.float64)) + 0.3


def stokes_weights(obs, mu, sigma):
    """obs [n, 4, n_obs], mu [n], sigma [4] -> W [n, 4, n_obs] (float64)."""
    S = np.asarray(obs, dtype=np.float64)
    n, _, n_obs = S.shape
    sig = np.asarray(sigma, dtype=np.float64).reshape(4)
    wI = w_stokes_i(S[:, 0, :].max(axis=1), mu)
    W = np.empty((n, 4, n_obs))
    W[:, 0, :] = (wI * wI / (sig[0] * sig[0]))[:, None]
    for s in (1, 2, 3):
        W[:, s, :] = 1.0 / (sig[s] * sig[s])
    return W
