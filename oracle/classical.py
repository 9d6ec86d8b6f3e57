"""FP64 oracle of the classical initial guess -- TEST INFRASTRUCTURE.

The paper's non-network initialisation (Sect. 5) takes B and gamma from the
magnetograph formula and the weak-field approximation (Jefferies & Mickey
1991) where the polarisation is weak, and the azimuth from the linear
polarisation (Auer et al. 1977).  Written out here from those definitions,
per pixel, on the observed samples:

* observed wavelength of sample k: the centroid of its filter row;
* continuum I_c: the largest observed intensity; line depression
  d_k = I_c - I_k;
* v: the centre of gravity of the depression, v = c * lambda_cog / lambda0;
* weak field, longitudinal: V = -C_Z B_par dI/dlambda (Eq. 7 constant C_Z),
  solved by least squares over the samples;
* weak field, transverse: |Q + iU| = (C_Z B_perp)^2 / 4 |d2I/dlambda2|,
  least squares for B_perp^2 (set to 0 if negative);
* azimuth: 2 psi = atan2(sum_k U_k, sum_k Q_k), the linear polarisation
  integrated over the observed samples (the paper cites Auer et al. 1977
  and calls it more reliable than half the arctangent of U/Q, without
  printing it; read here as the line-integrated ratio, which is exact for
  transverse fields and insensitive to the sign change of Q between the
  line core and the sigma components of strong fields);
* derivatives of I by finite differences on the (non-uniform) sample grid:
  central first differences, three-point second differences, the end
  samples taking their neighbour's second difference;
* B = sqrt(B_par^2 / alpha0^2 + B_perp^2 / alpha0), gamma = atan2(B_perp /
  sqrt(alpha0), B_par / alpha0) with the default filling factor alpha0 = 0.6
  (the weak-field signals scale with alpha B cos gamma and alpha B^2 sin^2
  gamma); Doppler width, damping, eta0 and alpha from the default model;
  S0, S1 = 0.3 I_c, 0.7 I_c; then the box projection.
* polarisation level: max_k sqrt(Q_k^2 + U_k^2 + V_k^2) / I_c (the paper
  switches between methods at 6%), undefined (NaN) when I_c <= 0.
* where a denominator vanishes (no depression, no slope or no curvature of
  I) the corresponding estimate is 0.

combined_init puts the two initialisations of Sect. 5 together: a model
from elsewhere (the network's) keeps everything but the azimuth, which is
always the classical one, and B and gamma, which are the classical ones
where the polarisation level is below the threshold (a NaN level keeps the
base's); a pixel with non-finite samples keeps the base model.
"""
import numpy as np

C_KMS = 299792.458
ALPHA0 = 0.6


def sample_offsets(filt, fine_offset_mA):
    """Observed wavelength of each filter row: its centroid [mA]."""
    F = np.asarray(filt, dtype=np.float64)
    return F @ np.asarray(fine_offset_mA, dtype=np.float64) / F.sum(axis=1)


def _d1(I, x):
    g = np.empty_like(I)
    g[:, 1:-1] = (I[:, 2:] - I[:, :-2]) / (x[2:] - x[:-2])
    g[:, 0] = (I[:, 1] - I[:, 0]) / (x[1] - x[0])
    g[:, -1] = (I[:, -1] - I[:, -2]) / (x[-1] - x[-2])
    return g


def _d2(I, x):
    g = np.empty_like(I)
    h0 = x[1:-1] - x[:-2]
    h1 = x[2:] - x[1:-1]
    g[:, 1:-1] = 2.0 * (h0 * I[:, 2:] - (h0 + h1) * I[:, 1:-1] + h1 * I[:, :-2]) / (
        h0 * h1 * (h0 + h1))
    g[:, 0] = g[:, 1]
    g[:, -1] = g[:, -2]
    return g


def classical_init(obs, x_mA, lambda0_A, cz_mA_per_G, default_model, project):
    """obs [n, 4, n_obs] -> (starting models [n, 10], polarisation level [n])."""
    S = np.asarray(obs, dtype=np.float64)
    I, Q, U, V = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    x = np.asarray(x_mA, dtype=np.float64)
    Ic = I.max(axis=1)
    d = Ic[:, None] - I

    def ratio(num, den):
        out = np.zeros_like(num)
        np.divide(num, den, out=out, where=den != 0.0)
        return out

    lam_cog = ratio((d * x).sum(axis=1), d.sum(axis=1))
    v = C_KMS * lam_cog / (lambda0_A * 1000.0)
    Ip = _d1(I, x)
    Ipp = _d2(I, x)
    b_par = -ratio((V * Ip).sum(axis=1), cz_mA_per_G * (Ip * Ip).sum(axis=1))
    L = np.sqrt(Q * Q + U * U)
    b_perp2 = 4.0 * ratio((L * np.abs(Ipp)).sum(axis=1), cz_mA_per_G ** 2 * (Ipp * Ipp).sum(axis=1))
    b_perp = np.sqrt(np.maximum(b_perp2, 0.0))
    psi = 0.5 * np.degrees(np.arctan2(U.sum(axis=1), Q.sum(axis=1)))
    bl = b_par / ALPHA0
    bt = b_perp / np.sqrt(ALPHA0)
    M = np.tile(np.asarray(default_model, dtype=np.float64), (S.shape[0], 1))
    M[:, 0] = np.sqrt(bl * bl + bt * bt)
    M[:, 1] = np.degrees(np.arctan2(bt, bl))
    M[:, 2] = psi
    M[:, 3] = v
    M[:, 7] = 0.3 * Ic
    M[:, 8] = 0.7 * Ic
    M = np.array([project(m) for m in M])
    pmax = np.sqrt(Q * Q + U * U + V * V).max(axis=1)
    pol = np.full_like(Ic, np.nan)
    np.divide(pmax, Ic, out=pol, where=Ic > 0.0)
    return M, pol


def combined_init(obs, base, pol_threshold, x_mA, lambda0_A, cz_mA_per_G, default_model,
                  project):
    """obs [n, 4, n_obs], base [n, 10] -> (starting models [n, 10], polarisation
    level [n])."""
    S = np.asarray(obs, dtype=np.float64)
    finite = np.isfinite(S).all(axis=(1, 2))
    M = np.array(base, dtype=np.float64)
    pol = np.full(S.shape[0], np.nan)
    if finite.any():
        Mc, pc = classical_init(S[finite], x_mA, lambda0_A, cz_mA_per_G, default_model, project)
        pol[finite] = pc
        sub = M[finite]
        sub[:, 2] = Mc[:, 2]
        low = pc < pol_threshold  # False for a NaN level
        sub[low, 0:2] = Mc[low, 0:2]
        M[finite] = sub
    return np.array([project(m) for m in M]), pol
