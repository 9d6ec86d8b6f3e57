"""Seeded synthetic inputs for the Milne-Eddington inversion.

This module only draws random numbers and lays out instrument descriptions;
it holds none of the inversion's arithmetic (no Voigt functions, no
absorption matrix, no radiative transfer, no fitting).  Both the GPU path
and the CPU oracle take their inputs from here.

Workloads (the paper's Hinode/HMI data are not available, so every input is
synthetic; shapes follow the paper's HMI set-up of Sect. 1 and Sect. 5):

* ``hmi``: Fe I 6173.3356 A, g_eff 2.5 (Table 1), synthesis on 101 points
  spanning +-600 mA, observed through 6 Gaussian filters (FWHM 76 mA) centred
  at +-34.4, +-103.2, +-172 mA, each row normalised to unit sum.
* ``fine``: Fe I 6302.4936 A (Sect. 3.1), 112 samples at 21.5 mA (the Hinode
  sampling of Sect. 4.1) seen through a 25 mA-FWHM Gaussian instrumental
  profile; synthesis on a x4 grid padded by 8 points per side (464 points),
  15-tap rows.

Full disk: the pixels of a 4096 x 4096 image inside the disk of
centre (2047.5, 2047.5) and radius 2048 (13,176,792 pixels, row-major), 80%
quiet (B ~ U[0,200] G) and 20% active (B ~ U[500,3500] G); active pixels are
a seeded union of random discs (spatially clustered load), or i.i.d. in the
variant; the other parameters follow the synthetic priors.

Parameter priors (every workload): B ~ U[0,3000] G, cos(gamma) ~ U[-1,1],
psi ~ U[0,180) deg, v ~ U[-3,3] km/s, Doppler width ~ U[20,50] mA,
a ~ U[0,0.5], eta0 ~ U[1,30], S0 ~ U[0.1,0.5], S1 = 1 - S0,
alpha ~ U[0.2,1].  Noise: N(0, 1e-3) added to every observed sample.
"""
from dataclasses import dataclass

import numpy as np

NPAR = 10
FWHM_TO_SIGMA = 1.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)))

# Sizes and seeds of the workloads.
CONFIGS = {
    "hmi_64x64": dict(n=64 * 64, seed=1000),
    "hmi_512x512": dict(n=512 * 512, seed=1001),
    "full_disk": dict(grid=4096, seed=1002),
    "learned_train": dict(n=10_000_000, seed=1003),
    "learned_control": dict(n=250_000, seed=1103),
    "learned_heldout": dict(n=1_000_000, seed=2003),
    "mixed_fine": dict(n=1_000_000, seed=1004),
    "mixed_hmi": dict(n=1_000_000, seed=1104),
}


@dataclass
class InstrumentSpec:
    name: str
    lambda0_A: float
    geff: float
    fine_offset_mA: np.ndarray  # [n_fine]
    filter: np.ndarray          # [n_obs, n_fine]
    obs_offset_mA: np.ndarray   # [n_obs] nominal centres

    @property
    def n_fine(self):
        return self.fine_offset_mA.shape[0]

    @property
    def n_obs(self):
        return self.filter.shape[0]


def hmi_instrument(n_fine=101, span_mA=600.0, fwhm_mA=76.0,
                   centres_mA=(-172.0, -103.2, -34.4, 34.4, 103.2, 172.0)):
    fine = np.linspace(-span_mA, span_mA, n_fine)
    sig = fwhm_mA * FWHM_TO_SIGMA
    c = np.asarray(centres_mA, dtype=np.float64)
    F = np.exp(-0.5 * ((fine[None, :] - c[:, None]) / sig) ** 2)
    F /= F.sum(axis=1, keepdims=True)
    return InstrumentSpec("hmi", 6173.3356, 2.5, fine, F, c)


def fine_instrument(n_obs=112, step_mA=21.5, oversample=4, pad=8, fwhm_mA=25.0, half_taps=7):
    obs = (np.arange(n_obs) - (n_obs - 1) / 2.0) * step_mA
    h = step_mA / oversample
    n_fine = n_obs * oversample + 2 * pad
    fine = obs[0] + (np.arange(n_fine) - pad) * h
    sig = fwhm_mA * FWHM_TO_SIGMA
    F = np.zeros((n_obs, n_fine))
    for j in range(n_obs):
        k0 = pad + oversample * j
        ks = np.arange(k0 - half_taps, k0 + half_taps + 1)
        w = np.exp(-0.5 * ((fine[ks] - obs[j]) / sig) ** 2)
        F[j, ks] = w / w.sum()
    return InstrumentSpec("fine", 6302.4936, 2.5, fine, F, obs)


def draw_params(n, seed, b_range=None):
    """[n, 10] float64 parameter vectors in API units."""
    rng = np.random.default_rng(seed)
    P = np.empty((n, NPAR))
    lo, hi = (0.0, 3000.0) if b_range is None else b_range
    P[:, 0] = rng.uniform(lo, hi, n)
    P[:, 1] = np.degrees(np.arccos(rng.uniform(-1.0, 1.0, n)))
    P[:, 2] = rng.uniform(0.0, 180.0, n)
    P[:, 3] = rng.uniform(-3.0, 3.0, n)
    P[:, 4] = rng.uniform(20.0, 50.0, n)
    P[:, 5] = rng.uniform(0.0, 0.5, n)
    P[:, 6] = rng.uniform(1.0, 30.0, n)
    P[:, 7] = rng.uniform(0.1, 0.5, n)
    P[:, 8] = 1.0 - P[:, 7]
    P[:, 9] = rng.uniform(0.2, 1.0, n)
    return P


def draw_noise(n, n_obs, seed, sigma=1e-3):
    """[n, 4, n_obs] float64 Gaussian noise (stream separate from params)."""
    rng = np.random.default_rng([*np.atleast_1d(seed).tolist(), 7])
    return rng.normal(0.0, sigma, size=(n, 4, n_obs))


def weights(n_obs, sigma=1e-3, w=(1.0, 1.0, 1.0, 1.0)):
    """[4, n_obs] float32 W = w^2 / sigma^2 (Eq. 1)."""
    W = np.empty((4, n_obs), np.float32)
    for s in range(4):
        W[s, :] = (w[s] ** 2) / sigma ** 2
    return W


def default_model():
    """The plain-LM starting model: midpoints of the synthetic priors."""
    return np.array([1500.0, 90.0, 90.0, 0.0, 35.0, 0.25, 15.5, 0.3, 0.7, 0.6])


def disk_mask(grid=4096):
    """Boolean [grid, grid] solar-disk mask centred on the grid, radius grid/2."""
    c = (grid - 1) / 2.0
    y, x = np.mgrid[0:grid, 0:grid]
    return (x - c) ** 2 + (y - c) ** 2 <= (grid / 2.0) ** 2


def disk_mu(grid=4096):
    """mu = cos(heliocentric angle) of each disk pixel, in the disk's
    row-major order: sqrt(1 - rho^2), rho the distance from the centre over
    the radius grid/2."""
    c = (grid - 1) / 2.0
    y, x = np.mgrid[0:grid, 0:grid]
    rho2 = ((x - c) ** 2 + (y - c) ** 2) / (grid / 2.0) ** 2
    return np.sqrt(np.clip(1.0 - rho2[disk_mask(grid)], 0.0, 1.0))


def full_disk(grid=4096, seed=1002, clustered=True, active_frac=0.2, r_range=(16.0, 128.0)):
    """Config-2 parameters.  Returns (P [n, 10] float64 in disk row-major
    order, active [n] bool, mask [grid, grid] bool).

    Clustered: discs with centres uniform over the bounding square and radii
    ~ U[r_range] are added until the active pixels cover at least
    active_frac of the disk.  I.i.d.: each disk pixel is active with
    probability active_frac."""
    mask = disk_mask(grid)
    n = int(mask.sum())
    rng = np.random.default_rng([seed, 11])
    if clustered:
        img = np.zeros((grid, grid), dtype=bool)
        target = active_frac * n
        covered = 0
        while covered < target:
            cx, cy = rng.uniform(0.0, grid, 2)
            r = rng.uniform(*r_range)
            x0, x1 = max(int(cx - r), 0), min(int(cx + r) + 2, grid)
            y0, y1 = max(int(cy - r), 0), min(int(cy + r) + 2, grid)
            if x0 >= x1 or y0 >= y1:
                continue
            yy, xx = np.mgrid[y0:y1, x0:x1]
            disc = (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
            sub = img[y0:y1, x0:x1]
            covered += int((disc & ~sub & mask[y0:y1, x0:x1]).sum())
            sub |= disc
        active = img[mask]
    else:
        active = rng.random(n) < active_frac
    P = draw_params(n, seed)
    quiet_B = rng.uniform(0.0, 200.0, n)
    active_B = rng.uniform(500.0, 3500.0, n)
    P[:, 0] = np.where(active, active_B, quiet_B)
    return P, active, mask
