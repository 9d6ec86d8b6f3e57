"""Pins of the oracle's classical initial guess (Sect. 5: weak-field /
magnetograph B and gamma, linear-polarisation azimuth, line position)."""
import numpy as np
import pytest

import oracle
from oracle import classical
import workloads as wl


@pytest.fixture(scope="module")
def hmi():
    spec = wl.hmi_instrument()
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    x = classical.sample_offsets(spec.filter, spec.fine_offset_mA)
    cz = oracle.zeeman_constant(spec.lambda0_A, spec.geff)
    return spec, oi, x, cz


def _init(spec, oi, x, cz, P):
    obs = oracle.forward_batch(oi, np.atleast_2d(P))
    return classical.classical_init(obs, x, spec.lambda0_A, cz, wl.default_model(),
                                    oracle.project)


def test_sample_offsets_are_the_filter_centres(hmi):
    spec, oi, x, cz = hmi
    np.testing.assert_allclose(x, [-172.0, -103.2, -34.4, 34.4, 103.2, 172.0], atol=1e-9)


def test_field_free_and_unshifted_lines(hmi):
    spec, oi, x, cz = hmi
    M = np.array([0.0, 40.0, 70.0, 0.0, 30.0, 0.2, 10.0, 0.25, 0.75, 0.8])
    M0, pol = _init(spec, oi, x, cz, M)
    assert M0[0, 0] == 0.0 and pol[0] == 0.0
    assert abs(M0[0, 3]) < 1e-9  # symmetric line on symmetric samples
    # the outermost HMI samples lie in the line wing: the continuum estimate
    # (largest observed I) is a little below the true S0 + S1 = 1
    assert 0.9 < M0[0, 7] + M0[0, 8] < 1.0


def test_velocity_sign_and_scale(hmi):
    spec, oi, x, cz = hmi
    P = np.tile([0.0, 40.0, 70.0, 0.0, 30.0, 0.2, 10.0, 0.25, 0.75, 0.8], (5, 1))
    P[:, 3] = [-2.0, -1.0, 0.0, 1.0, 2.0]
    v = _init(spec, oi, x, cz, P)[0][:, 3]
    assert np.all(np.diff(v) > 0) and np.all(np.sign(v[[0, 1, 3, 4]]) == [-1, -1, 1, 1])
    np.testing.assert_allclose(v, P[:, 3], atol=0.4)


def test_azimuth_rotates_with_the_model(hmi):
    """Q and U turn by 2 delta when psi turns by delta: the estimate turns by
    delta and the field strengths do not change."""
    spec, oi, x, cz = hmi
    base = np.array([600.0, 70.0, 20.0, 0.3, 30.0, 0.2, 12.0, 0.3, 0.7, 0.9])
    for delta in (13.0, 47.0, 101.0):
        m = base.copy()
        m[2] += delta
        a, _ = _init(spec, oi, x, cz, base)
        b, _ = _init(spec, oi, x, cz, m)
        d = (b[0, 2] - a[0, 2] - delta) % 180.0
        assert min(d, 180.0 - d) < 1e-6
        np.testing.assert_allclose(b[0, [0, 1, 3]], a[0, [0, 1, 3]], rtol=1e-9)


@pytest.mark.parametrize("which", ["hmi", "fine"])
def test_azimuth_exact_for_transverse_fields(which):
    """gamma = 90 deg: no Faraday rotation, so Q and U are one profile times
    cos 2 psi and sin 2 psi; the estimate is psi at any field strength and
    line shift, including fields whose sigma components lie outside the
    line core (where Q changes sign across the line)."""
    spec = wl.hmi_instrument() if which == "hmi" else wl.fine_instrument()
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    x = classical.sample_offsets(spec.filter, spec.fine_offset_mA)
    cz = oracle.zeeman_constant(spec.lambda0_A, spec.geff)
    rows = [[B, 90.0, psi, v, 30.0, 0.2, 12.0, 0.3, 0.7, 1.0]
            for B in (50.0, 300.0, 1500.0, 3500.0) for v in (-2.0, 0.0, 1.5)
            for psi in (10.0, 75.0, 140.0)]
    P = np.array(rows)
    M0, _ = _init(spec, oi, x, cz, P)
    d = (M0[:, 2] - P[:, 2] + 90.0) % 180.0 - 90.0
    assert np.abs(d).max() < 1e-6, np.abs(d).max()


def test_inclination_mirrors(hmi):
    spec, oi, x, cz = hmi
    a, _ = _init(spec, oi, x, cz, [300.0, 35.0, 50.0, 0.0, 30.0, 0.2, 12.0, 0.3, 0.7, 0.9])
    b, _ = _init(spec, oi, x, cz, [300.0, 145.0, 50.0, 0.0, 30.0, 0.2, 12.0, 0.3, 0.7, 0.9])
    assert a[0, 1] == pytest.approx(180.0 - b[0, 1], abs=1e-6)
    assert a[0, 0] == pytest.approx(b[0, 0], rel=1e-9)


def test_weak_field_recovery_and_linearity(hmi):
    """Weak longitudinal fields: the estimate of the flux density alpha B cos
    gamma is linear in B, and exact up to the finite differences across the
    68.8 mA sample spacing: within 5% for a line the samples resolve (Doppler
    width 45 mA), with the error shrinking as the line widens."""
    spec, oi, x, cz = hmi

    def flux(B, dld):
        M, _ = _init(spec, oi, x, cz, [B, 0.0, 0.0, 0.0, dld, 0.2, 12.0, 0.3, 0.7, 1.0])
        return M[0, 0] * np.cos(np.radians(M[0, 1])) * classical.ALPHA0

    out = np.array([flux(B, 30.0) for B in (10.0, 20.0, 40.0)])
    np.testing.assert_allclose(out / out[0], [1.0, 2.0, 4.0], rtol=2e-3)
    assert flux(20.0, 45.0) == pytest.approx(20.0, rel=0.05)
    err = [abs(flux(20.0, w) / 20.0 - 1.0) for w in (20.0, 30.0, 45.0)]
    assert err[0] > err[1] > err[2]


def _mixed_set(spec, oi, n=24, seed=5):
    """Weak and strong polarisation in one set: one atmosphere with fields
    from 0 to 2000 G (the level rises with the field over this range)."""
    P = np.tile([0.0, 60.0, 30.0, 0.2, 30.0, 0.2, 10.0, 0.3, 0.7, 0.8], (n, 1))
    P[:, 0] = np.linspace(0.0, 2000.0, n)
    return P, oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, seed)


def test_combined_threshold_extremes(hmi):
    """Threshold 0: only the azimuth comes from the classical estimate;
    threshold +inf: B, gamma and azimuth do; the rest is always the base."""
    spec, oi, x, cz = hmi
    P, obs = _mixed_set(spec, oi)
    base = wl.draw_params(len(P), 77)
    cls, pol = classical.classical_init(obs, x, spec.lambda0_A, cz, wl.default_model(),
                                        oracle.project)
    args = (x, spec.lambda0_A, cz, wl.default_model(), oracle.project)
    m0, p0 = classical.combined_init(obs, base, 0.0, *args)
    np.testing.assert_array_equal(p0, pol)
    keep = [0, 1, 3, 4, 5, 6, 7, 8, 9]
    proj = np.array([oracle.project(b) for b in base])
    np.testing.assert_array_equal(m0[:, keep], proj[:, keep])
    np.testing.assert_array_equal(m0[:, 2], cls[:, 2])
    mi, _ = classical.combined_init(obs, base, np.inf, *args)
    np.testing.assert_array_equal(mi[:, :3], cls[:, :3])
    np.testing.assert_array_equal(mi[:, 3:], proj[:, 3:])


def test_combined_threshold_splits_by_polarisation(hmi):
    spec, oi, x, cz = hmi
    P, obs = _mixed_set(spec, oi)
    base = wl.draw_params(len(P), 78)
    cls, pol = classical.classical_init(obs, x, spec.lambda0_A, cz, wl.default_model(),
                                        oracle.project)
    thr = float(np.median(pol))
    low = pol < thr
    assert 0 < low.sum() < len(P)
    m, _ = classical.combined_init(obs, base, thr, x, spec.lambda0_A, cz, wl.default_model(),
                                   oracle.project)
    proj = np.array([oracle.project(b) for b in base])
    np.testing.assert_array_equal(m[low, :2], cls[low, :2])
    np.testing.assert_array_equal(m[~low, :2], proj[~low, :2])
    # the weakest fields are the ones taken from the weak-field estimate
    assert np.all(np.diff(pol) > 0) and low[:4].all() and not low[-4:].any()


def test_combined_non_finite_and_dark_pixels(hmi):
    """Non-finite samples keep the base model; a non-positive continuum has
    no polarisation level (NaN), so B and gamma stay the base's."""
    spec, oi, x, cz = hmi
    P, obs = _mixed_set(spec, oi, n=4)
    obs[1, 2, 3] = np.nan
    obs[2] = -np.abs(obs[2])
    base = wl.draw_params(4, 79)
    m, pol = classical.combined_init(obs, base, np.inf, x, spec.lambda0_A, cz,
                                     wl.default_model(), oracle.project)
    proj = np.array([oracle.project(b) for b in base])
    np.testing.assert_array_equal(m[1], proj[1])
    assert np.isnan(pol[1]) and np.isnan(pol[2]) and np.isfinite(pol[[0, 3]]).all()
    np.testing.assert_array_equal(m[2, :2], proj[2, :2])
