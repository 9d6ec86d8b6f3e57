"""Pins of the oracle's Voigt / Faraday-Voigt functions (Sect. 3.2, Eqs. 8-11).

The oracle's w(z) is checked against library routines and closed forms that
do not share its algorithm: scipy's wofz (the MIT Faddeeva package), dawsn,
erfcx and mpmath's arbitrary-precision erfc.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import dawsn, erfcx, wofz

import oracle

A_VALUES = [0.0, 1e-10, 1e-6, 1e-3, 0.02, 0.1, 0.25, 0.5, 0.9, 1.0, 1.7, 2.5, 2.99,
            3.0, 3.01, 4.0, 5.0]


def _u_grid():
    return np.concatenate([np.linspace(-12.0, 12.0, 2401), np.linspace(-300.0, 300.0, 1201),
                           [-7.0, -6.9999, 7.0, 1.0, -1.0, 0.9999, 1e-8, -1e-8, 0.0]])


def test_against_scipy_wofz_grid():
    u = _u_grid()
    worst = 0.0
    for a in A_VALUES:
        H, F = oracle.faddeeva(u, a)
        ref = wofz(u + 1j * a)
        err = np.abs((H + 1j * F) - ref) / np.abs(ref)
        worst = max(worst, float(err.max()))
    # scipy's own accuracy is ~1e-14 at a few points; the oracle's is ~1e-15
    assert worst < 5e-14


@pytest.mark.parametrize("u,a", [(-7.84, 1e-8), (6.99, 0.0), (3.0, 0.0), (0.999, 0.0),
                                 (2.0, 2.9), (0.5, 3.01), (100.0, 0.1), (250.0, 5.0),
                                 (-4.29, 0.0), (1.5, 1.2), (5.5, 0.3), (0.0, 0.0)])
def test_against_mpmath(u, a):
    mpmath.mp.dps = 40
    z = mpmath.mpc(u, a)
    ref = complex(mpmath.exp(-z * z) * mpmath.erfc(-1j * z))
    H, F = oracle.faddeeva(np.array([u]), a)
    assert abs(complex(H[0], F[0]) - ref) / abs(ref) < 1e-14


def test_closed_forms():
    u = np.linspace(-20, 20, 4001)
    H, F = oracle.faddeeva(u, 0.0)
    # a = 0: H = exp(-u^2), F = (2/sqrt(pi)) Dawson(u)
    np.testing.assert_allclose(H, np.exp(-u * u), rtol=0, atol=5e-16)
    np.testing.assert_allclose(F, 2.0 / math.sqrt(math.pi) * dawsn(u), rtol=2e-14, atol=1e-300)
    # u = 0: H = erfcx(a), F = 0
    a = np.linspace(0.0, 5.0, 501)
    H0, F0 = oracle.faddeeva(np.zeros_like(a), a)
    np.testing.assert_allclose(H0, erfcx(a), rtol=1e-14)
    assert np.all(F0 == 0.0)
    # large |z| asymptote w ~ i / (sqrt(pi) z)
    z = 1e4 + 3.0j
    Hb, Fb = oracle.faddeeva(np.array([z.real]), z.imag)
    asym = 1j / (math.sqrt(math.pi) * z)
    assert abs(complex(Hb[0], Fb[0]) - asym) / abs(asym) < 1e-8


def test_symmetry_in_u():
    u = np.linspace(0.01, 40, 997)
    for a in (0.0, 0.3, 2.0):
        Hp, Fp = oracle.faddeeva(u, a)
        Hm, Fm = oracle.faddeeva(-u, a)
        np.testing.assert_array_equal(Hp, Hm)
        np.testing.assert_array_equal(Fp, -Fm)


def _fd(fun, x, h):
    return (fun(x + h) - fun(x - h)) / (2 * h)


@pytest.mark.parametrize("a", [0.05, 0.3, 1.0, 2.2])
def test_eq8_eq9_derivatives(a):
    """Eq. 8: dH/da = -dF/du = -2/sqrt(pi) + 2aH + 2uF;  Eq. 9: dH/du = dF/da = 2aF - 2uH."""
    u = np.linspace(-6, 6, 121)
    H, F = oracle.faddeeva(u, a)
    alpha = -2 / math.sqrt(math.pi) + 2 * a * H + 2 * u * F
    beta = 2 * a * F - 2 * u * H
    h = 1e-5
    dH_da = _fd(lambda x: oracle.faddeeva(u, x)[0], a, h)
    dF_da = _fd(lambda x: oracle.faddeeva(u, x)[1], a, h)
    dH_du = (oracle.faddeeva(u + h, a)[0] - oracle.faddeeva(u - h, a)[0]) / (2 * h)
    dF_du = (oracle.faddeeva(u + h, a)[1] - oracle.faddeeva(u - h, a)[1]) / (2 * h)
    for got, want in ((dH_da, alpha), (dF_du, -alpha), (dH_du, beta), (dF_da, beta)):
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


@pytest.mark.parametrize("a", [0.1, 0.8])
def test_eq10_eq11_second_derivatives(a):
    """Eqs. 10-11 (used by the paper's Taylor table)."""
    u = np.linspace(-5, 5, 51)
    H, F = oracle.faddeeva(u, a)
    al = -2 / math.sqrt(math.pi) + 2 * a * H + 2 * u * F
    be = 2 * a * F - 2 * u * H
    h = 1e-4

    def Hf(uu, aa):
        return oracle.faddeeva(uu, aa)[0]

    d2H_da2 = (Hf(u, a + h) - 2 * H + Hf(u, a - h)) / h ** 2
    d2H_du2 = (Hf(u + h, a) - 2 * H + Hf(u - h, a)) / h ** 2
    d2H_dadu = (Hf(u + h, a + h) - Hf(u + h, a - h) - Hf(u - h, a + h) + Hf(u - h, a - h)) / (4 * h * h)
    eq10 = 2 * H + 2 * a * al + 2 * u * be
    eq11 = 2 * F + 2 * a * be - 2 * u * al
    np.testing.assert_allclose(d2H_da2, eq10, atol=2e-6)
    np.testing.assert_allclose(-d2H_du2, eq10, atol=2e-6)
    np.testing.assert_allclose(d2H_dadu, eq11, atol=2e-6)
