"""Pins of the oracle's Taylor-table Voigt evaluation (Sect. 3.2, Eqs. 10-13;
table 500 u x 100 a at steps of 0.05, as the paper sizes it)."""
import numpy as np
import pytest
from scipy.special import wofz

import oracle
import workloads as wl

STEP = 0.05


def test_nodes_are_the_faddeeva_function():
    rng = np.random.default_rng(3)
    for _ in range(50):
        i, j = int(rng.integers(0, 500)), int(rng.integers(0, 100))
        h, f = oracle.voigt_table_node(i, j)
        w = wofz(STEP * i + 1j * STEP * j)
        assert abs(h - w.real) < 1e-13 and abs(f - w.imag) < 1e-13
        for order in (1, 2):  # at a node the expansion returns the node
            H, F = oracle.voigt_taylor(order, np.array([STEP * i, -STEP * i]), STEP * j)
            assert H[0] == h and F[0] == f and H[1] == h and F[1] == -f


def test_second_derivatives_of_eqs_10_11():
    """The expansion's second-order coefficients are the second derivatives
    of H and F (Eqs. 10-11), checked on the exact function by differences."""
    rng = np.random.default_rng(4)
    e = 1e-3
    for _ in range(20):
        u, a = rng.uniform(-6, 6), rng.uniform(0.05, 3)
        w = lambda du, da: wofz((u + du) + 1j * (a + da))
        H, F = w(0, 0).real, w(0, 0).imag
        al = -2 / np.sqrt(np.pi) + 2 * a * H + 2 * u * F
        be = 2 * a * F - 2 * u * H
        P, Q = H + a * al + u * be, F + a * be - u * al
        Haa = (w(0, e).real - 2 * H + w(0, -e).real) / e ** 2
        Huu = (w(e, 0).real - 2 * H + w(-e, 0).real) / e ** 2
        Hau = (w(e, e).real - w(e, -e).real - w(-e, e).real + w(-e, -e).real) / (4 * e * e)
        Faa = (w(0, e).imag - 2 * F + w(0, -e).imag) / e ** 2
        assert Haa == pytest.approx(2 * P, abs=2e-5) and Huu == pytest.approx(-2 * P, abs=2e-5)
        assert Faa == pytest.approx(2 * Q, abs=2e-5) and Hau == pytest.approx(2 * Q, abs=2e-5)


def test_error_falls_with_the_order_of_the_expansion():
    """Off a node by d along u: the error of order k shrinks as d^(k+1)
    (a dropped or mis-signed term would change the ratio)."""
    u0, a0 = 40 * STEP, 20 * STEP
    for order, ratio in ((1, 4.0), (2, 8.0)):
        errs = []
        for d in (0.02, 0.01):
            H, F = oracle.voigt_taylor(order, np.array([u0 + d]), a0)
            w = wofz(u0 + d + 1j * a0)
            errs.append(abs(H[0] - w.real) + abs(F[0] - w.imag))
        assert errs[0] / errs[1] == pytest.approx(ratio, rel=0.15), (order, errs)


def test_figure_2_claim_first_order_below_1e4_at_a_1():
    """Fig. 2: at a = 1, over 1e6 frequencies, the first-order expansion
    stays within 1e-4 of the Voigt function (second order far below)."""
    u = np.linspace(-24.97, 24.97, 1_000_000)
    w = wofz(u + 1j)
    H1, F1 = oracle.voigt_taylor(1, u, 1.0)
    H2, F2 = oracle.voigt_taylor(2, u, 1.0)
    assert np.abs(H1 - w.real).max() < 1e-4
    assert np.abs(H2 - w.real).max() < 2e-6 and np.abs(F2 - w.imag).max() < 2e-6


def test_beyond_the_table_the_asymptotic_series():
    u = np.concatenate([np.linspace(24.98, 200, 500), -np.linspace(24.98, 200, 500)])
    a = np.random.default_rng(5).uniform(0, 5, u.size)
    H, F = oracle.voigt_taylor(2, u, a)
    w = wofz(u + 1j * a)
    assert np.max(np.abs(H - w.real) / np.abs(w.real)) < 1e-7
    assert np.max(np.abs(F - w.imag) / np.abs(w.imag)) < 1e-8


def test_synthesis_through_the_table_stays_close():
    """Whole forward model with the second-order table: within 1e-4 of the
    exact synthesis (the paper's accuracy claim carried to Stokes)."""
    spec = wl.hmi_instrument()
    ex = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    t2 = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter, voigt=2)
    t1 = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter, voigt=1)
    P = wl.draw_params(300, 6)
    Se, S2, S1 = (oracle.forward_batch(i, P) for i in (ex, t2, t1))
    assert np.abs(S2 - Se).max() < 1e-4
    assert np.abs(S2 - Se).max() < np.abs(S1 - Se).max()
