"""Pins of the oracle's Milne-Eddington forward model and Jacobian.

What fixes each part:
* Eq. 7 coefficients printed in Sect. 3.1 (golden fixture);
* the Unno-Rachkovsky closed form against the formal solution of the
  polarised transfer equation for a constant propagation matrix and a linear
  source function, S0 e1 + S1 K^-1 e1, computed with numpy.linalg.solve;
* exact invariants of the model (B = 0, alpha = 0, eta0 = 0, S1 = 0, angle
  symmetries, Doppler shift by one grid step, far wings);
* the weak-field limit V -> -alpha C_Z cos(gamma) dI/dlambda;
* the analytic Jacobian against central finite differences;
* the filter step as a plain matrix product.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
C_KMS = 299792.458


@pytest.fixture(scope="module")
def hmi():
    s = wl.hmi_instrument()
    return oracle.Instrument(s.lambda0_A, s.geff, s.fine_offset_mA, s.filter)


def _single_point_inst(dlam_mA, lambda0=6173.3356, geff=2.5):
    fine = np.atleast_1d(np.asarray(dlam_mA, dtype=np.float64))
    return oracle.Instrument(lambda0, geff, fine, np.eye(fine.size))


def _model(**kw):
    M = wl.default_model().copy()
    names = ["B", "gamma", "psi", "v", "dld", "a", "eta0", "S0", "S1", "alpha"]
    for k, v in kw.items():
        M[names.index(k)] = v
    return M


def test_eq7_printed_coefficients():
    g = json.load(open(os.path.join(GOLD, "eq7_zeeman.json")))
    for line in g["lines"]:
        cz = oracle.zeeman_constant(line["lambda0_A"], line["geff"])
        assert round(cz, line["digits"]) == pytest.approx(line["printed"], abs=1e-12)
    fe = g["fe6173"]
    cz = oracle.zeeman_constant(fe["lambda0_A"], fe["geff"])
    assert abs(cz - fe["formula_value"]) < 5e-8


def _propagation_matrix_stokes(M, dlam, lambda0=6173.3356, geff=2.5):
    """Independent check of the radiative-transfer step: build the 4x4
    propagation matrix K from H, F and solve K x = e1 with LAPACK."""
    B, gd, pd, v, dld, a, eta0, S0, S1, alpha = M
    g, chi = math.radians(gd), math.radians(pd)
    cz = 4.66685e-10 * geff * lambda0 ** 2
    up = (dlam - lambda0 * 1e3 * v / C_KMS) / dld
    ub, ur = up + cz * B / dld, up - cz * B / dld
    (Hp, Hb, Hr), (Fp, Fb, Fr) = oracle.faddeeva(np.array([up, ub, ur]), a)
    half = eta0 / 2
    eI = 1 + half * (Hp * math.sin(g) ** 2 + 0.5 * (Hb + Hr) * (1 + math.cos(g) ** 2))
    eQ = half * (Hp - 0.5 * (Hb + Hr)) * math.sin(g) ** 2 * math.cos(2 * chi)
    eU = half * (Hp - 0.5 * (Hb + Hr)) * math.sin(g) ** 2 * math.sin(2 * chi)
    eV = half * (Hr - Hb) * math.cos(g)
    rQ = half * (Fp - 0.5 * (Fb + Fr)) * math.sin(g) ** 2 * math.cos(2 * chi)
    rU = half * (Fp - 0.5 * (Fb + Fr)) * math.sin(g) ** 2 * math.sin(2 * chi)
    rV = half * (Fr - Fb) * math.cos(g)
    K = np.array([[eI, eQ, eU, eV],
                  [eQ, eI, rV, -rU],
                  [eU, -rV, eI, rQ],
                  [eV, rU, -rQ, eI]])
    e1 = np.array([1.0, 0, 0, 0])
    mag = S0 * e1 + S1 * np.linalg.solve(K, e1)
    nonmag = S0 + S1 / (1 + eta0 * Hp)
    out = alpha * mag
    out[0] += (1 - alpha) * nonmag
    return out


def test_unno_rachkovsky_vs_formal_solution():
    P = wl.draw_params(40, 77)
    P[:5, 6] = 500.0  # strong lines exercise the magneto-optical terms
    for M in P:
        for dlam in (-250.0, -60.0, -10.0, 0.0, 35.0, 140.0):
            S = oracle.synth_fine(_single_point_inst(dlam), M, deriv=False)[:, 0]
            ref = _propagation_matrix_stokes(M, dlam)
            np.testing.assert_allclose(S, ref, rtol=0, atol=1e-13)


def test_field_free_and_trivial_limits():
    dl = np.linspace(-500, 500, 41)
    inst = _single_point_inst(dl)
    for M in (_model(B=0.0), _model(alpha=0.0)):
        S = oracle.synth_fine(inst, M, deriv=False)
        assert np.all(S[1:] == 0.0)
    M = _model(alpha=0.0)
    S = oracle.synth_fine(inst, M, deriv=False)
    H, _ = oracle.faddeeva((dl - 0.0) / M[4], M[5])
    np.testing.assert_allclose(S[0], M[7] + M[8] / (1 + M[6] * H), rtol=1e-15)
    S = oracle.synth_fine(inst, _model(eta0=0.0), deriv=False)
    np.testing.assert_allclose(S[0], 0.3 + 0.7, rtol=1e-15)
    assert np.all(S[1:] == 0.0)
    S = oracle.synth_fine(inst, _model(S1=0.0), deriv=False)
    np.testing.assert_allclose(S[0], 0.3, rtol=1e-15)
    # far wings: continuum
    far = _single_point_inst([-1e6, 1e6])
    S = oracle.synth_fine(far, _model(B=2500.0, gamma=30.0), deriv=False)
    np.testing.assert_allclose(S[0], 1.0, atol=1e-9)
    assert np.all(np.abs(S[1:]) < 1e-9)
    # line centre, B = 0: I = S0 + S1 / (1 + eta0 erfcx(a))
    from scipy.special import erfcx
    c = _single_point_inst([0.0])
    for a in (0.0, 0.2, 1.3):
        M = _model(B=0.0, v=0.0, a=a, alpha=0.8)
        S = oracle.synth_fine(c, M, deriv=False)
        assert S[0, 0] == pytest.approx(M[7] + M[8] / (1 + M[6] * erfcx(a)), rel=1e-14)


def test_angle_invariants():
    dl = np.linspace(-400, 400, 33)
    inst = _single_point_inst(dl)
    base = dict(B=1800.0, v=0.7, a=0.3, eta0=12.0, alpha=0.7)
    S = oracle.synth_fine(inst, _model(gamma=0.0, psi=40.0, **base), deriv=False)
    assert np.max(np.abs(S[1:3])) < 1e-15
    S = oracle.synth_fine(inst, _model(gamma=90.0, psi=40.0, **base), deriv=False)
    assert np.max(np.abs(S[3])) < 1e-15
    S = oracle.synth_fine(inst, _model(gamma=90.0, psi=0.0, **base), deriv=False)
    assert np.max(np.abs(S[2])) < 1e-15
    # psi + theta rotates Q + iU by exp(2 i theta); psi + 180 changes nothing
    g, p, th = 63.0, 25.0, 37.0
    S1 = oracle.synth_fine(inst, _model(gamma=g, psi=p, **base), deriv=False)
    S2 = oracle.synth_fine(inst, _model(gamma=g, psi=p + th, **base), deriv=False)
    rot = (S1[1] + 1j * S1[2]) * np.exp(2j * math.radians(th))
    np.testing.assert_allclose(S2[1] + 1j * S2[2], rot, atol=1e-14)
    np.testing.assert_allclose(S2[[0, 3]], S1[[0, 3]], atol=1e-14)
    S3 = oracle.synth_fine(inst, _model(gamma=g, psi=p + 180.0, **base), deriv=False)
    np.testing.assert_allclose(S3, S1, atol=1e-14)
    # (gamma, psi) -> (180 - gamma, 180 - psi) maps (I,Q,U,V) -> (I,Q,-U,-V)
    S4 = oracle.synth_fine(inst, _model(gamma=180 - g, psi=180 - p, **base), deriv=False)
    np.testing.assert_allclose(S4, S1 * np.array([1, 1, -1, -1])[:, None], atol=1e-14)
    # gamma -> 180 - gamma keeps I and negates V
    S5 = oracle.synth_fine(inst, _model(gamma=180 - g, psi=p, **base), deriv=False)
    np.testing.assert_allclose(S5[0], S1[0], atol=1e-14)
    np.testing.assert_allclose(S5[3], -S1[3], atol=1e-14)
    # (-B, gamma) == (B, 180 - gamma)
    bneg = dict(base)
    bneg["B"] = -base["B"]
    S6 = oracle.synth_fine(inst, _model(gamma=g, psi=p, **bneg), deriv=False)
    np.testing.assert_allclose(S6, S5, atol=1e-14)


def test_doppler_shift_by_one_grid_step():
    """v = c * 12 mA / lambda0 moves the unfiltered profiles by exactly one
    12 mA grid step toward the red."""
    s = wl.hmi_instrument()
    inst = oracle.Instrument(s.lambda0_A, s.geff, s.fine_offset_mA, s.filter)
    v1 = C_KMS * 12.0 / (s.lambda0_A * 1e3)
    M0 = _model(B=1300.0, gamma=50.0, psi=20.0, v=0.0)
    M1 = _model(B=1300.0, gamma=50.0, psi=20.0, v=v1)
    S0 = oracle.synth_fine(inst, M0, deriv=False)
    S1 = oracle.synth_fine(inst, M1, deriv=False)
    np.testing.assert_allclose(S1[:, 1:], S0[:, :-1], atol=1e-13)


def test_weak_field_limit():
    """V / B -> -alpha C_Z cos(gamma) dI/dlambda, dI/dlambda = -(c/lambda0) dI/dv."""
    dl = np.linspace(-300, 300, 61)
    inst = _single_point_inst(dl)
    cz = 4.66685e-10 * 2.5 * 6173.3356 ** 2
    errs = []
    for B in (1.0, 0.5):
        M = _model(B=B, gamma=35.0, psi=10.0, v=0.4, alpha=0.65)
        S, dS = oracle.synth_fine(inst, M)
        dI_dlam = -(C_KMS / (6173.3356 * 1e3)) * dS[0, :, 3]
        pred = -M[9] * cz * math.cos(math.radians(35.0)) * dI_dlam * B
        errs.append(np.max(np.abs(S[3] - pred)) / np.max(np.abs(pred)))
    assert errs[0] < 2e-6 and errs[1] < 6e-7
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)  # error ~ B^2
    # Q ~ B^2 to leading order; the magneto-optical cross terms add a
    # relative O(B) correction, so the deviation of Q(2B)/Q(B) from 4 falls
    # linearly with B
    dev = []
    for B in (1.0, 0.1):
        Sa = oracle.synth_fine(inst, _model(B=B, gamma=60.0, psi=30.0), deriv=False)
        Sb = oracle.synth_fine(inst, _model(B=2 * B, gamma=60.0, psi=30.0), deriv=False)
        k = np.argmax(np.abs(Sa[1]))
        dev.append(abs(Sb[1, k] / Sa[1, k] - 4.0))
    assert dev[1] < 1e-3
    assert dev[0] / dev[1] == pytest.approx(10.0, rel=0.05)


@pytest.mark.parametrize("seed", [3, 4])
def test_jacobian_vs_finite_differences(hmi, seed):
    P = wl.draw_params(8, seed)
    P[0, 0] = 4000.0
    P[1, 6] = 300.0
    for M in P:
        S, J = oracle.forward(hmi, M, jac=True)
        for p in range(10):
            h = 1e-6 * max(abs(M[p]), 1.0)
            Mp, Mm = M.copy(), M.copy()
            Mp[p] += h
            Mm[p] -= h
            fd = (oracle.forward(hmi, Mp) - oracle.forward(hmi, Mm)) / (2 * h)
            scale = max(np.max(np.abs(J[:, :, p])), 1e-300)
            assert np.max(np.abs(fd - J[:, :, p])) / scale < 1e-6, (p, M)


def test_filter_is_matrix_product(hmi):
    s = wl.hmi_instrument()
    np.testing.assert_allclose(s.filter.sum(axis=1), 1.0, rtol=1e-15)
    # rows with mirrored centres are mirror images
    np.testing.assert_allclose(s.filter[0], s.filter[5][::-1], rtol=1e-13)
    M = wl.draw_params(1, 9)[0]
    Sf, dSf = oracle.synth_fine(hmi, M)
    S, J = oracle.forward(hmi, M, jac=True)
    np.testing.assert_allclose(S, Sf @ s.filter.T, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(J, np.einsum("ik,skp->sip", s.filter, dSf), rtol=1e-12, atol=1e-16)
