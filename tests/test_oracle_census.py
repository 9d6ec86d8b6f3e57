"""The oracle's operation census (oracle/census.py), pinned to closed forms
and invariants: the counts of the damped solve against the textbook
operation counts of equilibration, Cholesky and the two substitutions
(Golub and Van Loan), chi^2 and the normal equations against their
definitions (Eqs. 1-4), the synthesis count's linearity in points and taps,
and the counting build's results against the plain oracle's (the counters
change no arithmetic)."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import census
import workloads as wl


def _solve_count(n_free, seed=0):
    L = census.census_lib()
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(10, 10))
    H = A @ A.T + 10 * np.eye(10)
    g = rng.normal(size=10)
    mask = (1 << n_free) - 1
    d = np.empty(10)
    census.take()
    code = L.orc_solve(oracle._d(np.ascontiguousarray(H)), oracle._d(g), 1e-3, mask,
                       oracle._d(d))
    assert code == 0
    return census.take()


@pytest.mark.parametrize("n", [1, 4, 10])
def test_solve_count_is_the_textbook_count(n):
    c = _solve_count(n)
    # equilibration: n reciprocals, one triangle of C at 2 products each,
    # the damped diagonal and the scaled gradient
    eq = n + n * (n + 1) + 2 * n
    # Cholesky: column j takes 2j for its diagonal and 2j + 1 per entry
    # below it: n(n-1) + (n-1)n(2n-1)/6 in closed form (leading term n^3/3)
    chol = n * (n - 1) + (n - 1) * n * (2 * n - 1) // 6
    subst = 2 * n * n  # two triangular solves: n^2 each, at 2 operations per entry
    assert c["solve"] == eq + chol + subst + n
    assert c["special"] == 2 * n  # n square roots in equilibration, n in Cholesky


def _forward_counts(inst, M, jac):
    L = census.census_lib()
    S = np.empty((4, inst.n_obs))
    J = np.empty((4, inst.n_obs, 10)) if jac else None
    census.take()
    L.orc_forward(ctypes.byref(inst.c), oracle._d(np.ascontiguousarray(M)), oracle._d(S),
                  oracle._d(J) if jac else None)
    return census.take(), S, J


def test_counting_build_computes_what_the_oracle_computes():
    spec = wl.hmi_instrument()
    pts, Fk, _ = census.support(spec)
    for voigt in (0, 2):
        inst = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA[pts], Fk,
                                 voigt=voigt)
        for M in wl.draw_params(4, 5):
            _, S, J = _forward_counts(inst, M, True)
            S0, J0 = oracle.forward(inst, M, jac=True)
            np.testing.assert_array_equal(S, S0)
            np.testing.assert_array_equal(J, J0)


def test_synthesis_count_is_linear_in_points_and_taps():
    """values = points * (per-point cost) + 8 * taps (a multiply-add per tap
    and Stokes parameter), with a per-point cost that does not depend on the
    instrument; three Voigt evaluations per point."""
    M = wl.draw_params(1, 9)[0]
    M[3] = 0.0  # no Doppler shift: every u stays inside the table's range
    fine = np.linspace(-300.0, 300.0, 41)
    per_point = set()
    for n_pts, n_obs in ((1, 1), (7, 2), (41, 6)):
        F = np.zeros((n_obs, n_pts))
        rng = np.random.default_rng(n_pts)
        F[rng.random((n_obs, n_pts)) < 0.6] = 1.0
        F[0, :] = 1.0  # every point read
        inst = oracle.Instrument(6173.3356, 2.5, fine[:n_pts], F, voigt=2)
        c, _, _ = _forward_counts(inst, M, False)
        taps = int((F != 0).sum())
        assert c["voigt_calls"] == 3 * n_pts
        assert (c["value"] - 8 * taps) % n_pts == 0
        per_point.add((c["value"] - 8 * taps) // n_pts)
        cj, _, _ = _forward_counts(inst, M, True)
        assert cj["value"] == c["value"]
        # derivatives: at most the 10 components of every value operation
        # (a product or quotient costs up to 3 per component)
        assert 0 < cj["gradient"] <= 30 * (cj["value"] + 11 * 3 * n_pts)
    assert len(per_point) == 1


def test_taylor_evaluation_count():
    """Second-order Taylor evaluation inside the table (Eqs. 12-13): locating
    the node (2 divisions, 2 products), alpha and beta (Eqs. 8-9), the two
    offsets, the first-order terms and the second-order terms."""
    L = census.census_lib()
    u = np.array([1.23])
    a = np.array([0.37])
    H, F = np.empty(1), np.empty(1)
    for order, expect in ((1, 2 + 2 + 6 + 5 + 2 + 4 + 4), (2, 2 + 2 + 6 + 5 + 2 + 4 + 4 + 22)):
        census.take()
        L.orc_voigt_taylor_batch(order, 1, oracle._d(u), oracle._d(a), oracle._d(H),
                                 oracle._d(F))
        assert census.take()["voigt"] == expect


def test_chi2_and_normal_equation_counts():
    """chi^2: a difference, a weighted square and a sum per residual row and
    the division by the degrees of freedom (Eq. 1).  Normal equations per row
    with every Jacobian entry non-zero: w r once, w J and a multiply-add into
    J^T W r per entry, one triangle (55 entries) of J^T W J at a multiply-add
    each: 1 + 10 * 3 + 55 * 2."""
    res = census.census(wl.hmi_instrument(), 4)
    rows = 24
    assert res["chi2"] == 4 * rows + 1
    assert 0 < res["normal_equations"] <= rows * (1 + 10 * 3 + 55 * 2)
    assert res["points"] == 59 and res["taps"] == 186


def test_committed_census_is_current():
    """The committed census record is what the script writes today."""
    import os
    path = os.path.join(census.ROOT, "profiles", "flop_census.md")
    with open(path) as fh:
        kv = dict(line.strip("- `\n").split(": ", 1) for line in fh if line.startswith("- `"))
    res = census.census(wl.hmi_instrument(), 64)
    for k in census.KEYS:
        assert abs(float(kv["hmi." + k]) - res[k]) <= 1e-3 * max(1.0, abs(res[k])), k
