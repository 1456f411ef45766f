"""Pins of the oracle's species + T point-implicit Jacobian (the variant of Eq. 4.12 in
which T is not frozen but follows the composition at fixed density and internal energy,
as it does through the Newton solve of Sec. 4.2).

* it equals central differences of S(rho Y, T(rho Y)) with T re-solved by bisection-
  checked Newton at fixed e (an independent route: no dual numbers);
* it differs from the frozen-T Jacobian by a rank-one term (dS/dT)(dT/d rho Y)^T;
* element totals stay linear invariants (l^T J = 0), so a run conserves them;
* on one step it differs from the frozen-T variant by O(dt^2), one order above the step.
"""

import math

import numpy as np
import pytest

from cases import synthetic_mechanism, two_range_mechanism, BC_PERIODIC
from cases.amr import detailed_front_case


@pytest.fixture(scope="module", params=["one-range", "two-range"])
def mech(request):
    m = synthetic_mechanism()
    return m if request.param == "one-range" else two_range_mechanism(m, t_mid=1800.0)


def _state(mech, T, seed):
    rng = np.random.default_rng(seed)
    Y = rng.dirichlet(np.ones(mech.ns))
    rho = 1.7
    return rho, Y, rho * Y[:-1]


@pytest.mark.parametrize("T0", [1500.0, 2600.0])
def test_full_jacobian_matches_central_differences(oracle, mech, T0):
    rho, Y, rhoY = _state(mech, T0, 4)
    e, _ = oracle.mixture_e_cv(mech, Y, T0)
    J = oracle.full_jacobian(mech, rho, e, T0, rhoY)

    def S(ry):
        Yp = np.append(ry / rho, 1.0 - ry.sum() / rho)
        T = oracle.temperature(mech, Yp, e, T0)
        return oracle.production(mech, rho, T, ry)[:-1]

    scale = np.max(np.abs(J))
    for m in range(mech.ns - 1):
        h = 1e-6 * rho
        d = np.zeros_like(rhoY)
        d[m] = h
        fd = (S(rhoY + d) - S(rhoY - d)) / (2 * h)
        assert np.max(np.abs(fd - J[:, m])) <= 2e-6 * scale, m


def test_rank_one_difference_from_frozen(oracle, mech):
    rho, Y, rhoY = _state(mech, 2200.0, 9)
    e, _ = oracle.mixture_e_cv(mech, Y, 2200.0)
    Jf = oracle.full_jacobian(mech, rho, e, 2200.0, rhoY)
    _, J0 = oracle.production(mech, rho, 2200.0, rhoY, jacobian=True)
    sv = np.linalg.svd(Jf - J0, compute_uv=False)
    assert sv[0] > 1e-6 * np.max(np.abs(J0))
    assert sv[1] <= 1e-10 * sv[0]


def test_elements_are_invariants(oracle, mech):
    rho, Y, rhoY = _state(mech, 2400.0, 5)
    e, _ = oracle.mixture_e_cv(mech, Y, 2400.0)
    J = oracle.full_jacobian(mech, rho, e, 2400.0, rhoY)
    nt = mech.ns - 1
    L = mech.comp[:nt].T / mech.M[:nt] - mech.comp[nt][:, None] / mech.M[nt]
    assert np.max(np.abs(L @ J)) <= 1e-13 * np.max(np.abs(L)) * np.max(np.abs(J))


def test_run_conserves_and_differs_by_second_order(oracle):
    mech = synthetic_mechanism()
    c = detailed_front_case(nx=24, ny=16, mech=mech)
    c.bc = [BC_PERIODIC] * 4
    U0, T0 = oracle.case_state(c)
    U, _, _, _, _ = oracle.step(c, U0, T0, 3, full_jacobian=True)
    nt = mech.ns - 1

    def elements(Uc):
        rhoY = Uc[4:].reshape(nt, -1)
        rho = Uc[0].ravel()
        X = np.vstack([rhoY / mech.M[:nt, None], (rho - rhoY.sum(0))[None, :] / mech.M[nt]])
        return np.array([math.fsum((mech.comp[:, e] @ X).ravel()) for e in range(mech.comp.shape[1])])

    assert np.max(np.abs(elements(U) - elements(U0)) / elements(U0)) <= 1e-13
    c2 = detailed_front_case(nx=32, ny=8, mech=mech)
    V0, S0 = oracle.case_state(c2)
    diffs = []
    for dt in [2e-9, 1e-9, 5e-10]:
        a = oracle.step(c2, V0, S0, 1, dt_fixed=dt)[0]
        b = oracle.step(c2, V0, S0, 1, dt_fixed=dt, full_jacobian=True)[0]
        diffs.append(np.max(np.abs(a[4:] - b[4:])))
        assert np.max(np.abs(a[4:] - V0[4:])) > 1e3 * diffs[-1]
    for x, y in zip(diffs[:-1], diffs[1:]):
        assert 3.5 < x / y < 4.5, diffs


def test_full_jacobian_needs_chemistry(oracle):
    from cases import detonation_tube_case
    c = detonation_tube_case(nx=16, ny=8, seed=3)
    U, T = oracle.case_state(c)
    assert oracle.step(c, U, T, 1, full_jacobian=True, check=False)[4] == -1
