"""Pins of the oracle's two-range NASA-7 thermodynamics (Eq. 4.3-4.5 with the low- and
high-temperature coefficient sets in which NASA-7 data are published; the high set
applies for T >= t_mid).

* a second set equal to the first reproduces the one-range results bitwise (a whole
  9-species step);
* below t_mid every property equals that of the low set's one-range mechanism, at and
  above it that of the high set's, bitwise (the range selection, checked against the
  one-range path rather than a retyped polynomial);
* the constructed test mechanism is continuous in h, cp and s at t_mid, and its
  derivative identities hold in both ranges;
* Newton for T equals bisection for roots below and above t_mid.
"""

import copy

import numpy as np
import pytest

from cases import synthetic_mechanism, two_range_mechanism
from cases.amr import detailed_front_case


@pytest.fixture(scope="module")
def mechs():
    m = synthetic_mechanism()
    return m, two_range_mechanism(m, t_mid=1800.0)


def test_identical_sets_equal_one_range(oracle, mechs):
    m, _ = mechs
    m2 = copy.deepcopy(m)
    m2.nasa_high = m.nasa.copy()
    m2.t_mid = np.full(m.ns, 1500.0)
    c1 = detailed_front_case(nx=48, ny=16, mech=m)
    c2 = detailed_front_case(nx=48, ny=16, mech=m2)
    U1, T1 = oracle.case_state(c1)
    U2, T2 = oracle.case_state(c2)
    a = oracle.step(c1, U1, T1, 3)
    b = oracle.step(c2, U2, T2, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_range_selection(oracle, mechs):
    m, _ = mechs
    other = synthetic_mechanism(seed=777)
    lo, hi = copy.deepcopy(m), copy.deepcopy(m)
    hi.nasa = other.nasa.copy()
    two = copy.deepcopy(m)
    two.nasa_high = other.nasa.copy()
    two.t_mid = np.linspace(900.0, 2100.0, m.ns)
    for k in range(m.ns):
        for T in [300.0, 899.0, 1200.0, 1600.0, 2000.0, 2100.0, 2500.0, 4000.0]:
            ref = oracle.species_thermo(lo if T < two.t_mid[k] else hi, k, T)
            assert oracle.species_thermo(two, k, T) == ref
    rng = np.random.default_rng(8)
    for T in [700.0, 3000.0]:          # every species on one side of its t_mid
        Y = rng.dirichlet(np.ones(m.ns))
        ref = oracle.mixture_e_cv(lo if T < 900.0 else hi, Y, T)
        assert oracle.mixture_e_cv(two, Y, T) == ref


def test_constructed_mechanism_is_continuous(oracle, mechs):
    _, m2 = mechs
    Tm = 1800.0
    for k in range(m2.ns):
        below = oracle.species_thermo(m2, k, np.nextafter(Tm, 0.0))
        at = oracle.species_thermo(m2, k, Tm)
        for x, y in zip(below, at):
            assert y == pytest.approx(x, rel=1e-12)
        for T in [1000.0, 2600.0]:
            h = 1e-5 * T
            hp, _, sp = oracle.species_thermo(m2, k, T + h)
            hm, _, sm = oracle.species_thermo(m2, k, T - h)
            _, cp, _ = oracle.species_thermo(m2, k, T)
            assert (hp - hm) / (2 * h) == pytest.approx(cp, rel=1e-8)
            assert (sp - sm) / (2 * h) == pytest.approx(cp / T, rel=1e-8)
    # the two sets differ away from t_mid
    assert oracle.species_thermo(m2, 0, 3000.0)[1] != pytest.approx(
        oracle.species_thermo(mechs[0], 0, 3000.0)[1], rel=1e-4)


def test_newton_across_t_mid_equals_bisection(oracle, mechs):
    _, m2 = mechs
    rng = np.random.default_rng(12)
    for Ttrue in [900.0, 1700.0, 1800.5, 1950.0, 3200.0]:
        Y = rng.dirichlet(np.ones(m2.ns))
        e, _ = oracle.mixture_e_cv(m2, Y, Ttrue)
        for T0 in [300.0, 1799.0, 5000.0]:
            T = oracle.temperature(m2, Y, e, T0)
            lo, hi = 100.0, 8000.0
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if oracle.mixture_e_cv(m2, Y, mid)[0] < e:
                    lo = mid
                else:
                    hi = mid
            assert T == pytest.approx(0.5 * (lo + hi), rel=1e-13)
            assert T == pytest.approx(Ttrue, rel=1e-12)
