"""Pins of the oracle's thermodynamics and chemistry (paper Eq. 4.2-4.9, 4.12-4.13).

Independent references: finite differences of the NASA polynomials, bisection,
the calorically-perfect special case, a closed-form single reaction, central
differences of the rates, and chemical equilibrium from a separate Gibbs
(element-potential) minimization at fixed internal energy and density.
"""

import copy
import math

import numpy as np
import pytest

from cases import (Case, synthetic_mechanism, detonation_tube_case, MODEL_ONESTEP,
                   MODEL_DETAILED, BC_PERIODIC, BC_ZEROGRAD)
from cases.mechanism import Mechanism, fresh_mass_fractions, complete_mechanism
from cases.amr import detailed_front_case
import refsol

RU = 8.314472


@pytest.fixture(scope="module")
def mech():
    return synthetic_mechanism()


def _zero_d_case(mech, p, T, Y):
    W = np.zeros((4 + mech.ns - 1, 1, 1))
    W[0], W[3] = p, T
    W[4:, 0, 0] = Y[:-1]
    return Case(name="0d", model=MODEL_DETAILED, nx=1, ny=1, dx=1e-3, dy=1e-3,
                bc=[BC_ZEROGRAD] * 4, W=W, mech=mech)


# ------------------------------------------------------------------ thermo (P8)
def test_nasa_derivative_identities(oracle, mech):
    """dh/dT = cp and ds/dT = cp/T for every species (Eq. 4.3-4.5)."""
    for k in range(mech.ns):
        for T in [400.0, 1200.0, 2500.0, 4000.0]:
            h = 1e-5 * T
            hp, _, sp = oracle.species_thermo(mech, k, T + h)
            hm, _, sm = oracle.species_thermo(mech, k, T - h)
            _, cp, _ = oracle.species_thermo(mech, k, T)
            assert (hp - hm) / (2 * h) == pytest.approx(cp, rel=1e-8)
            assert (sp - sm) / (2 * h) == pytest.approx(cp / T, rel=1e-8)


def test_newton_root_equals_bisection(oracle, mech):
    rng = np.random.default_rng(4)
    for _ in range(10):
        Y = rng.dirichlet(np.ones(mech.ns))
        Ttrue = rng.uniform(500.0, 3500.0)
        e, _ = oracle.mixture_e_cv(mech, Y, Ttrue)
        for T0 in [300.0, 1000.0, 5000.0]:
            T = oracle.temperature(mech, Y, e, T0)
            lo, hi = 100.0, 8000.0
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if oracle.mixture_e_cv(mech, Y, mid)[0] < e:
                    lo = mid
                else:
                    hi = mid
            assert T == pytest.approx(0.5 * (lo + hi), rel=1e-13)
            assert T == pytest.approx(Ttrue, rel=1e-12)


def test_calorically_perfect_special_case(oracle):
    """a0 = gamma/(gamma-1), a1..a5 = 0 makes e = R T/(gamma-1): Newton gives the closed form."""
    g = 1.4
    nasa = np.zeros((2, 7))
    nasa[:, 0] = g / (g - 1.0)
    m = Mechanism(species=["X", "Y"], elements=["E"], comp=np.array([[1], [1]]),
                  M=np.array([0.029, 0.029]), nasa=nasa, A=np.zeros(0), b=np.zeros(0),
                  Ea=np.zeros(0), nu_f=np.zeros((0, 2), np.int32), nu_b=np.zeros((0, 2), np.int32),
                  tb=np.zeros((0, 2)), has_tb=np.zeros(0, np.int32),
                  reversible=np.zeros(0, np.int32), A_cgs=np.zeros(0), Ea_kcal=np.zeros(0))
    R = RU / 0.029
    for e in [1e5, 7.2e5, 3.3e6]:
        T = oracle.temperature(m, np.array([0.3, 0.7]), e, 1000.0)
        assert T == pytest.approx((g - 1.0) * e / R, rel=4e-16)


# ------------------------------------------------------------------ chemistry (P9)
def test_jacobian_matches_central_differences(oracle, mech):
    rng = np.random.default_rng(8)
    rho = 3.0
    for T in [1200.0, 2500.0]:
        Y = rng.dirichlet(np.ones(mech.ns)) * 0.5 + fresh_mass_fractions(mech) * 0.5
        rhoY = rho * Y[:-1]
        w, J = oracle.production(mech, rho, T, rhoY, jacobian=True)
        nt = mech.ns - 1
        for m_ in range(nt):
            h = 1e-6 * max(rhoY[m_], 1e-3)
            up, dn = rhoY.copy(), rhoY.copy()
            up[m_] += h
            dn[m_] -= h
            col = (oracle.production(mech, rho, T, up)[:nt] - oracle.production(mech, rho, T, dn)[:nt]) / (2 * h)
            scale = np.max(np.abs(J)) + 1e-300
            assert np.max(np.abs(col - J[:, m_])) <= 1e-6 * scale, (T, m_)


def _one_reaction_mech(k, reversible=False):
    """A -> B, first order, A = k, b = 0, Ea = 0; B is the complement species."""
    nasa = np.zeros((2, 7))
    nasa[:, 0] = 3.5
    return Mechanism(species=["A", "B"], elements=["E"], comp=np.array([[1], [1]]),
                     M=np.array([0.02, 0.02]), nasa=nasa, A=np.array([k]), b=np.zeros(1),
                     Ea=np.zeros(1), nu_f=np.array([[1, 0]], np.int32),
                     nu_b=np.array([[0, 1]], np.int32), tb=np.zeros((1, 2)),
                     has_tb=np.zeros(1, np.int32),
                     reversible=np.array([1 if reversible else 0], np.int32),
                     A_cgs=np.array([k]), Ea_kcal=np.zeros(1))


def test_single_irreversible_first_order_closed_form(oracle):
    k = 3.7e5
    m = _one_reaction_mech(k)
    rho, rhoY = 2.0, np.array([1.2])
    for dt in [1e-7, 1e-6, 1e-5, 1e-3]:
        out = oracle.point_implicit(m, rho, 1500.0, rhoY, dt)
        assert out[0] == pytest.approx(rhoY[0] - dt * k * rhoY[0] / (1.0 + dt * k), rel=1e-14)
    w = oracle.production(m, rho, 1500.0, rhoY)
    assert w[0] == pytest.approx(-k * rhoY[0], rel=1e-15)
    assert w[1] == pytest.approx(k * rhoY[0], rel=1e-15)


def test_point_implicit_small_dt_limit(oracle, mech):
    rho, T = 2.5, 2200.0
    Y = 0.5 * fresh_mass_fractions(mech) + 0.5 / mech.ns
    rhoY = rho * Y[:-1]
    w, J = oracle.production(mech, rho, T, rhoY, jacobian=True)
    w = w[:-1]
    tau = 1.0 / np.max(np.abs(J))          # fastest chemical time scale
    prev = None
    for dt in [1e-2 * tau, 1e-3 * tau, 1e-4 * tau]:
        d = (oracle.point_implicit(mech, rho, T, rhoY, dt) - rhoY) / dt
        err = np.max(np.abs(d - w)) / np.max(np.abs(w))
        if prev is not None:
            assert err < 0.2 * prev or err < 1e-9
        prev = err
    assert prev < 1e-4


def test_point_implicit_conserves_elements(oracle, mech):
    """Linear invariants l with l^T J = 0 are conserved exactly: element totals
    including the complement species (this pins the complement chain of J)."""
    rng = np.random.default_rng(3)
    rho = 2.0
    nt = mech.ns - 1
    L = mech.comp[:nt].T / mech.M[:nt] - mech.comp[nt][:, None] / mech.M[nt]
    for T in [1500.0, 3000.0]:
        Y = rng.dirichlet(np.ones(mech.ns))
        rhoY = rho * Y[:-1]
        _, J = oracle.production(mech, rho, T, rhoY, jacobian=True)
        # l^T J = 0 up to round-off of the largest entries
        assert np.max(np.abs(L @ J)) <= 1e-13 * np.max(np.abs(L)) * np.max(np.abs(J))
        tau = 1.0 / np.max(np.abs(J))
        for dt in [0.1 * tau, 10.0 * tau, 1e3 * tau]:
            out = oracle.point_implicit(mech, rho, T, rhoY, dt)
            d = L @ (out - rhoY)
            cond = np.linalg.cond(np.eye(len(rhoY)) - dt * J)
            assert np.max(np.abs(d)) <= 1e-15 * cond * np.max(np.abs(L @ rhoY)), (T, dt, d)


# ------------------------------------------------------------------ long-time limits (P5)
def test_onestep_ignition_reaches_closed_form_temperature(oracle):
    """Constant-volume adiabatic burn of the one-step model: T_f = T0 + (gamma-1) Q Y0 / R."""
    W = np.zeros((5, 1, 1))
    W[0], W[3], W[4] = 1.0, 5.0, 1.0     # T0 = p/(rho R) = 5 so that the burn takes O(10) time units
    c = Case(name="ign", model=MODEL_ONESTEP, nx=1, ny=1, dx=1.0, dy=1.0, bc=[BC_ZEROGRAD] * 4,
             W=W, gamma=1.2, R=1.0, Q=50.0, Ea=24.0, k=30.6973223365)
    U, T = oracle.case_state(c)
    U, T, _, _, _ = oracle.step(c, U, T, 15000, dt_fixed=2e-3)
    assert T[0, 0] == pytest.approx(5.0 + 0.2 * 50.0, rel=1e-12)
    assert U[4, 0, 0] < 1e-12


def test_detailed_equilibrium_consistency(oracle, mech):
    """At the independent Gibbs equilibrium (fixed e, rho, element totals):
    every reaction is in detailed balance in the oracle's rates (Eq. 4.7-4.9),
    the oracle's Newton returns the Gibbs temperature, and the point-implicit
    map leaves the state unchanged (its fixed points are S = 0)."""
    Y = fresh_mass_fractions(mech)
    c = _zero_d_case(mech, 20 * 101325.0, 1500.0, Y)
    U, T = oracle.case_state(c)
    rho, e = U[0, 0, 0], U[3, 0, 0] / U[0, 0, 0]
    X0 = np.r_[U[4:, 0, 0], rho - U[4:, 0, 0].sum()] / mech.M
    b = mech.comp.T.astype(float) @ X0
    Teq, Xeq = refsol.equilibrium_T(mech, rho, e, b)
    assert 300.0 < Teq < 5000.0
    Yeq = Xeq * mech.M / rho
    # Newton temperature of the Gibbs mixture at the same e
    assert oracle.temperature(mech, Yeq, e, 1500.0) == pytest.approx(Teq, rel=1e-10)
    # detailed balance reaction by reaction: forward and reverse rates agree
    rhoY = rho * Yeq[:-1]
    for i in range(mech.nr):
        sub = copy.deepcopy(mech)
        sel = np.zeros(mech.nr, bool)
        sel[i] = True
        for f in ["A", "b", "Ea", "nu_f", "nu_b", "tb", "has_tb", "reversible"]:
            setattr(sub, f, getattr(mech, f)[sel])
        w = oracle.production(sub, rho, Teq, rhoY)
        # the same reaction made irreversible gives the forward rate alone
        sub.reversible = np.zeros(1, np.int32)
        wf = oracle.production(sub, rho, Teq, rhoY)
        scale = np.max(np.abs(wf)) + 1e-300
        assert np.max(np.abs(w)) <= 1e-7 * scale, (i, np.max(np.abs(w)), scale)
    # fixed point of the point-implicit map
    out = oracle.point_implicit(mech, rho, Teq, rhoY, 1e-6)
    assert np.max(np.abs(out - rhoY)) <= 1e-9 * rho


def _reactor_start(mech, start):
    """Initial 0-D state: the fresh A2/B2/C2 mixture at 1500 K, or the same element
    amounts as free atoms A, B (with C2) at 600 K; 20 atm."""
    if start == "fresh-1500K":
        return 1500.0, fresh_mass_fractions(mech)
    Y = np.zeros(mech.ns)
    Y[mech.species.index("A")], Y[mech.species.index("B")] = 0.03, 0.23
    Y[mech.species.index("C2")] = 0.74
    return 600.0, Y


@pytest.mark.parametrize("start", ["atoms-600K", "fresh-1500K"])
def test_adiabatic_reactor_relaxes_to_gibbs_equilibrium(oracle, start):
    """Constant-volume adiabatic reactor with the complete-channel mechanism: the long-time
    limit of the point-implicit steps (Eq. 4.12-4.13) with the Newton temperature is the
    independent Gibbs equilibrium of the same thermo at the same rho, e and element totals
    (element potentials, scipy): T to 1e-9, mole fractions to 1e-7. From free atoms the
    recombination releases heat (an ignition, T 600 -> 921 K); from the fresh mixture at
    1500 K the molecules dissociate and T falls."""
    mech = complete_mechanism()
    T0, Y = _reactor_start(mech, start)
    c = _zero_d_case(mech, 20 * 101325.0, T0, Y)
    U, T = oracle.case_state(c)
    rho, e = U[0, 0, 0], U[3, 0, 0] / U[0, 0, 0]
    X0 = np.r_[U[4:, 0, 0], rho - U[4:, 0, 0].sum()] / mech.M
    b = mech.comp.T.astype(float) @ X0
    Teq, Xeq = refsol.equilibrium_T(mech, rho, e, b)
    for dt in (1e-10, 1e-9, 1e-8, 1e-7):
        U, T, _, _, _ = oracle.step(c, U, T, 200, dt_fixed=dt)
    X = np.r_[U[4:, 0, 0], rho - U[4:, 0, 0].sum()] / mech.M
    assert T[0, 0] == pytest.approx(Teq, rel=1e-9)
    assert np.max(np.abs(X - Xeq)) <= 1e-7 * X.sum()
    assert abs(Teq - T0) > 250.0                 # the reactor did change state
    if start == "atoms-600K":
        assert Teq > T0


# ------------------------------------------------------------------ conservation (P4)
def test_conservation_detailed_periodic(oracle, mech):
    c = detailed_front_case(nx=24, ny=16, dx=25e-6, mech=mech)
    c.bc = [BC_PERIODIC] * 4
    U0, T0 = oracle.case_state(c)
    U, T, _, _, _ = oracle.step(c, U0, T0, 5)
    mom_scale = math.fsum(np.abs(U0[1]).ravel()) + math.fsum(np.abs(U[2]).ravel())
    for f in range(4):
        s0, s1 = math.fsum(U0[f].ravel()), math.fsum(U[f].ravel())
        scale = mom_scale if f in (1, 2) else math.fsum(np.abs(U0[f]).ravel())
        assert abs(s1 - s0) <= 1e-13 * scale, f
    nt = mech.ns - 1

    def elements(Uc):
        rhoY = Uc[4:].reshape(nt, -1)
        rho = Uc[0].ravel()
        X = np.vstack([rhoY / mech.M[:nt, None], (rho - rhoY.sum(0))[None, :] / mech.M[nt]])
        return np.array([math.fsum((mech.comp[:, e] @ X).ravel()) for e in range(mech.comp.shape[1])])

    e0, e1 = elements(U0), elements(U)
    assert np.max(np.abs(e1 - e0) / e0) <= 1e-13
    # the chemistry did act
    assert np.max(np.abs(U[4:] - U0[4:])) > 0
