"""Closed-form pins of the oracle's reaction-rate factors (paper Eq. 4.6-4.9, the
one-step source of Sec. 4.3 item 3).

Each test is aimed at one factor that the equilibrium pins cannot see (detailed
balance cancels k_f and the third-body factor):
  * the Arrhenius temperature factor T^b exp(-E_a/(R_u T)) of Eq. 4.8, through a
    single irreversible first-order reaction whose point-implicit step has a closed
    form, at two temperatures and with b != 0, E_a != 0;
  * the third-body factor sum_j a_ij X_j of Eq. 4.7 with distinct efficiencies, the
    complement species included, against the rate written out by hand;
  * the reverse rate k_f / K_c of Eq. 4.9 far from equilibrium, with K_c formed here
    from the NASA-7 polynomials;
  * the one-step rate law -k rho Y exp(-E_a/T) through a 0-D constant-volume reactor
    at rho != 1, whose fuel fraction Y(t) is the inverse of the quadrature
    t(Y) = int_Y^Y0 dY' / (k Y' exp(-E_a / T(Y'))).
"""

import math

import numpy as np
import pytest
from scipy import integrate, optimize

from cases import Case, MODEL_ONESTEP, BC_ZEROGRAD
from cases.mechanism import Mechanism

RU = 8.314472
PATM = 101325.0


def _mech(species, M, nasa, A, b, Ea, nu_f, nu_b, tb=None, has_tb=None, rev=None):
    ns, nr = len(species), len(A)
    return Mechanism(species=list(species), elements=["E"], comp=np.ones((ns, 1), np.int64),
                     M=np.asarray(M, float), nasa=np.asarray(nasa, float),
                     A=np.asarray(A, float), b=np.asarray(b, float), Ea=np.asarray(Ea, float),
                     nu_f=np.asarray(nu_f, np.int32), nu_b=np.asarray(nu_b, np.int32),
                     tb=np.zeros((nr, ns)) if tb is None else np.asarray(tb, float),
                     has_tb=np.zeros(nr, np.int32) if has_tb is None else np.asarray(has_tb, np.int32),
                     reversible=np.zeros(nr, np.int32) if rev is None else np.asarray(rev, np.int32),
                     A_cgs=np.asarray(A, float), Ea_kcal=np.asarray(Ea, float) / 4184.0)


def _nasa_rows(n, seed):
    """Smooth, distinct single-range NASA-7 rows (cp > 0 on 300-4000 K)."""
    rng = np.random.default_rng(seed)
    rows = np.zeros((n, 7))
    rows[:, 0] = 3.0 + rng.uniform(0, 1.5, n)
    rows[:, 1] = rng.uniform(1e-4, 8e-4, n)
    rows[:, 2] = -rng.uniform(1e-8, 6e-8, n)
    rows[:, 3] = rng.uniform(0, 1e-12, n)
    rows[:, 4] = -rng.uniform(0, 1e-16, n)
    rows[:, 5] = rng.uniform(-1e4, 1e4, n)
    rows[:, 6] = rng.uniform(2.0, 6.0, n)
    return rows


def _h_over_R(a, T):
    return a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5 + a[5]


def _s_over_R(a, T):
    return a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4 + a[6]


# ------------------------------------------------------------------ Eq. 4.8: T^b exp(-Ea/(Ru T))
def test_arrhenius_temperature_factor_closed_form(oracle):
    """A -> B, first order, b = 0.7, E_a = 83.7 kJ/mol: with k(T) = A T^b exp(-E_a/(R_u T))
    the point-implicit update is rho Y_A - dt k rho Y_A / (1 + dt k) exactly, and
    wdot_A = -k rho Y_A; at two temperatures the ratio k(T2)/k(T1) fixes b and E_a/R_u."""
    A, b, Ea = 2.3e6, 0.7, 8.37e4
    m = _mech(["A", "B"], [0.02, 0.03], _nasa_rows(2, 1), [A], [b], [Ea],
              [[1, 0]], [[0, 1]])
    rho, rhoA = 1.7, 0.6
    ks = {}
    for T in [1100.0, 2300.0]:
        k = A * T**b * math.exp(-Ea / (RU * T))
        ks[T] = k
        w = oracle.production(m, rho, T, np.array([rhoA]))
        assert w[0] == pytest.approx(-k * rhoA, rel=1e-13)
        assert w[1] == pytest.approx(0.03 / 0.02 * k * rhoA, rel=1e-13)   # M_B * q
        for dt in [0.1 / k, 1.0 / k, 30.0 / k]:
            out = oracle.point_implicit(m, rho, T, np.array([rhoA]), dt)
            assert out[0] == pytest.approx(rhoA - dt * k * rhoA / (1.0 + dt * k), rel=1e-13)
    # the two temperatures see different k: the pins above constrain T^b and Ea/(Ru T)
    assert ks[2300.0] / ks[1100.0] > 50.0


def test_arrhenius_second_order_forward_rate(oracle):
    """A + A -> B (second order, units m^3/mol/s): wdot_A = -2 M_A k_f X_A^2 with
    X_A = rho Y_A / M_A, k_f = A T^b exp(-E_a/(R_u T)), b = -0.8."""
    A, b, Ea = 4.1e7, -0.8, 3.1e4
    M = [0.014, 0.028]
    m = _mech(["A", "B"], M, _nasa_rows(2, 2), [A], [b], [Ea], [[2, 0]], [[0, 1]])
    rho, rhoA = 0.9, 0.35
    for T in [800.0, 2600.0]:
        kf = A * T**b * math.exp(-Ea / (RU * T))
        XA = rhoA / M[0]
        q = kf * XA * XA
        w = oracle.production(m, rho, T, np.array([rhoA]))
        assert w[0] == pytest.approx(-2.0 * M[0] * q, rel=1e-13)
        assert w[1] == pytest.approx(1.0 * M[1] * q, rel=1e-13)


# ------------------------------------------------------------------ Eq. 4.7: sum_j a_ij X_j
def test_third_body_factor_with_distinct_efficiencies(oracle):
    """A + B + M -> AB + M with efficiencies (0.7, 1.9, 2.6, 0.4) on (A, B, AB, C), C the
    complement species: q = (sum_j a_j X_j) k_f X_A X_B, X_C = (rho - sum rho Y) / M_C."""
    M = np.array([0.011, 0.017, 0.028, 0.031])
    eff = np.array([0.7, 1.9, 2.6, 0.4])
    A, b, Ea = 6.0e5, 0.35, 1.2e4
    m = _mech(["A", "B", "AB", "C"], M, _nasa_rows(4, 3), [A], [b], [Ea],
              [[1, 1, 0, 0]], [[0, 0, 1, 0]], tb=[eff], has_tb=[1])
    rho = 2.2
    rhoY = np.array([0.31, 0.52, 0.44])          # rho Y_C = 0.93
    X = np.append(rhoY / M[:3], (rho - rhoY.sum()) / M[3])
    for T in [1300.0, 2100.0]:
        kf = A * T**b * math.exp(-Ea / (RU * T))
        ctb = float(np.dot(eff, X))
        q = ctb * kf * X[0] * X[1]
        w = oracle.production(m, rho, T, rhoY)
        expect = np.array([-M[0] * q, -M[1] * q, M[2] * q, 0.0])
        assert np.allclose(w, expect, rtol=1e-13, atol=0.0), (T, w, expect)
        # a flat sum over X (all efficiencies 1) would give this, which differs here
        assert abs(ctb - X.sum()) > 0.05 * ctb
    # the Jacobian of a third-body reaction carries a_j (R_f - R_b) beside ctb dR/dX
    T = 1700.0
    _, J = oracle.production(m, rho, T, rhoY, jacobian=True)
    kf = A * T**b * math.exp(-Ea / (RU * T))
    Rf = kf * X[0] * X[1]
    ctb = float(np.dot(eff, X))
    dq = np.array([ctb * kf * X[1] + eff[0] * Rf, ctb * kf * X[0] + eff[1] * Rf,
                   eff[2] * Rf, eff[3] * Rf])                # dq/dX_j
    dqdm = dq[:3] / M[:3] - dq[3] / M[3]                      # d/d(rho Y_m), complement chain
    nu = np.array([-1.0, -1.0, 1.0])
    Jx = (M[:3] * nu)[:, None] * dqdm[None, :]
    assert np.allclose(J, Jx, rtol=1e-12, atol=1e-12 * np.max(np.abs(Jx)))


def test_third_body_efficiency_of_the_complement_species(oracle):
    """Only the complement's efficiency changes: the rate changes by (a'_C - a_C) X_C k_f X_A X_B."""
    M = np.array([0.011, 0.017, 0.028, 0.031])
    base = np.array([1.0, 1.0, 1.0, 1.0])
    bumped = np.array([1.0, 1.0, 1.0, 3.5])
    rho, T = 1.3, 1900.0
    rhoY = np.array([0.2, 0.3, 0.1])
    XC = (rho - rhoY.sum()) / M[3]
    ws = []
    for eff in (base, bumped):
        m = _mech(["A", "B", "AB", "C"], M, _nasa_rows(4, 3), [1.0e6], [0.0], [0.0],
                  [[1, 1, 0, 0]], [[0, 0, 1, 0]], tb=[eff], has_tb=[1])
        ws.append(oracle.production(m, rho, T, rhoY))
    dq = 2.5 * XC * 1.0e6 * (rhoY[0] / M[0]) * (rhoY[1] / M[1])
    assert ws[1][2] - ws[0][2] == pytest.approx(M[2] * dq, rel=1e-12)


# ------------------------------------------------------------------ Eq. 4.9: k_b = k_f / K_c
def test_reverse_rate_far_from_equilibrium(oracle):
    """A + B <=> C + D (reversible, b != 0, E_a != 0) far from equilibrium:
    q = k_f X_A X_B - (k_f / K_c) X_C X_D with K_c = exp(sum nu (s/R - h/(R T))) (p_atm/(R_u T))^dn,
    here dn = 0; and A2 <=> 2 A (dn = 1) for the pressure factor."""
    M = np.array([0.012, 0.021, 0.018, 0.015, 0.04])
    nasa = _nasa_rows(5, 4)
    A, b, Ea = 3.3e5, -0.45, 2.2e4
    m = _mech(["A", "B", "C", "D", "N"], M, nasa, [A], [b], [Ea],
              [[1, 1, 0, 0, 0]], [[0, 0, 1, 1, 0]], rev=[1])
    rho = 1.9
    rhoY = np.array([0.11, 0.27, 0.36, 0.05])
    X = np.append(rhoY / M[:4], (rho - rhoY.sum()) / M[4])
    for T in [1000.0, 2700.0]:
        kf = A * T**b * math.exp(-Ea / (RU * T))
        g = sum(nu * (_s_over_R(nasa[j], T) - _h_over_R(nasa[j], T) / T)
                for j, nu in [(0, -1), (1, -1), (2, 1), (3, 1)])
        Kc = math.exp(g)
        q = kf * X[0] * X[1] - kf / Kc * X[2] * X[3]
        w = oracle.production(m, rho, T, rhoY)
        expect = np.array([-M[0] * q, -M[1] * q, M[2] * q, M[3] * q, 0.0])
        assert np.allclose(w, expect, rtol=1e-12, atol=0.0), (T, w, expect)
        assert abs(kf / Kc * X[2] * X[3]) > 1e-3 * abs(kf * X[0] * X[1])   # reverse term matters

    M2 = np.array([0.028, 0.014, 0.04])
    nasa2 = _nasa_rows(3, 5)
    m2 = _mech(["A2", "A", "N"], M2, nasa2, [A], [b], [Ea], [[1, 0, 0]], [[0, 2, 0]], rev=[1])
    rhoY2 = np.array([0.5, 0.2])
    X2 = np.append(rhoY2 / M2[:2], (rho - rhoY2.sum()) / M2[2])
    for T in [1500.0, 3100.0]:
        kf = A * T**b * math.exp(-Ea / (RU * T))
        g = 2 * (_s_over_R(nasa2[1], T) - _h_over_R(nasa2[1], T) / T) - \
            (_s_over_R(nasa2[0], T) - _h_over_R(nasa2[0], T) / T)
        Kc = math.exp(g) * (PATM / (RU * T))
        q = kf * X2[0] - kf / Kc * X2[1] ** 2
        w = oracle.production(m2, rho, T, rhoY2)
        assert w[0] == pytest.approx(-M2[0] * q, rel=1e-12)
        assert w[1] == pytest.approx(2.0 * M2[1] * q, rel=1e-12)


# ------------------------------------------------------------------ one-step rate law
def test_onestep_reactor_follows_rate_quadrature(oracle):
    """0-D constant-volume one-step reactor at rho = 2.5: Y obeys dY/dt = -k Y exp(-E_a/T)
    with T = T0 + (gamma-1) Q (Y0 - Y)/R. The oracle's Y(t) (RK3, dt small) equals the
    inverse of t(Y) = int_Y^Y0 dY'/(k Y' exp(-E_a/T(Y'))) to the RK3 error."""
    gamma, R, Q, Ea, k = 1.2, 1.0, 50.0, 24.0, 30.6973223365
    rho, T0, Y0 = 2.5, 5.0, 1.0
    W = np.zeros((5, 1, 1))
    W[0], W[3], W[4] = rho, rho * R * T0, Y0
    c = Case(name="reactor", model=MODEL_ONESTEP, nx=1, ny=1, dx=1.0, dy=1.0,
             bc=[BC_ZEROGRAD] * 4, W=W, gamma=gamma, R=R, Q=Q, Ea=Ea, k=k)

    def Tof(Y):
        return T0 + (gamma - 1.0) * Q * (Y0 - Y) / R

    def t_of(Y):
        val, _ = integrate.quad(lambda y: 1.0 / (k * y * math.exp(-Ea / Tof(y))), Y, Y0,
                                epsabs=0.0, epsrel=1e-13, limit=200)
        return val

    dt = 2e-3
    U, T = oracle.case_state(c)
    nsteps_total = 0
    for n in [500, 500, 1000, 1000]:
        U, T, _, _, _ = oracle.step(c, U, T, n, dt_fixed=dt)
        nsteps_total += n
        t = nsteps_total * dt
        Y = U[4, 0, 0] / U[0, 0, 0]
        assert U[0, 0, 0] == rho                          # no flux: density unchanged
        if Y > 1e-6:
            # Y(t) by inverting the quadrature
            Yq = optimize.brentq(lambda y: t_of(y) - t, 1e-12, Y0 * (1 - 1e-15), xtol=1e-15,
                                 rtol=1e-15)
            assert Y == pytest.approx(Yq, rel=2e-6, abs=1e-9), (t, Y, Yq)
        assert T[0, 0] == pytest.approx(Tof(Y), rel=1e-12)
