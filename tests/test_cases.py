"""Case generators and the closed-form case constants they use.

* Chapman-Jouguet state of the one-step model, checked against a direct
  numerical solve of the Rankine-Hugoniot jump with a sonic downstream state;
* ZND rate constant (half-reaction length 1), checked by an independent ODE
  integration of the steady wave;
* detonation dynamics of the oracle: a 1-D one-step detonation settles at the
  CJ speed (within 1 %);
* determinism and shapes of the seeded workloads.
"""

import math

import numpy as np
import pytest
from scipy.optimize import brentq

from cases import (cj_state, znd_rate_constant, detonation_tube_case, ensemble_case, amr_case,
                   sod_case, adjoint_case, synthetic_mechanism, Case, MODEL_ONESTEP,
                   BC_ZEROGRAD, BC_DIRICHLET, BC_SLIPWALL)
import refsol


def test_cj_state_from_jump_conditions():
    g, Q = 1.2, 50.0
    cj = cj_state(g, Q)
    # Hugoniot with heat release along the Rayleigh line; CJ = the minimum-speed tangency
    a = g / (g - 1.0)

    def disc(D):   # discriminant of the energy equation for the downstream speed at lam = 1
        m = D
        A_, B_, C_ = a - 0.5, a * (1.0 / m + D), a + 0.5 * D * D + Q
        return B_ * B_ - 4.0 * A_ * C_

    D = brentq(disc, 2.0, 20.0, xtol=1e-14, rtol=1e-15)
    assert cj["D"] == pytest.approx(D, rel=1e-11)
    assert cj["D"] == pytest.approx(6.809475, abs=1e-6)
    assert cj["p"] == pytest.approx(21.5313, abs=1e-4)
    # sonic downstream state
    c1 = math.sqrt(g * cj["p"] / cj["rho"])
    assert cj["w"] == pytest.approx(c1, rel=1e-12)


def test_znd_rate_constant_by_ode():
    g, Q, Ea = 1.2, 50.0, 24.0
    k = znd_rate_constant(g, Q, Ea)
    assert k == pytest.approx(30.6973223365, rel=1e-9)
    x_half = refsol.znd_half_length_ode(g, Q, Ea, k, cj_state(g, Q)["D"])
    assert x_half == pytest.approx(1.0, rel=1e-7)


@pytest.mark.slow
def test_oracle_detonation_runs_at_cj_speed(oracle):
    """1-D one-step detonation (gamma 1.2, Q 50, Ea 24) started at a closed end: the front
    speed averaged over the second half of the run is within 1 % of D_CJ, and the peak
    pressure is near the von Neumann value. (With an open, zero-gradient end the burned
    slab keeps acting as a piston and the wave stays overdriven.)"""
    g, Q, Ea = 1.2, 50.0, 24.0
    k = znd_rate_constant(g, Q, Ea)
    dx, nx = 0.1, 2400
    c = detonation_tube_case(nx=nx, ny=1, dx=dx, seed=1, noise=0.0, k=k, slab_frac=0.02)
    c.bc[0] = BC_SLIPWALL
    U, T = oracle.case_state(c)
    x = (np.arange(nx) + 0.5) * dx
    times, fronts = [], []
    t = 0.0
    while True:
        U, T, t, _, _ = oracle.step(c, U, T, 200, t=t)
        P = oracle.primitives(c, U, T)
        shocked = np.nonzero(P[3, 0] > 2.0)[0]
        times.append(t)
        fronts.append(x[shocked.max()])
        if fronts[-1] > x[-1] - 20.0:
            break
    times, fronts = np.array(times), np.array(fronts)
    _, p_vn, _, _ = __import__("cases").znd_profile(g, Q, 0.0)
    assert abs(P[3, 0].max() / p_vn - 1.0) < 0.05
    half = len(times) // 2
    speed = np.polyfit(times[half:], fronts[half:], 1)[0]
    assert abs(speed / cj_state(g, Q)["D"] - 1.0) < 0.01, speed


def test_generators_are_deterministic_and_shaped():
    a, b = detonation_tube_case(), detonation_tube_case()
    assert np.array_equal(a.W, b.W) and a.W.shape == (5, 128, 1024)
    assert a.bc == [BC_ZEROGRAD, BC_DIRICHLET, BC_SLIPWALL, BC_SLIPWALL]
    slab = a.W[3, 0] > 1.0
    assert slab.sum() == 51                          # x_c < 0.05 L_x
    assert np.all(np.abs(a.W[0, :, ~slab] - 1.0) <= 0.01)
    s = sod_case()
    assert s.W.shape == (4, 1, 400)
    e = ensemble_case()
    assert len(e.domains) == 64
    nd1 = sum(1 for d in e.domains if d.ny == 1)
    assert nd1 == 32
    assert all(d.nx % 8 == 0 for d in e.domains)
    assert all(30 <= d.Q <= 60 and 20 <= d.Ea <= 30 for d in e.domains)
    adj = adjoint_case()
    assert adj["case"].W.shape == (5, 64, 512) and adj["case"].dt_fixed > 0


@pytest.mark.slow
def test_amr_case_shape():
    m = synthetic_mechanism()
    assert m.ns == 9 and m.nr == 19
    assert np.linalg.matrix_rank(m.nu_b - m.nu_f) == 6
    # every reaction conserves elements
    assert np.all((m.nu_b - m.nu_f) @ m.comp == 0)
    c = amr_case(mech=m)
    nb = len(c.blocks)
    assert 550 <= nb <= 700, nb
    assert 1.8e6 <= c.valid_cells() <= 2.2e6
    assert set(np.unique(c.blocks["nx"])) <= {8, 16, 32, 64}
    assert c.W.shape[0] == 12
