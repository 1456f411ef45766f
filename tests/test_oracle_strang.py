"""Pins of the oracle's Strang splitting (Sec. 4.2: chemistry over dt/2, the RK3 flux
update over dt, chemistry over dt/2; dt from the state at the start of the step).

* on a spatially uniform state the flux update is the identity up to the RK
  combination's rounding, so a Strang step equals two point-implicit half steps
  (with the Newton temperature between them), taken directly from the chemistry
  routines;
* the Strang and Lie steps differ by O(dt^2): halving dt divides the difference by
  about 4 (a wrong half-step length, or a missing half, leaves an O(dt) difference);
* mass, momentum, energy and element totals stay conserved on a periodic grid;
* a block split of the grid reproduces the uniform grid bitwise;
* models without chemistry reject it.
"""

import math

import numpy as np
import pytest

from cases import synthetic_mechanism, detonation_tube_case, BC_PERIODIC
from cases.amr import detailed_front_case
from test_oracle_blocks import _split_uniform, _gather


@pytest.fixture(scope="module")
def mech():
    return synthetic_mechanism()


def test_uniform_state_is_two_half_steps(oracle, mech):
    c = detailed_front_case(nx=4, ny=4, mech=mech)
    c.bc = [BC_PERIODIC] * 4
    c.W[:] = c.W[:, :1, :1]             # every cell the burned state behind the front
    c.W[1:3] = 0.0
    U0, T0 = oracle.case_state(c)
    U, T, _, dts, _ = oracle.step(c, U0, T0, 1, strang=True)
    dt = dts[0]
    rho, E = U0[0, 0, 0], U0[3, 0, 0]
    rhoY = U0[4:, 0, 0].copy()
    Tc = T0[0, 0]
    for _ in range(2):
        rhoY = oracle.point_implicit(mech, rho, Tc, rhoY, 0.5 * dt)
        Y = np.append(rhoY / rho, 1.0 - rhoY.sum() / rho)
        Tc = oracle.temperature(mech, Y, E / rho, Tc)
    for j in range(4):
        for i in range(4):
            assert np.allclose(U[4:, j, i], rhoY, rtol=1e-12, atol=1e-14 * rho)
            assert T[j, i] == pytest.approx(Tc, rel=1e-12)
    # the chemistry acted, and not as one full step
    assert np.max(np.abs(rhoY - U0[4:, 0, 0])) > 1e-8 * rho
    L = oracle.step(c, U0, T0, 1)[0]
    assert np.max(np.abs(L[4:] - U[4:])) > 1e-12 * rho


def test_strang_lie_difference_is_second_order(oracle, mech):
    c = detailed_front_case(nx=32, ny=8, mech=mech)
    U0, T0 = oracle.case_state(c)
    diffs = []
    for dt in [2e-9, 1e-9, 5e-10]:
        lie = oracle.step(c, U0, T0, 1, dt_fixed=dt)[0]
        strang = oracle.step(c, U0, T0, 1, dt_fixed=dt, strang=True)[0]
        diffs.append(np.max(np.abs(lie[4:] - strang[4:])))
        # the step itself is first order in dt
        assert np.max(np.abs(lie[4:] - U0[4:])) > 1e3 * diffs[-1]
    for a, b in zip(diffs[:-1], diffs[1:]):
        assert 3.6 < a / b < 4.4, diffs


def test_strang_conserves(oracle, mech):
    c = detailed_front_case(nx=24, ny=16, dx=25e-6, mech=mech)
    c.bc = [BC_PERIODIC] * 4
    U0, T0 = oracle.case_state(c)
    U, T, _, _, _ = oracle.step(c, U0, T0, 4, strang=True)
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
    assert np.max(np.abs(U[4:] - U0[4:])) > 0


def test_strang_block_split_equals_uniform(oracle, mech):
    c = detailed_front_case(nx=48, ny=16, mech=mech)
    bc, recs = _split_uniform(c, [0, 16, 40, 48], [0, 8, 16])
    U, T = oracle.case_state(c)
    Ub, Tb = oracle.block_state(bc)
    U1, _, t1, _, _ = oracle.step(c, U, T, 3, strang=True)
    U2, _, t2, _, _ = oracle.step_blocks(bc, Ub, Tb, 3, strang=True)
    assert t2[0] == t1
    assert np.array_equal(_gather(U2, recs, U1.shape), U1)


def test_strang_needs_chemistry(oracle):
    c = detonation_tube_case(nx=16, ny=8, seed=3)
    U, T = oracle.case_state(c)
    st = oracle.step(c, U, T, 1, strang=True, check=False)[4]
    assert st == -1


def test_strang_crossover_one_level_equals_synchronous(oracle, mech):
    c = detailed_front_case(nx=32, ny=16, mech=mech)
    bc, _ = _split_uniform(c, [0, 16, 32], [0, 16])
    Ub, Tb = oracle.block_state(bc)
    a = oracle.step_blocks(bc, Ub, Tb, 2, strang=True)
    b = oracle.step_blocks(bc, Ub, Tb, 2, strang=True, crossover=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
