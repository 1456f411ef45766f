"""Pins of the oracle's convective part (WENO5 + Lax-Friedrichs + SSP-RK3 + ghosts).

Each test checks the oracle against something other than itself: the exact
Riemann solution, polynomial exactness, observed orders of accuracy, invariants
(constant states, conservation, mirror and transpose symmetry).
"""

import json
import math
import os

import numpy as np
import pytest

from cases import (Case, sod_case, detonation_tube_case, MODEL_CPG, MODEL_ONESTEP,
                   BC_PERIODIC, BC_ZEROGRAD, BC_SLIPWALL, BC_DIRICHLET)
import refsol

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _prim(O, case, U, T):
    return O.primitives(case, U, T)


# ------------------------------------------------------------------ WENO5 point pins
def test_weno5_linear_data_is_exact(oracle):
    # all smoothness indicators are equal on linear data, so the linear weights
    # (0.1, 0.6, 0.3) apply and every candidate gives the midpoint value
    for base, slope in [(0.0, 1.0), (3.5, -2.25), (-1e3, 7.0)]:
        f = base + slope * np.arange(-2, 3)
        assert oracle.weno5(f) == pytest.approx(base + slope * 0.5, rel=1e-14, abs=1e-12)


def test_weno5_polynomial_reconstruction_order(oracle):
    # cell averages of h(x) = sin(x): the reconstruction converges to h(x_{i+1/2})
    # at 5th order where the solution is smooth and monotone
    errs = []
    for h in [0.1, 0.05, 0.025]:
        xc = 0.3 + h * np.arange(-2, 3)
        avg = (np.cos(xc - h / 2) - np.cos(xc + h / 2)) / h
        errs.append(abs(oracle.weno5(avg) - math.sin(0.3 + h / 2)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] > 4.7, (errs, orders)


def test_weno5_picks_smooth_side_of_jump(oracle):
    # jump between cells i and i+1: the stencil S0 (i-2..i) is smooth; its weight dominates
    f = np.array([1.0, 1.0, 1.0, 0.0, 0.0])
    v = oracle.weno5(f)
    assert abs(v - 1.0) < 1e-6
    f = np.array([1.0, 1.0, 0.0, 0.0, 0.0])   # jump between i-1 and i: S2 (i..i+2) smooth
    assert abs(oracle.weno5(f)) < 1e-6


def test_weno5_odd_symmetry(oracle):
    rng = np.random.default_rng(1)
    for _ in range(20):
        f = rng.normal(size=5)
        assert oracle.weno5(-f) == -oracle.weno5(f)


# ------------------------------------------------------------------ Sod vs exact Riemann
def test_sod_normalized_vs_exact(oracle):
    """Normalized Sod problem: 400 cells, CFL 0.5, t = 0.2."""
    c = sod_case()
    U, T = oracle.case_state(c)
    U, T, t, dts, _ = oracle.step(c, U, T, 2000)
    assert t == pytest.approx(0.2, abs=1e-15)
    x = (np.arange(c.nx) + 0.5) * c.dx
    ex = refsol.riemann_sample(x, 0.2, 0.5, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    P = _prim(oracle, c, U, T)
    rho = P[0, 0]
    # plateaus (star states) and exact star values from the exact solver
    ps, us = refsol.riemann_star(1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert ps == pytest.approx(0.30313, abs=1e-5) and us == pytest.approx(0.92745, abs=1e-5)
    i55, i77 = int(0.55 / c.dx), int(0.77 / c.dx)
    assert abs(rho[i55] - ex[0, i55]) < 1e-3
    assert abs(rho[i77] - ex[0, i77]) < 1e-3
    assert abs(P[3, 0, i55] - ps) < 1e-3 and abs(P[1, 0, i55] - us) < 1e-3
    l1 = np.mean(np.abs(rho - ex[0]))
    assert l1 < 4e-3, l1
    # wave positions: shock location = where rho crosses midway between rho*_R and rho_R
    shock = x[np.argmax(rho < 0.5 * (0.26557 + 0.125))]
    assert abs(shock - 0.8504) < 2 * c.dx
    # nothing moves ahead of the rarefaction head / shock
    assert np.allclose(rho[x < 0.2], 1.0, atol=1e-4)
    assert np.allclose(rho[x > 0.9], 0.125, atol=1e-4)


def test_sod_paper_setup_vs_exact(oracle):
    """The paper's own Sod configuration (dimensional, CFL 0.2) against the exact solution."""
    g = json.load(open(os.path.join(GOLDEN, "sod_paper_setup.json")))
    nx = g["nx"]
    L = g["x_max"] - g["x_min"]
    dx = L / nx
    xc = g["x_min"] + (np.arange(nx) + 0.5) * dx
    left = xc < 0.0
    W = np.zeros((4, 1, nx))
    W[0, 0] = np.where(left, g["left"]["rho"], g["right"]["rho"])
    W[3, 0] = np.where(left, g["left"]["p"], g["right"]["p"])
    c = Case(name="sod_paper", model=MODEL_CPG, nx=nx, ny=1, dx=dx, dy=dx, bc=[BC_ZEROGRAD] * 4,
             W=W, gamma=g["gamma"], R=g["R"], cfl=g["cfl"], t_end=g["t_end"])
    U, T = oracle.case_state(c)
    U, T, t, _, _ = oracle.step(c, U, T, 5000)
    assert t == pytest.approx(g["t_end"], rel=1e-14)
    ex = refsol.riemann_sample(xc, g["t_end"], 0.0, g["left"]["rho"], 0.0, g["left"]["p"],
                               g["right"]["rho"], 0.0, g["right"]["p"], g["gamma"])
    P = _prim(oracle, c, U, T)
    assert np.mean(np.abs(P[0, 0] - ex[0])) < 4e-3
    assert np.mean(np.abs(P[3, 0] - ex[2])) / 1e5 < 4e-3
    # T = p / (rho R) of the perfect gas
    assert np.allclose(T[0], P[3, 0] / (P[0, 0] * g["R"]), rtol=1e-12)


# ------------------------------------------------------------------ orders of accuracy
def _wave_case(nx, ny=1, axis=0):
    n = nx
    dx = 1.0 / n
    W = np.zeros((4, ny if axis == 0 else n, n if axis == 0 else ny))
    x = (np.arange(n) + 0.5) * dx
    if axis == 0:
        W[0] = 1.0 + 0.2 * np.sin(2 * math.pi * x)[None, :]
        W[1] = 1.0
    else:
        W[0] = 1.0 + 0.2 * np.sin(2 * math.pi * x)[:, None]
        W[2] = 1.0
    W[3] = 1.0
    shape = W.shape[1:]
    return Case(name="wave", model=MODEL_CPG, nx=shape[1], ny=shape[0], dx=dx, dy=dx,
                bc=[BC_PERIODIC] * 4, W=W, gamma=1.4, R=1.0)


@pytest.mark.parametrize("axis", [0, 1])
def test_spatial_order_five(oracle, axis):
    """Advected density wave, dt ~ dx^(5/3) so the RK3 error shrinks like dx^5."""
    errs = []
    t_end = 0.5
    for n in [20, 40, 80]:
        c = _wave_case(n, ny=1 if axis == 0 else 1, axis=axis)
        if axis == 1:
            c.nx, c.ny = 1, n
        dt = 0.4 * (1.0 / n) ** (5.0 / 3.0)
        nst = int(math.ceil(t_end / dt))
        U, T = oracle.case_state(c)
        U, T, t, _, _ = oracle.step(c, U, T, nst, dt_fixed=t_end / nst)
        x = (np.arange(n) + 0.5) / n
        exact = 1.0 + 0.2 * np.sin(2 * math.pi * (x - t_end))
        errs.append(np.max(np.abs(U[0].ravel() - exact)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 4.5, (errs, orders)


def test_time_order_three(oracle):
    c = _wave_case(64)
    U0, T0 = oracle.case_state(c)
    t_end = 0.25

    def run(nst):
        U, T, _, _, _ = oracle.step(c, U0, T0, nst, dt_fixed=t_end / nst)
        return U[0]

    ref = run(1024)
    errs = [np.max(np.abs(run(n) - ref)) for n in [32, 64, 128]]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 2.8, (errs, orders)


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("model", [MODEL_CPG, MODEL_ONESTEP])
def test_constant_state_preserved(oracle, model):
    nx, ny = 24, 12
    nU = 4 if model == MODEL_CPG else 5
    W = np.zeros((nU, ny, nx))
    W[0], W[1], W[2], W[3] = 1.3, 0.7, -0.4, 2.1
    if model == MODEL_ONESTEP:
        W[4] = 0.0     # burned: no reaction, state must stay constant
    c = Case(name="const", model=model, nx=nx, ny=ny, dx=0.1, dy=0.07, bc=[BC_PERIODIC] * 4, W=W,
             gamma=1.3, R=1.0, Q=5.0, Ea=10.0, k=3.0, cfl=0.5)
    U0, T0 = oracle.case_state(c)
    U, T, _, _, _ = oracle.step(c, U0, T0, 100)
    for f in range(nU):
        assert np.all(U[f] == U[f].flat[0])          # every cell sees identical inputs
        assert abs(U[f].flat[0] - U0[f].flat[0]) <= 1e-14 * max(1.0, abs(U0[f].flat[0]))


def test_conservation_periodic_onestep(oracle):
    rng = np.random.default_rng(7)
    nx, ny = 32, 16
    W = np.zeros((5, ny, nx))
    W[0] = 1.0 + 0.2 * rng.uniform(size=(ny, nx))
    W[1] = 0.3 * rng.normal(size=(ny, nx))
    W[2] = 0.3 * rng.normal(size=(ny, nx))
    W[3] = 1.0 + rng.uniform(size=(ny, nx))
    W[4] = rng.uniform(size=(ny, nx))
    c = Case(name="cons", model=MODEL_ONESTEP, nx=nx, ny=ny, dx=0.05, dy=0.05,
             bc=[BC_PERIODIC] * 4, W=W, gamma=1.2, R=1.0, Q=2.0, Ea=3.0, k=1.0, cfl=0.4)
    U0, T0 = oracle.case_state(c)
    U, T, _, _, _ = oracle.step(c, U0, T0, 40)
    for f in range(4):
        s0, s1 = math.fsum(U0[f].ravel()), math.fsum(U[f].ravel())
        scale = math.fsum(np.abs(U0[f]).ravel())
        assert abs(s1 - s0) <= 1e-13 * scale, (f, s0, s1)
    # the fuel decreases only through the source term
    assert math.fsum(U[4].ravel()) < math.fsum(U0[4].ravel())


def test_slip_wall_no_mass_flux(oracle):
    """Mirror ghosts make the wall-face mass flux vanish exactly: total mass is
    conserved with walls on S/N and periodic E/W, and the wall-normal flux of
    every face is zero (checked by summing L over the grid)."""
    rng = np.random.default_rng(3)
    nx, ny = 16, 12
    W = np.zeros((4, ny, nx))
    W[0] = 1.0 + 0.3 * rng.uniform(size=(ny, nx))
    W[1] = 0.2 * rng.normal(size=(ny, nx))
    W[2] = 0.2 * rng.normal(size=(ny, nx))
    W[3] = 1.0 + rng.uniform(size=(ny, nx))
    c = Case(name="wall", model=MODEL_CPG, nx=nx, ny=ny, dx=0.1, dy=0.1,
             bc=[BC_PERIODIC, BC_PERIODIC, BC_SLIPWALL, BC_SLIPWALL], W=W, gamma=1.4, R=1.0)
    U, T = oracle.case_state(c)
    L = oracle.rhs(c, U, T)
    # sum of L_rho = -(sum of boundary face fluxes)/d = 0 when the wall fluxes vanish
    assert abs(math.fsum(L[0].ravel())) < 1e-12 * math.fsum(np.abs(L[0]).ravel())
    # tangential momentum also has zero flux through the wall (its ghost is even, p odd part absent)
    assert abs(math.fsum(L[1].ravel())) < 1e-12 * math.fsum(np.abs(L[1]).ravel())


def test_transpose_symmetry(oracle):
    """Swapping x and y (and u and v) transposes the result."""
    c = detonation_tube_case(nx=48, ny=16, seed=11)
    cT = detonation_tube_case(nx=48, ny=16, seed=11)
    WT = np.transpose(c.W, (0, 2, 1)).copy()
    WT[[1, 2]] = WT[[2, 1]]
    cT.W, cT.nx, cT.ny = WT, c.ny, c.nx
    cT.bc = [c.bc[2], c.bc[3], c.bc[0], c.bc[1]]
    fresh = c.bc_prim[1].copy()
    fresh[[1, 2]] = fresh[[2, 1]]
    cT.bc_prim = [None, None, None, fresh]
    U, T = oracle.case_state(c)
    UT, TT = oracle.case_state(cT)
    U, T, t, _, _ = oracle.step(c, U, T, 30)
    UT, TT, tT, _, _ = oracle.step(cT, UT, TT, 30)
    assert t == tT
    back = np.transpose(UT, (0, 2, 1))[[0, 2, 1, 3, 4]]
    for f in range(5):
        scale = np.max(np.abs(U[f])) + 1e-300
        assert np.max(np.abs(back[f] - U[f])) <= 1e-12 * scale, f


def test_mirror_symmetry_with_walls(oracle):
    """A y-symmetric state between slip walls stays mirror-symmetric (v odd)."""
    c = detonation_tube_case(nx=64, ny=16, seed=5)
    half = c.W[:, :8, :]
    c.W = np.concatenate([half, half[:, ::-1, :]], axis=1)
    c.W[2] = 0.0
    U, T = oracle.case_state(c)
    U, T, _, _, _ = oracle.step(c, U, T, 40)
    for f in range(5):
        m = U[f, ::-1, :] * (-1.0 if f == 2 else 1.0)
        assert np.max(np.abs(m - U[f])) <= 1e-12 * (np.max(np.abs(U[f])) + 1e-300)


def test_dirichlet_inflow_and_zero_gradient(oracle):
    """With a uniform fresh state, a Dirichlet side holding the same state and a
    zero-gradient side leave the state unchanged."""
    c = detonation_tube_case(nx=32, ny=8, seed=2)
    c.W[:] = c.bc_prim[1][:, None, None]
    U0, T0 = oracle.case_state(c)
    c.k = 0.0
    U, T, _, _, _ = oracle.step(c, U0, T0, 10)
    assert np.max(np.abs(U - U0)) < 1e-13


def test_cfl_time_step_formula(oracle):
    c = detonation_tube_case(nx=64, ny=16, seed=9)
    U, T = oracle.case_state(c)
    P = oracle.primitives(c, U, T)
    s = np.max((np.abs(P[1]) + P[5]) / c.dx + (np.abs(P[2]) + P[5]) / c.dy)
    _, _, t, dts, _ = oracle.step(c, U, T, 1)
    assert dts[0] == pytest.approx(c.cfl / s, rel=1e-15)
    # t_end clips the last step and later steps do nothing
    _, _, t, dts, _ = oracle.step(c, U, T, 5, t_end=2.5 * dts[0])
    assert t == pytest.approx(2.5 * dts[0], rel=1e-14)
    assert dts[3] == 0.0 and dts[4] == 0.0
