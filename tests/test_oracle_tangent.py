"""The oracle's forward-mode derivative of the probe loss (dual numbers through
the whole discrete map) against central finite differences.

This is what the hand-written adjoint is later checked against: the tangent
gives <grad L, v> exactly for any direction v (Q, Ea, initial density).
"""

import numpy as np
import pytest

from cases import adjoint_case


def _small():
    a = adjoint_case(nx=48, ny=16, nsteps=12)
    c = a["case"]
    probes = np.array([16 * 48 + 6, 15 * 48 + 6, 0 * 48 + 12, 15 * 48 + 12], dtype=np.int32)
    return c, probes, np.array([1.0, 0.5, 2.0, 1.0])


@pytest.mark.parametrize("which", ["Q", "Ea", "rho0"])
def test_tangent_matches_central_differences(oracle, which):
    c, probes, w = _small()
    probes = probes % (c.nx * c.ny)
    n = 12
    rng = np.random.default_rng(2)
    dW = np.zeros_like(c.W)
    if which == "rho0":
        # outside the ignition slab: inside it all cells tie for the maximum wave speed,
        # where the max is not differentiable and finite differences see the largest
        # one-sided derivative rather than the lowest-index tie-break
        dW[0] = rng.normal(size=c.W.shape[1:])
        dW[0][:, c.W[3, 0] > 1.0] = 0.0
    dQ = 1.0 if which == "Q" else 0.0
    dEa = 1.0 if which == "Ea" else 0.0
    L, dL = oracle.loss_tangent(c, c.W, n, probes, w, c.dt_fixed, dW0=dW, dQ=dQ, dEa=dEa)

    def loss_at(h):
        cc = adjoint_case(nx=48, ny=16, nsteps=12)["case"]
        cc.Q += h * dQ
        cc.Ea += h * dEa
        val, _ = oracle.loss_tangent(cc, c.W + h * dW, n, probes, w, c.dt_fixed)
        return val

    scale = {"Q": c.Q, "Ea": c.Ea, "rho0": 1.0}[which]
    h = 1e-6 * scale
    fd = (loss_at(h) - loss_at(-h)) / (2 * h)
    assert dL == pytest.approx(fd, rel=1e-5), (dL, fd)
    assert np.isfinite(L) and L > 0


@pytest.mark.parametrize("field", [0, 1, 3, 5])
def test_detailed_tangent_matches_central_differences(oracle, field):
    """The detailed model (NASA-7 Newton for T, point-implicit chemistry): the dual-number
    tangent of the probe loss along p, u, T and B2 directions equals central differences
    (h = 1e-7 relative). The state has no zero speed and no tied wave-speed maximum, so
    the loss is differentiable there."""
    from cases.amr import detailed_adjoint_case
    a = detailed_adjoint_case(nx=24, ny=12)
    c, probes, w = a["case"], a["probe_cell"], a["probe_w"]
    U, T = oracle.case_state(c)
    _, _, _, dts, _ = oracle.step(c, U, T, 1, cfl=a["cfl_dt"])
    dt = float(dts[0])
    rng = np.random.default_rng(10 + field)
    dW = np.zeros_like(c.W)
    dW[field] = rng.normal(size=c.W.shape[1:]) * np.abs(c.W[field]).max()
    n = 4
    L, dL = oracle.loss_tangent(c, c.W, n, probes, w, dt, dW0=dW)
    h = 1e-7
    Lp, _ = oracle.loss_tangent(c, c.W + h * dW, n, probes, w, dt)
    Lm, _ = oracle.loss_tangent(c, c.W - h * dW, n, probes, w, dt)
    fd = (Lp - Lm) / (2 * h)
    assert dL == pytest.approx(fd, rel=1e-5), (dL, fd)
    assert np.isfinite(L) and L > 0
