"""GPU discrete adjoint (janc_adjoint) against the oracle's exact tangents and
central finite differences.

* dL/dQ and dL/dEa against the oracle's dual-number tangents (<= 1e-10 relative);
* <dL/dW0, v> along seeded directions against the oracle's tangent (<= 1e-10);
* the full gradient of a 1-3 step trajectory on an 8 x 4 grid, element by
  element, against oracle tangents along every basis direction, for three sets of
  boundary rules (every ghost rule in both sweeps);
* central differences (h = 1e-6 relative) of the GPU loss on Q and Ea at the full
  adjoint workload (<= 1e-5);
* the checkpoint interval does not change the result (bitwise);
* the full adjoint workload: 512 x 64, 400 steps, checkpoints every 20;
* torch autograd through the adjoint (both models).
"""

import numpy as np
import pytest

import oracle
import paper_2504_13750_amd as janc
from cases import adjoint_case, detonation_tube_case, BC_PERIODIC, BC_SLIPWALL, BC_ZEROGRAD, BC_DIRICHLET
from gpu_util import torch_dev

pytestmark = pytest.mark.gpu


def _gpu_adjoint(case, nsteps, probes, w, ckpt, W=None, Q=None, Ea=None):
    print(f"[gpu] janc_adjoint {case.nx}x{case.ny} nsteps={nsteps} ckpt={ckpt}", flush=True)
    torch, dev = torch_dev()
    ctx = janc.Context(janc.ONESTEP)
    ph = janc.make_physics(case.gamma, case.R, case.Q if Q is None else Q,
                           case.Ea if Ea is None else Ea, case.k)
    W0 = torch.tensor(case.W if W is None else W, dtype=torch.float64, device=dev)
    loss, gW, gth = ctx.adjoint(janc.grid_of(case), ph, janc.make_time(0.0, case.dt_fixed, 0.0),
                                W0, nsteps, ckpt, probes, w)
    ctx.sync_status()
    out = loss.item(), gW.cpu().numpy(), gth.cpu().numpy()
    ctx.close()
    return out


def _small(nx=48, ny=16):
    a = adjoint_case(nx=nx, ny=ny, nsteps=12)
    c = a["case"]
    probes = np.array([(ny // 2) * nx + 6, (ny - 1) * nx + 6, 12, (ny - 1) * nx + 12], np.int32)
    return c, probes, np.array([1.0, 0.5, 2.0, 1.0])


def test_parameter_gradients_match_oracle_tangents():
    c, probes, w = _small()
    L, gW, gth = _gpu_adjoint(c, 12, probes, w, ckpt=5)
    Lo, dQ = oracle.loss_tangent(c, c.W, 12, probes, w, c.dt_fixed, dQ=1.0)
    _, dEa = oracle.loss_tangent(c, c.W, 12, probes, w, c.dt_fixed, dEa=1.0)
    print(f"  loss gpu {L:.15e} oracle {Lo:.15e}; dQ {gth[0]:.12e} vs {dQ:.12e}; "
          f"dEa {gth[1]:.12e} vs {dEa:.12e}", flush=True)
    assert L == pytest.approx(Lo, rel=1e-12)
    assert gth[0] == pytest.approx(dQ, rel=1e-10, abs=0.0)
    assert gth[1] == pytest.approx(dEa, rel=1e-10, abs=0.0)


def _untied(nx=48, ny=16, seed=31):
    """The small tube with a little y velocity and pressure noise everywhere (ignition
    slab included), so that the wave-speed maxima are attained at single cells with
    v != 0: there the discrete map is differentiable. (In the uniform slab the maxima
    tie and v is zero up to rounding, where max and |v| have no derivative and two
    implementations may select different subgradients.)"""
    c, probes, w = _small(nx, ny)
    rng = np.random.default_rng(seed)
    c.W[2] = 0.02 * rng.uniform(-1.0, 1.0, size=c.W.shape[1:])
    c.W[3] *= 1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=c.W.shape[1:])
    return c, probes, w


@pytest.mark.parametrize("field", [0, 1, 2, 3, 4])
def test_directional_gradient_matches_oracle(field):
    c, probes, w = _untied()
    L, gW, gth = _gpu_adjoint(c, 12, probes, w, ckpt=4)
    rng = np.random.default_rng(100 + field)
    v = np.zeros_like(c.W)
    v[field] = rng.normal(size=c.W.shape[1:])
    _, dv = oracle.loss_tangent(c, c.W, 12, probes, w, c.dt_fixed, dW0=v)
    got = float(np.sum(gW * v))
    print(f"  field {field}: <g, v> gpu {got:.12e} oracle {dv:.12e}", flush=True)
    assert got == pytest.approx(dv, rel=1e-10, abs=0.0)


# boundary sets (W, E, S, N): the tube's; periodic everywhere; slip wall W, zero-gradient
# E, a Dirichlet inflow S (the fresh state) and zero-gradient N -- every ghost rule on
# both sweeps, with the ghost positions that one cell owns merged per side
_BCS = {"tube": None,
        "periodic": ([BC_PERIODIC] * 4, [None] * 4),
        "mixed": ([BC_SLIPWALL, BC_ZEROGRAD, BC_DIRICHLET, BC_ZEROGRAD],
                  [None, None, np.array([1.0, 0.0, 0.1, 1.0, 1.0]), None])}


@pytest.mark.parametrize("bcs", ["tube", "periodic", "mixed"])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_full_gradient_brute_force_tiny_grid(nsteps, bcs):
    c, _, _ = _small(nx=8, ny=4)
    if _BCS[bcs] is not None:
        c.bc, c.bc_prim = list(_BCS[bcs][0]), list(_BCS[bcs][1])
    c.W[3] = 1.0 + 0.3 * np.random.default_rng(5).uniform(size=c.W.shape[1:])  # no ties in max
    c.W[0] = 1.0 + 0.2 * np.random.default_rng(6).uniform(size=c.W.shape[1:])
    c.W[1] = 0.1 * np.random.default_rng(7).normal(size=c.W.shape[1:])
    probes = np.array([5, 17, 30], np.int32)
    w = np.array([1.0, -0.5, 2.0])
    L, gW, gth = _gpu_adjoint(c, nsteps, probes, w, ckpt=2)
    ref = np.zeros_like(c.W)
    for f in range(5):
        for j in range(c.ny):
            for i in range(c.nx):
                e = np.zeros_like(c.W)
                e[f, j, i] = 1.0
                ref[f, j, i] = oracle.loss_tangent(c, c.W, nsteps, probes, w, c.dt_fixed, dW0=e)[1]
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(gW - ref)) / scale
    print(f"  brute force {bcs} {nsteps} steps: max |g - ref| / max|ref| = {err:.2e}", flush=True)
    assert err <= 1e-10


def test_coinciding_probes_match_oracle():
    """Probes that share a cell are applied together, in probe order: gradients along a
    random direction in all fields and dL/dQ still equal the oracle's tangents. (Weights
    of one sign: a dL/dQ that cancels to a small fraction of its terms has no relative
    accuracy to test.)"""
    c, probes, w = _untied()
    probes = np.array([probes[0], probes[0], probes[1], probes[0], probes[2]], np.int32)
    w = np.array([1.0, 0.25, 0.5, 2.0, 1.5])
    L, gW, gth = _gpu_adjoint(c, 8, probes, w, ckpt=3)
    Lo, dQ = oracle.loss_tangent(c, c.W, 8, probes, w, c.dt_fixed, dQ=1.0)
    v = np.random.default_rng(77).normal(size=c.W.shape)
    _, dv = oracle.loss_tangent(c, c.W, 8, probes, w, c.dt_fixed, dW0=v)
    got = float(np.sum(gW * v))
    print(f"  loss {L:.15e} / {Lo:.15e}; dQ {gth[0]:.12e} / {dQ:.12e}; <g, v> {got:.12e} / "
          f"{dv:.12e}", flush=True)
    assert L == pytest.approx(Lo, rel=1e-12)
    assert gth[0] == pytest.approx(dQ, rel=1e-10, abs=0.0)
    assert got == pytest.approx(dv, rel=1e-10, abs=0.0)


@pytest.mark.parametrize("bad", ["count", "cell"])
def test_bad_probes_rejected(bad):
    c, probes, w = _small()
    if bad == "count":
        probes = np.resize(probes, 9).astype(np.int32)
        w = np.ones(9)
    else:
        probes = probes.copy()
        probes[1] = c.nx * c.ny
    torch, dev = torch_dev()
    ctx = janc.Context(janc.ONESTEP)
    W0 = torch.tensor(c.W, dtype=torch.float64, device=dev)
    with pytest.raises(janc.JancError) as ei:
        ctx.adjoint(janc.grid_of(c), janc.physics_of(c), janc.make_time(0.0, c.dt_fixed, 0.0),
                    W0, 4, 2, probes, w)
    assert ei.value.code == -1
    ctx.close()


def test_checkpoint_interval_does_not_change_result():
    c, probes, w = _small()
    a = _gpu_adjoint(c, 12, probes, w, ckpt=12)
    b = _gpu_adjoint(c, 12, probes, w, ckpt=5)
    d = _gpu_adjoint(c, 12, probes, w, ckpt=1)
    assert a[0] == b[0] == d[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[1], d[1])
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[2], d[2])


def test_adjoint_tube_512x64_400_steps():
    """512 x 64 tube, 400 steps, checkpoints every 20: parameter gradients against the
    oracle's tangents and central differences; a density direction against the oracle."""
    a = adjoint_case()
    c, probes, w, k = a["case"], a["probe_cell"], a["probe_w"], a["ckpt_every"]
    L, gW, gth = _gpu_adjoint(c, 400, probes, w, ckpt=k)
    Lo, dQ = oracle.loss_tangent(c, c.W, 400, probes, w, c.dt_fixed, dQ=1.0)
    _, dEa = oracle.loss_tangent(c, c.W, 400, probes, w, c.dt_fixed, dEa=1.0)
    print(f"  loss {L:.15e} / {Lo:.15e}; dQ {gth[0]:.10e} / {dQ:.10e}; dEa {gth[1]:.10e} / "
          f"{dEa:.10e}", flush=True)
    assert L == pytest.approx(Lo, rel=1e-12)
    assert gth[0] == pytest.approx(dQ, rel=1e-10, abs=0.0)
    assert gth[1] == pytest.approx(dEa, rel=1e-10, abs=0.0)
    rng = np.random.default_rng(9)
    v = np.zeros_like(c.W)
    v[0] = rng.normal(size=c.W.shape[1:])
    v[0][:, c.W[3, 0] > 1.0] = 0.0
    _, dv = oracle.loss_tangent(c, c.W, 400, probes, w, c.dt_fixed, dW0=v)
    got = float(np.sum(gW * v))
    print(f"  <dL/drho0, v> gpu {got:.10e} oracle {dv:.10e}", flush=True)
    assert got == pytest.approx(dv, rel=1e-9, abs=0.0)
    for q, name in [(0, "Q"), (1, "Ea")]:
        base = c.Q if q == 0 else c.Ea
        h = 1e-6 * base
        Lp = _gpu_adjoint(c, 400, probes, w, ckpt=k, **{name: base + h})[0]
        Lm = _gpu_adjoint(c, 400, probes, w, ckpt=k, **{name: base - h})[0]
        fd = (Lp - Lm) / (2 * h)
        print(f"  d/d{name}: adjoint {gth[q]:.10e} fd {fd:.10e}", flush=True)
        assert gth[q] == pytest.approx(fd, rel=1e-5, abs=0.0)


def test_probe_loss_autograd_function():
    """torch autograd through the adjoint: gradients equal janc_adjoint's (bitwise, scaled by
    the incoming gradient) and the oracle's tangents; the detailed model through the same
    function."""
    import torch
    from paper_2504_13750_amd.autograd import probe_loss
    c, probes, w = _small()
    _, dev = torch_dev()
    ctx = janc.Context(janc.ONESTEP)
    g = janc.grid_of(c)
    W0 = torch.tensor(c.W, dtype=torch.float64, device=dev, requires_grad=True)
    theta = torch.tensor([c.Q, c.Ea], dtype=torch.float64, device=dev, requires_grad=True)
    L = probe_loss(ctx, g, c.gamma, c.R, c.k, c.dt_fixed, W0, theta, 12, 5, probes, w)
    gW, gth = torch.autograd.grad(3.0 * L, (W0, theta))
    Ld, gWd, gthd = _gpu_adjoint(c, 12, probes, w, ckpt=5)
    assert L.item() == Ld
    assert np.array_equal(gW.cpu().numpy(), 3.0 * gWd) and np.array_equal(gth.cpu().numpy(), 3.0 * gthd)
    _, dQ = oracle.loss_tangent(c, c.W, 12, probes, w, c.dt_fixed, dQ=1.0)
    assert gth[0].item() == pytest.approx(3.0 * dQ, rel=1e-10)
    ctx.close()
    # the detailed model: dL/dW0 through autograd equals janc_adjoint's, dL/dtheta is zero
    from test_gpu_adjoint_detailed import _case, _gpu_adjoint as _det_adjoint
    cd, pd, wd = _case(16, 8, 3)
    dctx = janc.Context(janc.DETAILED, cd.mech)
    Wd = torch.tensor(cd.W, dtype=torch.float64, device=dev, requires_grad=True)
    th0 = torch.zeros(2, dtype=torch.float64, device=dev, requires_grad=True)
    Ldet = probe_loss(dctx, janc.grid_of(cd), 0.0, 0.0, 0.0, cd.dt_fixed, Wd, th0, 3, 2, pd, wd)
    gWdet, gthdet = torch.autograd.grad(2.0 * Ldet, (Wd, th0))
    Lr, gWr, _ = _det_adjoint(cd, 3, pd, wd, ckpt=2)
    assert Ldet.item() == Lr
    assert np.array_equal(gWdet.cpu().numpy(), 2.0 * gWr)
    assert np.all(gthdet.cpu().numpy() == 0.0)
    dctx.close()
