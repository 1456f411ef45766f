"""The chemistry kernel specialised to the mechanism's structure (the default of a
detailed-model context) against the generic kernel (janc_set_chem_kernel), bitwise: the
specialisation changes where the cell's values live (registers instead of LDS columns),
not the arithmetic. Uniform fronts of four mechanisms (9 species one and two NASA-7
ranges, the 6-species chemkin mechanism, 12 species), the 30-reaction complete mechanism
in a 0-D reactor, Strang splitting, the small 3-level AMR hierarchy in both advances and
the 637-block workload; the species + T Jacobian uses the generic kernel either way. The
reversed chemistry kernel of the detailed adjoint follows the same selection and is checked
the same way: loss and gradient of a 6-step adjoint run, bitwise, for three mechanisms
(9 species with one and two NASA-7 ranges, the 30-reaction complete mechanism)."""

import numpy as np
import pytest

import paper_2504_13750_amd as janc
from cases import synthetic_mechanism, two_range_mechanism
from cases.amr import detailed_front_case, amr_case
from gpu_util import run_uniform, run_blocks

pytestmark = pytest.mark.gpu


def _ctx(mech, mode):
    ctx = janc.Context(janc.DETAILED, mech)
    ctx.chem_kernel = mode
    assert ctx.chem_kernel == mode
    return ctx


def _uniform_pair(case, nsteps, **kw):
    out = []
    for mode in (janc.CHEM_GENERIC, janc.CHEM_SPECIALIZED):
        ctx = _ctx(case.mech, mode)
        print(f"[gpu] chem kernel mode {mode}", flush=True)
        out.append(run_uniform(case, nsteps, ctx=ctx, **kw))
        ctx.close()
    (Ua, Ta, ta, da), (Ub, Tb, tb, db) = out
    assert np.array_equal(Ua, Ub) and np.array_equal(Ta, Tb) and ta == tb and np.array_equal(da, db)
    return Ub


def test_default_is_specialised_and_switchable():
    ctx = janc.Context(janc.DETAILED, synthetic_mechanism())
    assert ctx.chem_kernel == janc.CHEM_SPECIALIZED
    ctx.chem_kernel = janc.CHEM_GENERIC
    assert ctx.chem_kernel == janc.CHEM_GENERIC
    with pytest.raises(janc.JancError):
        ctx.chem_kernel = 7
    ctx.close()
    one = janc.Context(janc.ONESTEP)
    assert one.chem_kernel == janc.CHEM_GENERIC
    with pytest.raises(janc.JancError):
        one.chem_kernel = janc.CHEM_SPECIALIZED
    one.close()


@pytest.mark.parametrize("which", ["synthetic-9", "two-range-9", "chemkin-6", "inert-12"])
def test_front_generic_equals_specialised_bitwise(which):
    from test_gpu_species_counts import six_species_mechanism, twelve_species_mechanism
    if which in ("synthetic-9", "two-range-9"):
        mech = synthetic_mechanism() if which == "synthetic-9" else two_range_mechanism(synthetic_mechanism())
        c = detailed_front_case(nx=48, ny=40, mech=mech)
    elif which == "chemkin-6":
        c = _hotspot6(six_species_mechanism())
    else:
        from cases import Case
        mech = twelve_species_mechanism()
        base = detailed_front_case(nx=40, ny=24)
        W = np.zeros((4 + mech.ns - 1, base.ny, base.nx))
        W[:4] = base.W[:4]
        W[4:12] = base.W[4:12]
        W[12:15] = np.array([0.02, 0.03, 0.04])[:, None, None]
        c = Case(name="front12", model=base.model, nx=base.nx, ny=base.ny, dx=base.dx, dy=base.dy,
                 bc=base.bc, W=W, mech=mech, cfl=0.5)
    U = _uniform_pair(c, 4)
    assert np.all(np.isfinite(U))


def _hotspot6(mech):
    import math
    from cases import Case, MODEL_DETAILED, BC_ZEROGRAD, BC_SLIPWALL
    nx, ny, dx = 40, 24, 2e-5
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(xc, yc)
    r2 = ((X - 0.4 * nx * dx) ** 2 + (Y - 0.5 * ny * dx) ** 2) / (6 * dx) ** 2
    W = np.zeros((4 + mech.ns - 1, ny, nx))
    W[0] = 5 * 101325.0 * (1.0 + 2.0 * np.exp(-r2))
    W[1] = 30.0
    W[2] = 10.0 * np.sin(2 * math.pi * X / (nx * dx))
    W[3] = 1100.0 + 1400.0 * np.exp(-r2)
    Yf = {"X2": 0.08, "Y2": 0.22, "XY": 0.02, "Y": 0.01}
    for k, sp in enumerate(mech.species[:-1]):
        W[4 + k] = Yf.get(sp, 0.0)
    return Case(name="hotspot6", model=MODEL_DETAILED, nx=nx, ny=ny, dx=dx, dy=dx,
                bc=[BC_ZEROGRAD, BC_ZEROGRAD, BC_SLIPWALL, BC_SLIPWALL], W=W, mech=mech, cfl=0.5)


def test_strang_and_full_jacobian_generic_equals_specialised_bitwise():
    c = detailed_front_case(nx=48, ny=40)
    _uniform_pair(c, 3, split=janc.SPLIT_STRANG)
    _uniform_pair(c, 3, jac=janc.JAC_FULL)


def test_complete_mechanism_reactor_generic_equals_specialised_bitwise():
    from cases.mechanism import complete_mechanism
    from test_oracle_floors import reactor_case
    c = reactor_case(complete_mechanism(), "fresh-1500K", n=8)
    _uniform_pair(c, 20, dt_fixed=1e-8)


@pytest.mark.parametrize("which", ["small-9sp", "amr-637-blocks"])
def test_amr_generic_equals_specialised_bitwise(which):
    from test_gpu_blocks import _small_detailed_amr
    bc = _small_detailed_amr() if which == "small-9sp" else amr_case()
    crosses = (0, janc.PLAN_CROSSOVER) if which == "small-9sp" else (0,)
    for cross in crosses:
        res = []
        for mode in (janc.CHEM_GENERIC, janc.CHEM_SPECIALIZED):
            ctx = _ctx(bc.mech, mode)
            res.append(run_blocks(bc, 3, ctx=ctx, flags=cross))
            ctx.close()
        (Ua, Ta, ta), (Ub, Tb, tb) = res
        assert np.array_equal(Ua, Ub) and np.array_equal(Ta, Tb) and np.array_equal(ta, tb)


@pytest.mark.parametrize("which", ["synthetic-9", "two-range-9", "complete-9-30"])
def test_adjoint_generic_equals_specialised_bitwise(which):
    from cases.amr import detailed_adjoint_case
    from cases.mechanism import complete_mechanism
    from gpu_util import torch_dev
    from test_gpu_adjoint_detailed import _dt
    base = synthetic_mechanism()
    # the complete mechanism at a slower common rate (1e9): at its default (1e13) the
    # frozen-T point-implicit step of this hot front drives states out of the admissible
    # range within the six steps, in the oracle as on the GPU
    mech = {"synthetic-9": base, "two-range-9": two_range_mechanism(base),
            "complete-9-30": complete_mechanism(A_cgs=1e9)}[which]
    a = detailed_adjoint_case(nx=32, ny=16, nsteps=6, mech=mech)
    c = a["case"]
    c.dt_fixed = _dt(c, a["cfl_dt"])
    torch, dev = torch_dev()
    out = []
    for mode in (janc.CHEM_GENERIC, janc.CHEM_SPECIALIZED):
        print(f"[gpu] janc_adjoint {which} chem kernel mode {mode}", flush=True)
        ctx = _ctx(mech, mode)
        W0 = torch.tensor(c.W, dtype=torch.float64, device=dev)
        loss, gW, gth = ctx.adjoint(janc.grid_of(c), janc.physics_of(c), janc.make_time(0.0, c.dt_fixed, 0.0),
                                    W0, 6, 3, a["probe_cell"], a["probe_w"])
        ctx.sync_status()
        out.append((loss.item(), gW.cpu().numpy(), gth.cpu().numpy()))
        ctx.close()
    (La, Ga, ta), (Lb, Gb, tb) = out
    assert La == Lb and np.array_equal(Ga, Gb) and np.array_equal(ta, tb)
    assert np.all(np.isfinite(Gb)) and np.max(np.abs(Gb[4:])) > 0
