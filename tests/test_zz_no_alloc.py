"""The allocation-free entry point janc_step_noalloc against janc_step (GPU).

janc_step_noalloc runs the same kernels as janc_step with every workspace (stage
states, reductions, plan tables) in the library's static scratch array, launched
directly instead of through a captured graph; both forms give bitwise-identical
results, so it is held to equality with janc_step. Two calls in a row share the
array, the second on a smaller grid; a grid beyond the array is rejected.
"""

import numpy as np
import pytest

import paper_2504_13750_amd as janc
from cases import detonation_tube_case
from cases.amr import detailed_front_case
from gpu_util import context_for, torch_dev

pytestmark = pytest.mark.gpu


def _run(case, nsteps, noalloc, ctx):
    torch, dev = torch_dev()
    phys = janc.physics_of(case)
    U, T = ctx.init_state(phys, torch.tensor(case.W, dtype=torch.float64, device=dev))
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    dts = torch.zeros(nsteps, dtype=torch.float64, device=dev)
    step = ctx.step_noalloc if noalloc else ctx.step
    print(f"[gpu] {'janc_step_noalloc' if noalloc else 'janc_step'} {case.name} "
          f"{case.nx}x{case.ny} nsteps={nsteps}", flush=True)
    step(janc.grid_of(case), phys, janc.time_of(case), U, T, nsteps, t, dts)
    ctx.sync_status()
    return U.cpu().numpy(), T.cpu().numpy(), t.item(), dts.cpu().numpy()


@pytest.mark.parametrize("model", ["onestep", "detailed"])
def test_noalloc_equals_step_two_calls(model):
    if model == "onestep":
        big = detonation_tube_case(nx=384, ny=96, seed=31)
        small = detonation_tube_case(nx=100, ny=20, seed=32)
        nsteps = 12
    else:
        big = detailed_front_case(nx=96, ny=48)
        small = detailed_front_case(nx=40, ny=16)
        nsteps = 3
    ctx = context_for(big)
    ref = [_run(c, nsteps, False, ctx) for c in (big, small)]
    got = [_run(c, nsteps, True, ctx) for c in (big, small)]
    ctx.close()
    for (Ur, Tr, tr, dr), (Ug, Tg, tg, dg), c in zip(ref, got, (big, small)):
        print(f"  {c.name}: max |dU| {np.max(np.abs(Ug - Ur)):.3e}, t {tg:.15e} / {tr:.15e}",
              flush=True)
        assert np.array_equal(Ug, Ur)
        assert np.array_equal(Tg, Tr)
        assert tg == tr
        assert np.array_equal(dg, dr)


def test_noalloc_rejects_grids_beyond_the_scratch():
    """The 9-species model needs 16 * 13 bytes per cell: 600 x 600 cells exceed 64 MiB."""
    torch, dev = torch_dev()
    c = detailed_front_case(nx=24, ny=8)
    ctx = context_for(c)
    nx, ny = 600, 600
    U = torch.ones((ctx.nfields, ny, nx), dtype=torch.float64, device=dev)
    T = torch.ones((ny, nx), dtype=torch.float64, device=dev)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    grid = janc.make_grid(nx, ny, c.dx, c.dy, c.bc, c.bc_prim)
    print("[gpu] janc_step_noalloc 600x600 (rejected)", flush=True)
    with pytest.raises(janc.JancError) as ei:
        ctx.step_noalloc(grid, janc.physics_of(c), janc.time_of(c), U, T, 1, t)
    assert ei.value.code == -1
    assert "static scratch" in str(ei.value)
    # the context still works afterwards, through both entry points
    Ur, _, _, _ = _run(c, 2, False, ctx)
    Ug, _, _, _ = _run(c, 2, True, ctx)
    assert np.array_equal(Ug, Ur)
    ctx.close()
