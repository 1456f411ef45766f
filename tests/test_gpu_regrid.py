"""GPU layer update (janc_regrid, janc_regrid_fill) against the oracle.

Bar: the new block tables are integer data and must be identical; the new pools are
copies and injections and must be bitwise equal to the oracle's fill of the same
state; a run that steps, updates the layers and steps again stays within 1e-10 per
conserved field of the oracle doing the same.
"""

import numpy as np
import pytest

import oracle
import paper_2504_13750_amd as janc
from cases import BlockCase, synthetic_mechanism, amr_case
from gpu_util import init_blocks, context_for, rel_err, torch_dev
from test_oracle_regrid import _base_case, _smooth_bump, _with_table, _table

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _small_detailed_amr():
    mech = synthetic_mechanism()
    return amr_case(mech=mech, nx0=128, ny0=64, dx0=25e-6 * 1024 / 128 / 4, nlevels=3,
                    widths=(0.28e-3, 0.2e-3), blk0=32, nsteps=3)


CASES = {
    "jump-2lev": lambda: _base_case(jump_at=77),
    "bump-3lev": lambda: _base_case(nlevels=3, rho=_smooth_bump),
    "front-9sp-3lev": _small_detailed_amr,
    "amr-9sp-1024x512-full": amr_case,
    "two-domains-3lev": lambda: __import__("test_gpu_blocks")._amr_pair()[0],
}
PARAMS = {"jump-2lev": (0.01, 3, 8), "bump-3lev": (0.02, 4, 8), "front-9sp-3lev": (0.05, 4, 8),
          "amr-9sp-1024x512-full": (0.05, 4, 8), "two-domains-3lev": (0.005, 4, 8)}


@pytest.mark.parametrize("name", list(CASES))
def test_regrid_table_and_fill_match_oracle(name):
    c = CASES[name]()
    thr, buf, sub = PARAMS[name]
    print(f"[gpu] janc_regrid {name} blocks={len(c.blocks)} thr={thr} buffer={buf} sub={sub}",
          flush=True)
    ctx = context_for(c)
    plan = ctx.plan(janc.domains_of(c), c.blocks, c.pool_cells)
    U, T = init_blocks(ctx, c)
    blocks, pool = ctx.regrid(plan, U, thr, buf, sub)
    Uh, Th = U.cpu().numpy(), T.cpu().numpy()
    ob, opool = oracle.regrid(c, Uh, thr, buf, sub)
    assert _table(blocks) == _table(ob) and pool == opool
    assert (blocks["level"] > 0).any()
    new_plan = ctx.plan(janc.domains_of(c), blocks, pool)
    Un, Tn = ctx.regrid_fill(plan, U, T, new_plan)
    oU, oT = oracle.regrid_fill(c, Uh, Th, ob, opool)
    assert np.array_equal(Un.cpu().numpy(), oU) and np.array_equal(Tn.cpu().numpy(), oT)
    new_plan.close()
    plan.close()
    ctx.close()


def test_step_regrid_step_vs_oracle():
    c = _small_detailed_amr()
    thr, buf, sub = PARAMS["front-9sp-3lev"]
    print("[gpu] step / regrid / step front-9sp-3lev", flush=True)
    torch, dev = torch_dev()
    ctx = context_for(c)
    plan = ctx.plan(janc.domains_of(c), c.blocks, c.pool_cells)
    U, T = init_blocks(ctx, c)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.step_blocks(plan, janc.time_of(c), U, T, 3, t)
    blocks, pool = ctx.regrid(plan, U, thr, buf, sub)
    new_plan = ctx.plan(janc.domains_of(c), blocks, pool)
    Un, Tn = ctx.regrid_fill(plan, U, T, new_plan)
    ctx.step_blocks(new_plan, janc.time_of(c), Un, Tn, 3, t)
    ctx.sync_status()
    # oracle: the same sequence from the same initial primitives
    Uo, To = oracle.block_state(c)
    Uo, To, to, _, _ = oracle.step_blocks(c, Uo, To, 3)
    ob, opool = oracle.regrid(c, Uo, thr, buf, sub)
    assert _table(blocks) == _table(ob)
    Uo, To = oracle.regrid_fill(c, Uo, To, ob, opool)
    n = _with_table(c, ob, opool)
    Uo, To, to, _, _ = oracle.step_blocks(n, Uo, To, 3, t=to)
    e = rel_err(Un.cpu().numpy(), Uo)
    eT = rel_err(Tn.cpu().numpy()[None], To[None])[0]
    print(f"  regrid run: blocks {len(c.blocks)} -> {len(blocks)}, per-field rel err "
          f"{np.array2string(e, precision=2)}, T {eT:.2e}", flush=True)
    assert np.all(e <= TOL) and eT <= TOL
    assert t.item() == pytest.approx(to[0], rel=1e-12)
    for p in (new_plan, plan):
        p.close()
    ctx.close()


def test_regrid_rejects_bad_parameters():
    c = _base_case(jump_at=77)
    ctx = context_for(c)
    plan = ctx.plan(janc.domains_of(c), c.blocks, c.pool_cells)
    U, T = init_blocks(ctx, c)
    for thr, buf, sub in [(-1.0, 2, 8), (0.1, -1, 8), (0.1, 2, 6), (0.1, 2, 256)]:
        with pytest.raises(janc.JancError) as ei:
            ctx.regrid(plan, U, thr, buf, sub)
        assert ei.value.code == -1
    plan.close()
    ctx.close()


def test_adaptive_run_vs_oracle():
    """Steps with a layer update every 4 steps (AdaptiveRun) against the oracle doing the
    same sequence: 10 steps, updates after steps 4 and 8."""
    from paper_2504_13750_amd.amr import AdaptiveRun
    c = _small_detailed_amr()
    thr, buf, sub = PARAMS["front-9sp-3lev"]
    print("[gpu] AdaptiveRun front-9sp-3lev, 10 steps, update every 4", flush=True)
    torch, dev = torch_dev()
    ctx = context_for(c)
    U, T = init_blocks(ctx, c)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    run = AdaptiveRun(ctx, janc.domains_of(c), c.blocks, c.pool_cells, U, T, janc.time_of(c), t,
                      (thr, buf, sub), every=4)
    run.advance(3)
    run.advance(7)
    ctx.sync_status()
    assert run.steps == 10 and run.updates == 2
    Uo, To = oracle.block_state(c)
    n, to = c, None
    for chunk in (4, 4, 2):
        Uo, To, to, _, _ = oracle.step_blocks(n, Uo, To, chunk, t=to)
        if chunk == 4:
            ob, opool = oracle.regrid(n, Uo, thr, buf, sub)
            Uo, To = oracle.regrid_fill(n, Uo, To, ob, opool)
            n = _with_table(c, ob, opool)
    assert _table(run.blocks) == _table(n.blocks)
    e = rel_err(run.U.cpu().numpy(), Uo)
    eT = rel_err(run.T.cpu().numpy()[None], To[None])[0]
    print(f"  adaptive run: {len(run.blocks)} blocks, per-field rel err "
          f"{np.array2string(e, precision=2)}, T {eT:.2e}", flush=True)
    assert np.all(e <= TOL) and eT <= TOL
    assert t.item() == pytest.approx(to[0], rel=1e-12)
    run.close()
    ctx.close()


def test_adaptive_run_crossover_vs_oracle():
    """The same with the crossover advance (a step is one level-0 step)."""
    from paper_2504_13750_amd.amr import AdaptiveRun
    c = _small_detailed_amr()
    thr, buf, sub = PARAMS["front-9sp-3lev"]
    print("[gpu] AdaptiveRun crossover front-9sp-3lev, 3 steps, update every 2", flush=True)
    torch, dev = torch_dev()
    ctx = context_for(c)
    U, T = init_blocks(ctx, c)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    run = AdaptiveRun(ctx, janc.domains_of(c), c.blocks, c.pool_cells, U, T, janc.time_of(c), t,
                      (thr, buf, sub), every=2, flags=janc.PLAN_CROSSOVER)
    run.advance(3)
    ctx.sync_status()
    Uo, To = oracle.block_state(c)
    Uo, To, to, _, _ = oracle.step_blocks(c, Uo, To, 2, crossover=True)
    ob, opool = oracle.regrid(c, Uo, thr, buf, sub)
    Uo, To = oracle.regrid_fill(c, Uo, To, ob, opool)
    n = _with_table(c, ob, opool)
    Uo, To, to, _, _ = oracle.step_blocks(n, Uo, To, 1, t=to, crossover=True)
    assert _table(run.blocks) == _table(ob)
    e = rel_err(run.U.cpu().numpy(), Uo)
    print(f"  adaptive crossover run: per-field rel err {np.array2string(e, precision=2)}",
          flush=True)
    assert np.all(e <= TOL)
    run.close()
    ctx.close()


def test_regrid_capacity_reported():
    """janc_regrid with too small an output table returns JANC_EINVAL and the length needed."""
    import ctypes as C
    from paper_2504_13750_amd import _lib as L
    c = _base_case(jump_at=77)
    ctx = context_for(c)
    plan = ctx.plan(janc.domains_of(c), c.blocks, c.pool_cells)
    U, T = init_blocks(ctx, c)
    full, pool = ctx.regrid(plan, U, 0.01, 3, 8)
    out = np.zeros(2, dtype=janc.BLOCK_DTYPE)
    n, p = C.c_int(0), C.c_longlong(0)
    params = L.janc_regrid_params(0.01, 3, 8)
    st = L.lib().janc_regrid(ctx.h, plan.h, C.byref(params), C.c_void_p(U.data_ptr()),
                             out.ctypes.data_as(C.c_void_p), 2, C.byref(n), C.byref(p),
                             C.c_void_p(torch_dev()[0].cuda.current_stream().cuda_stream))
    assert st == -1 and n.value == len(full) and p.value == pool
    plan.close()
    ctx.close()
