"""Helpers that run the HIP library through its C ABI on seeded cases."""

import numpy as np

import paper_2504_13750_amd as janc


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def rel_err(a, b):
    """max_cells |a_f - b_f| / max_cells |b_f| per field (field-max normalization)."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    out = []
    for f in range(a.shape[0]):
        scale = np.max(np.abs(b[f]))
        d = np.max(np.abs(a[f] - b[f]))
        out.append(d / scale if scale > 0 else d)
    return np.array(out)


def context_for(case):
    return janc.Context(case.model, case.mech)


def run_uniform(case, nsteps, ctx=None, dt_fixed=None, t_end=None, cfl=None, W=None, split=0,
                jac=0):
    """init_state + janc_step on the GPU; returns numpy (U, T, t, dt_log)."""
    print(f"[gpu] janc_step {case.name} model={case.model} {case.nx}x{case.ny} nsteps={nsteps} "
          f"split={split} jac={jac}", flush=True)
    torch, dev = torch_dev()
    own = ctx is None
    ctx = ctx or context_for(case)
    phys = janc.physics_of(case)
    Wt = torch.tensor(case.W if W is None else W, dtype=torch.float64, device=dev)
    U, T = ctx.init_state(phys, Wt)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=dev)
    kw = {}
    if dt_fixed is not None:
        kw["dt_fixed"] = dt_fixed
    if t_end is not None:
        kw["t_end"] = t_end
    if cfl is not None:
        kw["cfl"] = cfl
    kw["split"] = split
    kw["jac"] = jac
    ctx.step(janc.grid_of(case), phys, janc.time_of(case, **kw), U, T, nsteps, t, dts)
    ctx.sync_status()
    out = (U.cpu().numpy(), T.cpu().numpy(), t.item(), dts.cpu().numpy()[:nsteps])
    if own:
        ctx.close()
    return out


def init_blocks(ctx, bcase):
    """Conserved pool from the primitive pool, domain by domain, on the GPU."""
    torch, dev = torch_dev()
    W = torch.tensor(bcase.W, dtype=torch.float64, device=dev)
    U = torch.zeros_like(W)
    T = torch.zeros(bcase.pool_cells, dtype=torch.float64, device=dev)
    for b in bcase.blocks:
        dom = bcase.domains[int(b["domain"])]
        s, n = int(b["offset"]), int(b["nx"]) * int(b["ny"])
        u, tt = ctx.init_state(janc.physics_of(dom), W[:, s:s + n].contiguous())
        U[:, s:s + n] = u
        T[s:s + n] = tt
    return U, T


def run_blocks(bcase, nsteps, ctx=None, flags=0, tile=0, keep=False, split=0, jac=0):
    print(f"[gpu] janc_step_blocks {bcase.name} blocks={len(bcase.blocks)} "
          f"pool={bcase.pool_cells} nsteps={nsteps} flags={flags} tile={tile} split={split} jac={jac}",
          flush=True)
    torch, dev = torch_dev()
    own = ctx is None
    ctx = ctx or context_for(bcase)
    plan = ctx.plan(janc.domains_of(bcase), bcase.blocks, bcase.pool_cells, flags)
    if tile:
        plan.set_tile(tile)
    U, T = init_blocks(ctx, bcase)
    t = torch.zeros(len(bcase.domains), dtype=torch.float64, device=dev)
    ctx.step_blocks(plan, janc.time_of(bcase, split=split, jac=jac), U, T, nsteps, t)
    ctx.sync_status()
    out = (U.cpu().numpy(), T.cpu().numpy(), t.cpu().numpy())
    plan.close()
    if own:
        ctx.close()
    return out
