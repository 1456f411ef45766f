"""Time loop of an adaptive run: steps of a block hierarchy with a layer update every
`every` steps (the main loop of Alg. 2; the paper's AMR runs update every 40 steps,
Sec. 5.2.3). Every step and every update runs in the HIP library (janc_step_blocks,
janc_regrid, janc_regrid_fill); this class only keeps the current plan and pools.
"""

from . import Context, PLAN_DEFAULT


class AdaptiveRun:
    """An adaptive hierarchy advanced on one device.

    ctx: Context; domains: janc_domain array (domains_of); blocks / pool_cells: the
    initial table; U, T: its pools (device tensors); time: janc_time; t: device tensor of
    per-domain times; regrid: (threshold, buffer, sub) of janc_regrid_params; every:
    steps between layer updates; flags: plan flags (e.g. PLAN_CROSSOVER).
    """

    def __init__(self, ctx: Context, domains, blocks, pool_cells, U, T, time, t, regrid,
                 every=40, flags=PLAN_DEFAULT, stream=None):
        self.ctx, self.domains, self.time, self.t = ctx, domains, time, t
        self.regrid_params = tuple(regrid)
        self.every, self.flags, self.stream = int(every), int(flags), stream
        if self.every < 1:
            raise ValueError("every must be >= 1")
        self.blocks = blocks
        self.plan = ctx.plan(domains, blocks, pool_cells, flags)
        self.U, self.T = U, T
        self.steps = 0          # steps taken since the start
        self.updates = 0

    def update_layers(self):
        """One layer update: new table from the current state, new plan, filled pools."""
        thr, buf, sub = self.regrid_params
        blocks, pool = self.ctx.regrid(self.plan, self.U, thr, buf, sub, stream=self.stream)
        plan = self.ctx.plan(self.domains, blocks, pool, self.flags)
        U, T = self.ctx.regrid_fill(self.plan, self.U, self.T, plan, stream=self.stream)
        self.plan.close()
        self.plan, self.blocks, self.U, self.T = plan, blocks, U, T
        self.updates += 1

    def advance(self, nsteps):
        """nsteps steps, with a layer update whenever the step count reaches a multiple of
        `every` (after that step)."""
        left = int(nsteps)
        while left > 0:
            n = min(left, self.every - self.steps % self.every)
            self.ctx.step_blocks(self.plan, self.time, self.U, self.T, n, self.t,
                                 stream=self.stream)
            self.steps += n
            left -= n
            if self.steps % self.every == 0:
                self.update_layers()

    def close(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None
