"""Host logic of AdaptiveRun (the adaptive time loop): step chunks and update points,
checked with a stand-in context that records the calls (no GPU)."""

import numpy as np

from paper_2504_13750_amd.amr import AdaptiveRun


class _Plan:
    def __init__(self, log, tag):
        self.log, self.tag = log, tag

    def close(self):
        self.log.append(("close", self.tag))


class _Ctx:
    def __init__(self):
        self.log, self.nplans = [], 0

    def plan(self, domains, blocks, pool, flags):
        self.nplans += 1
        self.log.append(("plan", self.nplans, pool, flags))
        return _Plan(self.log, self.nplans)

    def step_blocks(self, plan, time, U, T, n, t, stream=None):
        self.log.append(("step", plan.tag, n))

    def regrid(self, plan, U, thr, buf, sub, stream=None):
        self.log.append(("regrid", plan.tag, thr, buf, sub))
        return np.zeros(3), 100 + plan.tag

    def regrid_fill(self, old, U, T, new, stream=None):
        self.log.append(("fill", old.tag, new.tag))
        return "U%d" % new.tag, "T%d" % new.tag


def test_chunks_and_updates():
    ctx = _Ctx()
    run = AdaptiveRun(ctx, None, np.zeros(2), 50, "U0", "T0", None, None, (0.1, 2, 8), every=4,
                      flags=4)
    run.advance(3)
    run.advance(7)
    steps = [e for e in ctx.log if e[0] == "step"]
    assert steps == [("step", 1, 3), ("step", 1, 1), ("step", 2, 4), ("step", 3, 2)]
    assert run.steps == 10 and run.updates == 2
    assert ("regrid", 1, 0.1, 2, 8) in ctx.log and ("fill", 1, 2) in ctx.log
    assert ("fill", 2, 3) in ctx.log and ("close", 1) in ctx.log and ("close", 2) in ctx.log
    assert [e for e in ctx.log if e[0] == "plan"] == [("plan", 1, 50, 4), ("plan", 2, 101, 4),
                                                      ("plan", 3, 102, 4)]
    assert run.U == "U3" and run.T == "T3"
    run.advance(0)
    assert run.steps == 10
    run.close()
    assert ctx.log[-1] == ("close", 3)


def test_update_after_exact_multiple():
    ctx = _Ctx()
    run = AdaptiveRun(ctx, None, np.zeros(2), 50, "U0", "T0", None, None, (0.1, 2, 8), every=5)
    run.advance(5)
    assert run.updates == 1 and [e for e in ctx.log if e[0] == "step"] == [("step", 1, 5)]
    run.advance(4)
    assert run.updates == 1
    run.advance(1)
    assert run.updates == 2
