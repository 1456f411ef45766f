"""Pins of the oracle's crossover advance (paper Fig. 2a, Alg. 2): the deepest level
first, two steps of a level per step of the next coarser level, dt_l = dt_0 / 2^l.

* with one level the crossover advance is the synchronous advance, bitwise;
* a level 1 that covers the whole domain, advanced with a fixed dt_0, is the uniform
  fine grid advanced twice as often with dt_0 / 2, bitwise, and level 0 becomes its
  four-to-one mean;
* a constant state survives a 3-level crossover step, and its dt_0 is 4 times the
  synchronous dt (the CFL bound with level-0 spacing over all levels, bitwise).

How a partially refined level couples to the coarser state between the coarse steps
has no closed form: beyond these checks it is "parity unpinned" (oracle and HIP path
agree with each other only).
"""

import numpy as np

from cases import detonation_tube_case, Domain, BlockCase, MODEL_ONESTEP, BC_PERIODIC, \
    BC_SLIPWALL, BC_ZEROGRAD
from cases.common import make_blocks
from test_oracle_blocks import _split_uniform, _gather, _small_amr


def test_single_level_crossover_equals_synchronous(oracle):
    c = detonation_tube_case(nx=96, ny=32, seed=41)
    bc, _ = _split_uniform(c, [0, 40, 96], [0, 16, 32])
    U, T = oracle.block_state(bc)
    a = oracle.step_blocks(bc, U, T, 15)
    b = oracle.step_blocks(bc, U, T, 15, crossover=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def _full_refinement():
    fine = detonation_tube_case(nx=64, ny=32, dx=0.025, seed=29)
    fine.bc = [BC_ZEROGRAD, BC_ZEROGRAD, BC_SLIPWALL, BC_SLIPWALL]
    fine.bc_prim = [None] * 4
    nx0, ny0 = 32, 16
    coarseW = 0.25 * (fine.W[:, 0::2, 0::2] + fine.W[:, 0::2, 1::2] + fine.W[:, 1::2, 0::2]
                      + fine.W[:, 1::2, 1::2])
    recs = [(0, 0, 0, 0, nx0, ny0)] + [(0, 1, i0, j0, 32, 16) for j0 in (0, 16) for i0 in (0, 32)]
    W = [coarseW.reshape(5, -1)] + [fine.W[:, j0:j0 + 16, i0:i0 + 32].reshape(5, -1)
                                    for (_, _, i0, j0, _, _) in recs[1:]]
    dom = Domain(nx=nx0, ny=ny0, dx=0.05, dy=0.05, bc=fine.bc, nlevels=2, gamma=fine.gamma,
                 R=1.0, Q=fine.Q, Ea=fine.Ea, k=fine.k)
    bcase = BlockCase(name="full", model=MODEL_ONESTEP, domains=[dom], blocks=make_blocks(recs),
                      W=np.concatenate(W, axis=1), cfl=0.5)
    return fine, bcase, recs, nx0, ny0


def test_full_refinement_crossover_is_two_fine_steps(oracle):
    fine, bcase, recs, nx0, ny0 = _full_refinement()
    dt0 = 1.2e-3        # fine steps of 6e-4, under the fine grid's CFL-0.5 step (7.0e-4)
    Uf, Tf = oracle.case_state(fine)
    Ub, Tb = oracle.block_state(bcase)
    U1, _, t1, _, _ = oracle.step(fine, Uf, Tf, 12, dt_fixed=dt0 / 2)
    U2, _, t2, dts, _ = oracle.step_blocks(bcase, Ub, Tb, 6, dt_fixed=dt0, crossover=True)
    assert np.all(dts[:, 0] == dt0)
    assert abs(t2[0] - 6 * dt0) <= 1e-15 and abs(t1 - t2[0]) <= 1e-15
    G = _gather(U2[:, nx0 * ny0:], [(0, 0, i0, j0, 32, 16) for (_, _, i0, j0, _, _) in recs[1:]],
                U1.shape)
    assert np.array_equal(G, U1)
    mean = ((U1[:, 0::2, 0::2] + U1[:, 0::2, 1::2]) + (U1[:, 1::2, 0::2] + U1[:, 1::2, 1::2])) * 0.25
    assert np.array_equal(U2[:, :nx0 * ny0].reshape(5, ny0, nx0), mean)


def test_constant_state_crossover(oracle):
    bc = _small_amr()
    bc.W[:] = np.array([1.3, 0.4, 0.0, 2.0, 0.0])[:, None]
    bc.domains[0].bc = [BC_PERIODIC, BC_PERIODIC, BC_SLIPWALL, BC_SLIPWALL]
    U0, T0 = oracle.block_state(bc)
    U, T, _, dts, _ = oracle.step_blocks(bc, U0, T0, 3, crossover=True)
    for f in range(5):
        assert np.max(np.abs(U[f] - U0[f])) <= 1e-14 * max(1.0, np.max(np.abs(U0[f])))
    _, _, _, dsync, _ = oracle.step_blocks(bc, U0, T0, 1)
    assert dts[0, 0] == 4.0 * dsync[0, 0]
