"""Pins of the oracle's block-table path (paper Sec. 3.1.3-3.1.4, Alg. 2-3).

* decomposition invariance: a uniform grid split into level-0 blocks of
  uneven sizes gives the uniform result bitwise (ghosts from neighbours are
  the same cells the uniform stencil reads);
* ensemble independence: domains advanced together equal each alone;
* a level that covers the whole domain reproduces the uniform fine grid and
  its parent level becomes the four-to-one mean;
* ring cells hold the injection of the coarser level, restricted cells the
  mean of their four children, and a constant state survives a 3-level
  hierarchy unchanged.

The coarse-fine coupling itself has no closed form: beyond these checks and the
symmetry and convergence pins of test_oracle_amr_symmetry.py its parity is
"parity unpinned" (oracle and HIP path agree with each other only).
"""

import numpy as np
import pytest

from cases import (detonation_tube_case, ensemble_case, amr_case, synthetic_mechanism, Domain,
                   BlockCase, MODEL_ONESTEP, MODEL_CPG, BC_PERIODIC, BC_SLIPWALL, BC_ZEROGRAD)
from cases.common import make_blocks
from cases.amr import build_hierarchy


def _split_uniform(case, xs, ys):
    """Tile a uniform case with level-0 blocks at x cuts xs and y cuts ys."""
    recs, cols = [], []
    for j0, j1 in zip(ys[:-1], ys[1:]):
        for i0, i1 in zip(xs[:-1], xs[1:]):
            recs.append((0, 0, i0, j0, i1 - i0, j1 - j0))
    blocks = make_blocks(recs)
    W = np.concatenate([case.W[:, j0:j0 + ny, i0:i0 + nx].reshape(case.nU, -1)
                        for (_, _, i0, j0, nx, ny) in recs], axis=1)
    dom = Domain(nx=case.nx, ny=case.ny, dx=case.dx, dy=case.dy, bc=list(case.bc), nlevels=1,
                 gamma=case.gamma, R=case.R, Q=case.Q, Ea=case.Ea, k=case.k,
                 bc_prim=list(case.bc_prim))
    return BlockCase(name="split", model=case.model, domains=[dom], blocks=blocks, W=W,
                     mech=case.mech, cfl=case.cfl), recs


def _gather(U, recs, shape):
    out = np.zeros(shape)
    off = 0
    for (_, _, i0, j0, nx, ny) in recs:
        out[:, j0:j0 + ny, i0:i0 + nx] = U[:, off:off + nx * ny].reshape(-1, ny, nx)
        off += nx * ny
    return out


def test_block_decomposition_invariance(oracle):
    c = detonation_tube_case(nx=128, ny=32, seed=17)
    bc, recs = _split_uniform(c, [0, 24, 64, 72, 128], [0, 8, 24, 32])
    U, T = oracle.case_state(c)
    Ub, Tb = oracle.block_state(bc)
    U1, T1, t1, _, _ = oracle.step(c, U, T, 25)
    U2, T2, t2, _, _ = oracle.step_blocks(bc, Ub, Tb, 25)
    assert t2[0] == t1
    G = _gather(U2, recs, U1.shape)
    assert np.array_equal(G, U1)


def test_ensemble_domains_are_independent(oracle):
    e = ensemble_case(n1d=2, n2d=2, seed=99)
    U, T = oracle.block_state(e)
    Ua, Ta, ta, _, _ = oracle.step_blocks(e, U, T, 15)
    for d in range(len(e.domains)):
        b = e.blocks[d]
        sub = BlockCase(name="one", model=e.model, domains=[e.domains[d]],
                        blocks=make_blocks([(0, 0, 0, 0, int(b["nx"]), int(b["ny"]))]),
                        W=e.W[:, b["offset"]:b["offset"] + b["nx"] * b["ny"]], cfl=e.cfl)
        s = slice(int(b["offset"]), int(b["offset"] + b["nx"] * b["ny"]))
        U1, T1, t1, _, _ = oracle.step_blocks(sub, U[:, s], T[s], 15)
        assert np.array_equal(U1, Ua[:, s])
        assert t1[0] == ta[d]


def test_full_refinement_reproduces_fine_grid(oracle):
    """Level 1 covering the whole domain = the uniform fine grid; level 0 = its 2x2 mean."""
    fine = detonation_tube_case(nx=64, ny=32, dx=0.025, seed=23)
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
    Uf, Tf = oracle.case_state(fine)
    Ub, Tb = oracle.block_state(bcase)
    U1, _, t1, _, _ = oracle.step(fine, Uf, Tf, 12)
    U2, _, t2, _, _ = oracle.step_blocks(bcase, Ub, Tb, 12)
    assert t2[0] == t1
    G = _gather(U2[:, nx0 * ny0:], [(0, 0, i0, j0, 32, 16) for (_, _, i0, j0, _, _) in recs[1:]],
                U1.shape)
    assert np.array_equal(G, U1)
    mean = ((U1[:, 0::2, 0::2] + U1[:, 0::2, 1::2]) + (U1[:, 1::2, 0::2] + U1[:, 1::2, 1::2])) * 0.25
    assert np.array_equal(U2[:, :nx0 * ny0].reshape(5, ny0, nx0), mean)


def _small_amr(model=MODEL_ONESTEP, seed=5):
    """A 3-level hierarchy on a 128 x 64 base with one-step physics (fast oracle)."""
    phi, geo = build_hierarchy(128, 64, 0.05, 3, (1.0, 0.7), blk0=32, seed=seed, margin=6)
    recs = [(0, lev, i0, j0, nx, ny) for (lev, i0, j0, nx, ny) in geo]
    blocks = make_blocks(recs)
    rng = np.random.default_rng(seed)
    parts = []
    for (_, lev, i0, j0, nx, ny) in recs:
        dx = 0.05 / (1 << lev)
        xc = (i0 + np.arange(nx) + 0.5) * dx
        yc = (j0 + np.arange(ny) + 0.5) * dx
        X, Y = np.meshgrid(xc, yc)
        W = np.zeros((5, ny, nx))
        W[0] = 1.0 + 0.3 * np.exp(-((X - 3.2) ** 2 + (Y - 1.6) ** 2))
        W[1] = 0.2 * np.sin(X)
        W[2] = 0.1 * np.cos(2 * Y)
        W[3] = 1.0 + 2.0 * np.exp(-((X - 2.0) ** 2 + (Y - 1.0) ** 2) / 0.3)
        W[4] = 1.0
        parts.append(W.reshape(5, -1))
    dom = Domain(nx=128, ny=64, dx=0.05, dy=0.05, bc=[BC_ZEROGRAD, BC_ZEROGRAD, BC_SLIPWALL,
                 BC_SLIPWALL], nlevels=3, gamma=1.2, R=1.0, Q=50.0, Ea=24.0, k=30.0)
    return BlockCase(name="amr_small", model=model, domains=[dom], blocks=blocks,
                     W=np.concatenate(parts, axis=1), cfl=0.5)


def _lookup(blocks, lev, I, J):
    for n, b in enumerate(blocks):
        if b["level"] == lev and b["i0"] <= I < b["i0"] + b["nx"] and b["j0"] <= J < b["j0"] + b["ny"]:
            return n
    return -1


def test_ring_rule_from_definition(oracle):
    bc = _small_amr()
    flags = oracle.ring_flags(bc)
    blocks = bc.blocks
    dom = bc.domains[0]
    cover = {}
    for lev in range(3):
        m = np.zeros((dom.ny << lev, dom.nx << lev), bool)
        for b in blocks[blocks["level"] == lev]:
            m[b["j0"]:b["j0"] + b["ny"], b["i0"]:b["i0"] + b["nx"]] = True
        cover[lev] = m
    nring = 0
    for b in blocks:
        lev = int(b["level"])
        m = cover[lev]
        H, Wd = m.shape
        for j in range(b["ny"]):
            for i in range(b["nx"]):
                I, J = b["i0"] + i, b["j0"] + j
                ring = False
                for d in (1, 2, 3):
                    for (a, c) in ((I - d, J), (I + d, J), (I, J - d), (I, J + d)):
                        if 0 <= a < Wd and 0 <= c < H and not m[c, a]:
                            ring = True
                f = flags[b["offset"] + j * b["nx"] + i]
                assert f == (1 if ring else 0)
                nring += ring
    assert nring > 0
    assert not np.any(flags[:dom.nx * dom.ny])      # level 0 covers everything: no ring


def test_restriction_and_ring_injection(oracle):
    bc = _small_amr()
    U, T = oracle.block_state(bc)
    U, T, _, _, _ = oracle.step_blocks(bc, U, T, 3)
    flags = oracle.ring_flags(bc)
    blocks = bc.blocks

    def cell(lev, I, J):
        n = _lookup(blocks, lev, I, J)
        b = blocks[n]
        return int(b["offset"] + (J - b["j0"]) * b["nx"] + (I - b["i0"]))

    checked = 0
    for b in blocks[blocks["level"] >= 1]:
        lev = int(b["level"])
        for cj in range(b["j0"] // 2, (b["j0"] + b["ny"]) // 2):
            for ci in range(b["i0"] // 2, (b["i0"] + b["nx"]) // 2):
                ch = [cell(lev, 2 * ci + (q & 1), 2 * cj + (q >> 1)) for q in range(4)]
                parent = cell(lev - 1, ci, cj)
                if any(flags[c] for c in ch):
                    # ring children are the injection of the final coarse value
                    for c in ch:
                        if flags[c]:
                            assert np.array_equal(U[:, c], U[:, parent])
                    continue
                mean = ((U[:, ch[0]] + U[:, ch[1]]) + (U[:, ch[2]] + U[:, ch[3]])) * 0.25
                assert np.array_equal(U[:, parent], mean)
                checked += 1
    assert checked > 100


def test_constant_state_on_hierarchy(oracle):
    bc = _small_amr()
    bc.W[:] = np.array([1.3, 0.4, 0.0, 2.0, 0.0])[:, None]   # burned, uniform, moving along walls
    bc.domains[0].bc = [BC_PERIODIC, BC_PERIODIC, BC_SLIPWALL, BC_SLIPWALL]
    U0, T0 = oracle.block_state(bc)
    U, T, _, _, _ = oracle.step_blocks(bc, U0, T0, 5)
    for f in range(5):
        assert np.max(np.abs(U[f] - U0[f])) <= 1e-14 * max(1.0, np.max(np.abs(U0[f])))


def test_invalid_blocks_are_untouched(oracle):
    c = detonation_tube_case(nx=64, ny=16, seed=3)
    bc, recs = _split_uniform(c, [0, 32, 64], [0, 16])
    extra = np.zeros(1, dtype=bc.blocks.dtype)
    extra[0] = (0, 0, 0, 0, 8, 8, bc.pool_cells, 0, 0)      # invalid block: reserved, not solved
    bc.blocks = np.concatenate([bc.blocks, extra])
    bc.W = np.concatenate([bc.W, np.full((5, 64), 7.0)], axis=1)
    U, T = oracle.block_state(bc)
    U2, _, _, _, _ = oracle.step_blocks(bc, U, T, 3)
    assert np.array_equal(U2[:, -64:], U[:, -64:])


def test_bad_tables_are_rejected(oracle):
    c = detonation_tube_case(nx=64, ny=16, seed=3)
    bc, _ = _split_uniform(c, [0, 32, 64], [0, 16])
    U, T = oracle.block_state(bc)
    bad = bc.blocks.copy()
    bad[1]["i0"] = 16                                      # overlap + gap
    bc.blocks = bad
    _, _, _, _, st = oracle.step_blocks(bc, U, T, 1, check=False)
    assert st == -1
