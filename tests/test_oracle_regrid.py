"""Pins of the oracle's layer update (regridding: Sec. 3.1.2 masked and buffer cells,
fixed subregions; Sec. 3.1.4 one-to-four refinement and unaltered blocks; Alg. 2).

* a straight density jump masks exactly the two cell columns beside it, so the refined
  subregions are those within `buffer` cells of those columns (closed form);
* a uniform state refines nothing, and a huge threshold refines nothing;
* new blocks hold the one-to-four injection of their parents, cell by cell;
* from a base-layer-only start the update is idempotent: a second update on the
  filled hierarchy returns the same table and bitwise the same pools;
* blocks that survive an update keep their data bitwise;
* refined blocks nest in solved cells of their parent layer (no ring cells below them).
"""

import numpy as np
import pytest

from cases import Domain, BlockCase, MODEL_ONESTEP, BC_ZEROGRAD, BC_SLIPWALL
from cases.common import make_blocks


def _base_case(nx=128, ny=64, blk=64, nlevels=2, jump_at=None, rho=None):
    recs = [(0, 0, i0, j0, blk, blk) for j0 in range(0, ny, blk) for i0 in range(0, nx, blk)]
    blocks = make_blocks(recs)
    W = np.zeros((5, nx * ny))
    off = 0
    for (_, _, i0, j0, bx, by) in recs:
        I, J = np.meshgrid(np.arange(i0, i0 + bx), np.arange(j0, j0 + by))
        r = np.ones_like(I, dtype=float)
        if jump_at is not None:
            r = np.where(I >= jump_at, 2.0, 1.0)
        if rho is not None:
            r = rho(I, J)
        W[0, off:off + bx * by] = r.ravel()
        W[3, off:off + bx * by] = 1.0
        W[4, off:off + bx * by] = 1.0
        off += bx * by
    dom = Domain(nx=nx, ny=ny, dx=0.05, dy=0.05, bc=[BC_ZEROGRAD, BC_ZEROGRAD, BC_SLIPWALL,
                 BC_SLIPWALL], nlevels=nlevels, gamma=1.2, R=1.0, Q=50.0, Ea=24.0, k=30.0)
    return BlockCase(name="regrid", model=MODEL_ONESTEP, domains=[dom], blocks=blocks, W=W,
                     cfl=0.5)


def _with_table(bcase, blocks, pool):
    return BlockCase(name=bcase.name, model=bcase.model, domains=bcase.domains, blocks=blocks,
                     W=np.zeros((bcase.nU, pool)), mech=bcase.mech, cfl=bcase.cfl)


def _table(blocks):
    return [tuple(int(b[k]) for k in ("domain", "level", "i0", "j0", "nx", "ny", "offset"))
            for b in blocks]


@pytest.mark.parametrize("buffer,sub", [(0, 8), (3, 8), (4, 16), (9, 12)])
def test_jump_refines_closed_form(oracle, buffer, sub):
    js = 77
    c = _base_case(jump_at=js)
    U, T = oracle.block_state(c)
    blocks, pool = oracle.regrid(c, U, threshold=0.01, buffer=buffer, sub=sub)
    masked = {js - 1, js}
    expect = [tuple(int(b[k]) for k in ("domain", "level", "i0", "j0", "nx", "ny"))
              for b in c.blocks]
    for b in c.blocks:
        i0, j0, nx, ny = int(b["i0"]), int(b["j0"]), int(b["nx"]), int(b["ny"])
        for y0 in range(0, ny, sub):
            for x0 in range(0, nx, sub):
                w, h = min(sub, nx - x0), min(sub, ny - y0)
                lo, hi = i0 + x0 - buffer, i0 + x0 + w - 1 + buffer
                if any(lo <= m <= hi for m in masked):
                    expect.append((0, 1, 2 * (i0 + x0), 2 * (j0 + y0), 2 * w, 2 * h))
    got = [t[:6] for t in _table(blocks)]
    assert got == expect
    offs = np.cumsum([0] + [b["nx"] * b["ny"] for b in blocks])
    assert list(blocks["offset"]) == list(offs[:-1]) and pool == offs[-1]
    assert len(got) > len(c.blocks)


def test_nothing_to_refine(oracle):
    c = _base_case(nlevels=3)
    U, _ = oracle.block_state(c)
    blocks, pool = oracle.regrid(c, U, threshold=1e-3, buffer=4, sub=8)
    assert _table(blocks) == _table(c.blocks) and pool == c.pool_cells
    c2 = _base_case(nlevels=3, jump_at=70)
    U2, _ = oracle.block_state(c2)
    blocks, _ = oracle.regrid(c2, U2, threshold=10.0, buffer=4, sub=8)
    assert _table(blocks) == _table(c2.blocks)


def _smooth_bump(I, J):
    return 1.0 + 0.8 * np.exp(-((I - 60.0) ** 2 + (J - 30.0) ** 2) / 60.0)


def test_injection_nesting_and_idempotence(oracle):
    c = _base_case(nlevels=3, rho=_smooth_bump)
    U, T = oracle.block_state(c)
    blocks, pool = oracle.regrid(c, U, threshold=0.02, buffer=4, sub=8)
    assert (blocks["level"] == 2).any()
    n = _with_table(c, blocks, pool)
    Un, Tn = oracle.regrid_fill(c, U, T, blocks, pool)
    # one-to-four injection from the parent layer, every field and T
    cover = {}
    for k, b in enumerate(blocks):
        for j in range(b["ny"]):
            for i in range(b["nx"]):
                cover[(int(b["level"]), int(b["i0"]) + i, int(b["j0"]) + j)] = int(b["offset"]) + j * int(b["nx"]) + i
    for b in blocks[blocks["level"] > 0]:
        lev = int(b["level"])
        for j in range(b["ny"]):
            for i in range(b["nx"]):
                c_f = int(b["offset"]) + j * int(b["nx"]) + i
                c_p = cover[(lev - 1, (int(b["i0"]) + i) // 2, (int(b["j0"]) + j) // 2)]
                assert np.array_equal(Un[:, c_f], Un[:, c_p]) and Tn[c_f] == Tn[c_p]
    # level 0 is copied
    for b_old, b_new in zip(c.blocks, blocks[:len(c.blocks)]):
        so = slice(int(b_old["offset"]), int(b_old["offset"]) + int(b_old["nx"]) * int(b_old["ny"]))
        sn = slice(int(b_new["offset"]), int(b_new["offset"]) + int(b_new["nx"]) * int(b_new["ny"]))
        assert np.array_equal(U[:, so], Un[:, sn]) and np.array_equal(T[so], Tn[sn])
    # refined blocks sit on solved (non-ring) parent cells
    ring = oracle.ring_flags(n)
    for b in blocks[blocks["level"] > 1]:
        for j in range(0, b["ny"], 2):
            for i in range(0, b["nx"], 2):
                cp = cover[(int(b["level"]) - 1, (int(b["i0"]) + i) // 2, (int(b["j0"]) + j) // 2)]
                assert ring[cp] == 0
    # a second update of the filled hierarchy changes nothing
    blocks2, pool2 = oracle.regrid(n, Un, threshold=0.02, buffer=4, sub=8)
    assert _table(blocks2) == _table(blocks) and pool2 == pool
    Un2, Tn2 = oracle.regrid_fill(n, Un, Tn, blocks2, pool2)
    assert np.array_equal(Un2, Un) and np.array_equal(Tn2, Tn)


def test_surviving_blocks_keep_their_data(oracle):
    c = _base_case(nlevels=3, rho=_smooth_bump)
    U, T = oracle.block_state(c)
    blocks, pool = oracle.regrid(c, U, threshold=0.02, buffer=4, sub=8)
    n = _with_table(c, blocks, pool)
    Un, Tn = oracle.regrid_fill(c, U, T, blocks, pool)
    # evolve the refined hierarchy so fine data differ from injected values
    Un, Tn, _, _, _ = oracle.step_blocks(n, Un, Tn, 3)
    # a second structure appears far from the first
    for b in blocks[blocks["level"] == 0]:
        o = int(b["offset"])
        I, J = np.meshgrid(np.arange(b["i0"], b["i0"] + b["nx"]), np.arange(b["j0"], b["j0"] + b["ny"]))
        bump = 0.5 * np.exp(-((I - 112.0) ** 2 + (J - 50.0) ** 2) / 20.0).ravel()
        Un[0, o:o + bump.size] += bump
    blocks2, pool2 = oracle.regrid(n, Un, threshold=0.02, buffer=4, sub=8)
    Un2, Tn2 = oracle.regrid_fill(n, Un, Tn, blocks2, pool2)
    old = {t[:6]: t[6] for t in _table(blocks)}
    kept = 0
    for t in _table(blocks2):
        if t[:6] in old and t[1] > 0:
            kept += 1
            so, sn = old[t[:6]], t[6]
            size = t[4] * t[5]
            assert np.array_equal(Un[:, so:so + size], Un2[:, sn:sn + size])
            assert np.array_equal(Tn[so:so + size], Tn2[sn:sn + size])
    assert kept > 0 and len(blocks2) > len(blocks)
