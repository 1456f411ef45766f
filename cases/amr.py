"""Block-structured AMR hierarchy with a wrinkled reacting front (9 species).

Geometry follows the block concepts of the paper (Sec. 3.1): level 0 tiles the
domain with equal blocks; each finer level (ratio 2) is built from fixed,
aligned subregions of that level's index space. Subregions of 64 x 64 cells are
split quad-wise down to 8 x 8 so that blocks of 8 x 8 .. 64 x 64 cover the
refinement band |x - x_f(y)| < w_l around the front
x_f(y) = 0.5 Lx + 0.05 Lx sin(6 pi y / Ly + phi). A level-l subregion is only
allowed where every level-(l-1) cell within 6 cells of its parents is covered,
which keeps levels properly nested with a margin wider than the 3-cell stencil
reach.

State: behind the front T = 2500 K, p = 20 atm, u = 600 m/s; ahead T = 1200 K,
p = 1 atm, u = 0; premixed composition everywhere; tanh blend over 4 finest
cells. Primitive layout per cell: [p, u, v, T, Y_1 .. Y_{Ns-1}].
"""

import math

import numpy as np
from scipy.ndimage import binary_erosion

from .common import (BlockCase, Case, Domain, make_blocks, MODEL_DETAILED, BC_ZEROGRAD,
                     BC_SLIPWALL)
from .mechanism import Mechanism, synthetic_mechanism, fresh_mass_fractions

ATM = 101325.0


def _morton(i, j):
    key = 0
    for bit in range(16):
        key |= ((i >> bit) & 1) << (2 * bit) | ((j >> bit) & 1) << (2 * bit + 1)
    return key


def front_primitives(mech: Mechanism, xc, yc, Lx, Ly, phi, dx_fine):
    """Primitive state [p, u, v, T, Y_1..] at cell centres (xc, yc) of any level."""
    xf = 0.5 * Lx + 0.05 * Lx * np.sin(6.0 * math.pi * yc / Ly + phi)
    s = 0.5 * (1.0 - np.tanh((xc - xf) / (4.0 * dx_fine)))   # 1 behind, 0 ahead
    Y = fresh_mass_fractions(mech)
    W = np.zeros((4 + mech.ns - 1,) + np.shape(xc))
    W[0] = s * 20.0 * ATM + (1.0 - s) * ATM
    W[1] = s * 600.0
    W[3] = s * 2500.0 + (1.0 - s) * 1200.0
    for k in range(mech.ns - 1):
        W[4 + k] = Y[k]
    return W


def _quad_blocks(need8, allowed8, top=8, fill=0.3):
    """Quadtree cover of the 8x8 regions marked needed, in aligned 64x64 subregions.

    need8/allowed8 are [H8, W8] boolean maps of 8x8-cell regions. A subregion
    becomes one block when it is entirely allowed and at least `fill` of its
    8x8 regions are needed; otherwise it is split in four. Returns a list of
    (i0, j0, n) in cells.
    """
    H8, W8 = need8.shape
    out = []

    def rec(r0, c0, n8):
        sub = need8[r0:r0 + n8, c0:c0 + n8]
        if not sub.any():
            return
        full = (sub.shape == (n8, n8) and sub.mean() >= fill
                and allowed8[r0:r0 + n8, c0:c0 + n8].all())
        if full or n8 == 1:
            out.append((c0 * 8, r0 * 8, n8 * 8))
            return
        h = n8 // 2
        for dr in (0, h):
            for dc in (0, h):
                rec(r0 + dr, c0 + dc, h)

    for r0 in range(0, H8, top):
        for c0 in range(0, W8, top):
            rec(r0, c0, top)
    return out


def build_hierarchy(nx0, ny0, dx0, nlevels, widths, blk0=64, seed=13751, margin=6):
    """Return (phi, [list of (level, i0, j0, nx, ny)]) for a wrinkled-front hierarchy."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = rng.uniform(0.0, 2.0 * math.pi)
    Lx, Ly = nx0 * dx0, ny0 * dx0
    blocks = [(0, i0, j0, blk0, blk0) for j0 in range(0, ny0, blk0) for i0 in range(0, nx0, blk0)]
    cover_prev = np.ones((ny0, nx0), dtype=bool)
    for lev in range(1, nlevels):
        nx, ny = nx0 << lev, ny0 << lev
        dx = dx0 / (1 << lev)
        # cells of level lev whose parent neighbourhood is covered at lev-1
        er = binary_erosion(cover_prev, structure=np.ones((2 * margin + 1, 2 * margin + 1)),
                            border_value=1)
        allowed = np.repeat(np.repeat(er, 2, axis=0), 2, axis=1)
        yc = (np.arange(ny) + 0.5) * dx
        xc = (np.arange(nx) + 0.5) * dx
        xf = 0.5 * Lx + 0.05 * Lx * np.sin(6.0 * math.pi * yc / Ly + phi)
        band = np.abs(xc[None, :] - xf[:, None]) < widths[lev - 1]
        need = band & allowed
        need8 = need.reshape(ny // 8, 8, nx // 8, 8).any(axis=(1, 3))
        allowed8 = allowed.reshape(ny // 8, 8, nx // 8, 8).all(axis=(1, 3))
        need8 &= allowed8
        lev_blocks = _quad_blocks(need8, allowed8)
        cover = np.zeros((ny, nx), dtype=bool)
        for (i0, j0, n) in lev_blocks:
            cover[j0:j0 + n, i0:i0 + n] = True
        lev_blocks.sort(key=lambda b: _morton(b[0] // 8, b[1] // 8))
        blocks += [(lev, i0, j0, n, n) for (i0, j0, n) in lev_blocks]
        cover_prev = cover
    return phi, blocks


def amr_case(mech: Mechanism = None, nx0: int = 1024, ny0: int = 512, dx0: float = 25e-6,
             nlevels: int = 3, widths=(1.9e-3, 1.5e-3), blk0: int = 64, seed: int = 13751,
             cfl: float = 0.5, nsteps: int = 50) -> BlockCase:
    if mech is None:
        mech = synthetic_mechanism()
    phi, geo = build_hierarchy(nx0, ny0, dx0, nlevels, widths, blk0=blk0, seed=seed)
    Lx, Ly = nx0 * dx0, ny0 * dx0
    dxf = dx0 / (1 << (nlevels - 1))
    recs, prims = [], []
    for (lev, i0, j0, nx, ny) in geo:
        dx = dx0 / (1 << lev)
        xc = (i0 + np.arange(nx) + 0.5) * dx
        yc = (j0 + np.arange(ny) + 0.5) * dx
        X, Y = np.meshgrid(xc, yc)
        prims.append(front_primitives(mech, X, Y, Lx, Ly, phi, dxf).reshape(4 + mech.ns - 1, -1))
        recs.append((0, lev, i0, j0, nx, ny))
    dom = Domain(nx=nx0, ny=ny0, dx=dx0, dy=dx0,
                 bc=[BC_ZEROGRAD, BC_ZEROGRAD, BC_SLIPWALL, BC_SLIPWALL], nlevels=nlevels)
    return BlockCase(name=f"amr{nx0}x{ny0}L{nlevels}", model=MODEL_DETAILED, domains=[dom],
                     blocks=make_blocks(recs), W=np.concatenate(prims, axis=1), mech=mech,
                     cfl=cfl, nsteps=nsteps)


def detailed_front_case(nx: int = 128, ny: int = 64, dx: float = 25e-6, mech: Mechanism = None,
                        seed: int = 13751, cfl: float = 0.5, nsteps: int = 10) -> Case:
    """Uniform-grid version of the front state (9 species), for the uniform path."""
    if mech is None:
        mech = synthetic_mechanism()
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = rng.uniform(0.0, 2.0 * math.pi)
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(xc, yc)
    W = front_primitives(mech, X, Y, nx * dx, ny * dx, phi, dx)
    return Case(name=f"front{nx}x{ny}", model=MODEL_DETAILED, nx=nx, ny=ny, dx=dx, dy=dx,
                bc=[BC_ZEROGRAD, BC_ZEROGRAD, BC_SLIPWALL, BC_SLIPWALL], W=W, mech=mech,
                cfl=cfl, nsteps=nsteps)


def detailed_adjoint_case(nx: int = 32, ny: int = 16, dx: float = 25e-6, nsteps: int = 8,
                          seed: int = 2504, cfl_dt: float = 0.4, mech: Mechanism = None) -> dict:
    """Adjoint workload of the detailed model: the 9-species front state with a seeded
    velocity field (u shifted by 40 m/s, v = 25 + 15 sin(2 pi x / L_x) m/s) and +-0.5 %
    noise on p and T, so that no speed is zero and no two cells tie for the largest wave
    speed (|v| and the max are then differentiable at the state). Fixed dt = cfl_dt over
    the CFL bound of the initial state; zero-gradient W/E, slip walls S/N; probes at two
    wall cells and two interior cells."""
    if mech is None:
        mech = synthetic_mechanism()
    c = detailed_front_case(nx=nx, ny=ny, dx=dx, mech=mech, nsteps=nsteps)
    rng = np.random.Generator(np.random.PCG64(seed))
    W = c.W.copy()
    xc = (np.arange(nx) + 0.5) / nx
    W[1] = W[1] + 40.0
    W[2] = 25.0 + 15.0 * np.sin(2.0 * math.pi * xc)[None, :] * np.ones((ny, 1))
    W[0] = W[0] * (1.0 + 0.005 * rng.uniform(-1.0, 1.0, size=W[0].shape))
    W[3] = W[3] * (1.0 + 0.005 * rng.uniform(-1.0, 1.0, size=W[3].shape))
    c.W = W
    probes = [(nx // 4, 0), (3 * nx // 4, ny - 1), (nx // 2, ny // 2), (nx // 8, ny // 3)]
    probe_cell = np.array([j * nx + i for (i, j) in probes], dtype=np.int32)
    probe_w = np.array([1.0, 0.5, 2.0, 1.0])
    return {"case": c, "probe_cell": probe_cell, "probe_w": probe_w, "cfl_dt": cfl_dt}
