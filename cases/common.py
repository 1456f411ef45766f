"""Case containers and enumerations shared by the generators.

Primitive vector layout per model (one row per field, x fastest):

* CPG (calorically perfect gas):       [rho, u, v, p]
* ONESTEP (one-step Arrhenius model):  [rho, u, v, p, Y]      (Y = fuel mass fraction)
* DETAILED (NASA-7 + mass action):     [p, u, v, T, Y_1 .. Y_{Ns-1}]

The conserved state of the paper (Sec. 4.1, Eq. 4.1) has the same number of
rows: [rho, rho u, rho v, E, rho Y_1 .. rho Y_{Ns-1}]; the last species is the
complement 1 - sum(Y).
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Boundary kinds, sides ordered W, E, S, N.
BC_PERIODIC = 0
BC_ZEROGRAD = 1
BC_SLIPWALL = 2
BC_DIRICHLET = 3

MODEL_CPG = 0
MODEL_ONESTEP = 1
MODEL_DETAILED = 2

BLOCK_DTYPE = np.dtype([
    ("domain", np.int32), ("level", np.int32), ("i0", np.int32), ("j0", np.int32),
    ("nx", np.int32), ("ny", np.int32), ("offset", np.int64), ("valid", np.int32),
    ("pad", np.int32),
])


def n_fields(model: int, ns: int = 0) -> int:
    if model == MODEL_CPG:
        return 4
    if model == MODEL_ONESTEP:
        return 5
    return 4 + ns - 1


@dataclass
class Case:
    """A uniform grid (paper Sec. 4.2: Cartesian grid with 3 ghost layers)."""
    name: str
    model: int
    nx: int
    ny: int
    dx: float
    dy: float
    bc: List[int]
    W: np.ndarray                      # primitives [nU, ny, nx]
    gamma: float = 1.4
    R: float = 1.0
    Q: float = 0.0
    Ea: float = 0.0
    k: float = 0.0
    mech: Optional[object] = None
    bc_prim: List[Optional[np.ndarray]] = field(default_factory=lambda: [None] * 4)
    cfl: float = 0.5
    dt_fixed: float = 0.0
    t_end: float = 0.0
    nsteps: int = 1

    @property
    def nU(self) -> int:
        return self.W.shape[0]

    @property
    def cells(self) -> int:
        return self.nx * self.ny


@dataclass
class Domain:
    """One independent problem of a block table: a level-0 grid plus refinement levels."""
    nx: int
    ny: int
    dx: float
    dy: float
    bc: List[int]
    nlevels: int = 1
    gamma: float = 1.4
    R: float = 1.0
    Q: float = 0.0
    Ea: float = 0.0
    k: float = 0.0
    bc_prim: List[Optional[np.ndarray]] = field(default_factory=lambda: [None] * 4)


@dataclass
class BlockCase:
    """A block table over one pool: AMR levels (paper Sec. 3.1) and/or ensemble instances."""
    name: str
    model: int
    domains: List[Domain]
    blocks: np.ndarray                 # BLOCK_DTYPE records
    W: np.ndarray                      # primitives [nU, pool_cells]
    mech: Optional[object] = None
    cfl: float = 0.5
    dt_fixed: float = 0.0
    t_end: float = 0.0
    nsteps: int = 1

    @property
    def nU(self) -> int:
        return self.W.shape[0]

    @property
    def pool_cells(self) -> int:
        return self.W.shape[1]

    def valid_cells(self) -> int:
        b = self.blocks[self.blocks["valid"] != 0]
        return int(np.sum(b["nx"].astype(np.int64) * b["ny"]))


def make_blocks(records) -> np.ndarray:
    """records: iterable of (domain, level, i0, j0, nx, ny); offsets are packed in order."""
    recs = list(records)
    out = np.zeros(len(recs), dtype=BLOCK_DTYPE)
    off = 0
    for n, (d, lev, i0, j0, nx, ny) in enumerate(recs):
        out[n] = (d, lev, i0, j0, nx, ny, off, 1, 0)
        off += nx * ny
    return out
