"""Sod shock tube (paper Sec. 5.1 (1)), in the normalized textbook form.

400 cells on [0, 1], interface at x = 0.5, left (rho, u, p) = (1, 0, 1), right
(0.125, 0, 0.1), gamma = 1.4, zero-gradient ("non-reflecting") ends, CFL 0.5 up
to t = 0.2. One cell in y, so the y sweep is absent.
"""

import numpy as np

from .common import Case, MODEL_CPG, BC_ZEROGRAD


def sod_case(nx: int = 400, gamma: float = 1.4, cfl: float = 0.5, t_end: float = 0.2,
             nsteps: int = 2000) -> Case:
    dx = 1.0 / nx
    xc = (np.arange(nx) + 0.5) * dx
    left = xc < 0.5
    W = np.zeros((4, 1, nx))
    W[0, 0] = np.where(left, 1.0, 0.125)
    W[3, 0] = np.where(left, 1.0, 0.1)
    return Case(name=f"sod{nx}", model=MODEL_CPG, nx=nx, ny=1, dx=dx, dy=dx,
                bc=[BC_ZEROGRAD] * 4, W=W, gamma=gamma, R=1.0, cfl=cfl,
                t_end=t_end, nsteps=nsteps)
