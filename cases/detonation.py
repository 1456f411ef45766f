"""One-step Arrhenius detonation workloads (nondimensional).

Model (the user source-term path of the paper, Sec. 4.3 item 3): two species,
fuel -> product, one transported mass fraction Y (the fuel), rate
dY/dt = -k Y exp(-Ea / T), chemical energy Y*Q per unit mass. Units: pre-shock
rho0 = p0 = 1 so R T0 = 1, R = 1, and the length unit is the half-reaction
length of the steady ZND wave, so with 20 cells per half-reaction length the
grid spacing is 0.05.

This module computes the case constants that follow from the model in closed
form or by quadrature (Chapman-Jouguet state, ZND rate constant) and builds
seeded initial conditions. It is case preparation, not the solver.
"""

import math

import numpy as np
from scipy.integrate import quad

from .common import (Case, Domain, BlockCase, make_blocks, MODEL_ONESTEP,
                     BC_ZEROGRAD, BC_SLIPWALL, BC_DIRICHLET)


def cj_state(gamma: float, Q: float, rho0: float = 1.0, p0: float = 1.0) -> dict:
    """Chapman-Jouguet detonation of the one-step model (same gamma both sides)."""
    c0 = math.sqrt(gamma * p0 / rho0)
    K = (gamma * gamma - 1.0) * Q / (2.0 * c0 * c0)
    M = math.sqrt(1.0 + K) + math.sqrt(K)
    D = c0 * M
    p_cj = (p0 + rho0 * D * D) / (gamma + 1.0)
    # Sonic downstream state: rho1 w^2 = gamma p1 together with rho1 w = rho0 D.
    w = gamma * p_cj / (rho0 * D)
    rho_cj = rho0 * D / w
    return {"D": D, "M": M, "c0": c0, "p": p_cj, "rho": rho_cj, "w": w,
            "u_lab": D - w}


def znd_profile(gamma: float, Q: float, lam, rho0: float = 1.0, p0: float = 1.0):
    """Steady ZND state at reaction progress lam = 1 - Y, in the shock frame.

    Returns (w, p, rho, T) with w the flow speed relative to the shock.
    """
    cj = cj_state(gamma, Q, rho0, p0)
    D = cj["D"]
    m = rho0 * D
    a = gamma / (gamma - 1.0)
    H0 = a * p0 / rho0 + 0.5 * D * D
    lam = np.asarray(lam, dtype=float)
    A = a - 0.5
    B = a * (p0 / m + D)
    C = H0 + lam * Q
    disc = np.maximum(B * B - 4.0 * A * C, 0.0)
    w = (B - np.sqrt(disc)) / (2.0 * A)
    p = p0 + m * (D - w)
    rho = m / w
    T = p / rho
    return w, p, rho, T


def znd_rate_constant(gamma: float, Q: float, Ea: float, half_length: float = 1.0) -> float:
    """Pre-exponential factor k that puts the ZND half-reaction point at half_length.

    x(1/2) = (1/k) * int_0^{1/2} w / ((1 - lam) exp(-Ea/T)) dlam.
    """
    def integrand(lam):
        w, _, _, T = znd_profile(gamma, Q, lam)
        return float(w / ((1.0 - lam) * math.exp(-Ea / T)))
    val, _ = quad(integrand, 0.0, 0.5, epsabs=1e-13, epsrel=1e-13, limit=200)
    return val / half_length


def _tube_primitives(nx, ny, dx, gamma, Q, slab_frac, noise, rng, slab_pressure_factor=3.0):
    cj = cj_state(gamma, Q)
    Lx = nx * dx
    xc = (np.arange(nx) + 0.5) * dx
    slab = xc < slab_frac * Lx
    W = np.zeros((5, ny, nx))
    xi = rng.uniform(-1.0, 1.0, size=(ny, nx))
    rho = 1.0 + noise * xi
    rho[:, slab] = 1.0
    W[0] = rho
    W[3] = np.where(slab[None, :], slab_pressure_factor * cj["p"], 1.0)
    W[4] = np.where(slab[None, :], 0.0, 1.0)
    return W


def detonation_tube_case(nx: int = 1024, ny: int = 128, gamma: float = 1.2, Q: float = 50.0,
                         Ea: float = 24.0, dx: float = 0.05, slab_frac: float = 0.05,
                         noise: float = 0.01, seed: int = 2504, cfl: float = 0.5,
                         nsteps: int = 1000, k: float = None) -> Case:
    """2-D detonation tube: slip walls S/N, zero-gradient outflow W, Dirichlet fresh inflow E.

    Ignition slab (first slab_frac of the length): p = 3 p_CJ, rho = 1, u = v = 0,
    burned (Y = 0). Elsewhere p = 1, rho = 1 + noise*xi with xi ~ U[-1, 1] per cell
    from a seeded PCG64 stream, Y = 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if k is None:
        k = znd_rate_constant(gamma, Q, Ea)
    W = _tube_primitives(nx, ny, dx, gamma, Q, slab_frac, noise, rng)
    fresh = np.array([1.0, 0.0, 0.0, 1.0, 1.0])
    bc = [BC_ZEROGRAD, BC_DIRICHLET, BC_SLIPWALL, BC_SLIPWALL]
    return Case(name=f"det{nx}x{ny}", model=MODEL_ONESTEP, nx=nx, ny=ny, dx=dx, dy=dx,
                bc=bc, W=W, gamma=gamma, R=1.0, Q=Q, Ea=Ea, k=k,
                bc_prim=[None, fresh, None, None], cfl=cfl, nsteps=nsteps)


def adjoint_case(nx: int = 512, ny: int = 64, nsteps: int = 400, seed: int = 5120,
                 cfl_dt: float = 0.4) -> dict:
    """Adjoint workload: the 2-D one-step tube at nx x ny with a fixed dt.

    dt = cfl_dt / max((|u|+c)/dx + (|v|+c)/dy) of the nominal initial state, which
    for u = v = 0 is cfl_dt / (2 c_max / dx) with c_max the slab sound speed.
    Probes are four wall cells; the loss is the time-integrated probe pressure.
    """
    case = detonation_tube_case(nx=nx, ny=ny, seed=seed, nsteps=nsteps)
    p_max = case.W[3].max()
    c_max = math.sqrt(case.gamma * p_max / 1.0)
    case.dt_fixed = cfl_dt / (c_max / case.dx + c_max / case.dy)
    probes = [(nx // 8, 0), (nx // 8, ny - 1), (nx // 4, 0), (nx // 4, ny - 1)]
    probe_cell = np.array([j * nx + i for (i, j) in probes], dtype=np.int32)
    probe_w = np.ones(len(probes))
    return {"case": case, "probe_cell": probe_cell, "probe_w": probe_w,
            "ckpt_every": 20}


def ensemble_case(n1d: int = 32, n2d: int = 32, seed: int = 2025, nsteps: int = 500,
                  gamma: float = 1.2, dx: float = 0.05) -> BlockCase:
    """Ensemble of independent one-step detonation instances of uneven sizes.

    1-D instances: nx = 256 * 32**u rounded to a multiple of 8 (ny = 1).
    2-D instances: nx = 128 * 4**u rounded to a multiple of 32, ny = nx / 4.
    Q ~ U[30, 60], Ea ~ U[20, 30]; k from the ZND half-reaction length of each
    instance; each instance is one domain (its own CFL time step) and one block.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    domains, recs, prims = [], [], []
    fresh = np.array([1.0, 0.0, 0.0, 1.0, 1.0])
    shapes = []
    for n in range(n1d):
        u = rng.uniform()
        nx = int(round(256 * 32 ** u / 8.0)) * 8
        shapes.append((nx, 1))
    for n in range(n2d):
        u = rng.uniform()
        nx = int(round(128 * 4 ** u / 32.0)) * 32
        shapes.append((nx, nx // 4))
    for d, (nx, ny) in enumerate(shapes):
        Q = rng.uniform(30.0, 60.0)
        Ea = rng.uniform(20.0, 30.0)
        k = znd_rate_constant(gamma, Q, Ea)
        W = _tube_primitives(nx, ny, dx, gamma, Q, 0.05, 0.01, rng)
        bc = [BC_ZEROGRAD, BC_DIRICHLET, BC_SLIPWALL, BC_SLIPWALL]
        domains.append(Domain(nx=nx, ny=ny, dx=dx, dy=dx, bc=bc, nlevels=1, gamma=gamma,
                              R=1.0, Q=Q, Ea=Ea, k=k, bc_prim=[None, fresh, None, None]))
        recs.append((d, 0, 0, 0, nx, ny))
        prims.append(W.reshape(5, -1))
    blocks = make_blocks(recs)
    return BlockCase(name=f"ensemble{n1d}+{n2d}", model=MODEL_ONESTEP, domains=domains,
                     blocks=blocks, W=np.concatenate(prims, axis=1), cfl=0.5, nsteps=nsteps)
