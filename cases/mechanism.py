"""Seeded synthetic 9-species / 19-reaction reversible mechanism.

The paper's H2-O2 mechanism and its thermo data are not available, so this
generator draws a mechanism with the same shape (Sec. 4.1, Eq. 4.3-4.9):
elements {A, B, C}; species A2, B2, A, B, AB, A2B, AB2, A2B2, C2, where C2 is an
inert diluent that is the last (complement) species and appears only as a third
body. Reactions are element-balanced bimolecular exchanges X + Y <=> Z + W and
third-body recombinations X + Y (+M) <=> Z (+M), drawn until the stoichiometric
matrix reaches rank Ns - 1 - rank(reacting elements) = 6, so that chemical
equilibrium of all reactions is the Gibbs minimum at fixed element totals.

Rates: A = 10^U[8, 14] (cm-mol-s), b = U[-1, 1], Ea = U[0, 40] kcal/mol,
third-body efficiencies U[0.5, 2.5]. NASA-7 (single temperature range):
a0..a4 = template * (1 + U[-0.05, 0.05]) with template
(3.5, 4e-4, -4e-8, 1e-12, -1e-16), a5 = U[-1.5e4, 1.5e4] K (C2: 0),
a6 = 3 * (1 + U[-0.05, 0.05]). SI conversion: A * 1e-6^(order-1), Ea * 4184.
"""

import itertools
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

SPECIES = ["A2", "B2", "A", "B", "AB", "A2B", "AB2", "A2B2", "C2"]
ELEMENTS = ["A", "B", "C"]
COMP = np.array([[2, 0, 0], [0, 2, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0],
                 [2, 1, 0], [1, 2, 0], [2, 2, 0], [0, 0, 2]], dtype=np.int64)
ATOMIC_MASS = np.array([2.0e-3, 16.0e-3, 14.0e-3])  # kg/mol, synthetic
NASA_TEMPLATE = np.array([3.5, 4.0e-4, -4.0e-8, 1.0e-12, -1.0e-16])


@dataclass
class Mechanism:
    species: List[str]
    elements: List[str]
    comp: np.ndarray          # [ns, nel]
    M: np.ndarray             # [ns] kg/mol
    nasa: np.ndarray          # [ns, 7]
    A: np.ndarray             # [nr] SI
    b: np.ndarray             # [nr]
    Ea: np.ndarray            # [nr] J/mol
    nu_f: np.ndarray          # [nr, ns] int
    nu_b: np.ndarray          # [nr, ns] int
    tb: np.ndarray            # [nr, ns] third-body efficiencies
    has_tb: np.ndarray        # [nr] int
    reversible: np.ndarray    # [nr] int
    A_cgs: np.ndarray
    Ea_kcal: np.ndarray
    nasa_high: Optional[np.ndarray] = None   # [ns, 7] high-temperature set (two-range NASA-7)
    t_mid: Optional[np.ndarray] = None       # [ns] K: the high set applies for T >= t_mid

    @property
    def ns(self) -> int:
        return len(self.species)

    @property
    def nr(self) -> int:
        return len(self.A)


def _candidates(nreact: int):
    """Element-balanced reactions among the 8 reacting species."""
    idx = range(nreact)
    pairs = list(itertools.combinations_with_replacement(idx, 2))
    exch, recomb = [], []
    for r in pairs:
        er = COMP[r[0]] + COMP[r[1]]
        for p in pairs:
            if p <= r:
                continue
            if np.array_equal(er, COMP[p[0]] + COMP[p[1]]):
                exch.append((r, p))
        for s in idx:
            if np.array_equal(er, COMP[s]):
                recomb.append((r, (s,)))
    return exch, recomb


def synthetic_mechanism(seed: int = 13750, n_exchange: int = 14, n_recomb: int = 5,
                        max_tries: int = 1000) -> Mechanism:
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = len(SPECIES)
    nreact = ns - 1
    exch, recomb = _candidates(nreact)
    target_rank = nreact - np.linalg.matrix_rank(COMP[:nreact, :2])
    for _ in range(max_tries):
        ie = rng.choice(len(exch), size=n_exchange, replace=False)
        ir = rng.choice(len(recomb), size=n_recomb, replace=False)
        rx = [exch[i] for i in ie] + [recomb[i] for i in ir]
        nr = len(rx)
        nu_f = np.zeros((nr, ns), dtype=np.int32)
        nu_b = np.zeros((nr, ns), dtype=np.int32)
        for i, (r, p) in enumerate(rx):
            for s in r:
                nu_f[i, s] += 1
            for s in p:
                nu_b[i, s] += 1
        if np.linalg.matrix_rank(nu_b - nu_f) == target_rank:
            break
    else:
        raise RuntimeError("no full-rank reaction set found")
    has_tb = np.array([0] * n_exchange + [1] * n_recomb, dtype=np.int32)
    tb = np.zeros((nr, ns))
    tb[has_tb == 1] = rng.uniform(0.5, 2.5, size=(int(has_tb.sum()), ns))
    A_cgs = 10.0 ** rng.uniform(8.0, 14.0, size=nr)
    b = rng.uniform(-1.0, 1.0, size=nr)
    Ea_kcal = rng.uniform(0.0, 40.0, size=nr)
    order = nu_f.sum(axis=1) + has_tb
    A_si = A_cgs * (1e-6) ** (order - 1)
    nasa = np.zeros((ns, 7))
    nasa[:, :5] = NASA_TEMPLATE[None, :] * (1.0 + rng.uniform(-0.05, 0.05, size=(ns, 5)))
    nasa[:, 5] = rng.uniform(-1.5e4, 1.5e4, size=ns)
    nasa[-1, 5] = 0.0
    nasa[:, 6] = 3.0 * (1.0 + rng.uniform(-0.05, 0.05, size=ns))
    M = COMP.astype(float) @ ATOMIC_MASS
    return Mechanism(species=list(SPECIES), elements=list(ELEMENTS), comp=COMP.copy(), M=M,
                     nasa=nasa, A=A_si, b=b, Ea=Ea_kcal * 4184.0, nu_f=nu_f, nu_b=nu_b,
                     tb=tb, has_tb=has_tb, reversible=np.ones(nr, dtype=np.int32),
                     A_cgs=A_cgs, Ea_kcal=Ea_kcal)


def fresh_mass_fractions(mech: Mechanism) -> np.ndarray:
    """Premixed composition Y(A2, B2, C2) = (0.03, 0.23, 0.74), all others zero."""
    Y = np.zeros(mech.ns)
    Y[mech.species.index("A2")] = 0.03
    Y[mech.species.index("B2")] = 0.23
    Y[mech.species.index("C2")] = 0.74
    return Y


def two_range_mechanism(mech: Mechanism, t_mid: float = 1800.0, eps: float = 0.05,
                        seed: int = 13752) -> Mechanism:
    """The same mechanism with two-range NASA-7 thermodynamics: below t_mid the
    original coefficients, above it a second set whose cp/R differs by
    eps_k (T - t_mid)^2 / t_mid^2 (eps_k ~ eps U[0.5, 1]) and whose a5, a6 keep h and s
    continuous at t_mid, so cp, dcp/dT, h and s are all continuous there."""
    rng = np.random.default_rng(seed)
    low = np.array(mech.nasa, dtype=float)
    high = low.copy()
    e = eps * rng.uniform(0.5, 1.0, size=mech.ns)
    Tm = float(t_mid)
    d0, d1, d2 = e, -2.0 * e / Tm, e / Tm ** 2        # added to a0, a1, a2
    high[:, 0] += d0
    high[:, 1] += d1
    high[:, 2] += d2
    high[:, 5] -= Tm * (d0 + d1 * Tm / 2.0 + d2 * Tm ** 2 / 3.0)      # h continuous
    high[:, 6] -= d0 * np.log(Tm) + d1 * Tm + d2 * Tm ** 2 / 2.0       # s continuous
    out = Mechanism(**{k: getattr(mech, k) for k in mech.__dataclass_fields__})
    out.nasa_high = high
    out.t_mid = np.full(mech.ns, Tm)
    return out


def complete_mechanism(base: Mechanism = None, A_cgs: float = 1e13) -> Mechanism:
    """Every element-balanced exchange and recombination among the 8 reacting species of
    `base` (19 + 11 = 30 reversible reactions, third body M with unit efficiencies) on the
    same species and NASA-7 data, with one fast temperature-independent rate A = A_cgs.

    Every species is linked to every other by some channel, so a constant-volume reactor
    relaxes to the Gibbs equilibrium of the mixture within a few thousand short steps (the
    seeded 19-reaction set stalls in a partial equilibrium). The equilibrium itself does
    not depend on the rates."""
    if base is None:
        base = synthetic_mechanism()
    ns = base.ns
    exch, recomb = _candidates(ns - 1)
    rx = exch + recomb
    nr = len(rx)
    nu_f = np.zeros((nr, ns), dtype=np.int32)
    nu_b = np.zeros((nr, ns), dtype=np.int32)
    for i, (r, p) in enumerate(rx):
        for s in r:
            nu_f[i, s] += 1
        for s in p:
            nu_b[i, s] += 1
    has_tb = np.array([0] * len(exch) + [1] * len(recomb), dtype=np.int32)
    tb = np.zeros((nr, ns))
    tb[has_tb == 1] = 1.0
    order = nu_f.sum(axis=1) + has_tb
    a_cgs = np.full(nr, float(A_cgs))
    return Mechanism(species=list(base.species), elements=list(base.elements),
                     comp=base.comp.copy(), M=base.M.copy(), nasa=base.nasa.copy(),
                     A=a_cgs * (1e-6) ** (order - 1), b=np.zeros(nr), Ea=np.zeros(nr),
                     nu_f=nu_f, nu_b=nu_b, tb=tb, has_tb=has_tb,
                     reversible=np.ones(nr, dtype=np.int32), A_cgs=a_cgs, Ea_kcal=np.zeros(nr))
