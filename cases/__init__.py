"""Seeded synthetic workloads for the reacting-flow step (arXiv 2504.13750).

This package holds input generators only. Every case is described by primitive
fields (density or pressure, velocities, pressure or temperature, mass
fractions), boundary kinds, physics constants and, for block-structured cases,
block geometry. It holds none of the solver's arithmetic: the conversion to
conserved variables, the equation of state, fluxes, chemistry and AMR coupling
live separately in the CPU oracle and in the HIP library, and both consume the
same generated inputs.

The paper's own workloads (a 9-species H2-O2 mechanism, Cantera thermo data,
OpenFOAM cases) are not available, so every workload here is synthetic with the
shapes of the paper's test cases (Sec. 5.1 Sod tube, Sec. 5.2 detonation tube,
Sec. 5.2.3 AMR run, Sec. 6.2 adjoint problem).
"""

from .common import (BC_PERIODIC, BC_ZEROGRAD, BC_SLIPWALL, BC_DIRICHLET,
                     MODEL_CPG, MODEL_ONESTEP, MODEL_DETAILED,
                     Case, BlockCase, Domain)
from .sod import sod_case
from .detonation import (cj_state, znd_rate_constant, znd_profile,
                         detonation_tube_case, adjoint_case, ensemble_case)
from .mechanism import synthetic_mechanism, two_range_mechanism, Mechanism
from .amr import amr_case

__all__ = [
    "BC_PERIODIC", "BC_ZEROGRAD", "BC_SLIPWALL", "BC_DIRICHLET",
    "MODEL_CPG", "MODEL_ONESTEP", "MODEL_DETAILED",
    "Case", "BlockCase", "Domain",
    "sod_case", "cj_state", "znd_rate_constant", "znd_profile",
    "detonation_tube_case", "adjoint_case", "ensemble_case",
    "synthetic_mechanism", "two_range_mechanism", "Mechanism", "amr_case",
]
