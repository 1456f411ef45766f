"""The chemistry kernels specialised to a mechanism's structure (janc_rtc.hip: the forward
point-implicit step and its reverse in the adjoint) are generated and compiled with hipRTC
for gfx950 on the host (no device needed) for mechanisms of
different shapes: the seeded 9-species mechanism (one and two NASA-7 ranges), the
30-reaction complete mechanism, the hand-written 6-species chemkin mechanism, a
12-species mechanism with inert species, and a 2-species mechanism with an irreversible
reaction of a repeated reactant; a mechanism without kernels is rejected. Their results are
checked against the generic kernels on the GPU (test_gpu_chem_spec.py)."""

import copy

import numpy as np
import pytest

import paper_2504_13750_amd as janc
from cases import synthetic_mechanism, two_range_mechanism
from cases.mechanism import complete_mechanism


def _two_species():
    """The seeded mechanism cut to its first two species (equal molar masses) with one
    irreversible reaction 2 S0 -> 2 S1: a repeated reactant and a repeated product."""
    m = copy.deepcopy(synthetic_mechanism())
    m.species = m.species[:2]
    m.comp = m.comp[:2]
    m.M = m.M[:2].copy()
    m.M[1] = m.M[0]
    m.nasa = m.nasa[:2]
    m.A, m.b, m.Ea = np.array([1e6]), np.array([0.5]), np.array([2.0e4])
    m.nu_f = np.array([[2, 0]], np.int32)
    m.nu_b = np.array([[0, 2]], np.int32)
    m.tb = np.ones((1, 2))
    m.has_tb = np.array([0], np.int32)
    m.reversible = np.array([0], np.int32)
    return m


def _mechanisms():
    from test_gpu_species_counts import six_species_mechanism, twelve_species_mechanism
    base = synthetic_mechanism()
    return {"synthetic-9": base, "two-range-9": two_range_mechanism(base),
            "complete-9-30": complete_mechanism(), "chemkin-6": six_species_mechanism(),
            "inert-12": twelve_species_mechanism(), "two-species": _two_species()}


@pytest.mark.parametrize("name", ["synthetic-9", "two-range-9", "complete-9-30", "chemkin-6",
                                  "inert-12", "two-species"])
def test_specialised_chemistry_kernel_compiles(name):
    m = _mechanisms()[name]
    st, log = janc.chem_kernel_check(m)
    assert st == 0, log


def test_mechanism_without_kernels_rejected():
    from test_gpu_species_counts import twelve_species_mechanism
    m = twelve_species_mechanism()
    m13 = copy.deepcopy(m)
    m13.species = m.species[:-1] + ["G2", m.species[-1]]
    m13.comp = np.concatenate([m.comp[:-1], m.comp[-1:], m.comp[-1:]])
    m13.M = np.concatenate([m.M[:-1], m.M[-1:], m.M[-1:]])
    m13.nasa = np.concatenate([m.nasa[:-1], m.nasa[-1:], m.nasa[-1:]])
    z = np.zeros((m.nr, 1), np.int32)
    ins = lambda a, c: np.concatenate([a[..., :-1], c, a[..., -1:]], axis=-1)
    m13.nu_f = ins(m.nu_f, z).astype(np.int32)
    m13.nu_b = ins(m.nu_b, z).astype(np.int32)
    m13.tb = ins(m.tb, np.ones((m.nr, 1)))
    st, log = janc.chem_kernel_check(m13)
    assert st == -1 and "ns 2..12" in log
