"""The chemkin / NASA-7 reader (paper Sec. 4.1 and 5.1: chemkin-format mechanism in
cm-mol-s-cal-K, NASA-7 thermo) and writer.

* a hand-written mechanism text checks every conversion against values worked out by
  hand here (A to SI by molecularity, Ea units, third-body efficiencies, reversibility,
  two temperature ranges, default t_mid, custom atomic weights, complement species last);
* the seeded synthetic mechanism survives write -> parse (thermo to the 8 decimals of
  the fixed 15-column fields, rates exactly or to one rounding);
* unsupported or malformed input is rejected.
"""

import numpy as np
import pytest

from paper_2504_13750_amd import chemkin
from cases import synthetic_mechanism, two_range_mechanism

TEXT = """! a small invented mechanism (not a published one)
ELEM X/10.0/ Y/20.0/ Z/5.0/
END
SPECIES
X2 Y2 XY X2Y Y Z2
END
THERMO ALL
   300.000  1000.000  5000.000
X2                      X   2               G   300.000  5000.000 1200.00      1
 3.10000000E+00 5.00000000E-04-1.00000000E-07 2.00000000E-11-1.00000000E-15    2
-1.00000000E+03 4.00000000E+00 3.00000000E+00 6.00000000E-04-2.00000000E-07    3
 3.00000000E-11-2.00000000E-15-9.00000000E+02 5.00000000E+00                   4
Y2                      Y   2               G   300.000  5000.000 1200.00      1
 3.20000000E+00 5.00000000E-04-1.00000000E-07 2.00000000E-11-1.00000000E-15    2
-1.10000000E+03 4.10000000E+00 3.30000000E+00 6.00000000E-04-2.00000000E-07    3
 3.00000000E-11-2.00000000E-15-8.00000000E+02 5.10000000E+00                   4
XY                      X   1Y   1          G   300.000  5000.000 1200.00      1
 3.40000000E+00 5.00000000E-04-1.00000000E-07 2.00000000E-11-1.00000000E-15    2
 2.00000000E+03 4.20000000E+00 3.50000000E+00 6.00000000E-04-2.00000000E-07    3
 3.00000000E-11-2.00000000E-15 2.10000000E+03 5.20000000E+00                   4
X2Y                     X   2Y   1          G   300.000  5000.000 1200.00      1
 3.60000000E+00 5.00000000E-04-1.00000000E-07 2.00000000E-11-1.00000000E-15    2
-5.00000000E+03 4.30000000E+00 3.70000000E+00 6.00000000E-04-2.00000000E-07    3
 3.00000000E-11-2.00000000E-15-4.90000000E+03 5.30000000E+00                   4
Y                       Y   1               G   300.000  5000.000 1200.00      1
 2.50000000E+00 0.00000000E+00 0.00000000E+00 0.00000000E+00 0.00000000E+00    2
 3.00000000E+04 4.00000000E+00 2.50000000E+00 0.00000000E+00 0.00000000E+00    3
 0.00000000E+00 0.00000000E+00 3.00000000E+04 4.00000000E+00                   4
Z2                      Z   2               G   300.000  5000.000              1
 3.50000000E+00 0.00000000E+00 0.00000000E+00 0.00000000E+00 0.00000000E+00    2
 0.00000000E+00 3.00000000E+00 3.50000000E+00 0.00000000E+00 0.00000000E+00    3
 0.00000000E+00 0.00000000E+00 0.00000000E+00 3.00000000E+00                   4
END
REACTIONS  CAL/MOLE
X2 + Y2 <=> 2XY          2.0E+13   0.5   1000.0   ! bimolecular
2XY=X2Y + Y              1.5E+12  -0.2   250.0
DUPLICATE
XY+XY=X2Y + Y            1.0E+11   0.0   0.0
DUPLICATE
X2 + Y + M => X2Y + M    1.0E+15  -1.0   0.0
  Z2/0.5/ X2/2.5/
END
"""


def test_hand_written_mechanism():
    m = chemkin.parse(TEXT, complement="Z2")
    assert m.species == ["X2", "Y2", "XY", "X2Y", "Y", "Z2"]
    assert np.allclose(m.M, [0.020, 0.040, 0.030, 0.040, 0.020, 0.010], rtol=0, atol=1e-15)
    assert m.nr == 4
    # A to SI: bimolecular x 1e-6, termolecular (third body) x 1e-12
    assert m.A[0] == pytest.approx(2.0e13 * 1e-6, rel=1e-15)
    assert m.A[3] == pytest.approx(1.0e15 * 1e-12, rel=1e-15)
    assert m.Ea[0] == pytest.approx(1000.0 * 4.184, rel=1e-15)
    assert list(m.b) == [0.5, -0.2, 0.0, -1.0]
    assert list(m.reversible) == [1, 1, 1, 0] and list(m.has_tb) == [0, 0, 0, 1]
    assert list(m.nu_f[0]) == [1, 1, 0, 0, 0, 0] and list(m.nu_b[0]) == [0, 0, 2, 0, 0, 0]
    for i in (1, 2):
        assert list(m.nu_f[i]) == [0, 0, 2, 0, 0, 0] and list(m.nu_b[i]) == [0, 0, 0, 1, 1, 0]
    assert list(m.nu_f[3]) == [1, 0, 0, 0, 1, 0] and list(m.nu_b[3]) == [0, 0, 0, 1, 0, 0]
    assert list(m.tb[3]) == [2.5, 1.0, 1.0, 1.0, 1.0, 0.5] and not m.tb[0].any()
    # two ranges: high set from line 2 and the head of line 3, low set after it
    assert m.t_mid[0] == 1200.0 and m.t_mid[5] == 1000.0       # Z2 takes the default
    assert list(m.nasa_high[0]) == [3.1, 5e-4, -1e-7, 2e-11, -1e-15, -1000.0, 4.0]
    assert list(m.nasa[0]) == [3.0, 6e-4, -2e-7, 3e-11, -2e-15, -900.0, 5.0]


def test_complement_is_moved_last():
    txt = TEXT.replace("X2 Y2 XY X2Y Y Z2", "Z2 X2 Y2 XY X2Y Y")
    m = chemkin.parse(txt, complement="Z2")
    assert m.species == ["X2", "Y2", "XY", "X2Y", "Y", "Z2"]
    assert list(m.tb[3]) == [2.5, 1.0, 1.0, 1.0, 1.0, 0.5]
    assert list(m.nu_f[3]) == [1, 0, 0, 0, 1, 0]


def _check_roundtrip(m, r):
    assert r.species == m.species and r.elements == m.elements
    assert np.array_equal(r.comp, m.comp)
    assert np.allclose(r.M, m.M, rtol=1e-15, atol=0)
    q = np.vectorize(lambda v: float(f"{v:15.8E}"))
    assert np.array_equal(r.nasa, q(m.nasa))
    assert np.allclose(r.A, m.A, rtol=2e-16 * 4, atol=0)
    assert np.array_equal(r.b, m.b)
    assert np.allclose(r.Ea, m.Ea, rtol=2e-16 * 4, atol=0)
    for f in ("nu_f", "nu_b", "has_tb", "reversible"):
        assert np.array_equal(getattr(r, f), getattr(m, f)), f
    assert np.array_equal(r.tb[m.has_tb == 1], m.tb[m.has_tb == 1])


def test_synthetic_mechanism_roundtrip():
    m = synthetic_mechanism()
    txt = chemkin.write(m, atomic_weights={"A": 2.0, "B": 16.0, "C": 14.0})
    r = chemkin.parse(txt, atomic_weights=None, complement="C2")
    _check_roundtrip(m, r)
    assert r.nasa_high is None and r.t_mid is None


def test_two_range_roundtrip():
    m = two_range_mechanism(synthetic_mechanism(), t_mid=1800.0)
    txt = chemkin.write(m, atomic_weights={"A": 2.0, "B": 16.0, "C": 14.0})
    r = chemkin.parse(txt, complement="C2")
    _check_roundtrip(m, r)
    q = np.vectorize(lambda v: float(f"{v:15.8E}"))
    assert np.array_equal(r.nasa_high, q(m.nasa_high))
    assert np.array_equal(r.t_mid, m.t_mid)


def test_separate_thermo_text():
    mech_part, rest = TEXT.split("THERMO ALL")
    thermo_part, reac_part = rest.split("END\nREACTIONS")
    m1 = chemkin.parse(TEXT)
    m2 = chemkin.parse(mech_part + "REACTIONS" + reac_part, thermo="THERMO ALL" + thermo_part + "END\n")
    assert m1.species == m2.species and np.array_equal(m1.nasa, m2.nasa)
    assert np.array_equal(m1.A, m2.A)


@pytest.mark.parametrize("old,new", [
    ("X2 + Y + M => X2Y + M", "X2 + Y2 + M => X2Y + M"),             # not balanced
    ("  Z2/0.5/ X2/2.5/", "  LOW / 1.0 2.0 3.0 /"),                     # fall-off data
    ("X2 + Y + M => X2Y + M", "X2 + Y (+M) => X2Y (+M)"),             # fall-off form
    ("X2 + Y + M => X2Y + M", "X2 + Q + M => X2Y + M"),               # unknown species
    ("REACTIONS  CAL/MOLE", "REACTIONS  MOLECULES"),                    # units
    ("X2 + Y2 <=> 2XY", "X2 + Y2 <=> 1.5XY"),                         # stoichiometry
    ("SPECIES\nX2", "SPECIES\nW2 X2"),                                 # no thermo data
])
def test_rejected_input(old, new):
    assert old in TEXT
    with pytest.raises(chemkin.ChemkinError):
        chemkin.parse(TEXT.replace(old, new), complement="Z2")
