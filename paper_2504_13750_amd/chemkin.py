"""Chemkin-format mechanism and NASA-7 thermodynamic data: reader and writer.

The paper reads its detailed mechanism in chemkin format (units cm-mol-s-cal-K) and takes
the species thermodynamics as NASA-7 polynomials (Sec. 4.1, Eq. 4.3-4.9; Sec. 5.1). This
module turns such text into the arrays the library's janc_mech expects, in SI units:

* ELEMENTS, with optional atomic weights written NAME/weight/ (g/mol); standard weights
  are known for H, He, C, N, O, Ar;
* SPECIES;
* THERMO [ALL]: fixed-column four-line NASA-7 records with a high- and a low-temperature
  coefficient set and their common temperature t_mid (the default temperatures of the
  THERMO line apply where a record leaves t_mid blank). The thermo records may also come
  from a separate text;
* REACTIONS [energy units] [MOLES]: elementary reactions A + B <=> C + D (reversible),
  => (irreversible) or = (reversible), integer stoichiometric coefficients (2OH or 2 OH),
  third bodies + M with efficiency lines NAME/value/ (default 1), DUPLICATE. Energy units:
  CAL/MOLE (default), KCAL/MOLE, JOULES/MOLE, KJOULES/MOLE, KELVINS.

Conversions: A from cm-mol-s to SI by (1e-6)^(order - 1), order = forward molecularity plus
one for a third body; Ea to J/mol. Species are reordered so that the complement species
(the inert diluent whose mass fraction is 1 - sum of the others, N2 or AR by default) comes
last. A mechanism whose high and low sets coincide for every species is returned with one
range (nasa_high = t_mid = None).

Not supported (ChemkinError): pressure-dependent reactions ((+M), LOW, TROE, SRI, PLOG),
explicit reverse parameters (REV), reaction orders (FORD, RORD), MOLECULES units,
non-integer stoichiometry, unbalanced reactions.
"""

import re
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

RU = 8.314472   # J/(mol K), the library's gas constant (KELVINS activation energies)

STANDARD_WEIGHTS = {"H": 1.00794, "HE": 4.002602, "C": 12.0107, "N": 14.0067, "O": 15.9994,
                    "AR": 39.948}
ENERGY_UNITS = {"CAL/MOLE": 4.184, "KCAL/MOLE": 4184.0, "JOULES/MOLE": 1.0,
                "KJOULES/MOLE": 1000.0, "KELVINS": RU}
UNSUPPORTED = ("LOW", "TROE", "SRI", "PLOG", "REV", "FORD", "RORD", "CHEB", "LT", "RLT",
               "HIGH", "TDEP", "EXCI", "JAN", "FIT1", "MOME", "XSMI", "USRPROG")


class ChemkinError(ValueError):
    pass


@dataclass
class Mechanism:
    """A mechanism in the library's layout (SI): the attributes janc_mech is built from."""
    species: List[str]
    elements: List[str]
    comp: np.ndarray          # [ns, nel] atoms of each element
    M: np.ndarray             # [ns] kg/mol
    nasa: np.ndarray          # [ns, 7] low-temperature set (the only set with one range)
    A: np.ndarray             # [nr] SI
    b: np.ndarray             # [nr]
    Ea: np.ndarray            # [nr] J/mol
    nu_f: np.ndarray          # [nr, ns]
    nu_b: np.ndarray          # [nr, ns]
    tb: np.ndarray            # [nr, ns] third-body efficiencies (rows of non-third-body: 0)
    has_tb: np.ndarray        # [nr]
    reversible: np.ndarray    # [nr]
    nasa_high: Optional[np.ndarray] = None   # [ns, 7] used for T >= t_mid
    t_mid: Optional[np.ndarray] = None       # [ns] K

    @property
    def ns(self) -> int:
        return len(self.species)

    @property
    def nr(self) -> int:
        return len(self.A)


def _strip(line: str) -> str:
    return line.split("!", 1)[0].rstrip()


def _num(s: str) -> float:
    return float(s.strip().upper().replace("D", "E"))


def _sections(text: str):
    """Split chemkin text into (keyword line tokens, body lines) per section."""
    out, cur, body = [], None, []
    for raw in text.splitlines():
        line = _strip(raw)
        if not line.strip():
            continue
        tok = line.split()
        key = tok[0].upper()
        if cur is None:
            for name, pre in (("ELEMENTS", "ELEM"), ("SPECIES", "SPEC"), ("THERMO", "THER"),
                              ("REACTIONS", "REAC")):
                if key.startswith(pre):
                    cur, body = (name, [t.upper() for t in tok[1:]]), []
                    break
            else:
                raise ChemkinError(f"text outside a section: {raw!r}")
            continue
        if key == "END":
            out.append((cur, body))
            cur = None
            continue
        body.append(raw.split("!", 1)[0].rstrip("\n"))
    if cur is not None:
        out.append((cur, body))   # a final section may omit END
    return out


def _parse_thermo(header: List[str], lines: List[str]):
    """NASA-7 records: name -> (composition dict, low[7], high[7], t_mid)."""
    lines = [l for l in lines if l.strip()]
    t_mid_default = None
    if lines and not (len(lines[0]) >= 80 and lines[0][79] == "1"):
        vals = lines[0].split()
        try:
            t_mid_default = _num(vals[1])
            lines = lines[1:]
        except (IndexError, ValueError):
            pass
    recs = {}
    if len(lines) % 4:
        raise ChemkinError("thermo records must have four lines each")
    for k in range(0, len(lines), 4):
        l1, l2, l3, l4 = (l.ljust(80) for l in lines[k:k + 4])
        name = l1[:18].split()[0].upper()
        comp = {}
        for q in range(4):
            f = l1[24 + 5 * q:29 + 5 * q]
            el, cnt = f[:2].strip().upper(), f[2:].strip()
            if el and cnt and int(float(cnt)) != 0:
                comp[el] = comp.get(el, 0) + int(float(cnt))
        tm = l1[65:73].strip()
        t_mid = _num(tm) if tm else t_mid_default
        if t_mid is None:
            raise ChemkinError(f"species {name}: no t_mid")
        c = []
        for l in (l2, l3, l4):
            for q in range(5):
                f = l[15 * q:15 * q + 15]
                if f.strip():
                    c.append(_num(f))
        if len(c) < 14:
            raise ChemkinError(f"species {name}: expected 14 NASA-7 coefficients")
        recs[name] = (comp, np.array(c[7:14]), np.array(c[0:7]), float(t_mid))
    return recs


_SPEC = re.compile(r"^(\d*)\s*(.+)$")


def _side(text: str, species: Dict[str, int], where: str):
    """Stoichiometry of one side: ({species index: coefficient}, third body?)."""
    if "(+" in text.replace(" ", ""):
        raise ChemkinError(f"pressure-dependent (fall-off) reaction not supported: {where}")
    nu, tb = {}, False
    for part in [p.strip() for p in text.split("+") if p.strip()]:
        if part.upper() == "M":
            tb = True
            continue
        m = _SPEC.match(part)
        coef, name = m.group(1), m.group(2).strip().upper()
        if name not in species:
            raise ChemkinError(f"unknown species {name!r} in {where}")
        if re.search(r"[./]", coef):
            raise ChemkinError(f"non-integer stoichiometry in {where}")
        nu[species[name]] = nu.get(species[name], 0) + (int(coef) if coef else 1)
    return nu, tb


def parse(text: str, thermo: Optional[str] = None, complement: Optional[str] = None,
          atomic_weights: Optional[Dict[str, float]] = None) -> Mechanism:
    """Mechanism from chemkin text (and optional separate thermo text)."""
    secs = _sections(text)
    if thermo is not None:
        tsecs = _sections(thermo if thermo.lstrip().upper().startswith("THER") else
                          "THERMO\n" + thermo)
        secs += [s for s in tsecs if s[0][0] == "THERMO"]
    weights = dict(STANDARD_WEIGHTS)
    if atomic_weights:
        weights.update({k.upper(): float(v) for k, v in atomic_weights.items()})
    elements, species, trecs, reac_hdr, reac_lines = [], [], {}, [], []
    for (name, hdr), body in secs:
        if name == "ELEMENTS":
            for t in (hdr + " ".join(body).split()):
                m = re.match(r"^([A-Za-z]+)(?:/\s*([^/]+)\s*/)?$", t)
                if not m:
                    raise ChemkinError(f"bad element entry {t!r}")
                el = m.group(1).upper()
                if m.group(2):
                    weights[el] = _num(m.group(2))
                elements.append(el)
        elif name == "SPECIES":
            species += [t.upper() for t in hdr + " ".join(body).split()]
        elif name == "THERMO":
            trecs.update(_parse_thermo(hdr, body))
        else:
            reac_hdr, reac_lines = hdr, body
    if len(set(species)) != len(species):
        raise ChemkinError("duplicate species")
    for el in elements:
        if el not in weights:
            raise ChemkinError(f"no atomic weight for element {el}")
    unit = 4.184
    for t in reac_hdr:
        if t in ENERGY_UNITS:
            unit = ENERGY_UNITS[t]
        elif t == "MOLECULES":
            raise ChemkinError("MOLECULES units not supported")
        elif t not in ("MOLES",):
            raise ChemkinError(f"unknown REACTIONS unit {t}")
    sidx = {s: k for k, s in enumerate(species)}
    rx = []   # (nu_f, nu_b, tb?, rev, A, b, Ea, eff)
    for raw in reac_lines:
        line = raw.strip()
        if not line:
            continue
        if "=" in line:
            tok = line.split()
            if len(tok) < 4:
                raise ChemkinError(f"reaction line needs A, b, Ea: {raw!r}")
            A, b, Ea = (_num(x) for x in tok[-3:])
            eq = " ".join(tok[:-3])
            arrow = "<=>" if "<=>" in eq else ("=>" if "=>" in eq else "=")
            parts = eq.split(arrow)
            if len(parts) != 2:
                raise ChemkinError(f"bad reaction equation {eq!r}")
            lhs, rhs, rev = parts[0], parts[1], arrow != "=>"
            nf, tf = _side(lhs, sidx, eq)
            nb, tbk = _side(rhs, sidx, eq)
            if tf != tbk:
                raise ChemkinError(f"third body on one side only: {eq}")
            rx.append([nf, nb, tf, rev, A, b, Ea * unit, {}, eq])
            continue
        key = line.split("/")[0].split()[0].upper()
        if key in ("DUP", "DUPLICATE"):
            continue
        if key in UNSUPPORTED:
            raise ChemkinError(f"auxiliary keyword not supported: {line!r}")
        if not rx or not rx[-1][2]:
            raise ChemkinError(f"efficiencies without a third-body reaction: {line!r}")
        for name, val in re.findall(r"([^\s/]+)\s*/\s*([^/]+?)\s*/", line):
            nm = name.upper()
            if nm not in sidx:
                raise ChemkinError(f"unknown species {nm!r} in efficiencies")
            rx[-1][7][sidx[nm]] = _num(val)
    missing = [s for s in species if s not in trecs]
    if missing:
        raise ChemkinError(f"no thermo data for {missing}")
    # complement species last
    if complement is None:
        complement = "N2" if "N2" in sidx else ("AR" if "AR" in sidx else species[-1])
    complement = complement.upper()
    if complement not in sidx:
        raise ChemkinError(f"complement species {complement} not in the mechanism")
    order = [k for k in range(len(species)) if species[k] != complement] + [sidx[complement]]
    ns, nr, ne = len(species), len(rx), len(elements)
    comp = np.zeros((ns, ne), dtype=np.int64)
    for k, s in enumerate(species):
        for el, n in trecs[s][0].items():
            if el not in elements:
                raise ChemkinError(f"species {s} contains undeclared element {el}")
            comp[k, elements.index(el)] += n
    nu_f = np.zeros((nr, ns), dtype=np.int32)
    nu_b = np.zeros((nr, ns), dtype=np.int32)
    tb = np.zeros((nr, ns))
    has_tb = np.zeros(nr, dtype=np.int32)
    rev = np.zeros(nr, dtype=np.int32)
    A = np.zeros(nr)
    bb = np.zeros(nr)
    Ea = np.zeros(nr)
    for i, (nf, nb_, t, r, a, b_, e, eff, eq) in enumerate(rx):
        for k, v in nf.items():
            nu_f[i, k] = v
        for k, v in nb_.items():
            nu_b[i, k] = v
        if not np.array_equal(nu_f[i] @ comp, nu_b[i] @ comp):
            raise ChemkinError(f"reaction not element-balanced: {eq}")
        if t:
            has_tb[i] = 1
            tb[i, :] = 1.0
            for k, v in eff.items():
                tb[i, k] = v
        rev[i] = 1 if r else 0
        A[i], bb[i], Ea[i] = a, b_, e
    A = A * (1e-6) ** (nu_f.sum(axis=1) + has_tb - 1)
    w = np.array([weights[el] for el in elements]) * 1e-3
    low = np.array([trecs[s][1] for s in species])
    high = np.array([trecs[s][2] for s in species])
    tmid = np.array([trecs[s][3] for s in species])
    two = not np.array_equal(low, high)
    return Mechanism(species=[species[k] for k in order], elements=elements,
                     comp=comp[order], M=(comp[order].astype(float) @ w), nasa=low[order],
                     A=A, b=bb, Ea=Ea, nu_f=nu_f[:, order], nu_b=nu_b[:, order],
                     tb=tb[:, order], has_tb=has_tb, reversible=rev,
                     nasa_high=high[order] if two else None, t_mid=tmid[order] if two else None)


def load(path: str, thermo_path: Optional[str] = None, **kw) -> Mechanism:
    """parse() of a mechanism file (and an optional separate thermo file)."""
    with open(path) as fh:
        text = fh.read()
    thermo = None
    if thermo_path is not None:
        with open(thermo_path) as fh:
            thermo = fh.read()
    return parse(text, thermo, **kw)


def _fmt15(x: float) -> str:
    return f"{x:15.8E}"


def write(mech, atomic_weights: Optional[Dict[str, float]] = None, t_low: float = 200.0,
          t_high: float = 6000.0, t_mid: float = 1000.0) -> str:
    """Chemkin text (ELEMENTS, SPECIES, THERMO ALL, REACTIONS KCAL/MOLE MOLES) of a
    mechanism in the library's layout; A written in cm-mol-s, Ea in kcal/mol. Thermo
    coefficients use the standard 15-column fields (8 decimals); a one-range mechanism is
    written with equal high and low sets."""
    weights = dict(STANDARD_WEIGHTS)
    if atomic_weights:
        weights.update({k.upper(): float(v) for k, v in atomic_weights.items()})
    out = ["ELEMENTS"]
    out += [f"{el}/{weights[el.upper()]!r}/" for el in mech.elements]
    out += ["END", "SPECIES", " ".join(mech.species), "END", "THERMO ALL",
            f"{t_low:10.3f}{t_mid:10.3f}{t_high:10.3f}"]
    for k, s in enumerate(mech.species):
        els = [(el, int(mech.comp[k, e])) for e, el in enumerate(mech.elements) if mech.comp[k, e]]
        if len(els) > 4:
            raise ChemkinError(f"species {s}: more than 4 elements")
        ef = "".join(f"{el:<2s}{n:>3d}" for el, n in els).ljust(20)
        hi = mech.nasa_high[k] if mech.nasa_high is not None else mech.nasa[k]
        tm = float(mech.t_mid[k]) if mech.t_mid is not None else t_mid
        out.append(f"{s:<18s}{'':6s}{ef}G{t_low:10.3f}{t_high:10.3f}{tm:8.2f}".ljust(79) + "1")
        c = list(hi) + list(mech.nasa[k])
        out.append("".join(_fmt15(v) for v in c[0:5]).ljust(79) + "2")
        out.append("".join(_fmt15(v) for v in c[5:10]).ljust(79) + "3")
        out.append("".join(_fmt15(v) for v in c[10:14]).ljust(79) + "4")
    out += ["END", "REACTIONS KCAL/MOLE MOLES"]
    for i in range(mech.nr):
        def side(nu):
            terms = []
            for k in np.nonzero(nu)[0]:
                terms.append((f"{nu[k]}" if nu[k] > 1 else "") + mech.species[k])
            if mech.has_tb[i]:
                terms.append("M")
            return " + ".join(terms)
        arrow = " <=> " if mech.reversible[i] else " => "
        order = int(mech.nu_f[i].sum()) + int(mech.has_tb[i])
        A = float(mech.A[i]) / (1e-6) ** (order - 1)
        out.append(f"{side(mech.nu_f[i])}{arrow}{side(mech.nu_b[i])}   {A!r} {float(mech.b[i])!r} "
                   f"{float(mech.Ea[i]) / 4184.0!r}")
        if mech.has_tb[i]:
            eff = [f"{mech.species[k]}/{float(mech.tb[i, k])!r}/" for k in range(mech.ns)
                   if mech.tb[i, k] != 1.0]
            if eff:
                out.append("    " + " ".join(eff))
    out.append("END")
    return "\n".join(out) + "\n"
