"""Independent reference solutions used to pin the oracle (no solver code shared).

* exact Riemann solver for the Euler equations of a perfect gas (Toro, "Riemann
  Solvers and Numerical Methods for Fluid Dynamics", ch. 4), for the Sod tube;
* chemical equilibrium by Gibbs (Helmholtz) minimization with element
  potentials at fixed internal energy, density and element totals, for the
  long-time limit of the adiabatic constant-volume reactor;
* an independent ODE integration of the steady ZND wave.
"""

import math

import numpy as np
from scipy.optimize import brentq, minimize
from scipy.integrate import solve_ivp

RU = 8.314472
PATM = 101325.0


# ------------------------------------------------------------------ exact Riemann
def _fK(p, rhoK, pK, cK, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rhoK)
        B = (g - 1.0) / (g + 1.0) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
    else:       # rarefaction
        f = 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)
    return f


def riemann_star(rl, ul, pl, rr, ur, pr, g=1.4):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    fn = lambda p: _fK(p, rl, pl, cl, g) + _fK(p, rr, pr, cr, g) + (ur - ul)
    ps = brentq(fn, 1e-12, 10.0 * max(pl, pr), xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_fK(ps, rr, pr, cr, g) - _fK(ps, rl, pl, cl, g))
    return ps, us


def riemann_sample(x, t, x0, rl, ul, pl, rr, ur, pr, g=1.4):
    """Exact (rho, u, p) at positions x and time t for an initial jump at x0."""
    ps, us = riemann_star(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((3, len(x)))
    gm = (g - 1.0) / (g + 1.0)
    for n, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if ps > pl:
                SL = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= SL:
                    out[:, n] = (rl, ul, pl)
                else:
                    out[:, n] = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:
                SHL = ul - cl
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                STL = us - cs
                if s <= SHL:
                    out[:, n] = (rl, ul, pl)
                elif s >= STL:
                    out[:, n] = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2.0 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2.0 * (ul - s))
                    rho = rl * (c / cl) ** (2.0 / (g - 1))
                    out[:, n] = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                SR = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= SR:
                    out[:, n] = (rr, ur, pr)
                else:
                    out[:, n] = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:
                SHR = ur + cr
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                STR = us + cs
                if s >= SHR:
                    out[:, n] = (rr, ur, pr)
                elif s <= STR:
                    out[:, n] = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2.0 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2.0 * (ur - s))
                    rho = rr * (c / cr) ** (2.0 / (g - 1))
                    out[:, n] = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out


# ------------------------------------------------------------------ Gibbs equilibrium
def _nasa_terms(a, T):
    h = a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5 + a[5]
    s = a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4 + a[6]
    return h, s  # h/R (K), s/R (-)


def equilibrium_at_T(mech, T, b_elem, lam0=None):
    """Concentrations X (mol/m^3) minimizing the Helmholtz energy at fixed T, V and
    element totals b_elem (mol/m^3), by the convex dual in the element potentials."""
    ns = mech.ns
    g0 = np.zeros(ns)
    for k in range(ns):
        h, s = _nasa_terms(mech.nasa[k], T)
        g0[k] = h / T - s            # mu0_k / (R T) at p0 = 1 atm
    n = mech.comp.astype(float)      # [ns, nel]
    c0 = PATM / (RU * T)

    def X_of(lam):
        return c0 * np.exp(np.clip(n @ lam - g0, -700, 700))

    def dual(lam):   # convex: sum_k X_k(lam) - b . lam
        X = X_of(lam)
        return X.sum() - b_elem @ lam, n.T @ X - b_elem

    def hess(lam):
        X = X_of(lam)
        return (n * X[:, None]).T @ n

    if lam0 is None:
        # start where every species holds a comparable share of the element totals
        target = np.log(np.maximum(b_elem.mean() / ns, 1e-300) / c0) + g0
        lam, *_ = np.linalg.lstsq(n, target, rcond=None)
    else:
        lam = lam0.copy()
    # Newton on the strictly convex dual, with backtracking
    for _ in range(500):
        f, gr = dual(lam)
        H = hess(lam)
        step = np.linalg.lstsq(H, gr, rcond=None)[0]
        t = 1.0
        while True:
            f2, _ = dual(lam - t * step)
            if f2 <= f - 1e-4 * t * gr @ step or t < 1e-12:
                break
            t *= 0.5
        lam = lam - t * step
        if np.max(np.abs(gr) / np.maximum(b_elem, 1e-300)) < 1e-15:
            break
    return X_of(lam), lam


def equilibrium_T(mech, rho, e_mass, b_elem, T_lo=300.0, T_hi=6000.0):
    """Adiabatic constant-volume equilibrium: T such that the equilibrium mixture at T
    has internal energy e_mass (J/kg) at density rho."""
    cache = {"lam": None}

    def resid(T):
        X, lam = equilibrium_at_T(mech, T, b_elem, cache["lam"])
        cache["lam"] = lam
        e_vol = 0.0
        for k in range(mech.ns):
            h, _ = _nasa_terms(mech.nasa[k], T)
            e_vol += X[k] * RU * (h - T)
        return e_vol - rho * e_mass

    T = brentq(resid, T_lo, T_hi, xtol=1e-12, rtol=1e-15, maxiter=300)
    X, _ = equilibrium_at_T(mech, T, b_elem, cache["lam"])
    return T, X


# ------------------------------------------------------------------ ZND by ODE integration
def znd_half_length_ode(gamma, Q, Ea, k, D):
    """Distance behind the shock where lam = 1/2, integrating d lam/dx along the
    Rayleigh line with the Rankine-Hugoniot energy balance solved pointwise."""
    rho0 = p0 = 1.0
    m = rho0 * D
    a = gamma / (gamma - 1.0)
    H0 = a * p0 / rho0 + 0.5 * D * D

    def w_of(lam):
        # energy a p w/m + w^2/2 = H0 + lam Q with p = p0 + m (D - w); subsonic root
        f = lambda w: a * (p0 + m * (D - w)) * w / m + 0.5 * w * w - H0 - lam * Q
        w_sonic = a * (p0 / m + D) / (2.0 * (a - 0.5))
        return brentq(f, 1e-9, w_sonic, xtol=1e-15, rtol=1e-15)

    def rhs(x, y):
        lam = min(y[0], 0.999999)
        w = w_of(lam)
        p = p0 + m * (D - w)
        T = p * w / m
        return [k * (1.0 - lam) * math.exp(-Ea / T) / w]

    ev = lambda x, y: y[0] - 0.5
    ev.terminal = True
    sol = solve_ivp(rhs, (0.0, 100.0), [0.0], events=ev, rtol=1e-12, atol=1e-14, method="DOP853")
    return float(sol.t_events[0][0])
