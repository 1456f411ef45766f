"""CPU oracle for the reacting-flow step of arXiv 2504.13750 (test infrastructure).

A plain FP64 C++ implementation (janc_oracle.cpp) of what the HIP library
computes, loaded through ctypes. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does. It shares no code with the HIP library: both consume the seeded
primitive inputs of the `cases` package and nothing else.
"""

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

D = C.c_double
I = C.c_int
PD = C.POINTER(C.c_double)
PI = C.POINTER(C.c_int)


class OMech(C.Structure):
    _fields_ = [("ns", I), ("nr", I), ("M", PD), ("nasa", PD), ("A", PD), ("b", PD), ("Ea", PD),
                ("nuf", PI), ("nub", PI), ("tb", PD), ("has_tb", PI), ("rev", PI),
                ("nasa_high", PD), ("t_mid", PD)]


class OPhys(C.Structure):
    _fields_ = [("model", I), ("gamma", D), ("R", D), ("Q", D), ("Ea", D), ("k", D)]


class OGrid(C.Structure):
    _fields_ = [("nx", I), ("ny", I), ("dx", D), ("dy", D), ("bc", I * 4)]


class OTime(C.Structure):
    _fields_ = [("cfl", D), ("dt_fixed", D), ("t_end", D), ("split", I), ("jac", I)]


class ODomain(C.Structure):
    _fields_ = [("nx", I), ("ny", I), ("dx", D), ("dy", D), ("bc", I * 4), ("nlevels", I),
                ("gamma", D), ("R", D), ("Q", D), ("Ea", D), ("k", D)]


ST_OK, ST_EINVAL, ST_NONFINITE, ST_NEWTON, ST_NEGATIVE = 0, -1, -4, -5, -6


class OracleError(RuntimeError):
    pass


def lib():
    """The oracle library. JANC_ORACLE_VARIANT=fma selects the build with fused
    multiply-add contraction, used only to measure round-off floors."""
    global _LIB
    if _LIB is None:
        variant = os.environ.get("JANC_ORACLE_VARIANT") or None
        path = _build.lib_path(variant)
        src = os.path.join(_HERE, "janc_oracle.cpp")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build(variant=variant)
        _LIB = C.CDLL(path)
        _LIB.oracle_weno5.restype = D
        _LIB.oracle_max_threads.restype = I
    return _LIB


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _p(a, t=PD):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class _MechView:
    """Keeps the numpy buffers alive while the C view is used."""

    def __init__(self, mech):
        self.keep = []
        if mech is None:
            self.ptr = None
            return
        def k(a, f):
            a = f(a)
            self.keep.append(a)
            return a
        M = k(mech.M, _f64); nasa = k(mech.nasa, _f64); A = k(mech.A, _f64)
        b = k(mech.b, _f64); Ea = k(mech.Ea, _f64); nuf = k(mech.nu_f, _i32)
        nub = k(mech.nu_b, _i32); tb = k(mech.tb, _f64); htb = k(mech.has_tb, _i32)
        rev = k(mech.reversible, _i32)
        hi = tm = None
        if getattr(mech, "nasa_high", None) is not None:
            hi = k(mech.nasa_high, _f64)
            tm = k(mech.t_mid, _f64)
        self.s = OMech(len(mech.M), len(mech.A), _p(M), _p(nasa), _p(A), _p(b), _p(Ea),
                       _p(nuf, PI), _p(nub, PI), _p(tb), _p(htb, PI), _p(rev, PI),
                       None if hi is None else _p(hi), None if tm is None else _p(tm))
        self.ptr = C.byref(self.s)


def _phys(case):
    return OPhys(case.model, case.gamma, case.R, case.Q, case.Ea, case.k)


def _grid(case):
    return OGrid(case.nx, case.ny, case.dx, case.dy, (I * 4)(*case.bc))


def _bc_prim(nU, bc, bc_prim):
    out = np.zeros((4, nU))
    for s in range(4):
        if bc_prim[s] is not None:
            out[s] = bc_prim[s]
    return out


def _check(st, what):
    if st != ST_OK:
        raise OracleError(f"oracle {what} failed with status {st}")


# ------------------------------------------------------------------ state conversion
def init_state(model, W, mech=None, gamma=1.4, R=1.0, Q=0.0):
    """Primitive [nU, ...] -> (U [nU, ...], T [...]) for one model."""
    W = _f64(W)
    shape = W.shape[1:]
    n = int(np.prod(shape))
    U = np.zeros_like(W)
    T = np.zeros(shape)
    mv = _MechView(mech)
    ph = OPhys(model, gamma, R, Q, 0.0, 0.0)
    st = lib().oracle_init_state(C.byref(ph), mv.ptr, C.c_longlong(n), _p(W), _p(U), _p(T))
    _check(st, "init_state")
    return U, T


def case_state(case):
    return init_state(case.model, case.W, case.mech, case.gamma, case.R, case.Q)


def primitives(case, U, T):
    U = _f64(U)
    T = _f64(T)
    n = int(np.prod(T.shape))
    out = np.zeros((6,) + T.shape)
    mv = _MechView(case.mech)
    ph = _phys(case)
    st = lib().oracle_primitives(C.byref(ph), mv.ptr, C.c_longlong(n), _p(U), _p(T), _p(out))
    _check(st, "primitives")
    return out


# ------------------------------------------------------------------ uniform grid
def rhs(case, U, T):
    U = _f64(U).copy()
    T = _f64(T).copy()
    L = np.zeros_like(U)
    mv = _MechView(case.mech)
    ph, g = _phys(case), _grid(case)
    bp = _bc_prim(case.nU, case.bc, case.bc_prim)
    st = lib().oracle_rhs(C.byref(g), C.byref(ph), mv.ptr, _p(bp), _p(U), _p(T), _p(L))
    _check(st, "rhs")
    return L


def step(case, U, T, nsteps, t=0.0, cfl=None, dt_fixed=None, t_end=None, check=True,
         strang=False, full_jacobian=False):
    """Advance nsteps; returns (U, T, t, dt_log, status).

    strang=False: chemistry over dt after the RK stages (Lie); True: over dt/2 before
    and after them (Strang splitting, Sec. 4.2). full_jacobian: the point-implicit
    Jacobian lets T follow the composition at fixed rho and e (species + T variant)."""
    U = _f64(U).copy()
    T = _f64(T).copy()
    mv = _MechView(case.mech)
    ph, g = _phys(case), _grid(case)
    tm = OTime(case.cfl if cfl is None else cfl,
               case.dt_fixed if dt_fixed is None else dt_fixed,
               case.t_end if t_end is None else t_end, 1 if strang else 0,
               1 if full_jacobian else 0)
    bp = _bc_prim(case.nU, case.bc, case.bc_prim)
    tt = D(t)
    dts = np.zeros(max(nsteps, 1))
    st = lib().oracle_step(C.byref(g), C.byref(ph), mv.ptr, _p(bp), C.byref(tm), _p(U), _p(T),
                           I(nsteps), C.byref(tt), _p(dts))
    if check:
        _check(st, "step")
    return U, T, tt.value, dts[:nsteps], st


def loss_tangent(case, W0, nsteps, probe_cell, probe_w, dt_fixed, dW0=None, dQ=0.0, dEa=0.0):
    """Probe loss and its directional derivative along (dW0, dQ, dEa) (forward-mode dual numbers)."""
    W0 = _f64(W0)
    dW = None if dW0 is None else _f64(dW0)
    mv = _MechView(case.mech)
    ph, g = _phys(case), _grid(case)
    bp = _bc_prim(case.nU, case.bc, case.bc_prim)
    pc = _i32(probe_cell)
    pw = _f64(probe_w)
    loss, dloss = D(0.0), D(0.0)
    st = lib().oracle_loss_tangent(C.byref(g), C.byref(ph), mv.ptr, _p(bp), D(dt_fixed), _p(W0),
                                   None if dW is None else _p(dW), D(dQ), D(dEa), I(nsteps),
                                   I(len(pc)), _p(pc, PI), _p(pw), C.byref(loss), C.byref(dloss))
    _check(st, "loss_tangent")
    return loss.value, dloss.value


# ------------------------------------------------------------------ block tables
def _domains(bcase):
    arr = (ODomain * len(bcase.domains))()
    for d, dom in enumerate(bcase.domains):
        arr[d] = ODomain(dom.nx, dom.ny, dom.dx, dom.dy, (I * 4)(*dom.bc), dom.nlevels,
                         dom.gamma, dom.R, dom.Q, dom.Ea, dom.k)
    return arr


def block_state(bcase):
    """Conserved pool state from the primitive pool, domain by domain."""
    U = np.zeros_like(bcase.W)
    T = np.zeros(bcase.pool_cells)
    for b in bcase.blocks:
        dom = bcase.domains[b["domain"]]
        s = slice(int(b["offset"]), int(b["offset"]) + int(b["nx"]) * int(b["ny"]))
        u, t = init_state(bcase.model, bcase.W[:, s], bcase.mech, dom.gamma, dom.R, dom.Q)
        U[:, s] = u
        T[s] = t
    return U, T


def step_blocks(bcase, U, T, nsteps, t=None, cfl=None, dt_fixed=None, t_end=None, check=True,
                crossover=False, strang=False, full_jacobian=False):
    """Advance a block table nsteps; returns (U, T, t[ndom], dt_log[nsteps, ndom], status).

    crossover=False: synchronous advance (paper Fig. 2b); True: crossover advance (Fig. 2a,
    Alg. 2), where a step is one level-0 step (dt_log holds dt_0). strang as in step()."""
    U = _f64(U).copy()
    T = _f64(T).copy()
    nd = len(bcase.domains)
    nU = bcase.nU
    mv = _MechView(bcase.mech)
    doms = _domains(bcase)
    bp = np.zeros((nd, 4, nU))
    for d, dom in enumerate(bcase.domains):
        bp[d] = _bc_prim(nU, dom.bc, dom.bc_prim)
    blocks = np.ascontiguousarray(bcase.blocks)
    tm = OTime(bcase.cfl if cfl is None else cfl,
               bcase.dt_fixed if dt_fixed is None else dt_fixed,
               bcase.t_end if t_end is None else t_end, 1 if strang else 0,
               1 if full_jacobian else 0)
    tt = np.zeros(nd) if t is None else _f64(t).copy()
    dts = np.zeros((max(nsteps, 1), nd))
    st = lib().oracle_step_blocks(I(bcase.model), mv.ptr, I(nd), doms, _p(bp), I(len(blocks)),
                                  blocks.ctypes.data_as(C.c_void_p),
                                  C.c_longlong(bcase.pool_cells), C.byref(tm), _p(U), _p(T),
                                  I(nsteps), _p(tt), _p(dts), I(1 if crossover else 0))
    if check:
        _check(st, "step_blocks")
    return U, T, tt, dts[:nsteps], st


def ring_flags(bcase):
    flags = np.zeros(bcase.pool_cells, dtype=np.uint8)
    doms = _domains(bcase)
    blocks = np.ascontiguousarray(bcase.blocks)
    ns = bcase.mech.ns if bcase.mech is not None else 0
    st = lib().oracle_ring_flags(I(bcase.model), I(ns), I(len(bcase.domains)), doms,
                                 I(len(blocks)), blocks.ctypes.data_as(C.c_void_p),
                                 C.c_longlong(bcase.pool_cells),
                                 flags.ctypes.data_as(C.POINTER(C.c_ubyte)))
    _check(st, "ring_flags")
    return flags


class ORegrid(C.Structure):
    _fields_ = [("threshold", D), ("buffer", I), ("sub", I)]


def regrid(bcase, U, threshold, buffer, sub):
    """New block table of a hierarchy by the density-gradient criterion (layer update of
    Sec. 3.1.2 / 3.1.4): returns (blocks [BLOCK_DTYPE], pool_cells)."""
    doms = _domains(bcase)
    blocks = np.ascontiguousarray(bcase.blocks)
    ns = bcase.mech.ns if bcase.mech is not None else 0
    bc_rho = np.zeros((len(bcase.domains), 4))
    for d, dom in enumerate(bcase.domains):
        for q in range(4):
            if dom.bc_prim is not None and dom.bc_prim[q] is not None:
                bc_rho[d, q] = float(dom.bc_prim[q][0])
    cfg = ORegrid(float(threshold), int(buffer), int(sub))
    U = _f64(U)
    cap = 1024
    while True:
        out = np.zeros(cap, dtype=blocks.dtype)
        n, pool = I(0), C.c_longlong(0)
        st = lib().oracle_regrid(I(bcase.model), I(ns), I(len(bcase.domains)), doms, _p(bc_rho),
                                 I(len(blocks)), blocks.ctypes.data_as(C.c_void_p),
                                 C.c_longlong(bcase.pool_cells), _p(U), C.byref(cfg),
                                 out.ctypes.data_as(C.c_void_p), I(cap), C.byref(n),
                                 C.byref(pool))
        if st == ST_EINVAL and n.value > cap:
            cap = n.value
            continue
        _check(st, "regrid")
        return out[:n.value].copy(), int(pool.value)


def regrid_fill(bcase, U, T, blocks, pool_cells):
    """Pools of a new table (from regrid): unaltered blocks copied, new blocks injected
    one-to-four from the new coarser layer. Returns (U, T)."""
    doms = _domains(bcase)
    old = np.ascontiguousarray(bcase.blocks)
    new = np.ascontiguousarray(blocks)
    ns = bcase.mech.ns if bcase.mech is not None else 0
    U, T = _f64(U), _f64(T)
    Un = np.zeros((U.shape[0], pool_cells))
    Tn = np.zeros(pool_cells)
    st = lib().oracle_regrid_fill(I(bcase.model), I(ns), I(len(bcase.domains)), doms,
                                  I(len(old)), old.ctypes.data_as(C.c_void_p),
                                  C.c_longlong(bcase.pool_cells), _p(U), _p(T), I(len(new)),
                                  new.ctypes.data_as(C.c_void_p), C.c_longlong(pool_cells),
                                  _p(Un), _p(Tn))
    _check(st, "regrid_fill")
    return Un, Tn


# ------------------------------------------------------------------ point functions for pins
def weno5(f):
    f = _f64(f)
    return lib().oracle_weno5(_p(f))


def species_thermo(mech, k, T):
    mv = _MechView(mech)
    h, cp, s = D(), D(), D()
    lib().oracle_species_thermo(mv.ptr, I(k), D(T), C.byref(h), C.byref(cp), C.byref(s))
    return h.value, cp.value, s.value


def mixture_e_cv(mech, Y, T):
    mv = _MechView(mech)
    Y = _f64(Y)
    e, cv = D(), D()
    lib().oracle_mixture_e_cv(mv.ptr, _p(Y), D(T), C.byref(e), C.byref(cv))
    return e.value, cv.value


def temperature(mech, Y, e, Tguess):
    mv = _MechView(mech)
    Y = _f64(Y)
    T = D()
    st = lib().oracle_temperature(mv.ptr, _p(Y), D(e), D(Tguess), C.byref(T))
    _check(st, "temperature")
    return T.value


def production(mech, rho, T, rhoY, jacobian=False):
    mv = _MechView(mech)
    rhoY = _f64(rhoY)
    w = np.zeros(mech.ns)
    nt = mech.ns - 1
    J = np.zeros((nt, nt)) if jacobian else None
    lib().oracle_production(mv.ptr, D(rho), D(T), _p(rhoY), _p(w),
                            _p(J) if jacobian else None)
    return (w, J) if jacobian else w


def full_jacobian(mech, rho, e, T, rhoY):
    """dS/d(rho Y_1..rho Y_{Ns-1}) with T following the composition at fixed rho and e."""
    mv = _MechView(mech)
    rhoY = _f64(rhoY).copy()
    nt = mech.ns - 1
    J = np.zeros((nt, nt))
    st = lib().oracle_full_jacobian(mv.ptr, D(rho), D(e), D(T), _p(rhoY), _p(J))
    _check(st, "full_jacobian")
    return J


def point_implicit(mech, rho, T, rhoY, dt):
    mv = _MechView(mech)
    r = _f64(rhoY).copy()
    st = lib().oracle_point_implicit(mv.ptr, D(rho), D(T), _p(r), D(dt))
    _check(st, "point_implicit")
    return r
