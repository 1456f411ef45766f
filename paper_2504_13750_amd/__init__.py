"""MI355X-native per-time-step core update of the JANC reacting-flow solver.

Python binding of the C ABI in include/janc.h (libjanc.so, hand-written HIP
kernels for gfx950). This module only marshals arguments: torch tensors supply
device memory (FP64, SoA, x fastest) and the stream; every step of the update
runs in the library's kernels. There is no CPU fallback: without the built
library every call raises.

Paper: "JANC: A cost-effective, differentiable compressible reacting flow
solver featured with JAX-based adaptive mesh refinement", arXiv 2504.13750.

Minimal use (a 9-species mechanism read from chemkin text, one uniform grid)::

    import torch, paper_2504_13750_amd as janc
    from paper_2504_13750_amd import chemkin
    mech = chemkin.parse(open("mech.inp").read(), open("thermo.dat").read())
    ctx = janc.Context(janc.DETAILED, mech)
    grid = janc.make_grid(nx, ny, dx, dy, [janc.BC_ZEROGRAD] * 4, [None] * 4)
    phys = janc.make_physics()
    U, T = ctx.init_state(phys, W)            # W: [p, u, v, T, Y_1..Y_{Ns-1}] on cuda:0
    t = torch.zeros(1, dtype=torch.float64, device=W.device)
    ctx.step(grid, phys, janc.make_time(cfl=0.5, split=janc.SPLIT_STRANG), U, T, 100, t)
    ctx.sync_status()

Block tables (AMR hierarchies, ensembles): Context.plan + Context.step_blocks; layer
updates: Context.regrid + Context.regrid_fill, or amr.AdaptiveRun for the time loop;
gradients: Context.adjoint, or autograd.probe_loss inside torch autograd.
"""

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import LibraryMissing

CPG, ONESTEP, DETAILED = 0, 1, 2
BC_PERIODIC, BC_ZEROGRAD, BC_SLIPWALL, BC_DIRICHLET = 0, 1, 2, 3
PLAN_DEFAULT, PLAN_PER_BLOCK, PLAN_NO_GRAPH, PLAN_CROSSOVER, PLAN_PER_LEVEL = 0, 1, 2, 4, 8
PLAN_AUTOTUNE = 16
PLAN_RESOLVE_HALOS = 32
CHEM_GENERIC, CHEM_SPECIALIZED = 0, 1
AUTOTUNE_CANDIDATES = [(16, 0), (16, 1), (32, 0), (32, 1), (64, 0), (64, 1)]
SPLIT_LIE, SPLIT_STRANG = 0, 1
JAC_FROZEN_T, JAC_FULL = 0, 1
STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENONFINITE", -5: "ENEWTON",
          -6: "ENEGATIVE"}

BLOCK_DTYPE = np.dtype([
    ("domain", np.int32), ("level", np.int32), ("i0", np.int32), ("j0", np.int32),
    ("nx", np.int32), ("ny", np.int32), ("offset", np.int64), ("valid", np.int32),
    ("pad", np.int32),
])


class JancError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"janc error {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _dptr(x, numel=None, name="array"):
    """Device pointer of a contiguous FP64 CUDA tensor (or None)."""
    if x is None:
        return None
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and x.numel() != numel:
        raise ValueError(f"{name} has {x.numel()} elements, expected {numel}")
    return C.c_void_p(x.data_ptr())


# ------------------------------------------------------------------ structs
def make_grid(nx, ny, dx, dy, bc, bc_prim=None):
    g = L.janc_grid()
    g.nx, g.ny, g.dx, g.dy = int(nx), int(ny), float(dx), float(dy)
    for s in range(4):
        g.bc[s] = int(bc[s])
        if bc_prim is not None and bc_prim[s] is not None:
            v = np.asarray(bc_prim[s], dtype=np.float64)
            for f in range(len(v)):
                g.bc_prim[s][f] = float(v[f])
    return g


def make_physics(gamma=1.4, R=1.0, Q=0.0, Ea=0.0, k=0.0):
    return L.janc_physics(float(gamma), float(R), float(Q), float(Ea), float(k))


def make_time(cfl=0.5, dt_fixed=0.0, t_end=0.0, split=0, jac=0):
    """split: SPLIT_LIE (chemistry over dt after the RK stages) or SPLIT_STRANG
    (chemistry over dt/2 before and after them); jac: JAC_FROZEN_T or JAC_FULL
    (point-implicit Jacobian with T following the composition)."""
    return L.janc_time(float(cfl), float(dt_fixed), float(t_end), int(split), int(jac))


def grid_of(case):
    return make_grid(case.nx, case.ny, case.dx, case.dy, case.bc, case.bc_prim)


def physics_of(obj):
    return make_physics(obj.gamma, obj.R, obj.Q, obj.Ea, obj.k)


def time_of(case, **over):
    kw = dict(cfl=case.cfl, dt_fixed=case.dt_fixed, t_end=case.t_end)
    kw.update(over)
    return make_time(**kw)


def domains_of(bcase):
    arr = (L.janc_domain * len(bcase.domains))()
    for d, dom in enumerate(bcase.domains):
        arr[d].grid = make_grid(dom.nx, dom.ny, dom.dx, dom.dy, dom.bc, dom.bc_prim)
        arr[d].phys = physics_of(dom)
        arr[d].nlevels = int(dom.nlevels)
    return arr


class _Mech:
    def __init__(self, mech):
        def f64(a):
            return np.ascontiguousarray(a, dtype=np.float64)

        def i32(a):
            return np.ascontiguousarray(a, dtype=np.int32)
        self.keep = [f64(mech.M), f64(mech.nasa), f64(mech.A), f64(mech.b), f64(mech.Ea),
                     i32(mech.nu_f), i32(mech.nu_b), f64(mech.tb), i32(mech.has_tb),
                     i32(mech.reversible)]
        hi = getattr(mech, "nasa_high", None)
        if hi is not None:
            self.keep += [f64(hi), f64(mech.t_mid)]
        k = self.keep
        pd = lambda a: a.ctypes.data_as(L.PD)
        pi = lambda a: a.ctypes.data_as(L.PI)
        self.s = L.janc_mech(len(mech.M), len(mech.A), pd(k[0]), pd(k[1]), pd(k[2]), pd(k[3]),
                             pd(k[4]), pi(k[5]), pi(k[6]), pd(k[7]), pi(k[8]), pi(k[9]),
                             pd(k[10]) if hi is not None else None,
                             pd(k[11]) if hi is not None else None)


# ------------------------------------------------------------------ context
class Plan:
    def __init__(self, ctx, handle, ndom, pool_cells):
        self.ctx, self.h, self.ndom, self.pool_cells = ctx, handle, ndom, pool_cells

    def set_tile(self, width):
        self.ctx._check(L.lib().janc_plan_set_tile(self.h, int(width)))

    def set_schedule(self, width, linear):
        self.ctx._check(L.lib().janc_plan_set_schedule(self.h, int(width), int(linear)))

    def autotune(self, time, U, T, reps=5, stream=None):
        """janc_plan_autotune: returns ((tile width, linear order) kept, {candidate: median
        ms of one RK stage triple})."""
        choice = (C.c_int * 2)()
        ms = (C.c_double * 6)()
        self.ctx._check(L.lib().janc_plan_autotune(
            self.ctx.h, self.h, C.byref(time), _dptr(U, self.ctx.nfields * self.pool_cells, "U"),
            _dptr(T, self.pool_cells, "T"), int(reps), choice, ms,
            C.c_void_p(_stream_handle(stream))))
        times = {AUTOTUNE_CANDIDATES[q]: ms[q] for q in range(6) if ms[q] >= 0.0}
        return (choice[0], choice[1]), times

    def stats(self):
        """dict(cells, ring_cells, blocks, tiles) of the plan."""
        out = (C.c_longlong * 4)()
        self.ctx._check(L.lib().janc_plan_stats(self.h, out))
        return {"cells": out[0], "ring_cells": out[1], "blocks": out[2], "tiles": out[3]}

    def close(self):
        if self.h:
            L.lib().janc_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chem_kernel_check(mech):
    """janc_chem_kernel_check: generate and compile (hipRTC, no device) the chemistry
    kernels specialised to `mech` (the forward point-implicit step and its reverse in the
    adjoint); returns (status, compiler log)."""
    m = _Mech(mech)
    buf = C.create_string_buffer(1 << 16)
    st = L.lib().janc_chem_kernel_check(C.byref(m.s), buf, len(buf))
    return int(st), buf.value.decode(errors="replace")


class Context:
    """A library context (janc_create) on one HIP device for one model."""

    def __init__(self, model, mech=None, device=0):
        lib = L.lib()
        self.model = int(model)
        self._mech = _Mech(mech) if mech is not None else None
        h = C.c_void_p()
        st = lib.janc_create(C.byref(h), self.model,
                             C.byref(self._mech.s) if self._mech else None, int(device))
        if st != 0:
            raise JancError(st, "janc_create failed")
        self.h = h
        self.device = int(device)

    @property
    def nfields(self):
        return int(L.lib().janc_num_fields(self.h))

    @property
    def chem_kernel(self):
        """janc_get_chem_kernel: CHEM_GENERIC or CHEM_SPECIALIZED (the default of a
        detailed-model context once its specialised kernel is built; the forward step and
        the adjoint's reversed chemistry follow it, with bitwise the same results)."""
        mode = C.c_int()
        self._check(L.lib().janc_get_chem_kernel(self.h, C.byref(mode)))
        return mode.value

    @chem_kernel.setter
    def chem_kernel(self, mode):
        self._check(L.lib().janc_set_chem_kernel(self.h, int(mode)))

    def _check(self, st):
        if st != 0:
            msg = L.lib().janc_last_error(self.h)
            raise JancError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            L.lib().janc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_status(self, stream=None):
        self._check(L.lib().janc_sync_status(self.h, C.c_void_p(_stream_handle(stream))))

    def init_state(self, phys, W, stream=None):
        """Primitive W [nfields, ...] (device) -> (U, T) (new device tensors)."""
        torch = _torch()
        if W.dim() < 2 or W.shape[0] != self.nfields:
            raise ValueError(f"W must have {self.nfields} fields in its leading dimension, "
                             f"got shape {tuple(W.shape)}")
        n = W[0].numel()
        U = torch.empty_like(W)
        T = torch.empty(W.shape[1:], dtype=torch.float64, device=W.device)
        self._check(L.lib().janc_init_state(self.h, C.byref(phys), C.c_longlong(n),
                                            _dptr(W, name="W"), _dptr(U), _dptr(T),
                                            C.c_void_p(_stream_handle(stream))))
        return U, T

    def step(self, grid, phys, time, U, T, nsteps, t, dt_log=None, stream=None):
        n = grid.nx * grid.ny
        if dt_log is not None and dt_log.numel() < int(nsteps):
            raise ValueError(f"dt_log has {dt_log.numel()} elements, the call writes {int(nsteps)}")
        self._check(L.lib().janc_step(self.h, C.byref(grid), C.byref(phys), C.byref(time),
                                      _dptr(U, self.nfields * n, "U"), _dptr(T, n, "T"),
                                      int(nsteps), _dptr(t, 1, "t"),
                                      _dptr(dt_log, None, "dt_log"),
                                      C.c_void_p(_stream_handle(stream))))

    def step_noalloc(self, grid, phys, time, U, T, nsteps, t, dt_log=None, stream=None):
        """Context.step through janc_step_noalloc: no device allocation; every workspace
        lives in the library's static scratch array (JANC_NOALLOC_SCRATCH_BYTES per device),
        shared by every call on the device."""
        n = grid.nx * grid.ny
        if dt_log is not None and dt_log.numel() < int(nsteps):
            raise ValueError(f"dt_log has {dt_log.numel()} elements, the call writes {int(nsteps)}")
        self._check(L.lib().janc_step_noalloc(self.h, C.byref(grid), C.byref(phys), C.byref(time),
                                              _dptr(U, self.nfields * n, "U"), _dptr(T, n, "T"),
                                              int(nsteps), _dptr(t, 1, "t"),
                                              _dptr(dt_log, None, "dt_log"),
                                              C.c_void_p(_stream_handle(stream))))

    def plan(self, domains, blocks, pool_cells, flags=PLAN_DEFAULT):
        blocks = np.ascontiguousarray(blocks, dtype=BLOCK_DTYPE)
        h = C.c_void_p()
        self._check(L.lib().janc_plan_create(self.h, len(domains), domains, len(blocks),
                                             blocks.ctypes.data_as(C.c_void_p),
                                             C.c_longlong(int(pool_cells)), int(flags),
                                             C.byref(h)))
        return Plan(self, h, len(domains), int(pool_cells))

    def step_blocks(self, plan, time, U, T, nsteps, t, stream=None):
        self._check(L.lib().janc_step_blocks(self.h, plan.h, C.byref(time),
                                             _dptr(U, self.nfields * plan.pool_cells, "U"),
                                             _dptr(T, plan.pool_cells, "T"), int(nsteps),
                                             _dptr(t, plan.ndom, "t"),
                                             C.c_void_p(_stream_handle(stream))))

    def regrid(self, plan, U, threshold, buffer, sub, stream=None):
        """Layer update of a plan's hierarchy from the state U (janc_regrid): returns the
        new block table (BLOCK_DTYPE records, offsets packed) and its pool length."""
        params = L.janc_regrid_params(float(threshold), int(buffer), int(sub))
        cap = max(1024, 4 * int(plan.stats()["blocks"]))
        while True:
            out = np.zeros(cap, dtype=BLOCK_DTYPE)
            n, pool = C.c_int(0), C.c_longlong(0)
            st = L.lib().janc_regrid(self.h, plan.h, C.byref(params),
                                     _dptr(U, self.nfields * plan.pool_cells, "U"),
                                     out.ctypes.data_as(C.c_void_p), cap, C.byref(n),
                                     C.byref(pool), C.c_void_p(_stream_handle(stream)))
            if st == -1 and n.value > cap:
                cap = n.value
                continue
            self._check(st)
            return out[:n.value].copy(), int(pool.value)

    def regrid_fill(self, old_plan, U, T, new_plan, stream=None):
        """Pools of new_plan from the state (U, T) of old_plan (janc_regrid_fill): new
        device tensors (U_new, T_new)."""
        torch = _torch()
        Un = torch.empty((self.nfields, new_plan.pool_cells), dtype=torch.float64, device=U.device)
        Tn = torch.empty(new_plan.pool_cells, dtype=torch.float64, device=U.device)
        self._check(L.lib().janc_regrid_fill(self.h, old_plan.h,
                                             _dptr(U, self.nfields * old_plan.pool_cells, "U"),
                                             _dptr(T, old_plan.pool_cells, "T"), new_plan.h,
                                             _dptr(Un), _dptr(Tn),
                                             C.c_void_p(_stream_handle(stream))))
        return Un, Tn

    def profile_step(self, plan, time, U, T, t, stream=None):
        """One step with HIP events around each launch group; returns milliseconds of
        [stage 1, stage 2, stage 3, chemistry, restriction, ring refill]."""
        ms = (C.c_double * 6)()
        self._check(L.lib().janc_profile_step(self.h, plan.h, C.byref(time),
                                              _dptr(U, self.nfields * plan.pool_cells, "U"),
                                              _dptr(T, plan.pool_cells, "T"),
                                              _dptr(t, plan.ndom, "t"), ms,
                                              C.c_void_p(_stream_handle(stream))))
        return [ms[q] for q in range(6)]

    def adjoint(self, grid, phys, time, W0, nsteps, ckpt_every, probe_cell, probe_w,
                stream=None):
        """Returns (loss, dL/dW0, dL/dtheta) as device tensors ([1], [nfields, ny, nx], [2]).
        W0 holds the model's primitives (init_state's layout); dL/dtheta = (dL/dQ, dL/dEa)
        for the one-step model, zeros for the detailed model."""
        torch = _torch()
        pc = np.ascontiguousarray(probe_cell, dtype=np.int32)
        pw = np.ascontiguousarray(probe_w, dtype=np.float64)
        loss = torch.zeros(1, dtype=torch.float64, device=W0.device)
        gW = torch.zeros_like(W0)
        gth = torch.zeros(2, dtype=torch.float64, device=W0.device)
        self._check(L.lib().janc_adjoint(self.h, C.byref(grid), C.byref(phys), C.byref(time),
                                         _dptr(W0, self.nfields * grid.nx * grid.ny, "W0"), int(nsteps),
                                         int(ckpt_every), len(pc), pc.ctypes.data_as(L.PI),
                                         pw.ctypes.data_as(L.PD), _dptr(loss), _dptr(gW),
                                         _dptr(gth), C.c_void_p(_stream_handle(stream))))
        return loss, gW, gth


def load():
    """Load the HIP library (raises LibraryMissing when it is not built)."""
    return L.lib()
