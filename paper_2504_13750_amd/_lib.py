"""ctypes view of include/janc.h and the loader of the in-tree libjanc.so."""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjanc.so")

MAX_FIELDS = 16

D = C.c_double
I = C.c_int
PD = C.POINTER(C.c_double)
PI = C.POINTER(C.c_int)
VP = C.c_void_p


class janc_mech(C.Structure):
    _fields_ = [("ns", I), ("nr", I), ("M", PD), ("nasa", PD), ("A", PD), ("b", PD), ("Ea", PD),
                ("nu_f", PI), ("nu_b", PI), ("tb", PD), ("has_tb", PI), ("reversible", PI),
                ("nasa_high", PD), ("t_mid", PD)]


class janc_physics(C.Structure):
    _fields_ = [("gamma", D), ("R", D), ("Q", D), ("Ea", D), ("k", D)]


class janc_grid(C.Structure):
    _fields_ = [("nx", I), ("ny", I), ("dx", D), ("dy", D), ("bc", I * 4),
                ("bc_prim", (D * MAX_FIELDS) * 4)]


class janc_time(C.Structure):
    _fields_ = [("cfl", D), ("dt_fixed", D), ("t_end", D), ("split", C.c_int), ("jac", C.c_int)]


class janc_domain(C.Structure):
    _fields_ = [("grid", janc_grid), ("phys", janc_physics), ("nlevels", I)]


class janc_block(C.Structure):
    _fields_ = [("domain", I), ("level", I), ("i0", I), ("j0", I), ("nx", I), ("ny", I),
                ("offset", C.c_longlong), ("valid", I), ("pad", I)]


assert C.sizeof(janc_block) == 40


class janc_regrid_params(C.Structure):
    _fields_ = [("threshold", D), ("buffer", I), ("sub", I)]

_LIB = None

EXPORTS = {
    "janc_create": (I, [C.POINTER(VP), I, C.POINTER(janc_mech), I]),
    "janc_destroy": (None, [VP]),
    "janc_last_error": (C.c_char_p, [VP]),
    "janc_num_fields": (I, [VP]),
    "janc_set_chem_kernel": (I, [VP, I]),
    "janc_get_chem_kernel": (I, [VP, PI]),
    "janc_chem_kernel_check": (I, [C.POINTER(janc_mech), C.c_char_p, I]),
    "janc_sync_status": (I, [VP, VP]),
    "janc_init_state": (I, [VP, C.POINTER(janc_physics), C.c_longlong, VP, VP, VP, VP]),
    "janc_step": (I, [VP, C.POINTER(janc_grid), C.POINTER(janc_physics), C.POINTER(janc_time),
                      VP, VP, I, VP, VP, VP]),
    "janc_step_noalloc": (I, [VP, C.POINTER(janc_grid), C.POINTER(janc_physics),
                              C.POINTER(janc_time), VP, VP, I, VP, VP, VP]),
    "janc_plan_create": (I, [VP, I, C.POINTER(janc_domain), I, VP, C.c_longlong, I,
                             C.POINTER(VP)]),
    "janc_plan_destroy": (None, [VP]),
    "janc_plan_set_tile": (I, [VP, I]),
    "janc_plan_set_schedule": (I, [VP, I, I]),
    "janc_plan_autotune": (I, [VP, VP, C.POINTER(janc_time), VP, VP, I, C.POINTER(I),
                               C.POINTER(C.c_double), VP]),
    "janc_plan_stats": (I, [VP, C.POINTER(C.c_longlong)]),
    "janc_step_blocks": (I, [VP, VP, C.POINTER(janc_time), VP, VP, I, VP, VP]),
    "janc_profile_step": (I, [VP, VP, C.POINTER(janc_time), VP, VP, VP, C.POINTER(C.c_double),
                              VP]),
    "janc_adjoint": (I, [VP, C.POINTER(janc_grid), C.POINTER(janc_physics), C.POINTER(janc_time),
                         VP, I, I, I, PI, PD, VP, VP, VP, VP]),
    "janc_regrid": (I, [VP, VP, C.POINTER(janc_regrid_params), VP, VP, I, C.POINTER(I),
                        C.POINTER(C.c_longlong), VP]),
    "janc_regrid_fill": (I, [VP, VP, VP, VP, VP, VP, VP, VP]),
}


class LibraryMissing(RuntimeError):
    pass


def lib():
    """Load libjanc.so; fails loudly when the HIP library has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} not found: build the HIP library first "
                "(python -m paper_2504_13750_amd.build)")
        # One HIP runtime per process: torch brings its own; importing it first makes
        # libjanc bind to that runtime instead of loading a second one beside it.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB
