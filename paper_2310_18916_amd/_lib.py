"""ctypes declarations of libgsis.so (see include/gsis.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsis.so")

GSIS_OK = 0
STATUS = {0: "GSIS_OK", -1: "GSIS_EINVAL", -2: "GSIS_ESTATE", -3: "GSIS_ENOMEM", -4: "GSIS_EDEVICE",
          -5: "GSIS_ENOTFINITE", -6: "GSIS_EDIVERGED"}
NMOM = {0: 14, 1: 18}
PHASES = ("prep", "sweep", "moments", "macro", "residual", "recon")


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("nvx", C.c_int), ("nvy", C.c_int), ("nvz", C.c_int),
        ("vmin", C.c_double * 3), ("vmax", C.c_double * 3),
        ("species", C.c_int), ("Kn", C.c_double), ("omega", C.c_double),
        ("dr", C.c_double), ("Zr", C.c_double), ("A", C.c_double * 4),
        ("inv_dt", C.c_double), ("vdf_dtype", C.c_int), ("conservative", C.c_int),
        ("macro_cfl", C.c_double), ("order", C.c_int), ("limiter_k", C.c_double),
    ]


# name -> (restype, argtypes), in the order of include/gsis.h
_P, _I, _D, _SZ = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_DP = C.POINTER(C.c_double)
SIGNATURES = {
    "gsis_create": (_I, [C.POINTER(_P), C.POINTER(Config)]),
    "gsis_destroy": (_I, [_P]),
    "gsis_set_solid_mask": (_I, [_P, _P, _SZ]),
    "gsis_set_velocity_nodes": (_I, [_P, C.c_int, _P, C.c_int]),
    "gsis_set_velocity_list": (_I, [_P, _P, C.c_int]),
    "gsis_set_spatial_mesh": (_I, [_P, C.c_int, _P, C.c_int, _P, _P, _P, _P]),
    "gsis_precondition": (_I, [_P, C.c_int, C.c_int]),
    "gsis_set_boundary": (_I, [_P, _I, _I, _DP, _D, _D]),
    "gsis_set_wall_flux": (_I, [_P, _I]),
    "gsis_workspace_size": (_I, [_P, C.POINTER(_SZ)]),
    "gsis_bind_workspace": (_I, [_P, _P, _SZ]),
    "gsis_set_stream": (_I, [_P, _P]),
    "gsis_init_maxwellian": (_I, [_P, _D, _DP, _D, _D]),
    "gsis_kinetic_step": (_I, [_P, _I]),
    "gsis_moments": (_I, [_P, _P, _I]),
    "gsis_gsis_correct": (_I, [_P, _I]),
    "gsis_residual": (_I, [_P, _DP]),
    "gsis_residual_noalloc": (_I, [_P, _DP]),
    "gsis_get_vdf": (_I, [_P, _P, _P]),
    "gsis_set_vdf": (_I, [_P, _P, _P]),
    "gsis_state_size": (_I, [_P, C.POINTER(_SZ)]),
    "gsis_get_state": (_I, [_P, _P]),
    "gsis_set_state": (_I, [_P, _P]),
    "gsis_set_tile": (_I, [_P, _I, _I, _I, _I]),
    "gsis_get_tile": (_I, [_P, C.POINTER(C.c_int)]),
    "gsis_autotune": (_I, [_P, _I, C.POINTER(C.c_int), _DP, _I, C.POINTER(C.c_int)]),
    "gsis_tile_shapes": (_I, [C.POINTER(C.c_int), _I, C.POINTER(C.c_int)]),
    "gsis_get_vdf_nodes": (_I, [_P, C.POINTER(C.c_int), _I, _P]),
    "gsis_profile_enable": (_I, [_P, _I]),
    "gsis_profile_read": (_I, [_P, _DP, C.POINTER(C.c_longlong), _I]),
    "gsis_pass_count": (_I, [_P, C.POINTER(C.c_longlong)]),
    "gsis_last_error": (C.c_char_p, [_P]),
    "gsis_batch_create": (_I, [C.POINTER(_P), C.POINTER(_P), _I]),
    "gsis_batch_destroy": (_I, [_P]),
    "gsis_batch_workspace_size": (_I, [_P, C.POINTER(_SZ)]),
    "gsis_batch_bind_workspace": (_I, [_P, _P, _SZ]),
    "gsis_batch_set_stream": (_I, [_P, _P]),
    "gsis_batch_set_tile": (_I, [_P, _I, _I, _I, _I]),
    "gsis_batch_get_tile": (_I, [_P, C.POINTER(C.c_int)]),
    "gsis_batch_autotune": (_I, [_P, _I, C.POINTER(C.c_int), _DP, _I, C.POINTER(C.c_int)]),
    "gsis_batch_init_maxwellian": (_I, [_P, _D, _DP, _D, _D]),
    "gsis_batch_run": (_I, [_P, _I, _I, _I]),
    "gsis_batch_residuals": (_I, [_P, _DP, _I, C.POINTER(C.c_int)]),
    "gsis_batch_last_run_ms": (_I, [_P, _DP]),
    "gsis_batch_last_error": (C.c_char_p, [_P]),
}

_lib = None


def lib():
    """Load libgsis.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python paper_2310_18916_amd/csrc/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
