"""ctypes binding of libpadjoint.so (the C ABI in include/pa.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Loading fails loudly when the library is missing; there is no CPU
fallback.
"""

import ctypes
import os
from ctypes import POINTER, Structure, byref, c_double, c_int32, c_size_t, c_uint64, c_void_p, c_char_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpadjoint.so")

PA_OK = 0
ERRORS = {-1: "PA_EINVAL", -2: "PA_ENOMEM", -3: "PA_EDEVICE", -4: "PA_ENONFINITE",
          -5: "PA_ELINESEARCH", -6: "PA_EUNSUPPORTED"}


class PaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Physics(Structure):
    _fields_ = [("nu", c_double), ("mu", c_double), ("dt", c_double), ("forcing_amp", c_double),
                ("forcing_k", c_int32), ("reserved", c_int32)]


class Obs(Structure):
    _fields_ = [("stride", c_int32), ("n_times", c_int32), ("steps", POINTER(c_int32)),
                ("values", c_void_p)]


class Kernel(Structure):
    _fields_ = [("kind", c_int32), ("metric", c_int32), ("param", c_double)]


class EnsembleAcc(Structure):
    _fields_ = [("lambda_sum", c_void_p), ("energy_sum", c_void_p), ("shell_sum", c_void_p),
                ("count", ctypes.c_int64)]


TILE_FIELDS = ("row_variant", "row_teams", "adj_variant", "adj_teams", "col_variant", "col_block", "col_split")


class Tiles(Structure):
    _fields_ = [(name, c_int32) for name in TILE_FIELDS]


EXPORTS = {
    "pa_create": (c_int32, [POINTER(Physics), c_int32, c_int32, c_void_p, POINTER(c_void_p)]),
    "pa_destroy": (c_int32, [c_void_p]),
    "pa_set_stream": (c_int32, [c_void_p, c_void_p]),
    "pa_last_error": (c_char_p, []),
    "pa_get_shape": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "pa_workspace_bytes": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "pa_checkpoint_bytes": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_size_t)]),
    "pa_init_field": (c_int32, [c_void_p, POINTER(c_uint64), c_int32, c_double, c_double, c_void_p,
                                c_void_p, c_size_t]),
    "pa_forward": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), c_void_p, c_void_p, c_void_p,
                             c_int32, c_void_p, c_void_p, c_size_t]),
    "pa_adjoint_gradient": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), c_void_p, c_void_p,
                                      c_int32, c_void_p, c_size_t]),
    "pa_adjoint_gradient_noalloc": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), c_void_p, c_void_p,
                                              c_int32]),
    "pa_adjoint_from_checkpoints": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), c_void_p,
                                              c_void_p, c_int32, c_void_p, c_size_t]),
    "pa_precondition": (c_int32, [c_void_p, POINTER(Kernel), c_double, c_void_p, c_void_p, c_void_p,
                                  c_size_t]),
    "pa_assimilate": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), POINTER(Kernel), c_int32,
                                c_int32, c_int32, c_int32, POINTER(c_double), POINTER(c_int32), c_void_p,
                                c_size_t]),
    "pa_assimilate_kernels": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), POINTER(Kernel), c_int32,
                                        c_int32, c_int32, c_int32, POINTER(c_double), POINTER(c_int32), c_void_p,
                                        c_size_t]),
    "pa_assimilate_members": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), POINTER(Kernel), c_int32,
                                        c_int32, c_int32, c_int32, POINTER(c_double), POINTER(c_int32), c_void_p,
                                        c_size_t]),
    "pa_assimilate_state_bytes": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_size_t)]),
    "pa_assimilate_ex": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(Obs), POINTER(Kernel), c_int32, c_int32,
                                   c_int32, c_int32, c_int32, POINTER(c_double), POINTER(c_int32), c_void_p,
                                   c_void_p, c_size_t, c_void_p, c_size_t]),
    "pa_adjoint_impulse": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p,
                                     c_void_p, POINTER(EnsembleAcc), c_int32, c_void_p, c_size_t]),
    "pa_ensemble_acc_bytes": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_size_t), POINTER(c_size_t),
                                        POINTER(c_size_t)]),
    "pa_ensemble_stats": (c_int32, [c_void_p, POINTER(EnsembleAcc), c_int32, c_int32, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
    "pa_set_tiles": (c_int32, [c_void_p, POINTER(Tiles)]),
    "pa_get_tiles": (c_int32, [c_void_p, POINTER(Tiles)]),
    "pa_set_sobolev": (c_int32, [c_void_p, c_double]),
    "pa_set_checkpoint_slots": (c_int32, [c_void_p, c_int32]),
    "pa_set_cancel_flags": (c_int32, [c_void_p, c_void_p]),
    "pa_is_device_memory": (c_int32, [c_void_p, POINTER(c_int32)]),
    "pa_get_checkpoint_slots": (c_int32, [c_void_p, POINTER(c_int32)]),
    "pa_checkpoint_advances": (c_int32, [c_int32, c_int32, POINTER(ctypes.c_int64)]),
    "pa_checkpoint_schedule": (c_int32, [c_int32, c_int32, c_void_p, ctypes.c_int64, POINTER(ctypes.c_int64)]),
    "pa_first_guess": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_size_t]),
    "pa_shell_growth": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_double, c_double, c_void_p, c_void_p]),
    "pa_profile_start": (c_int32, [c_void_p, c_int32, c_int32]),
    "pa_profile_stop": (c_int32, [c_void_p, POINTER(ctypes.c_int64), POINTER(ctypes.c_int64), POINTER(c_double)]),
}

_lib = None


def load(path=None):
    """Load the library (once) and declare every export's signature."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it first (python -m paper_2602_14016_amd.build)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(code):
    if code != PA_OK:
        msg = load().pa_last_error()
        raise PaError(code, msg.decode() if msg else "")
    return code
