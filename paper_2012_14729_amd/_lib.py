"""ctypes declarations of the C ABI in include/lbm.h (argument marshalling only).

Loads the in-tree libpflbm.so and fails loudly when it is missing: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpflbm.so")

FORMS = ("stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2")
LBM_OK, LBM_E_INVAL, LBM_E_HIP, LBM_E_DIVERGED, LBM_E_UNSUPPORTED = 0, -1, -2, -3, -4


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("wall_x", C.c_int32), ("wall_y", C.c_int32),
        ("u_wall_lo", C.c_double), ("u_wall_hi", C.c_double),
        ("rho1", C.c_double), ("rho2", C.c_double),
        ("nu1", C.c_double), ("nu2", C.c_double),
        ("sigma", C.c_double), ("W", C.c_double),
        ("M", C.c_double), ("tau_h", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double),
        ("rho0", C.c_double), ("eps_n", C.c_double),
    ]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "lbm_workspace_bytes": (C.c_int, [C.POINTER(LbmParams), C.POINTER(C.c_size_t)]),
    "lbm_init": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(LbmParams), C.c_void_p, C.c_size_t, C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "lbm_moments": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p]),
    "lbm_hydro_pressure": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "lbm_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "lbm_get_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "lbm_state_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "lbm_save": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_restore": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_step_blobs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "lbm_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_kernel_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "lbm_destroy": (C.c_int, [C.c_void_p]),
    "lbm_batch_workspace_bytes": (C.c_int, [C.POINTER(LbmParams), C.c_int32, C.POINTER(C.c_size_t)]),
    "lbm_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(LbmParams), C.POINTER(C.c_int32), C.c_int32,
                                   C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.c_void_p]),
    "lbm_batch_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lbm_batch_moments": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "lbm_batch_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "lbm_batch_config": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double)]),
    "lbm_batch_tile_shape": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_batch_destroy": (C.c_int, [C.c_void_p]),
    "lbm_adjoint_workspace_bytes": (C.c_int, [C.POINTER(LbmParams), C.POINTER(C.c_size_t)]),
    "lbm_adjoint_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbm_adjoint_reset": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_adjoint_seed_phi_misfit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "lbm_adjoint_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_adjoint_step_blob": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    "lbm_adjoint_step_blob_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                                C.c_void_p]),
    "lbm_adjoint_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "lbm_adjoint_param_grads": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "lbm_adjoint_destroy": (C.c_int, [C.c_void_p]),
    "lbm_last_error": (C.c_char_p, []),
    "lbm_version": (C.c_char_p, []),
}


def exported_names():
    return tuple(_SIGS)


def lib():
    """The loaded library; raises if libpflbm.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2012_14729_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != LBM_OK:
        raise LbmError(code, lib().lbm_last_error().decode())
    return code


def make_params(**kw) -> LbmParams:
    p = LbmParams()
    p.rho0 = float("nan")
    p.eps_n = 1e-6
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, int(v) if k in ("nx", "ny", "wall_x", "wall_y") else float(v))
    return p


def form_index(form) -> int:
    if isinstance(form, str):
        return FORMS.index(form.lower().replace("-", ""))
    return int(form)
