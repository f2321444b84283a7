"""ctypes binding of liblbm.so (include/lbm.h): argument marshalling only.

Every function here forwards plain pointers and sizes to the C ABI; all the
arithmetic of the method runs in the library's HIP kernels.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
STATUS = {0: "LBM_OK", -1: "LBM_E_NULL", -2: "LBM_E_SIZE", -3: "LBM_E_DTYPE", -4: "LBM_E_PARAM",
          -5: "LBM_E_UNSTABLE", -6: "LBM_E_HIP", -7: "LBM_E_NONFINITE", -8: "LBM_E_UNSUPPORTED"}
LBM_F32, LBM_F64 = 0, 1
LBM_PERIODIC, LBM_WALLS = 0, 1


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("visc_law", ctypes.c_int32), ("model", ctypes.c_int32), ("phase_eq", ctypes.c_int32),
        ("grad_scheme", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("phi_A", ctypes.c_double), ("phi_B", ctypes.c_double),
        ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
        ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
        ("sigma", ctypes.c_double), ("W", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("eta", ctypes.c_double),
        ("s_f", ctypes.c_double * 9), ("s_g", ctypes.c_double * 9),
        ("body_force", ctypes.c_double * 2), ("gravity", ctypes.c_double * 2),
        ("rho_ref", ctypes.c_double),
        ("theta", ctypes.c_double * 4),
        ("rho0", ctypes.c_double), ("eps_n", ctypes.c_double),
    ]


class LbmError(RuntimeError):
    def __init__(self, fn, code):
        msg = lib().lbm_status_string(code).decode()
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({msg})")
        self.code = code


_lib = None
P = ctypes.POINTER
vp = ctypes.c_void_p

# name -> argtypes (restype int unless listed in _RESTYPE)
_SIGS = {
    "lbm_status_string": [ctypes.c_int],
    "lbm_state_size": [P(LbmParams), P(ctypes.c_size_t)],
    "lbm_init": [P(LbmParams), vp, vp, vp, vp, vp],
    "lbm_step": [P(LbmParams), vp, ctypes.c_int64, vp],
    "lbm_levels_per_launch": [P(LbmParams), P(ctypes.c_int32)],
    "lbm_hydrostatic_pressure": [P(LbmParams), vp, vp, vp],
    "lbm_moments": [P(LbmParams), vp, vp, vp, vp, vp],
    "lbm_diagnostics": [P(LbmParams), vp, P(ctypes.c_double), vp],
    "lbm_export_state": [P(LbmParams), vp, vp, vp, vp, P(ctypes.c_int64), vp],
    "lbm_import_state": [P(LbmParams), vp, vp, vp, vp, ctypes.c_int64, vp],
    "lbm_tape_size": [P(LbmParams), ctypes.c_int32, P(ctypes.c_size_t)],
    "lbm_tape_record": [P(LbmParams), vp, vp, ctypes.c_int32, vp],
    "lbm_tape_restore": [P(LbmParams), vp, ctypes.c_int32, vp, vp],
    "lbm_adjoint_size": [P(LbmParams), P(ctypes.c_size_t)],
    "lbm_adjoint_phi": [P(LbmParams), vp, vp, vp, vp],
    "lbm_adjoint_step": [P(LbmParams), vp, ctypes.c_int32, vp, vp],
    "lbm_adjoint_run": [P(LbmParams), vp, ctypes.c_int32, ctypes.c_int32, vp, vp],
    "lbm_adjoint_init": [P(LbmParams), vp, vp, vp],
    "lbm_adjoint_params": [P(LbmParams), vp, P(ctypes.c_double), P(ctypes.c_int64), vp],
    "lbm_adjoint_export": [P(LbmParams), vp, vp, vp, vp, vp],
    "lbm_adjoint_import": [P(LbmParams), vp, vp, vp, vp, ctypes.c_int64, vp],
    "lbm_batch_create": [P(LbmParams), ctypes.c_int32, ctypes.c_int32, P(vp)],
    "lbm_batch_state_size": [vp, P(ctypes.c_size_t)],
    "lbm_batch_case_offset": [vp, ctypes.c_int32, P(ctypes.c_size_t)],
    "lbm_batch_init": [vp, vp, P(vp), P(vp), vp],
    "lbm_batch_step": [vp, vp, ctypes.c_int64, vp],
    "lbm_batch_tuning": [vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)],
    "lbm_batch_levels_per_launch": [vp, P(ctypes.c_int32)],
    "lbm_batch_destroy": [vp],
    "lbm_batch_step_noalloc": [P(LbmParams), ctypes.c_int32, vp, ctypes.c_int64, vp],
    "lbm_bandwidth_probe": [ctypes.c_int32, vp, vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, vp],
}
_RESTYPE = {"lbm_status_string": ctypes.c_char_p}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(or python paper_2111_00847_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = L
    return _lib


def check(fn: str, code: int) -> None:
    if code != LBM_OK:
        raise LbmError(fn, code)


def call(fn: str, *args) -> int:
    """Call an entry point and raise LbmError on a non-zero status."""
    code = getattr(lib(), fn)(*args)
    check(fn, code)
    return code
