"""ctypes loader for libqsim.so (built in-tree by paper_2009_01845_amd.build).

There is no fallback: if the library is missing, importing a function that
needs it raises immediately."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsim.so")

QS_OK, QS_E_INVALID, QS_E_NOMEM, QS_E_DEVICE, QS_E_UNSUPPORTED, QS_E_STATE = 0, -1, -2, -3, -4, -5
QS_C64, QS_C128 = 1, 2


class QsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qsim error {code}: {msg}")
        self.code = code


class Callbacks(C.Structure):
    _fields_ = [("every", C.c_int32), ("entropy_qubits", C.c_int32), ("energy", C.c_void_p),
                ("energies", C.POINTER(C.c_double)), ("entropies", C.POINTER(C.c_double))]


class Tune(C.Structure):
    _fields_ = [("tile_bits", C.c_int32), ("fuse_k", C.c_int32), ("use_mfma", C.c_int32),
                ("low_bits", C.c_int32), ("lane_ops", C.c_int32), ("reserved", C.c_int32 * 3)]


_st = C.c_int32
_p = C.c_void_p
_pp = C.POINTER(C.c_void_p)
_i32 = C.c_int32
_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_i64 = C.c_int64
_u64 = C.c_uint64

SIGNATURES = {
    "qs_version": (C.c_char_p, []),
    "qs_last_error": (C.c_char_p, []),
    "qs_state_create": (_st, [_i32, _i32, _p, _pp]),
    "qs_state_wrap": (_st, [_p, _i32, _i32, _p, _pp]),
    "qs_state_destroy": (_st, [_p]),
    "qs_state_info": (_st, [_p, _i32p, _i32p, _pp]),
    "qs_state_set_basis": (_st, [_p, _u64]),
    "qs_state_set_plus": (_st, [_p]),
    "qs_state_upload": (_st, [_p, _p]),
    "qs_state_download": (_st, [_p, _p]),
    "qs_state_copy": (_st, [_p, _p]),
    "qs_state_sync": (_st, [_p]),
    "qs_gate_matrix": (_st, [C.c_char_p, C.c_double, _f64p, _i32p]),
    "qs_apply": (_st, [_p, _f64p, _i32, _i32p, _i32, _i32p]),
    "qs_circuit_create": (_st, [_i32, _pp]),
    "qs_circuit_add_gate": (_st, [_p, _f64p, _i32, _i32p, _i32, _i32p]),
    "qs_circuit_add_rot": (_st, [_p, C.c_char, _i32, _i32, _i32, _i32p]),
    "qs_circuit_compile": (_st, [_p, C.POINTER(Tune)]),
    "qs_circuit_run": (_st, [_p, _p, _p, _i32]),
    "qs_circuit_info": (_st, [_p, _i32p, _i32p, _i32p]),
    "qs_circuit_pass_info": (_st, [_p, _i32, _i32p, _i32p, _i32p]),
    "qs_circuit_schedule": (_st, [_p, _i32p]),
    "qs_circuit_destroy": (_st, [_p]),
    "qs_circuit_create_density": (_st, [_i32, _pp]),
    "qs_circuit_add_channel": (_st, [_p, _i32, _f64p, _i32, _i32p]),
    "qs_density_set_pure": (_st, [_p, _p]),
    "qs_channel_kraus": (_st, [C.c_char_p, C.c_double, _f64p, _i32p, _i32p]),
    "qs_density_expectation": (_st, [_p, _p, _f64p]),
    "qs_density_trace": (_st, [_p, _f64p]),
    "qs_pauli_sum_create": (_st, [_i32, _i32, _f64p, C.POINTER(C.c_char_p), _pp]),
    "qs_ising_create": (_st, [_i32, _f64p, _f64p, _pp]),
    "qs_obs_destroy": (_st, [_p]),
    "qs_expectation": (_st, [_p, _p, _f64p]),
    "qs_expectation_async": (_st, [_p, _p, _p]),
    "qs_expectation_noalloc": (_st, [_p, _p, _p]),
    "qs_norm2": (_st, [_p, _f64p]),
    "qs_sample": (_st, [_p, _i32, _i32p, _i64, _u64, _f64p, C.POINTER(C.c_int64)]),
    "qs_adiabatic_run": (_st, [_p, _p, C.c_double, C.c_double, _i32, _f64p]),
    "qs_entanglement_entropy": (_st, [_p, _i32, _f64p]),
    "qs_adiabatic_run_callbacks": (_st, [_p, _p, C.c_double, C.c_double, _i32, C.POINTER(Callbacks), _f64p]),
    "qs_evolve": (_st, [_p, _p, _p, C.c_double, C.c_double, _i32, C.POINTER(Callbacks)]),
    "qs_adjoint": (_st, [_p, _f64p, _p, _p, _p, _f64p, _f64p]),
    "qs_batch_create": (_st, [_i32, _pp, _pp, _i32, _p, _pp]),
    "qs_batch_run": (_st, [_p, _f64p, _f64p, _f64p]),
    "qs_batch_destroy": (_st, [_p]),
    "qs_batch_autotune": (_st, [_p, _f64p, C.c_char_p]),
    "qs_batch_choice": (_st, [_p, _i32, C.POINTER(Tune)]),
    "qs_autotune": (_st, [_p, _p, _f64p, C.c_char_p]),
    "qs_profile_enable": (_st, [_i32]),
    "qs_profile_reset": (_st, []),
    "qs_profile_read": (_st, [_i32, C.POINTER(C.c_int64), _f64p]),
}

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2009_01845_amd.build`")
        # torch ships its own HIP runtime; loading it first makes the library
        # bind to that same runtime (a second copy, loaded from the system
        # ROCm, would not see the device that torch has opened)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(status: int):
    if status != QS_OK:
        raise QsError(status, lib().qs_last_error().decode())
