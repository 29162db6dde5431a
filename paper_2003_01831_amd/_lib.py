"""ctypes loader for libafq.so (the gfx950 HIP library built from csrc/).

Argument marshalling only: every step of the walker step runs in the library's
kernels. There is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafq.so")

AFQ_OK = 0
STATUS = {0: "AFQ_OK", -1: "AFQ_E_INVALID", -2: "AFQ_E_NOMEM", -3: "AFQ_E_HIP", -4: "AFQ_E_SINGULAR",
          -5: "AFQ_E_STATE", -6: "AFQ_E_UNSUPPORTED"}
PRECISION = {"fp64": 0, "cfp32": 1, "bf16x3": 2}
EXCHANGE_FORM = {"auto": 0, "cholesky": 1, "four_index": 2}
AFQ_HOST_PTRS = 1          # afq_system_create flag: h1, chol and phi_t are host pointers
PHASES = ["overlap", "pack", "exchange", "coulomb", "assemble", "abuild", "taylor", "weight", "qr", "msd_omega",
          "msd_sums"]

# every symbol declared in include/afq.h with its ctypes signature
_vp, _i, _d, _u64, _u32 = C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_uint32
SIGNATURES = {
    "afq_system_create": (_i, [C.POINTER(_vp), _i, _i, _i, _i, _vp, _vp, _vp, _d, _i, _vp, _u32]),
    "afq_system_set_precision": (_i, [_vp, _i]),
    "afq_system_set_msd": (_i, [_vp, _vp, _i, _vp, _vp]),
    "afq_system_set_background": (_i, [_vp, _i, _vp]),
    "afq_system_background": (_i, [_vp, C.POINTER(_i), _vp]),
    "afq_system_set_exchange_form": (_i, [_vp, _i]),
    "afq_system_exchange_form": (_i, [_vp, C.POINTER(_i), C.POINTER(_u64)]),
    "afq_kp_system_create": (_i, [C.POINTER(_vp), _i, _vp, _i, _i, _i, _i, _vp, _vp, _vp, _d, _i, _vp]),
    "afq_system_destroy": (_i, [_vp]),
    "afq_walkers_create": (_i, [C.POINTER(_vp), _vp, _i, _vp, _vp]),
    "afq_walkers_destroy": (_i, [_vp]),
    "afq_walkers_get": (_i, [_vp, _vp, _vp, _vp, _vp, C.POINTER(_u64)]),
    "afq_walkers_set": (_i, [_vp, _vp, _vp, _vp, _u64]),
    "afq_walkers_stats": (_i, [_vp, C.POINTER(_i), C.POINTER(C.c_int64)]),
    "afq_walkers_set_controls": (_i, [_vp, _d, _d]),
    "afq_walkers_comb": (_i, [_vp, _d, _vp, C.POINTER(_d)]),
    "afq_walkers_comb_noalloc": (_i, [_vp, _d, _vp, C.POINTER(_d)]),
    "afq_eshift_update": (_i, [_d, _d, _d, _d, _d, C.POINTER(_d)]),
    "afq_step": (_i, [_vp, _vp, _i, _d, _vp, _u64, _i, _d, _i, _vp, _vp, _vp, _vp]),
    "afq_energy": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "afq_energy_backward": (_i, [_vp, _vp, _d, _vp, _vp, _vp]),
    "afq_fields_generate": (_i, [_u64, _u32, _u64, _i, _i, _i, _vp, _vp]),
    "afq_autotune": (_i, [_vp, _vp, _i, _vp]),
    "afq_system_set_propagator_tile": (_i, [_vp, _i]),
    "afq_system_propagator_tile": (_i, [_vp, _vp]),
    "afq_exchange_variant": (_i, [_vp, _i, _i]),
    "afq_bp_begin": (_i, [_vp, _i]),
    "afq_bp_rdm1": (_i, [_vp, _i, _vp, C.POINTER(_d)]),
    "afq_bp_end": (_i, [_vp]),
    "afq_batch_create": (_i, [C.POINTER(_vp), _i, _vp, _vp]),
    "afq_batch_step": (_i, [_vp, _i, _d, _u64, _i, _vp, _i, _vp]),
    "afq_batch_destroy": (_i, [_vp]),
    "afq_trace_enable": (_i, [_i]),
    "afq_trace_reset": (_i, []),
    "afq_trace_query": (_i, [_i, C.POINTER(_d), C.POINTER(C.c_int64)]),
    "afq_last_error": (C.c_char_p, []),
    "afq_version": (_i, []),
}


class AfqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libafq.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2003_01831_amd.build` "
                           "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != AFQ_OK:
        msg = _lib.afq_last_error().decode() if _lib is not None else ""
        raise AfqError(code, msg)
    return code
