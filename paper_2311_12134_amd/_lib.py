"""ctypes loader for liblsms_kkr.so (argument marshalling only; every step runs in the HIP library).

There is deliberately no fallback: if the shared library is missing the import of a
compute entry point raises, so a GPU run can never silently use another path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsms_kkr.so")

c_int = ctypes.c_int
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P = ctypes.POINTER

LSMS_OK = 0
LSMS_E_ARG = -1
LSMS_E_CAPACITY = -2
LSMS_E_DEVICE = -3
LSMS_E_NOMEM = -4
LSMS_E_STATE = -5
LSMS_FP64 = 0
LSMS_SPLIT = 1
INFO_NOCONV = -1
INFO_BADINPUT = -2

_PROTOS = {
    "lsms_last_error": (ctypes.c_char_p, []),
    "lsms_create": (c_int, [c_int, c_int, c_size_t, P(c_void_p)]),
    "lsms_destroy": (c_int, [c_void_p]),
    "lsms_build_liz": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_double, c_int64, c_void_p, c_void_p,
                               c_void_p, P(c_int64)]),
    "lsms_build_liz_subset": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_double, c_int32, c_void_p, c_int64,
                                      c_void_p, c_void_p, c_void_p, P(c_int64)]),
    "lsms_tau_solve": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_int,
                               c_double, c_int, c_void_p, c_void_p, c_void_p, c_void_p, P(c_void_p), c_void_p]),
    "lsms_kubo_sigma": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lsms_kubo_sigma_noalloc": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_int32, c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lsms_kubo_sigma_tensor": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                       c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lsms_kubo_sigma_grad": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_int32, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "lsms_factors_free": (c_int, [c_void_p]),
    "lsms_batched_lu_solve": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_int, c_void_p,
                                      c_void_p]),
    "lsms_autotune_kernel": (c_int, [c_void_p, c_int, c_int, c_int, P(c_int), c_void_p, c_int, c_void_p]),
    "lsms_tuning_table": (c_int, [c_void_p, c_int, c_void_p]),
    "lsms_tuning_save": (c_int, [c_void_p, ctypes.c_char_p]),
    "lsms_tuning_load": (c_int, [c_void_p, ctypes.c_char_p]),
    "lsms_peak_probe": (c_int, [c_void_p, c_int, P(c_double), c_void_p]),
    "lsms_gaunt_table": (c_int, [c_void_p]),
    "lsms_set_profiling": (c_int, [c_void_p, c_int]),
    "lsms_set_tuning": (c_int, [c_void_p, c_int, c_int]),
    "lsms_get_tuning": (c_int, [c_void_p, c_int, P(c_int)]),
    "lsms_autotune": (c_int, [c_void_p, c_int, c_int, P(c_int), P(ctypes.c_float), c_void_p]),
    "lsms_kernel_stats": (c_int, [c_void_p, c_int, P(c_double), P(c_int64), P(c_double), P(c_double)]),
}

_lib = None


class LsmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lsms error %d: %s" % (code, msg))
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblsms_kkr.so is not built (run paper_2311_12134_amd.build.build()); "
                               "there is no other implementation of this path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != LSMS_OK:
        raise LsmsError(rc, lib().lsms_last_error().decode())
    return rc
