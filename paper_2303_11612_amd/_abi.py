"""ctypes declarations of the C ABI in include/tucker_rand.h.

Loading fails loudly if the HIP library has not been built; there is no
fallback implementation.
"""
import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtucker_rand.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tucker_rand.h")

TR_OK, TR_EINVAL, TR_ENOMEM, TR_EDEVICE, TR_ENOTSUP, TR_ENUMERIC = range(6)
TR_F64, TR_F32 = 0, 1
PROB = {"none": 0, "nearly_optimal": 1, "uniform": 2}
PREC = {"native": 0, "bf16": 1, "fp8e4m3": 2}
TR_DEV_NONFINITE, TR_DEV_ZERO_DIST, TR_DEV_BAD_INDEX = 0x1, 0x2, 0x4
# tr_params.flags bits
FLAGS = {"stabilized_power": 0x1, "unfused_power": 0x2, "related_form": 0x4}
KC = {"colnorms": 0, "sample": 1, "gather": 2, "power": 3, "factor": 4, "ttm": 5,
      "gaussian": 6}
MAX_ORDER = 8
# size of the fixed device scratch of tucker_rand_sthosvd_noalloc
NOALLOC_SCRATCH_BYTES = 128 << 20


class TrParams(ctypes.Structure):
    _fields_ = [
        ("order", c_int32), ("dims", POINTER(c_int64)), ("ranks", POINTER(c_int64)),
        ("oversample", c_int32), ("power", c_int32), ("prob", c_int32),
        ("samples", POINTER(c_int64)), ("seed", c_uint64), ("precision", c_int32),
        ("flags", c_uint32),
    ]


class TrDiag(ctypes.Structure):
    _fields_ = [
        ("indices", POINTER(c_void_p)), ("scales", POINTER(c_void_p)),
        ("sketch", POINTER(c_void_p)), ("sigma", POINTER(c_void_p)),
        ("status", c_void_p), ("timer", c_void_p), ("norms", c_void_p),
    ]


_SIGS = {
    "tucker_rand_status_string": (c_char_p, [c_int]),
    "tucker_rand_workspace_size": (c_int, [POINTER(TrParams), c_int, c_int, POINTER(c_size_t)]),
    "tucker_rand_thosvd": (c_int, [POINTER(TrParams), c_int, c_void_p, POINTER(c_void_p),
                                   c_void_p, c_void_p, c_size_t, POINTER(TrDiag), c_void_p]),
    "tucker_rand_sthosvd": (c_int, [POINTER(TrParams), c_int, c_void_p, POINTER(c_void_p),
                                    c_void_p, c_void_p, c_size_t, POINTER(TrDiag), c_void_p]),
    "tucker_rand_sthosvd_noalloc": (c_int, [POINTER(TrParams), c_int, c_void_p,
                                            POINTER(c_void_p), c_void_p, POINTER(TrDiag),
                                            c_void_p]),
    "tucker_rand_adaptive": (c_int, [POINTER(TrParams), c_int, c_int, c_double, c_int, c_void_p,
                                     POINTER(c_void_p), c_void_p, c_void_p, c_size_t,
                                     POINTER(c_int64), POINTER(c_double), POINTER(TrDiag),
                                     c_void_p]),
    "tucker_rand_sthosvd_csc": (c_int, [POINTER(TrParams), c_int, c_int64, c_void_p, c_void_p,
                                        c_void_p, POINTER(c_void_p), c_void_p, c_void_p,
                                        c_size_t, POINTER(TrDiag), c_void_p]),
    "tucker_rand_batch_workspace_size": (c_int, [c_int, POINTER(POINTER(TrParams)), c_int,
                                                 POINTER(c_size_t)]),
    "tucker_rand_sthosvd_batch": (c_int, [c_int, POINTER(POINTER(TrParams)), c_int,
                                          POINTER(c_void_p), POINTER(POINTER(c_void_p)),
                                          POINTER(c_void_p), c_void_p, c_size_t, c_void_p,
                                          c_void_p]),
    "tucker_rand_gaussian": (c_int, [c_int64, c_int64, c_int32, c_uint64, c_void_p, c_void_p]),
    "tucker_rand_colnorms": (c_int, [c_int, c_void_p, c_int64, c_int64, c_int64, c_void_p,
                                     c_void_p, c_void_p]),
    "tucker_rand_sample_workspace_size": (c_size_t, [c_int64]),
    "tucker_rand_sample": (c_int, [c_void_p, c_int64, c_int64, c_int, c_uint64, c_int32,
                                   c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "tucker_rand_gather": (c_int, [c_int, c_void_p, c_int64, c_int64, c_int64, c_void_p,
                                   c_int64, c_void_p, c_void_p]),
    "tucker_rand_power_workspace_size": (c_size_t, [c_int, c_int64, c_int64, c_int64, c_int64]),
    "tucker_rand_power": (c_int, [c_int, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int32,
                                  c_void_p, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]),
    "tucker_rand_factor_workspace_size": (c_size_t, [c_int64, c_int64, c_int64]),
    "tucker_rand_factor": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p]),
    "tucker_rand_ttm_workspace_size": (c_size_t, [c_int64, c_int64, c_int64, c_int64]),
    "tucker_rand_ttm": (c_int, [c_int, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64,
                                c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "tucker_rand_timer_create": (c_int, [c_int, c_uint32, POINTER(c_void_p)]),
    "tucker_rand_timer_destroy": (c_int, [c_void_p]),
    "tucker_rand_timer_reset": (c_int, [c_void_p]),
    "tucker_rand_timer_read": (c_int, [c_void_p, c_int, POINTER(c_double), POINTER(c_int64),
                                       POINTER(c_double), POINTER(c_int64)]),
}

_lib = None


def header_symbols():
    """Function names declared in include/tucker_rand.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tucker_rand_\w+)\s*\(", text)))


def lib():
    """The loaded HIP library (ctypes.CDLL) with argument types declared."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run "
                "`python -m paper_2303_11612_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().tucker_rand_status_string(code).decode()


class TuckerRandError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {status_string(code)} ({code})")
        self.code = code


def check(fn: str, code: int):
    if code != TR_OK:
        raise TuckerRandError(fn, code)
