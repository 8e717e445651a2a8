"""ctypes declarations of the stablel1 C ABI (include/stablel1.h).

torch is imported first on purpose: the library then binds to the HIP runtime
torch has already loaded (same soname), so one runtime serves the process.
"""
import ctypes
import os

import torch  # noqa: F401  (load order, see module docstring)

from .build import lib_path

F64, F32, BF16, FP8_E4M3 = 0, 1, 2, 3
OK, MAXITER, EINVAL, ESHAPE, EDTYPE, EHIP, ENOMEM, ESINGULAR, ELIMIT = 0, 1, -1, -2, -3, -4, -5, -6, -7
MAX_STAGES = 8
TRACE_FIELDS = 13
FLAG_NO_GRAPH = 1
FLAG_PROFILE = 2
FLAG_ENGINE_GRID = 4
FLAG_ENGINE_WG = 8
FLAG_ENGINE_HYBRID = 16
FLAG_TAIL_COLUMNS = 32
FLAG_ISTA = 64
FLAG_RULE_DST = 128
FLAG_NO_GEMM = 256
FLAG_RULE_DOME = 512
FLAG_HYBRID_GRID_FIRST = 1024
FLAG_GRID_SPLIT_STEP = 2048
FLAG_GRID_STEP = 4096
FLAG_PARK_ALL = 8192
GRID_KERNELS = 7
ENGINE_GRID, ENGINE_WG, ENGINE_HYBRID = 1, 2, 3

c_dict = ctypes.c_void_p
c_p = ctypes.c_void_p
c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_d = ctypes.c_double


class Opts(ctypes.Structure):
    _fields_ = [("Gamma", c_d), ("tol", c_d), ("margin", c_d), ("max_iter", c_i32), ("y_dtype", c_i32),
                ("chunk", c_i32), ("flags", c_i32), ("trace", c_p), ("trace_cap", c_i32), ("screen_every", c_i32),
                ("gemm_signals", c_i32), ("x0", c_p)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("sl1_dict_dense", c_i32, [ctypes.POINTER(c_dict), c_i32, c_i64, c_i64, c_p, c_p, c_p, c_d, c_p]),
    ("sl1_dict_kron", c_i32, [ctypes.POINTER(c_dict), c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_p, c_p, c_p, c_d,
                              c_p]),
    ("sl1_dict_faust", c_i32, [ctypes.POINTER(c_dict), c_i32, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                               c_p, c_p, c_p, c_p, c_d, c_p]),
    ("sl1_dict_free", c_i32, [c_dict]),
    ("sl1_dict_info", c_i32, [c_dict, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), ctypes.POINTER(c_d),
                              ctypes.POINTER(c_d)]),
    ("sl1_opts_default", c_i32, [ctypes.POINTER(Opts)]),
    ("sl1_solve", c_i32, [ctypes.POINTER(c_dict), c_i32, ctypes.POINTER(c_d), ctypes.POINTER(c_d), c_p, c_i64,
                          c_p, c_p, ctypes.POINTER(Opts), c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    ("sl1_solve_noalloc", c_i32, [ctypes.POINTER(c_dict), c_i32, ctypes.POINTER(c_d), ctypes.POINTER(c_d), c_p,
                                  c_i64, c_p, c_p, ctypes.POINTER(Opts), c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    ("sl1_lambda_max", c_i32, [c_dict, c_i64, c_p, c_i32, c_p, c_p]),
    ("sl1_dict_adjoint", c_i32, [c_dict, c_i64, c_p, c_i32, c_p, c_p, c_p]),
    ("sl1_grad", c_i32, [c_dict, c_i64, c_p, c_p, c_p, c_p, c_p, c_p, c_i32, c_p]),
    ("sl1_measure_rc", c_i32, [ctypes.POINTER(c_dict), c_i32, c_i64, ctypes.POINTER(c_d), c_p]),
    ("sl1_tune_kron", c_i32, [ctypes.POINTER(c_dict), c_i32, c_i64, ctypes.POINTER(c_i32), ctypes.POINTER(c_d), c_p]),
    ("sl1_dict_kron_tile", c_i32, [c_dict, c_i32, c_i32]),
    ("sl1_last_solve_clock", c_i32, [c_i64, c_i64, c_i64, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(c_d)]),
    ("sl1_last_solve_profile", c_i32, [c_i64, c_i64, c_i64, ctypes.POINTER(c_d), ctypes.POINTER(ctypes.c_longlong)]),
    ("sl1_last_solve_phases", c_i32, [c_i64, c_i64, c_i64, ctypes.POINTER(c_i32), ctypes.POINTER(c_d),
                                      ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(c_i32),
                                      ctypes.POINTER(c_i32)]),
    ("sl1_status_str", ctypes.c_char_p, [c_i32]),
    ("sl1_version", ctypes.c_char_p, []),
]

_LIB = None


def load(path=None):
    """Load libstablel1.so; raises if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"stablel1 HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or python paper_1812_06635_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class Stablel1Error(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load().sl1_status_str(code).decode()
        super().__init__(f"{where}: status {code} ({msg})")


def check(code, where, allow_warn=True):
    if code < 0 or (code > 0 and not allow_warn):
        raise Stablel1Error(code, where)
    return code
