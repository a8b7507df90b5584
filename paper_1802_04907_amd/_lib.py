"""ctypes declarations of the libqiht C ABI (include/qiht.h)."""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# QIHT_LIB_PATH selects another build of the same library (the host-
# sanitizer build of build.py, for instance).
LIB_PATH = os.environ.get("QIHT_LIB_PATH") or os.path.join(HERE, "libqiht.so")

QIHT_OK = 0
QIHT_FMT_BF16 = 116  # dense formats (include/qiht.h)
QIHT_FMT_E4M3 = 108
QIHT_ODD_LEVELS = 0x100  # odd level set, OR'd into a bit width
QIHT_NOALLOC_WORKSPACE_BYTES = 16 << 20  # the no-allocation solve's device array
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY",
                4: "DEVICE", 5: "NUMERIC"}
DTYPE = {"f64": 0, "f32": 1, "c64": 2, "c128": 3}
REASONS = {1: "converged", 2: "max_iters", 3: "stationary"}


class QihtParams(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("tol", C.c_double), ("k", C.c_double),
                ("c", C.c_double), ("max_backtracks", C.c_int32),
                ("mu_mode", C.c_int32), ("x0", C.c_void_p), ("support0", C.c_void_p),
                ("profile", C.c_int32), ("refit", C.c_int32)]


class QihtInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("reason", C.c_int32),
                ("backtracks", C.c_int32), ("capped_iterations", C.c_int32),
                ("mu_last", C.c_double), ("pass_ms", C.c_double),
                ("pass_launches", C.c_int32), ("full_selects", C.c_int32)]


class QihtProblem(C.Structure):
    _fields_ = [("q", C.c_void_p), ("yhat", C.c_void_p), ("s", C.c_int64),
                ("x_out", C.c_void_p), ("support_out", C.c_void_p)]


# name -> (restype, argtypes); every name is declared in include/qiht.h
SIGNATURES = {
    "qiht_default_params": (None, [C.POINTER(QihtParams)]),
    "qiht_quantize_matrix": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                       C.c_int, C.c_int, C.c_int, C.c_uint64,
                                       C.c_void_p, C.POINTER(C.c_void_p)]),
    "qiht_quantize_vector": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.c_int,
                                       C.c_uint64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.POINTER(C.c_double)]),
    "qiht_qmatrix_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                    C.POINTER(C.c_int), C.POINTER(C.c_double),
                                    C.POINTER(C.c_int64)]),
    "qiht_qmatrix_export_codes": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "qiht_qmatrix_row_exponents": (C.c_int, [C.c_void_p, C.c_void_p]),
    "qiht_qmatrix_free": (None, [C.c_void_p]),
    "qiht_niht_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64,
                                  C.POINTER(QihtParams), C.c_void_p, C.c_void_p,
                                  C.POINTER(QihtInfo), C.c_void_p]),
    "qiht_niht_solve_complex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64,
                                          C.POINTER(QihtParams), C.c_void_p, C.c_void_p,
                                          C.POINTER(QihtInfo), C.c_void_p]),
    "qiht_niht_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64,
                                          C.POINTER(QihtParams), C.c_void_p, C.c_void_p,
                                          C.POINTER(QihtInfo), C.c_void_p]),
    "qiht_niht_solve_fresh": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int,
                                        C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_uint64,
                                        C.c_int64, C.POINTER(QihtParams), C.c_void_p,
                                        C.c_void_p, C.POINTER(QihtInfo), C.c_void_p]),
    "qiht_niht_solve_batched": (C.c_int, [C.c_int32, C.POINTER(QihtProblem),
                                          C.POINTER(QihtParams),
                                          C.POINTER(QihtInfo), C.c_void_p]),
    "qiht_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "qiht_hard_threshold": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64,
                                      C.c_void_p, C.c_void_p]),
    "qiht_fourier_gradient": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64,
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "qiht_fourier_niht_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                          C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p]),
    "qiht_refit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                             C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_void_p, C.c_void_p]),
    "qiht_tune_report": (C.c_int64, [C.c_char_p, C.c_int64]),
    "qiht_last_error": (C.c_char_p, []),
    "qiht_version": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libqiht.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_1802_04907_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
