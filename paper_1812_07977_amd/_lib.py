"""ctypes declarations of libgs_fluid.so (the C ABI in include/gs_fluid.h and
include/gs_cnn.h).

Argument marshalling only: every computation runs in the library's kernels.
Loading fails loudly if the library has not been built; there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GS_FLUID_LIB selects another build of the same sources (the host-sanitized
# build used by the CPU sanitizer check)
LIB_PATH = os.environ.get("GS_FLUID_LIB") or os.path.join(HERE, "libgs_fluid.so")

GS_OK = 0
GS_ERR_ARG = -1
GS_ERR_HIP = -2
GS_ERR_NONPHYSICAL = -3
GS_ERR_STATE = -4

GS_BC_OUTFLOW = 0
GS_BC_PERIODIC = 1
GS_F64 = 0
GS_F32 = 1

# every symbol the header declares: (name, restype, argtypes)
_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)
_LL = ctypes.c_longlong

SIGNATURES = [
    ("gs_fluid_create", _I, [_I, _I, _I, _D, _D, _D, _D, _D, _I, _I, _VP, ctypes.POINTER(_VP)]),
    ("gs_fluid_dt", _I, [_VP, _VP, _PD]),
    ("gs_fluid_dt_last", _I, [_VP, _PD]),
    ("gs_fluid_step", _I, [_VP, _VP, _D]),
    ("gs_fluid_step_dt", _I, [_VP, _VP, _D, _PD]),
    ("gs_fluid_advance", _I, [_VP, _VP, _I, _D, _VP]),
    ("gs_fluid_advance_noalloc", _I, [_I, _I, _I, _D, _D, _D, _D, _D, _I, _I, _VP, _I, _D, _D,
                                      _VP, _VP, _VP, _VP]),
    ("gs_fluid_totals", _I, [_VP, _VP, _PD]),
    ("gs_fluid_sync", _I, [_VP]),
    ("gs_fluid_get_time", _I, [_VP, _PD]),
    ("gs_fluid_set_time", _I, [_VP, _D]),
    ("gs_fluid_set_stream", _I, [_VP, _VP]),
    ("gs_fluid_set_launch", _I, [_VP, _I, _I]),
    ("gs_fluid_profile", _I, [_VP, _I]),
    ("gs_fluid_kernel_ms", _I, [_VP, _I, _PD, _PI]),
    ("gs_fluid_workspace_bytes", _LL, [_I, _I, _I, _I]),
    ("gs_fluid_destroy", None, [_VP]),
    ("gs_fluid_last_error", ctypes.c_char_p, [_VP]),
    ("gs_fluid_stream_probe", _I, [_VP, _VP, _VP, _LL, _I, _VP]),
    # batched form (include/gs_batch.h)
    ("gs_batch_create", _I, [_I, _VP, _D, _D, _I, _I, _VP, _VP, ctypes.POINTER(_VP)]),
    ("gs_batch_set_launch", _I, [_VP, _I, _I]),
    ("gs_batch_autotune", _I, [_VP, ctypes.c_char_p, _PI, _PI, _PI]),
    ("gs_batch_advance", _I, [_VP, _I, _D, _I]),
    ("gs_batch_times", _I, [_VP, _PD]),
    ("gs_batch_sync", _I, [_VP]),
    ("gs_batch_destroy", None, [_VP]),
    ("gs_batch_last_error", ctypes.c_char_p, [_VP]),
    # learned-correction network (include/gs_cnn.h)
    ("gs_cnn_param_count", _I, []),
    ("gs_cnn_create", _I, [_I, _I, _I, _I, _D, _VP, ctypes.POINTER(_VP)]),
    ("gs_cnn_set_params", _I, [_VP, _VP]),
    ("gs_cnn_get_params", _I, [_VP, _VP]),
    ("gs_cnn_set_norm", _I, [_VP, _PD, _PD, _PD]),
    ("gs_cnn_set_features", _I, [_VP, _I, _D]),
    ("gs_cnn_forward", _I, [_VP, _VP, _VP]),
    ("gs_cnn_restrict", _I, [_VP, _VP, _VP]),
    ("gs_cnn_make_target", _I, [_VP, _VP, _VP, _VP]),
    ("gs_cnn_gradients", _I, [_VP, _VP, _VP, _VP, _PD]),
    ("gs_cnn_train_step", _I, [_VP, _VP, _VP, ctypes.c_float, _PD]),
    ("gs_cnn_correct", _I, [_VP, _VP]),
    ("gs_cnn_counts", _I, [_VP, _PI, _PI]),
    ("gs_cnn_set_stream", _I, [_VP, _VP]),
    ("gs_cnn_destroy", None, [_VP]),
    ("gs_cnn_last_error", ctypes.c_char_p, [_VP]),
]

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded library; raises LibraryMissing if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built; run `python -m paper_1812_07977_amd.build` "
                "(hipcc, gfx950). There is no CPU fallback.")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
