"""ctypes loader for ``libdas.so`` (the gfx950 delay-and-sum library).

There is no fallback: if the library has not been built this raises, naming
the build command.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdas.so")

DAS_OK = 0
DAS_EINVAL = -1
DAS_ESHAPE = -2
DAS_EDTYPE = -3
DAS_EALIGN = -4
DAS_EHIP = -5
DAS_ENOMEM = -6

DAS_IQ_C64 = 0
DAS_IQ_C16F = 1
DAS_IQ_C16BF = 2

# Every symbol include/das.h declares.
EXPORTED = ("das_plan_create", "das_execute", "das_execute_per_tx", "das_plan_destroy", "das_tx_plane_wave",
            "das_plan_query", "das_tile_order", "das_status_string", "das_last_error", "das_version",
            "das_kernel_variants", "das_choose_kernel_variant")

# Every symbol include/das_learn.h declares.
LEARN_EXPORTED = ("das_conv3d", "das_conv3d_wgrad", "das_conv3d_wgrad_work", "das_transpose_weights",
                  "das_avgpool2", "das_avgpool2_bwd", "das_upsample2", "das_upsample2_bwd", "das_add_mask",
                  "das_mse_residual", "das_adam", "das_f32_to_bf16", "das_compound_features", "das_compound_work",
                  "das_compound_rescale", "das_compound_output", "das_learn_last_error")

# Every symbol include/das_post.h declares.
POST_EXPORTED = ("das_bmode", "das_bmode_work", "das_power_doppler", "das_power_doppler_work",
                 "das_power_doppler_noalloc", "das_post_last_error")


class DasParams(ctypes.Structure):
    _fields_ = [("n_tx", ctypes.c_int32), ("n_elem", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_frames", ctypes.c_int32), ("n_vox", ctypes.c_int64), ("sound_speed", ctypes.c_double),
                ("fs", ctypes.c_double), ("f_demod", ctypes.c_double), ("t0", ctypes.c_double),
                ("f_number", ctypes.c_double), ("tukey_alpha", ctypes.c_double)]


class DasPlanInfo(ctypes.Structure):
    _fields_ = [("n_vox", ctypes.c_int64), ("n_slots", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("total_triples", ctypes.c_int64), ("active_triples", ctypes.c_int64),
                ("processed_triples", ctypes.c_int64), ("tile_dims", ctypes.c_int32 * 3),
                ("max_window", ctypes.c_int32), ("kernel_fc", ctypes.c_int32), ("kernel_pitch", ctypes.c_int32),
                ("kernel_groups", ctypes.c_int32)]


_lib = None


def load():
    """Load libdas.so once and declare the prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdas.so is not built (%s); run `python -m paper_2604_06257_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.das_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(DasParams), vp, vp, vp, vp]
    lib.das_plan_create.restype = ctypes.c_int
    lib.das_execute.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    lib.das_execute.restype = ctypes.c_int
    lib.das_execute_per_tx.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    lib.das_execute_per_tx.restype = ctypes.c_int
    lib.das_plan_destroy.argtypes = [vp]
    lib.das_plan_destroy.restype = ctypes.c_int
    lib.das_tx_plane_wave.argtypes = [vp, vp, i64, vp, i32, dbl, vp]
    lib.das_tx_plane_wave.restype = ctypes.c_int
    lib.das_plan_query.argtypes = [vp, ctypes.POINTER(DasPlanInfo)]
    lib.das_plan_query.restype = ctypes.c_int
    lib.das_tile_order.argtypes = [vp, i64, vp, i64, ctypes.POINTER(i64), vp]
    lib.das_tile_order.restype = ctypes.c_int
    lib.das_status_string.argtypes = [ctypes.c_int]
    lib.das_status_string.restype = ctypes.c_char_p
    lib.das_last_error.argtypes = []
    lib.das_last_error.restype = ctypes.c_char_p
    lib.das_version.argtypes = []
    lib.das_version.restype = ctypes.c_int
    lib.das_kernel_variants.argtypes = [vp, i32]
    lib.das_kernel_variants.restype = ctypes.c_int
    lib.das_choose_kernel_variant.argtypes = [i32, i32, ctypes.c_int64, ctypes.c_double, vp]
    lib.das_choose_kernel_variant.restype = ctypes.c_int
    _declare_learn(lib)
    _lib = lib
    return lib


def _declare_learn(lib):
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
    sig = {
        "das_conv3d": [vp, i32, i32, vp, vp, vp, i32, i32, i32, vp, i32, i32, i32, i32, i32, i32, i32, i32, i32, vp],
        "das_conv3d_wgrad": [vp, i32, i32, vp, i32, i32, vp, vp, vp, i64, i32, i32, i32, i32, i32, i32, vp],
        "das_conv3d_wgrad_work": [i32, i32, i32, i32, i32, i32],
        "das_transpose_weights": [vp, vp, i32, i32, vp],
        "das_avgpool2": [vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp],
        "das_avgpool2_bwd": [vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, i32, vp],
        "das_upsample2": [vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp],
        "das_upsample2_bwd": [vp, i32, i32, vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp],
        "das_add_mask": [vp, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, i32, i64, i32, vp],
        "das_mse_residual": [vp, i32, vp, vp, i64, vp, i32, vp, vp, vp],
        "das_adam": [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp],
        "das_f32_to_bf16": [vp, vp, i64, vp],
        "das_compound_features": [vp, i32, i64, f32, vp, i32, vp, vp, vp, vp],
        "das_compound_work": [i64],
        "das_compound_rescale": [vp, i64, vp, i32, vp, vp],
        "das_compound_output": [vp, i32, vp, i64, vp, vp, vp],
        "das_learn_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    post = {"das_bmode": [vp, i64, i32, f32, vp, vp, i64, vp], "das_bmode_work": [i64, i32],
            "das_power_doppler": [vp, i64, i32, i32, vp, vp, i64, vp], "das_power_doppler_work": [i64, i32],
            "das_power_doppler_noalloc": [vp, i64, i32, i32, vp, vp],
            "das_post_last_error": []}
    for name, args in post.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.das_bmode_work.restype = i64
    lib.das_power_doppler_work.restype = i64
    lib.das_post_last_error.restype = ctypes.c_char_p
    lib.das_conv3d_wgrad_work.restype = i64
    lib.das_compound_work.restype = i64
    lib.das_learn_last_error.restype = ctypes.c_char_p


class DasError(RuntimeError):
    """A negative status from libdas (HIP failure or allocation failure)."""

    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (load().das_status_string(status).decode(), status, message))
        self.status = status


class DasValueError(ValueError):
    """A negative status from libdas caused by the arguments."""

    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (load().das_status_string(status).decode(), status, message))
        self.status = status


def check(status, learn=False, post=False):
    """Raise on a negative libdas status (ValueError for argument errors)."""
    if status == DAS_OK:
        return
    lib = load()
    msg = (lib.das_post_last_error() if post else lib.das_learn_last_error() if learn else lib.das_last_error()).decode()
    if status in (DAS_EINVAL, DAS_ESHAPE, DAS_EDTYPE, DAS_EALIGN):
        raise DasValueError(status, msg)
    raise DasError(status, msg)
