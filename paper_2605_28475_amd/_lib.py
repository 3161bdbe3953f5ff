"""ctypes declarations of the C ABI in include/wefq.h (argument marshalling only)."""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwefq.so")

WEFQ_OK, WEFQ_EINVAL, WEFQ_ENOMEM, WEFQ_EHIP, WEFQ_EUNSUPPORTED, WEFQ_EBUDGET = range(6)
MAXWELL, HARD_SPHERE, VHS = 0, 1, 2
FP64, FP32, BF16X3, FP64_NAIVE, PREP_BILINEAR, PREP_RADIAL = 1, 2, 4, 8, 16, 32
RK_EULER, RK_HEUN, RK_SSP3, RK_CLASSIC4 = 1, 2, 3, 4
PROBE_MFMA_F32, PROBE_MFMA_F64, PROBE_MFMA_BF16, PROBE_VALU_F32, PROBE_VALU_F64 = range(5)

STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "EUNSUPPORTED", 5: "EBUDGET"}


MAX_BETA = 33          # WEFQ_MAX_BETA
RK_NOALLOC_BYTES = 64 << 20   # WEFQ_RK_NOALLOC_BYTES


class CoreDesc(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("gamma", ctypes.c_double), ("b0", ctypes.c_double),
                ("Kmax", ctypes.c_int32), ("Lmax", ctypes.c_int32),
                ("precisions", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("n_beta", ctypes.c_int32), ("beta", ctypes.POINTER(ctypes.c_double)),
                ("rad_pad", ctypes.c_int32), ("ang_pad", ctypes.c_int32)]


class CoreInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("NK", ctypes.c_int64), ("NQ", ctypes.c_int64),
                ("N_T", ctypes.c_int64), ("N_G", ctypes.c_int64), ("N_S", ctypes.c_int64),
                ("N_T_merged", ctypes.c_int64), ("N_G_merged", ctypes.c_int64),
                ("N_S_merged", ctypes.c_int64), ("quad_nodes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("flop_alg_per_cell", ctypes.c_double),
                ("gamma", ctypes.c_double), ("b0", ctypes.c_double), ("model", ctypes.c_int64),
                ("n_beta", ctypes.c_int64), ("beta", ctypes.c_double * MAX_BETA),
                ("radial_groups", ctypes.c_int64), ("rad_pad", ctypes.c_int64), ("ang_pad", ctypes.c_int64)]


class Segment(ctypes.Structure):
    _fields_ = [("core", ctypes.c_void_p), ("precision", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("f", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("B", ctypes.c_int64),
                ("ld_f", ctypes.c_int64), ("ld_q", ctypes.c_int64)]


class WefqError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"wefq {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

# (name, restype, argtypes)
_SIGNATURES = [
    ("wefq_build_core", ctypes.c_int, [ctypes.POINTER(CoreDesc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("wefq_core_info_get", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CoreInfo)]),
    ("wefq_core_download_R", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    ("wefq_core_save", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    ("wefq_core_load", ctypes.c_int, [ctypes.c_char_p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    ("wefq_mode_index", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int64)]),
    ("wefq_apply_Q", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]),
    ("wefq_radial_workspace", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("wefq_apply_Q_radial", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p]),
    ("wefq_dense_bytes", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    ("wefq_dense_assemble", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("wefq_apply_Q_dense", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p]),
    ("wefq_apply_J", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_void_p]),
    ("wefq_apply_Qfg", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_void_p]),
    ("wefq_check_conservation", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    ("wefq_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("wefq_last_error", ctypes.c_char_p, []),
    ("wefq_host_coo", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("wefq_host_gauss", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    ("wefq_tune_set", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("wefq_tune_get", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    ("wefq_plan_create", ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    ("wefq_plan_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("wefq_plan_launch_direct", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("wefq_plan_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
    ("wefq_plan_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("wefq_runner_create", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    ("wefq_runner_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    ("wefq_runner_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("wefq_rk_workspace", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64)]),
    ("wefq_rk_integrate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_void_p]),
    ("wefq_rk_integrate_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    ("wefq_peak_probe", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_void_p]),
]


def exported_symbols():
    return [name for name, _, _ in _SIGNATURES]


def lib():
    """Load libwefq.so; raises if the HIP extension has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with python -m paper_2605_28475_amd.build")
        # The device buffers and streams come from torch, which carries its own HIP runtime and
        # names it by a different file name: loading this library first would bring in the
        # system runtime as well, and two runtimes in one process do not share devices
        # (the library then finds no device).  Loaded after torch, it binds to torch's.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        handle = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status):
    if status != WEFQ_OK:
        msg = lib().wefq_last_error()
        raise WefqError(status, msg.decode() if msg else "")
