"""ctypes view of the C ABI in include/mrrr.h (libmrrr.so, built for gfx950).

Loading fails loudly when the library is missing: there is no CPU fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrrr.so")

MRRR_ALL, MRRR_INDEX, MRRR_VALUE = 0, 1, 2
COUNTER_NAMES = ("blocks", "nodes", "levels", "sturm_steps", "qds_steps", "singletons", "twisted",
                 "fallbacks", "child_reject", "workspace_mb", "wave_solves", "pool_rows", "ambiguous_left",
                 "workspace_bytes")
EXPORTS = ("mrrr_step", "mrrr_step_batched", "mrrr_step_backward", "mrrr_step_backward_batched",
           "mrrr_get_tuning", "mrrr_set_tuning", "mrrr_autotune_batched", "mrrr_profile_enable", "mrrr_profile_reset",
           "mrrr_profile_read", "mrrr_release", "mrrr_last_error", "mrrr_status_string", "mrrr_workspace_size",
           "mrrr_step_ws", "mrrr_get_limits", "mrrr_set_limits", "mrrr_step_noalloc",
           "mrrr_probe_division", "mrrr_backtransform", "mrrr_tridiagonalize",
           "mrrr_cholesky", "mrrr_sygst", "mrrr_trsm_lt", "mrrr_step_f32",
           "mrrr_syev", "mrrr_sygv", "mrrr_syevr", "mrrr_sygvr")
KERNELS = ("grid", "refine", "child", "vectors", "backward", "vectors_ckpt", "backtransform", "tridiag", "ghep")


class MrrrRange(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("il", ctypes.c_int64),
                ("iu", ctypes.c_int64), ("vl", ctypes.c_double), ("vu", ctypes.c_double)]


class MrrrInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("status", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("counters", ctypes.c_int64 * 16)]

    def as_dict(self):
        out = {"m": self.m, "status": self.status, "max_depth": self.max_depth}
        for k, name in enumerate(COUNTER_NAMES):
            out[name] = int(self.counters[k])
        return out


class MrrrTuning(ctypes.Structure):
    _fields_ = [("grid_density", ctypes.c_int32), ("refine_wave_slots", ctypes.c_int32),
                ("vec_wave_slots", ctypes.c_int32), ("vec_ckpt_min_run", ctypes.c_int32),
                ("vec_ckpt_min_n", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class MrrrLimits(ctypes.Structure):
    _fields_ = [("max_depth", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("child_growth_limit", ctypes.c_double)]


class MrrrKernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("work", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class MrrrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mrrr error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libmrrr.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1205_2107_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    PI64 = ctypes.POINTER(ctypes.c_int64)
    lib.mrrr_step.restype = ctypes.c_int
    lib.mrrr_step.argtypes = [I64, P, P, MrrrRange, P, P, I64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_step_f32.restype = ctypes.c_int
    lib.mrrr_step_f32.argtypes = [I64, P, P, MrrrRange, P, P, I64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_workspace_size.restype = ctypes.c_size_t
    lib.mrrr_workspace_size.argtypes = [I64, MrrrRange]
    lib.mrrr_step_ws.restype = ctypes.c_int
    lib.mrrr_step_ws.argtypes = [I64, P, P, MrrrRange, P, P, I64, P, ctypes.c_size_t, P, P]
    lib.mrrr_step_noalloc.restype = ctypes.c_int
    lib.mrrr_step_noalloc.argtypes = [I64, P, P, MrrrRange, P, P, I64, P, P]
    lib.mrrr_backtransform.restype = ctypes.c_int
    lib.mrrr_backtransform.argtypes = [I64, I64, P, I64, P, P, I64, P]
    lib.mrrr_tridiagonalize.restype = ctypes.c_int
    lib.mrrr_tridiagonalize.argtypes = [I64, P, I64, P, P, P, P]
    lib.mrrr_cholesky.restype = ctypes.c_int
    lib.mrrr_cholesky.argtypes = [I64, P, I64, PI64, P]
    lib.mrrr_sygst.restype = ctypes.c_int
    lib.mrrr_sygst.argtypes = [I64, P, I64, P, I64, P]
    lib.mrrr_trsm_lt.restype = ctypes.c_int
    lib.mrrr_trsm_lt.argtypes = [I64, I64, P, I64, P, I64, P]
    lib.mrrr_syev.restype = ctypes.c_int
    lib.mrrr_syev.argtypes = [I64, P, I64, P, P, I64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_sygv.restype = ctypes.c_int
    lib.mrrr_sygv.argtypes = [I64, P, I64, P, I64, P, P, I64, PI64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_syevr.restype = ctypes.c_int
    lib.mrrr_syevr.argtypes = [I64, P, I64, MrrrRange, P, P, I64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_sygvr.restype = ctypes.c_int
    lib.mrrr_sygvr.argtypes = [I64, P, I64, P, I64, MrrrRange, P, P, I64, PI64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_probe_division.restype = ctypes.c_int
    lib.mrrr_probe_division.argtypes = [I64, P, P, P, P]
    lib.mrrr_get_limits.restype = ctypes.c_int
    lib.mrrr_get_limits.argtypes = [ctypes.POINTER(MrrrLimits)]
    lib.mrrr_set_limits.restype = ctypes.c_int
    lib.mrrr_set_limits.argtypes = [ctypes.POINTER(MrrrLimits)]
    lib.mrrr_step_batched.restype = ctypes.c_int
    lib.mrrr_step_batched.argtypes = [I64, PI64, PI64, P, P, P, P, PI64, ctypes.POINTER(MrrrInfo), P]
    lib.mrrr_step_backward.restype = ctypes.c_int
    lib.mrrr_step_backward.argtypes = [I64, P, P, I64, P, P, I64, P, P, P]
    lib.mrrr_step_backward_batched.restype = ctypes.c_int
    lib.mrrr_step_backward_batched.argtypes = [I64, PI64, PI64, PI64, P, P, P, P, P, P, P]
    lib.mrrr_autotune_batched.restype = ctypes.c_int
    lib.mrrr_autotune_batched.argtypes = [I64, PI64, PI64, P, P, P, P, PI64, ctypes.POINTER(MrrrTuning), P]
    lib.mrrr_get_tuning.restype = ctypes.c_int
    lib.mrrr_get_tuning.argtypes = [ctypes.POINTER(MrrrTuning)]
    lib.mrrr_set_tuning.restype = ctypes.c_int
    lib.mrrr_set_tuning.argtypes = [ctypes.POINTER(MrrrTuning)]
    lib.mrrr_profile_enable.restype = ctypes.c_int
    lib.mrrr_profile_enable.argtypes = [ctypes.c_int]
    lib.mrrr_profile_reset.restype = ctypes.c_int
    lib.mrrr_profile_reset.argtypes = []
    lib.mrrr_profile_read.restype = ctypes.c_int
    lib.mrrr_profile_read.argtypes = [ctypes.c_int, ctypes.POINTER(MrrrKernelTime)]
    lib.mrrr_release.restype = ctypes.c_int
    lib.mrrr_release.argtypes = []
    lib.mrrr_last_error.restype = ctypes.c_char_p
    lib.mrrr_last_error.argtypes = []
    lib.mrrr_status_string.restype = ctypes.c_char_p
    lib.mrrr_status_string.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def check(rc):
    if rc != 0:
        msg = load().mrrr_last_error().decode(errors="replace")
        raise MrrrError(rc, msg)
