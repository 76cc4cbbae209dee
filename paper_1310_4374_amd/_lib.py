"""ctypes binding of libperiodic_sum.so (include/periodic_sum.h).

Argument marshalling only: every step of the method runs in the HIP library.
Importing this module on a machine without the built library raises at once;
there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libperiodic_sum.so")

(PS_OK, PS_E_INVALID, PS_E_NOT_NEUTRAL, PS_E_OUT_OF_BOX, PS_E_RANK, PS_E_NOMEM, PS_E_HIP, PS_E_UNSUPPORTED,
 PS_E_IO) = range(9)
PS_FP64, PS_FP32_ACC64 = 0, 1
PS_MEAN_ZERO, PS_MEAN_NONE = 0, 1
PS_BASIS_SPHERICAL, PS_BASIS_RBF = 0, 1

STATUS_NAMES = {0: "PS_OK", 1: "PS_E_INVALID", 2: "PS_E_NOT_NEUTRAL", 3: "PS_E_OUT_OF_BOX", 4: "PS_E_RANK",
                5: "PS_E_NOMEM", 6: "PS_E_HIP", 7: "PS_E_UNSUPPORTED", 8: "PS_E_IO"}

EXPORTS = ["periodic_sum_plan", "periodic_sum_eval", "periodic_sum_energy", "periodic_sum_energy_vjp",
           "periodic_sum_plan_batched", "periodic_sum_eval_batched", "periodic_sum_status", "periodic_sum_plan_info",
           "periodic_sum_plan_tables", "periodic_sum_last_coefficients", "periodic_sum_set_profiling",
           "periodic_sum_stage_times", "periodic_sum_autotune", "periodic_sum_near_counts", "periodic_sum_destroy",
           "periodic_sum_last_error", "periodic_sum_plan_save", "periodic_sum_plan_load", "periodic_sum_select",
           "periodic_sum_forward_epoch", "periodic_sum_eval_noalloc"]
STAGES = ["sort", "near", "bounds", "check", "solve", "mean", "pairs", "far"]


class ps_params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("p", ctypes.c_int32), ("R_b", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("precision", ctypes.c_int32), ("mean", ctypes.c_int32),
                ("rcond", ctypes.c_double), ("n_max", ctypes.c_int64), ("m_max", ctypes.c_int64),
                ("tile_targets", ctypes.c_int32), ("n_split", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("n_centres", ctypes.c_int32), ("centres", ctypes.POINTER(ctypes.c_double)),
                ("n_check", ctypes.c_int32), ("check_points", ctypes.POINTER(ctypes.c_double)),
                ("periodic", ctypes.c_int32), ("kernel", ctypes.c_int32), ("kappa", ctypes.c_double),
                ("dim", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ps_plan_info(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("P", ctypes.c_int32), ("L", ctypes.c_int32), ("n_images", ctypes.c_int32),
                ("rank", ctypes.c_int32), ("R0", ctypes.c_double), ("R_b", ctypes.c_double), ("cond", ctypes.c_double),
                ("n_near_last", ctypes.c_int64), ("tile_targets", ctypes.c_int32), ("n_split", ctypes.c_int32),
                ("nsys", ctypes.c_int32), ("mean_corners", ctypes.c_int32), ("profiled_evals", ctypes.c_int64),
                ("forward_epoch", ctypes.c_int64), ("periodic", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("kernel", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("tune_ms", ctypes.c_double), ("tune_second_ms", ctypes.c_double)]


class ps_select_row(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("p", ctypes.c_int32), ("n_solves", ctypes.c_int32),
                ("B_P", ctypes.c_double), ("err", ctypes.c_double), ("err_prec", ctypes.c_double),
                ("ms", ctypes.c_double), ("set_s", ctypes.c_double)]


class PeriodicSumError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """Load the library (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("libperiodic_sum.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_1310_4374_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        st = ctypes.c_int
        L.periodic_sum_plan.argtypes = [ctypes.POINTER(ps_params), ctypes.c_int, ctypes.POINTER(vp)]
        L.periodic_sum_plan.restype = st
        L.periodic_sum_plan_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(ps_params), ctypes.c_int, ctypes.POINTER(vp)]
        L.periodic_sum_plan_batched.restype = st
        L.periodic_sum_eval.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.periodic_sum_eval.restype = st
        L.periodic_sum_eval_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.periodic_sum_eval_noalloc.restype = st
        L.periodic_sum_energy.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.periodic_sum_energy.restype = st
        L.periodic_sum_energy_vjp.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32, i64, vp]
        L.periodic_sum_energy_vjp.restype = st
        L.periodic_sum_eval_batched.argtypes = [vp, ctypes.POINTER(i64), vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.periodic_sum_eval_batched.restype = st
        L.periodic_sum_status.argtypes = [vp, vp]
        L.periodic_sum_status.restype = st
        L.periodic_sum_plan_info.argtypes = [vp, ctypes.POINTER(ps_plan_info)]
        L.periodic_sum_plan_info.restype = st
        dp = ctypes.POINTER(ctypes.c_double)
        L.periodic_sum_plan_tables.argtypes = [vp, dp, dp, dp, dp]
        L.periodic_sum_plan_tables.restype = st
        L.periodic_sum_last_coefficients.argtypes = [vp, dp]
        L.periodic_sum_last_coefficients.restype = st
        L.periodic_sum_set_profiling.argtypes = [vp, ctypes.c_int32]
        L.periodic_sum_set_profiling.restype = st
        L.periodic_sum_stage_times.argtypes = [vp, dp, ctypes.c_int32]
        L.periodic_sum_stage_times.restype = st
        L.periodic_sum_autotune.argtypes = [vp, ctypes.POINTER(i64), vp, vp, vp, vp, vp, vp, vp, vp, dp, vp]
        L.periodic_sum_autotune.restype = st
        L.periodic_sum_near_counts.argtypes = [vp, ctypes.POINTER(i64), ctypes.c_int32]
        L.periodic_sum_near_counts.restype = st
        L.periodic_sum_destroy.argtypes = [vp]
        L.periodic_sum_destroy.restype = None
        L.periodic_sum_plan_save.argtypes = [vp, ctypes.c_char_p]
        L.periodic_sum_plan_save.restype = st
        L.periodic_sum_plan_load.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(vp)]
        L.periodic_sum_plan_load.restype = st
        L.periodic_sum_select.argtypes = [ctypes.POINTER(ps_params), ctypes.c_int, i64, vp, vp, vp, vp, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ps_select_row), ctypes.POINTER(ctypes.c_int32), vp]
        L.periodic_sum_select.restype = st
        L.periodic_sum_forward_epoch.argtypes = [vp, ctypes.POINTER(i64)]
        L.periodic_sum_forward_epoch.restype = st
        L.periodic_sum_last_error.argtypes = []
        L.periodic_sum_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status):
    if status != PS_OK:
        raise PeriodicSumError(status, lib().periodic_sum_last_error().decode())
