"""ctypes declarations of librbc (include/rbc.h).  Argument marshalling only."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbc.so")

RBC_OK, RBC_EINVAL, RBC_ESCHEME, RBC_ENOMEM, RBC_EHIP, RBC_EUNSUPPORTED, RBC_EBUSY = range(7)
MODES = {"full": 0, "signs": 1, "perms": 2, "none": 3}
PRECS = {"f64": 0, "f32": 1, "bf16x3": 2, "f16s": 3, "fp8c": 4}

c_i64 = ctypes.c_int64
c_dbl_p = ctypes.POINTER(ctypes.c_double)
c_i32_p = ctypes.POINTER(ctypes.c_int32)
c_vp = ctypes.c_void_p


class PlanInfo(ctypes.Structure):
    _fields_ = [("M", c_i64), ("K", c_i64), ("N", c_i64),
                ("Mp", c_i64), ("Kp", c_i64), ("Np", c_i64),
                ("mM", c_i64), ("mK", c_i64), ("mN", c_i64),
                ("n_leaves", c_i64),
                ("levels", ctypes.c_int32), ("n_groups", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32), ("tile_k", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t),
                ("off_S", ctypes.c_size_t), ("off_T", ctypes.c_size_t), ("off_P", ctypes.c_size_t),
                ("bytes_S", ctypes.c_size_t), ("bytes_T", ctypes.c_size_t), ("bytes_P", ctypes.c_size_t),
                ("off_aux", ctypes.c_size_t), ("bytes_aux", ctypes.c_size_t),
                ("n_scatter_groups", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchOptions(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("grid", ctypes.c_int32), ("timeout_ms", ctypes.c_int32),
                ("trace", ctypes.c_int32), ("task_bytes", c_i64), ("item_budget", c_i64),
                ("mode", ctypes.c_int32), ("order", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_items", c_i64), ("n_tasks", c_i64), ("n_counters", c_i64),
                ("scale_tasks", c_i64), ("gather_tasks", c_i64), ("leaf_tasks", c_i64),
                ("scatter_tasks", c_i64), ("gate_tasks", c_i64), ("levels", c_i64), ("launches", c_i64),
                ("workspace_bytes", ctypes.c_size_t),
                ("control_bytes", ctypes.c_size_t), ("grid", ctypes.c_int32), ("prec", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchItem(ctypes.Structure):
    _fields_ = [("region_offset", ctypes.c_size_t), ("region_bytes", ctypes.c_size_t), ("first_task", c_i64),
                ("gate_counter", ctypes.c_int32), ("done_counter", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); every function of include/rbc.h
SIGNATURES = {
    "rbc_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "rbc_last_error": (ctypes.c_char_p, []),
    "rbc_abi_version": (ctypes.c_int, []),
    "rbc_scheme_create": (ctypes.c_int, [ctypes.c_int] * 4 + [c_dbl_p] * 3 + [ctypes.c_double,
                                                                              ctypes.POINTER(c_vp)]),
    "rbc_scheme_builtin": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(c_vp)]),
    "rbc_scheme_info": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_int)] + [c_dbl_p] * 4),
    "rbc_scheme_tensors": (ctypes.c_int, [c_vp] + [c_dbl_p] * 3),
    "rbc_scheme_destroy": (None, [c_vp]),
    "rbc_draw": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, c_i32_p, c_i32_p]),
    "rbc_fold": (ctypes.c_int, [c_vp, c_i32_p, c_i32_p, ctypes.c_int] + [c_dbl_p] * 3),
    "rbc_plan_create": (ctypes.c_int, [c_i64, c_i64, c_i64, ctypes.c_int, ctypes.POINTER(c_vp),
                                       ctypes.c_int, ctypes.c_int, ctypes.POINTER(c_vp)]),
    "rbc_plan_get_info": (ctypes.c_int, [c_vp, ctypes.POINTER(PlanInfo)]),
    "rbc_plan_traffic": (ctypes.c_int, [c_vp, c_dbl_p]),
    "rbc_plan_destroy": (None, [c_vp]),
    "rbc_matmul": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, ctypes.c_uint64,
                                  ctypes.c_int, ctypes.c_int, c_vp, ctypes.c_size_t, c_vp]),
    "rbc_matmul_noalloc": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, ctypes.c_uint64,
                                          ctypes.c_int, ctypes.c_int, c_vp]),
    "rbc_matmul_draws": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_i32_p, c_i32_p,
                                        ctypes.c_int, c_vp, ctypes.c_size_t, c_vp]),
    "rbc_average_workspace": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "rbc_matmul_average": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, ctypes.POINTER(ctypes.c_uint64),
                                          c_i64, ctypes.c_int, ctypes.c_int, c_vp, ctypes.c_size_t, c_vp]),
    "rbc_accumulate": (ctypes.c_int, [c_vp, c_vp, ctypes.c_int, c_i64, c_i64, c_i64, ctypes.c_int, c_vp]),
    "rbc_accumulate_weighted": (ctypes.c_int, [c_vp, c_vp, ctypes.c_int, c_i64, c_i64, c_i64, ctypes.c_double,
                                               ctypes.c_int, c_vp]),
    "rbc_apa_ebc_weights": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), c_i64,
                                           ctypes.POINTER(ctypes.c_double)]),
    "rbc_matmul_apa_ebc": (ctypes.c_int, [ctypes.POINTER(c_vp), ctypes.POINTER(ctypes.c_double), c_i64, c_vp, c_i64,
                                          c_vp, c_i64, c_vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, c_vp,
                                          ctypes.c_size_t, c_vp]),
    "rbc_scale_f64": (ctypes.c_int, [c_vp, c_i64, ctypes.c_double, c_vp]),
    "rbc_stage_gather": (ctypes.c_int, [c_vp, ctypes.c_int, c_vp, c_i64, c_i32_p, c_i32_p, c_vp,
                                        ctypes.c_size_t, c_vp]),
    "rbc_stage_leaf": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "rbc_stage_scatter": (ctypes.c_int, [c_vp, c_i32_p, c_i32_p, ctypes.c_int, c_vp, c_i64, c_vp,
                                         ctypes.c_size_t, c_vp]),
    "rbc_plan_set_timing": (ctypes.c_int, [c_vp, ctypes.c_int]),
    "rbc_plan_set_leaf_gather": (ctypes.c_int, [c_vp, ctypes.c_int]),
    "rbc_plan_set_fusion": (ctypes.c_int, [c_vp, ctypes.c_int]),
    "rbc_peak_copy": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "rbc_peak_mfma": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, c_vp, c_dbl_p, c_vp]),
    "rbc_plan_get_leaf_gather": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "rbc_plan_set_leaf_scatter": (ctypes.c_int, [c_vp, ctypes.c_int]),
    "rbc_plan_get_leaf_scatter": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "rbc_plan_timing_collect": (ctypes.c_int, [c_vp, c_dbl_p, ctypes.POINTER(c_i64)]),
    "rbc_batch_create": (ctypes.c_int, [ctypes.POINTER(BatchOptions), ctypes.POINTER(c_vp)]),
    "rbc_batch_add": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, ctypes.c_uint64,
                                     ctypes.c_int, ctypes.c_int, ctypes.POINTER(c_i64)]),
    "rbc_batch_workspace": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "rbc_batch_prepare": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "rbc_batch_launch": (ctypes.c_int, [c_vp, c_vp, ctypes.c_int]),
    "rbc_batch_check": (ctypes.c_int, [c_vp, c_vp]),
    "rbc_batch_get_info": (ctypes.c_int, [c_vp, ctypes.POINTER(BatchInfo)]),
    "rbc_batch_trace": (ctypes.c_int, [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64), c_dbl_p]),
    "rbc_batch_set_grid": (ctypes.c_int, [c_vp, ctypes.c_int]),
    "rbc_batch_get_item": (ctypes.c_int, [c_vp, c_i64, ctypes.POINTER(BatchItem)]),
    "rbc_batch_task_table": (ctypes.c_int, [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]),
    "rbc_batch_destroy": (None, [c_vp]),
}

_lib = None


class RbcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


STATUS_NAMES = {RBC_OK: "ok", RBC_EINVAL: "RBC_EINVAL", RBC_ESCHEME: "RBC_ESCHEME",
                RBC_ENOMEM: "RBC_ENOMEM", RBC_EHIP: "RBC_EHIP", RBC_EUNSUPPORTED: "RBC_EUNSUPPORTED",
                RBC_EBUSY: "RBC_EBUSY"}


def lib():
    """The loaded library.  Raises if it has not been built: there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librbc.so is not built (%s); run python -m paper_1905_07439_amd.build"
                              % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != RBC_OK:
        msg = lib().rbc_last_error()
        raise RbcError(status, msg.decode() if msg else "")
    return status
