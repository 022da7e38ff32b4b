"""ctypes declarations of libbhx (include/bhx.h). Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# BHX_LIBRARY=checked loads libbhx_checked.so, the build with device-side
# invariant checks (failures reported as BH_E_CHECK)
LIB_PATH = os.path.join(HERE, "libbhx_checked.so" if os.environ.get("BHX_LIBRARY") == "checked"
                        else "libbhx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bhx.h")

(BH_OK, BH_E_INVALID, BH_E_NONFINITE, BH_E_CAPACITY, BH_E_OOM, BH_E_HIP, BH_E_STACK, BH_E_STATE,
 BH_E_CHECK) = range(9)
STATUS_NAMES = ["BH_OK", "BH_E_INVALID", "BH_E_NONFINITE", "BH_E_CAPACITY", "BH_E_OOM",
                "BH_E_HIP", "BH_E_STACK", "BH_E_STATE", "BH_E_CHECK"]
BH_FP64, BH_FP32C = 0, 1
BH_FLAG_COUNTS = 1
BH_FLAG_TIMING = 2
BH_FLAG_ADJOINT = 4
BH_FLAG_GRAPH = 8
BH_FLAG_QUAD = 16
BH_FLAG_MARKERS = 32


class bh_config(C.Structure):
    _fields_ = [("n_max", C.c_int64), ("leaf_size", C.c_int32), ("precision", C.c_int32),
                ("G", C.c_double), ("flags", C.c_uint32), ("walk_group", C.c_int32),
                ("max_scenes", C.c_int32)]


class bh_tree_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnodes", C.c_int64), ("depth", C.c_int32),
                ("pad", C.c_int32), ("info", C.c_void_p), ("mom", C.c_void_p),
                ("eps2", C.c_void_p), ("order", C.c_void_p), ("keys", C.c_void_p),
                ("box", C.c_double * 8), ("quad", C.c_void_p)]


class bh_stats_t(C.Structure):
    _fields_ = [("nnodes", C.c_int64), ("depth", C.c_int32), ("bucket_sort", C.c_int32),
                ("total_nodes_accepted", C.c_int64), ("total_leaf_pairs", C.c_int64),
                ("timed_evals", C.c_int64), ("build_ms", C.c_double), ("walk_ms", C.c_double)]


class bh_tune_result(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("walk_group", C.c_int32), ("ms_per_step", C.c_double)]


P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
SIGNATURES = {
    "bh_create": ([C.POINTER(bh_config), P, C.POINTER(P)], C.c_int),
    "bh_destroy": ([P], None),
    "bh_set_stream": ([P, P], C.c_int),
    "bh_sync": ([P], C.c_int),
    "bh_last_error": ([P], C.c_char_p),
    "bh_build_tree": ([P, P, P, P, I64], C.c_int),
    "bh_compute_accel": ([P, P, P, D, P, D, P, P, I64], C.c_int),
    "bh_compute_accel_direct": ([P, P, P, D, P, P, P, I64], C.c_int),
    "bh_step_leapfrog": ([P, P, P, P, D, P, D, D, I32, P, I64], C.c_int),
    "bh_step_euler": ([P, P, P, P, D, P, D, D, I32, I32, P, I64], C.c_int),
    "bh_contact_components": ([P, P, P, P, D, P, C.POINTER(I64), C.POINTER(I64), I64], C.c_int),
    "bh_walk_counts": ([P, P, I64], C.c_int),
    "bh_tree_export": ([P, C.POINTER(bh_tree_view)], C.c_int),
    "bh_stats": ([P, C.POINTER(bh_stats_t)], C.c_int),
    "bh_diagnostics": ([P, P, P, P, D, P, P, I64], C.c_int),
    "bh_gravity_dt_bound": ([P, P, P, I64, C.POINTER(D)], C.c_int),
    "bh_timing_reset": ([P], C.c_int),
    "bh_accel_vjp": ([P, P, P, D, P, D, P, P, P, I64], C.c_int),
    "bh_batched_accel": ([P, I32, P, P, P, D, P, D, P, P], C.c_int),
    "bh_autotune": ([C.POINTER(bh_config), P, I32, P, P, P, P, D, P, D, D, I32,
                     C.POINTER(bh_tune_result)], C.c_int),
    "bh_batched_step": ([P, I32, P, P, P, P, D, P, D, D, I32, P], C.c_int),
    "bh_leapfrog_vjp": ([P, P, P, P, P, D, P, D, D, I32, P, P, P, P, P, I64], C.c_int),
    "bh_leapfrog_vjp_stored": ([P, P, P, D, P, D, D, I32, P, P, P, P, I64], C.c_int),
    "bh_probe_fma": ([P, I32, I64, C.POINTER(D)], C.c_int),
    "bh_compute_accel_direct_noalloc": ([P, I32, D, P, P, D, P, P, P, I64], C.c_int),
}

_lib = None


class ExtensionMissing(RuntimeError):
    pass


def header_symbols(path: str = HEADER) -> list[str]:
    """Names of the functions include/bhx.h declares."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z_]+)\s*\(", text)))


def load():
    """Loads libbhx.so; raises ExtensionMissing when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ExtensionMissing(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1912_04197_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib
