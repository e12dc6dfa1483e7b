"""ctypes view of include/finger.h.  Loading fails loudly when libfinger.so
has not been built: there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfinger.so")

FINGER_OK = 0
FINGER_EINVAL = -1
FINGER_ENOMEM = -2
FINGER_EDEVICE = -3
FINGER_ENODEV = -4
FINGER_EOVERFLOW = -5
FINGER_EINTERNAL = -6
FINGER_ECORRUPT = -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENODEV",
                -5: "EOVERFLOW", -6: "EINTERNAL", -7: "ECORRUPT"}

L2, ANGULAR, IP = 0, 1, 2
ENTRY_PIVOT, ENTRY_DESCENT = -1, -2
CODE_F32, CODE_BF16, CODE_FP8E4M3 = 0, 1, 2
MODE_PLAIN, MODE_FINGER, MODE_GATED = 0, 1, 2
SIGMA_STD, SIGMA_VARIANCE = 0, 1
NCOUNTERS = 7
COUNTER_NAMES = ("expansions", "exact", "screened", "skipped", "visited", "preps", "status")

(T_P_F64, T_EIGVALS, T_P_F32, T_NODE_CC, T_NODE_PC, T_EDGE_ALPHA, T_EDGE_RHO,
 T_EDGE_CODES, T_EDGE_SCALE, T_SAMPLES, T_XY) = range(11)

EXPORTED = (
    "finger_build_params_init", "finger_build_tables", "finger_free_tables",
    "finger_tables_info_get", "finger_tables_read", "finger_search_params_init",
    "finger_search_workspace_size", "finger_search", "finger_estimate_edges",
    "finger_exact_knn_workspace_size", "finger_exact_knn", "finger_gate_attach",
    "finger_gate_param_count", "finger_mlp_forward", "finger_mlp_backward",
    "finger_adam_step", "finger_gate_targets", "finger_last_error",
    "finger_hierarchy_attach", "finger_descend", "finger_build_graph",
    "finger_mlp_backward_workspace_size", "finger_gate_calibrate", "finger_tables_export",
    "finger_tables_import", "finger_checksum64", "finger_search_noalloc",
    "finger_search_noalloc_capacity", "finger_build_graph_grouped",
)


class BuildParams(C.Structure):
    _fields_ = [
        ("rank", C.c_int32), ("code_type", C.c_int32), ("metric", C.c_int32),
        ("sigma_mode", C.c_int32), ("n_samples", C.c_int64), ("seed", C.c_uint64),
        ("pivots", C.c_void_p), ("n_pivots", C.c_int32), ("dm_override", C.c_int32),
        ("dm", C.c_double * 5), ("basis", C.c_void_p),
    ]


class SearchParams(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("k", C.c_int32), ("ef", C.c_int32), ("entry", C.c_int32),
        ("warmup", C.c_int32), ("k_max", C.c_int32),
        ("k_per_query", C.c_void_p), ("ef_per_query", C.c_void_p),
        ("ef_max", C.c_int32), ("persistent", C.c_int32), ("waves_per_cu", C.c_int32),
        ("visited_capacity", C.c_int32), ("spill_capacity", C.c_int32), ("visited_probe", C.c_int32),
        ("code_prefetch", C.c_int32), ("ef_classes", C.c_int32), ("gate_band", C.c_float),
        ("screen_layout", C.c_int32),
        ("log_features", C.c_void_p), ("log_targets", C.c_void_p),
        ("log_capacity", C.c_int64), ("log_count", C.c_void_p),
        ("kernel_events", C.c_void_p * 2),
    ]


class TablesInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("m", C.c_int32), ("rank", C.c_int32), ("max_degree", C.c_int32),
        ("code_type", C.c_int32), ("metric", C.c_int32), ("n_pivots", C.c_int32),
        ("n_samples_used", C.c_int64), ("mu", C.c_double), ("sigma", C.c_double),
        ("mu_hat", C.c_double), ("sigma_hat", C.c_double), ("eps", C.c_double),
        ("eps_gate", C.c_double), ("gate_attached", C.c_int32),
        ("edge_table_bytes", C.c_int64), ("corr_xy", C.c_double),
        ("hierarchy_top_level", C.c_int32), ("hierarchy_top", C.c_int32),
        ("hierarchy_rows", C.c_int64),
    ]


PROGRESS_FN = C.CFUNCTYPE(None, C.c_char_p, C.c_int64, C.c_int64, C.c_void_p)


class GraphStats(C.Structure):
    _fields_ = [
        ("sym_edges", C.c_int64), ("sym_degree_max", C.c_int32),
        ("components_before_repair", C.c_int32), ("edges_added", C.c_int64),
        ("ms_knn", C.c_double), ("ms_symmetrize", C.c_double), ("ms_prune", C.c_double),
        ("ms_repair", C.c_double),
    ]


_lib = None


def load() -> C.CDLL:
    """Load libfinger.so (built by ``python -m paper_2206_11408_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2206_11408_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    P = C.POINTER
    lib.finger_last_error.restype = C.c_char_p
    lib.finger_last_error.argtypes = []
    lib.finger_build_params_init.restype = None
    lib.finger_build_params_init.argtypes = [P(BuildParams)]
    lib.finger_search_params_init.restype = None
    lib.finger_search_params_init.argtypes = [P(SearchParams)]
    lib.finger_build_tables.restype = C.c_int
    lib.finger_build_tables.argtypes = [vp, i64, i32, vp, i32, P(BuildParams), P(vp), vp]
    lib.finger_free_tables.restype = None
    lib.finger_free_tables.argtypes = [vp]
    lib.finger_tables_info_get.restype = C.c_int
    lib.finger_tables_info_get.argtypes = [vp, P(TablesInfo)]
    lib.finger_tables_read.restype = C.c_int
    lib.finger_tables_read.argtypes = [vp, i32, vp, P(sz)]
    lib.finger_search_workspace_size.restype = C.c_int
    lib.finger_search_workspace_size.argtypes = [vp, i64, P(SearchParams), P(sz)]
    lib.finger_search.restype = C.c_int
    lib.finger_search.argtypes = [vp, vp, i64, P(SearchParams), vp, vp, vp, vp, sz, vp]
    lib.finger_estimate_edges.restype = C.c_int
    lib.finger_estimate_edges.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
    lib.finger_exact_knn_workspace_size.restype = C.c_int
    lib.finger_exact_knn_workspace_size.argtypes = [i64, i32, i64, i32, P(sz)]
    lib.finger_exact_knn.restype = C.c_int
    lib.finger_exact_knn.argtypes = [vp, i64, i32, vp, i64, i32, i32, vp, vp, vp, sz, vp]
    lib.finger_gate_attach.restype = C.c_int
    lib.finger_gate_attach.argtypes = [vp, vp, i32, i32, C.c_double]
    lib.finger_gate_param_count.restype = i64
    lib.finger_gate_param_count.argtypes = [i32, i32]
    lib.finger_mlp_forward.restype = C.c_int
    lib.finger_mlp_forward.argtypes = [vp, i32, i32, vp, i64, vp, vp]
    lib.finger_mlp_backward.restype = C.c_int
    lib.finger_mlp_backward.argtypes = [vp, i32, i32, vp, vp, i64, vp, vp, vp, sz, vp]
    lib.finger_mlp_backward_workspace_size.restype = C.c_int
    lib.finger_mlp_backward_workspace_size.argtypes = [i32, i32, i64, P(sz)]
    lib.finger_gate_calibrate.restype = C.c_int
    lib.finger_gate_calibrate.argtypes = [vp, i32, i32, vp, vp, i64, P(C.c_double), vp]
    lib.finger_tables_export.restype = C.c_int
    lib.finger_tables_export.argtypes = [vp, vp, P(sz)]
    lib.finger_tables_import.restype = C.c_int
    lib.finger_tables_import.argtypes = [vp, sz, vp, i64, i32, vp, i32, P(vp), vp]
    lib.finger_search_noalloc.restype = C.c_int
    lib.finger_search_noalloc.argtypes = [vp, vp, i64, P(SearchParams), vp, vp, vp, vp]
    lib.finger_search_noalloc_capacity.restype = sz
    lib.finger_search_noalloc_capacity.argtypes = []
    lib.finger_checksum64.restype = C.c_uint64
    lib.finger_checksum64.argtypes = [vp, sz]
    lib.finger_adam_step.restype = C.c_int
    lib.finger_adam_step.argtypes = [vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float,
                                     C.c_float, i32, vp]
    lib.finger_build_graph.restype = C.c_int
    lib.finger_build_graph.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, P(GraphStats),
                                       PROGRESS_FN, vp, vp]
    lib.finger_build_graph_grouped.restype = C.c_int
    lib.finger_build_graph_grouped.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, i64, vp,
                                               P(GraphStats), PROGRESS_FN, vp, vp]
    lib.finger_hierarchy_attach.restype = C.c_int
    lib.finger_hierarchy_attach.argtypes = [vp, vp, vp, i64, i32]
    lib.finger_descend.restype = C.c_int
    lib.finger_descend.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.finger_gate_targets.restype = C.c_int
    lib.finger_gate_targets.argtypes = [vp, vp, i64, i32, vp, vp]
    _lib = lib
    return lib


class FingerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int) -> None:
    if status != FINGER_OK:
        raise FingerError(status, load().finger_last_error().decode())
