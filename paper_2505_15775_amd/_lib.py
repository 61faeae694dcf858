"""ctypes mirror of include/alm_bm.h and the loader of libalmbm.so.

Argument marshalling only: every computation runs in the HIP library.  If the
library is missing or fails to load, importing this module raises; there is no
CPU fallback.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libalmbm.so")

OK = 0
NOT_CONVERGED = 1
STATUS_NAMES = {
    0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID_ARG", -2: "ERR_INVALID_PATTERN", -3: "ERR_HIP",
    -4: "ERR_OOM", -5: "ERR_NUMERIC", -6: "ERR_UNSUPPORTED",
}
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2}
CONS_DIAG = 0
CONS_TRACE_EDGES = 1
STEP_EXACT, STEP_FIXED = 0, 1
INNER_GD, INNER_LBFGS = 0, 1
RANK_ADAPT, RANK_FIXED = 0, 1


class AlmBmError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Desc(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("val", C.c_void_p),
        ("ell_width", C.c_int32),
        ("diag", C.c_void_p),
        ("j_coef", C.c_double),
        ("cons_kind", C.c_int32),
        ("m", C.c_int64),
        ("b", C.c_void_p),
        ("trace_coef", C.c_double),
        ("n_edges", C.c_int64),
        ("edge_i", C.c_void_p),
        ("edge_j", C.c_void_p),
        ("precision", C.c_int32),
        ("r_max", C.c_int32),
        ("lanczos_kmax", C.c_int32),
        ("validate", C.c_int32),
        ("rank_block_max", C.c_int32),
        ("lbfgs_memory_max", C.c_int32),
        ("hub_min_degree", C.c_int32),
    ]


class Options(C.Structure):
    _fields_ = [
        ("eps_kkt", C.c_double),
        ("sigma", C.c_double),
        ("max_outer", C.c_int32),
        ("max_inner", C.c_int32),
        ("step_rule", C.c_int32),
        ("eta_fixed", C.c_double),
        ("rank_policy", C.c_int32),
        ("r_cap", C.c_int32),
        ("tau_rank", C.c_double),
        ("expand_needs_inner", C.c_int32),
        ("inner_tol_scale", C.c_double),
        ("inner_tol_decay", C.c_double),
        ("lanczos_kmax", C.c_int32),
        ("lanczos_tol_rel", C.c_double),
        ("seed", C.c_uint64),
        ("graph_unroll", C.c_int32),
        ("verbose", C.c_int32),
        ("time_limit_s", C.c_double),
        ("bf16_promote", C.c_int32),
        ("refresh_every", C.c_int32),
        ("lanczos_restarts", C.c_int32),
        ("sigma_edges", C.c_double),
        ("sigma_growth", C.c_double),
        ("sigma_max", C.c_double),
        ("pinf_reduction", C.c_double),
        ("rank_block", C.c_int32),
        ("resume_outer", C.c_int32),
        ("resume_inner_tol", C.c_double),
        ("resume_pinf", C.c_double),
        ("inner_solver", C.c_int32),
        ("lbfgs_memory", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [
        ("outer", C.c_int32),
        ("inner_total", C.c_int64),
        ("rank", C.c_int32),
        ("expansions", C.c_int32),
        ("pobj", C.c_double),
        ("dobj", C.c_double),
        ("pinf", C.c_double),
        ("dinf", C.c_double),
        ("gap", C.c_double),
        ("kkt", C.c_double),
        ("lam_min", C.c_double),
        ("time_s", C.c_double),
        ("time_lanczos_s", C.c_double),
        ("promoted_at_outer", C.c_int32),
        ("time_promoted_s", C.c_double),
        ("sigma_final", C.c_double),
        ("sigma_increases", C.c_int32),
        ("inner_tol", C.c_double),
        ("lanczos_resid", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "alm_bm_create", "alm_bm_destroy", "alm_bm_objective_grad", "alm_bm_cost_apply", "alm_bm_line_search",
    "alm_bm_dual_update", "alm_bm_lanczos_min_eig", "alm_bm_solve", "alm_bm_kkt", "alm_bm_default_options", "alm_bm_last_error",
    "alm_bm_maxcut_cost_host", "alm_bm_abi_sizes", "alm_bm_gd_step", "alm_bm_set_tiles", "alm_bm_set_hub_threshold", "alm_bm_psd_step",
    "alm_bm_autotune",
    "alm_bm_inner_solve", "alm_bm_ws_features", "alm_bm_ws_pool", "alm_bm_ws_param_count", "alm_bm_ws_work_size",
    "alm_bm_ws_forward", "alm_bm_ws_loss_grad", "alm_bm_ws_adam", "alm_bm_ws_ridge_fit",
    "alm_bm_batch_create", "alm_bm_batch_destroy", "alm_bm_batch_offsets", "alm_bm_batch_solve",
    "alm_bm_batch_autotune", "alm_bm_lanczos_block", "alm_bm_ladder_factor",
    "alm_bm_objective_grad_noalloc", "alm_bm_block_moments", "alm_bm_gather_probe", "alm_bm_gather_probe_out_size",
]

vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
f64 = C.c_double


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libalmbm.so not built ({LIB_PATH}); run __graft_entry__.build() or "
                          "python paper_2505_15775_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "alm_bm_create": (i32, [C.POINTER(Desc), vp, C.POINTER(vp)]),
        "alm_bm_destroy": (i32, [vp]),
        "alm_bm_objective_grad": (i32, [vp, i32, vp, vp, f64, vp, vp, vp, vp]),
        "alm_bm_objective_grad_noalloc": (i32, [C.POINTER(Desc), i32, vp, vp, f64, vp, vp, vp, vp]),
        "alm_bm_cost_apply": (i32, [vp, i32, vp, vp, vp, vp]),
        "alm_bm_line_search": (i32, [vp, i32, vp, vp, vp, f64, vp, vp, vp]),
        "alm_bm_dual_update": (i32, [vp, vp, f64, vp, vp, vp]),
        "alm_bm_gd_step": (i32, [vp, i32, vp, vp, f64, vp, vp, vp, vp]),
        "alm_bm_lanczos_min_eig": (i32, [vp, vp, i32, f64, C.c_uint64, vp, vp, vp, vp, vp]),
        "alm_bm_solve": (i32, [vp, C.POINTER(Options), vp, C.POINTER(i32), vp, C.POINTER(Result), vp]),
        "alm_bm_kkt": (i32, [vp, i32, vp, vp, f64, vp, vp]),
        "alm_bm_default_options": (None, [C.POINTER(Options)]),
        "alm_bm_last_error": (C.c_char_p, []),
        "alm_bm_maxcut_cost_host": (i32, [i64, i64, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i64)]),
        "alm_bm_abi_sizes": (None, [C.POINTER(i64)]),
        "alm_bm_set_tiles": (i32, [vp, i32, i32]),
        "alm_bm_set_hub_threshold": (i32, [vp, i32, vp]),
        "alm_bm_psd_step": (i32, [i32, vp, vp, C.c_double, vp]),
        "alm_bm_block_moments": (i32, [vp, i32, vp, f64, vp, vp]),
        "alm_bm_gather_probe": (i32, [vp, i64, i32, vp, i64, vp, vp]),
        "alm_bm_gather_probe_out_size": (i64, []),
        "alm_bm_ws_features": (i32, [vp, vp, vp, vp]),
        "alm_bm_ws_pool": (i32, [vp, i64, vp, vp, vp]),
        "alm_bm_ws_param_count": (i64, [i32, i32]),
        "alm_bm_ws_work_size": (i64, [i32, i32, i32]),
        "alm_bm_ws_forward": (i32, [vp, i32, i32, vp, vp, i64, vp, vp, vp]),
        "alm_bm_ws_loss_grad": (i32, [vp, i32, i32, vp, vp, i64, vp, vp, vp, vp, vp, i32, vp]),
        "alm_bm_ws_adam": (i32, [vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp]),
        "alm_bm_ws_ridge_fit": (i32, [vp, vp, i32, i32, f64, vp]),
        "alm_bm_batch_create": (i32, [i32, vp, i32, vp, C.POINTER(vp)]),
        "alm_bm_batch_destroy": (i32, [vp]),
        "alm_bm_batch_offsets": (i32, [vp, vp]),
        "alm_bm_batch_solve": (i32, [vp, C.POINTER(Options), vp, vp, vp, vp, vp, vp]),
        "alm_bm_batch_autotune": (i32, [vp, i32, vp, vp, C.POINTER(i32), vp]),
        "alm_bm_lanczos_block": (i32, [vp, vp, i32, i32, C.c_uint64, vp, vp, vp, C.POINTER(i32), vp]),
        "alm_bm_ladder_factor": (i32, [vp, i32, vp, vp]),
        "alm_bm_inner_solve": (i32, [vp, C.POINTER(Options), i32, vp, vp, f64, i32, C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(f64), vp]),
        "alm_bm_autotune": (i32, [vp, i32, i32, C.POINTER(i32), C.POINTER(i32), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    sizes = (i64 * 3)()
    lib.alm_bm_abi_sizes(sizes)
    mine = (C.sizeof(Desc), C.sizeof(Options), C.sizeof(Result))
    if tuple(sizes) != mine:
        raise ImportError(f"ABI mismatch between alm_bm.h {tuple(sizes)} and the Python mirror {mine}")
    return lib


lib = _load()


def check(status, where):
    if status < 0:
        msg = lib.alm_bm_last_error()
        raise AlmBmError(status, where, msg.decode() if msg else "")
    return status


def default_options():
    o = Options()
    lib.alm_bm_default_options(C.byref(o))
    return o
