"""ctypes declarations of the C-ABI in include/psdp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsdp.so")

PSDP_OK = 0
PSDP_NOT_CONVERGED = 1
PSDP_FELL_BACK_FULL_EIG = 2
PSDP_PENDING = 3
PSDP_ERR_INVALID_ARG = -1
PSDP_ERR_HIP = -2
PSDP_ERR_OUT_OF_MEMORY = -3
PSDP_ERR_NUMERICAL = -4
PSDP_ERR_CAPACITY = -5

SIDE_AUTO, SIDE_POS, SIDE_NEG, SIDE_FULL = 0, 1, 2, 3
METHOD_LOBPCG, METHOD_BLOCK_KRYLOV, METHOD_TOP_R, METHOD_CHEBYSHEV = 0, 1, 2, 3
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2

# every symbol include/psdp.h declares
EXPORTED = [
    "psdp_default_options", "psdp_create", "psdp_destroy", "psdp_set_stream",
    "psdp_workspace_bytes", "psdp_project", "psdp_project_batched",
    "psdp_full_eig_project", "psdp_status_str", "psdp_profile_enable",
    "psdp_profile_get", "psdp_version", "psdp_block_product", "psdp_batched_tuning",
    "psdp_server_default_config", "psdp_server_create", "psdp_server_destroy",
    "psdp_server_open_session", "psdp_server_close_session", "psdp_server_submit",
    "psdp_server_wait", "psdp_server_drain", "psdp_server_session_block",
    "psdp_server_stats_get", "psdp_server_stats_reset", "psdp_full_eig_project_batched",
    "psdp_profile_filter", "psdp_certify_tail", "psdp_block_product_noalloc",
    "psdp_admm_default_options", "psdp_admm_solve", "psdp_transfer_stats",
]

ADMM_SOLVED, ADMM_MAX_ITER, ADMM_PRIMAL_INFEASIBLE, ADMM_DUAL_INFEASIBLE = 0, 1, 2, 3


class Options(ctypes.Structure):
    _fields_ = [
        ("side", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("refine_fp64", ctypes.c_int),
        ("ladder", ctypes.c_int),
        ("certify", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("side_threshold", ctypes.c_double),
        ("expand_cols", ctypes.c_int),
        ("pos_hint", ctypes.c_int),
        ("fallback_full", ctypes.c_int),
        ("block_guard", ctypes.c_int),
        ("batch_variant", ctypes.c_int),
        ("batch_graph", ctypes.c_int),
        ("bound_rel_max", ctypes.c_double),
        ("certify_delta", ctypes.c_double),
        ("warm_side", ctypes.c_int),
        ("method", ctypes.c_int),
        ("method_param", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("err_bound", ctypes.c_double),
        ("res_fro", ctypes.c_double),
        ("tail_est", ctypes.c_double),
        ("pi_fro", ctypes.c_double),
        ("theta_guard", ctypes.c_double),
        ("tol_used", ctypes.c_double),
        ("n_pos", ctypes.c_int),
        ("m_out", ctypes.c_int),
        ("iters", ctypes.c_int),
        ("side_used", ctypes.c_int),
        ("certified", ctypes.c_int),
        ("status", ctypes.c_int),
        ("expansions", ctypes.c_int),
        ("prec_final", ctypes.c_int),
        ("n_pos_full", ctypes.c_int),
        ("pos_est", ctypes.c_int),
        ("block_side", ctypes.c_int),
        ("cert_delta", ctypes.c_double),
        ("cert_eta", ctypes.c_double),
        ("trunc_bound", ctypes.c_double),
        ("spec_lower", ctypes.c_double),
        ("products", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Sdp(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("p", ctypes.c_int),
        ("C", ctypes.c_void_p),
        ("ldc", ctypes.c_int),
        ("nnz", ctypes.c_int),
        ("con", ctypes.POINTER(ctypes.c_int)),
        ("row", ctypes.POINTER(ctypes.c_int)),
        ("col", ctypes.POINTER(ctypes.c_int)),
        ("val", ctypes.POINTER(ctypes.c_double)),
        ("b", ctypes.POINTER(ctypes.c_double)),
    ]


class AdmmOptions(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("eps_abs", ctypes.c_double),
        ("eps_rel", ctypes.c_double),
        ("eps_inf", ctypes.c_double),
        ("exact", ctypes.c_int),
        ("tol_scale", ctypes.c_double),
        ("tol_power", ctypes.c_double),
        ("prec", ctypes.c_int),
        ("m_cap", ctypes.c_int),
        ("method", ctypes.c_int),
    ]


class AdmmInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("iters", ctypes.c_int),
        ("obj", ctypes.c_double),
        ("r_prim", ctypes.c_double),
        ("r_dual", ctypes.c_double),
        ("proj_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("proj_block", ctypes.c_int),
        ("proj_full", ctypes.c_int),
        ("proj_not_certified", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int),
        ("hbm_budget", ctypes.c_size_t),
        ("batch_lane", ctypes.c_int),
        ("small_n", ctypes.c_int),
        ("max_batch", ctypes.c_int),
        ("opt", Options),
    ]


class ServerResult(ctypes.Structure):
    _fields_ = [
        ("info", Info),
        ("ticket", ctypes.c_longlong),
        ("session", ctypes.c_int),
        ("lane", ctypes.c_int),
        ("batch_size", ctypes.c_int),
        ("queue_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_longlong),
        ("completed", ctypes.c_longlong),
        ("rejected", ctypes.c_longlong),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double),
        ("throughput", ctypes.c_double),
        ("hbm_held", ctypes.c_size_t),
        ("hbm_peak", ctypes.c_size_t),
        ("active", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("max_active", ctypes.c_int),
        ("batched_launches", ctypes.c_longlong),
        ("batched_requests", ctypes.c_longlong),
        ("lane_fallbacks", ctypes.c_longlong),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load libpsdp.so (built in-tree by paper_1912_02767_amd/build.py).

    Raises LibraryMissing when it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} not found: build it with `python -m paper_1912_02767_amd.build` "
            "(hipcc --offload-arch=gfx950); the projection has no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    lib.psdp_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.psdp_default_options.restype = None
    lib.psdp_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.psdp_create.restype = ctypes.c_int
    lib.psdp_destroy.argtypes = [vp]
    lib.psdp_destroy.restype = ctypes.c_int
    lib.psdp_set_stream.argtypes = [vp, vp]
    lib.psdp_set_stream.restype = ctypes.c_int
    lib.psdp_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_size_t)]
    lib.psdp_workspace_bytes.restype = ctypes.c_int
    lib.psdp_project.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int,
                                 ctypes.c_int, ip, vp, vp, ctypes.c_int,
                                 ctypes.POINTER(Options), ctypes.POINTER(Info)]
    lib.psdp_project.restype = ctypes.c_int
    lib.psdp_project_batched.argtypes = [vp, ctypes.c_int, ip, ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ip, ip, ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(Options),
                                         ctypes.POINTER(Info)]
    lib.psdp_project_batched.restype = ctypes.c_int
    lib.psdp_full_eig_project_batched.argtypes = [vp, ctypes.c_int, ip, ctypes.POINTER(vp),
                                                  ctypes.POINTER(vp), ip, ip, ctypes.POINTER(vp),
                                                  ctypes.POINTER(vp), ctypes.POINTER(Info)]
    lib.psdp_full_eig_project.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, vp,
                                          ctypes.c_int]
    lib.psdp_full_eig_project.restype = ctypes.c_int
    lib.psdp_block_product.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]
    lib.psdp_block_product.restype = ctypes.c_int
    lib.psdp_block_product_noalloc.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                               ctypes.c_int]
    lib.psdp_block_product_noalloc.restype = ctypes.c_int
    lib.psdp_admm_default_options.argtypes = [ctypes.POINTER(AdmmOptions)]
    lib.psdp_admm_default_options.restype = None
    lib.psdp_admm_solve.argtypes = [vp, ctypes.POINTER(Sdp), ctypes.POINTER(AdmmOptions), vp,
                                    ctypes.c_int, vp, vp, ctypes.c_int, ctypes.POINTER(AdmmInfo)]
    lib.psdp_admm_solve.restype = ctypes.c_int
    lib.psdp_certify_tail.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, ip, dp, dp]
    lib.psdp_certify_tail.restype = ctypes.c_int
    lib.psdp_status_str.argtypes = [ctypes.c_int]
    lib.psdp_status_str.restype = ctypes.c_char_p
    lib.psdp_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.psdp_profile_enable.restype = ctypes.c_int
    lib.psdp_batched_tuning.argtypes = [vp, ip, dp]
    lib.psdp_batched_tuning.restype = ctypes.c_int
    lib.psdp_profile_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_long), dp, dp, dp]
    lib.psdp_profile_get.restype = ctypes.c_int
    lib.psdp_profile_filter.argtypes = [vp, ctypes.c_char_p]
    lib.psdp_profile_filter.restype = ctypes.c_int
    llp = ctypes.POINTER(ctypes.c_longlong)
    lib.psdp_full_eig_project_batched.restype = ctypes.c_int
    lib.psdp_server_default_config.argtypes = [ctypes.POINTER(ServerConfig)]
    lib.psdp_server_default_config.restype = None
    lib.psdp_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ServerConfig)]
    lib.psdp_server_create.restype = ctypes.c_int
    lib.psdp_server_destroy.argtypes = [vp]
    lib.psdp_server_destroy.restype = ctypes.c_int
    lib.psdp_server_open_session.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
    lib.psdp_server_open_session.restype = ctypes.c_int
    lib.psdp_server_close_session.argtypes = [vp, ctypes.c_int]
    lib.psdp_server_close_session.restype = ctypes.c_int
    lib.psdp_server_submit.argtypes = [vp, ctypes.c_int, vp, vp, vp, llp]
    lib.psdp_server_submit.restype = ctypes.c_int
    lib.psdp_server_wait.argtypes = [vp, ctypes.c_longlong, ctypes.c_double,
                                     ctypes.POINTER(ServerResult)]
    lib.psdp_server_wait.restype = ctypes.c_int
    lib.psdp_server_drain.argtypes = [vp]
    lib.psdp_server_drain.restype = ctypes.c_int
    lib.psdp_server_session_block.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, ip]
    lib.psdp_server_session_block.restype = ctypes.c_int
    lib.psdp_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.psdp_server_stats_get.restype = ctypes.c_int
    lib.psdp_server_stats_reset.argtypes = [vp]
    lib.psdp_server_stats_reset.restype = ctypes.c_int
    lib.psdp_transfer_stats.argtypes = [llp, llp, llp, ctypes.c_int]
    lib.psdp_transfer_stats.restype = ctypes.c_int
    lib.psdp_version.argtypes = []
    lib.psdp_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_str(code: int) -> str:
    return load().psdp_status_str(int(code)).decode()
