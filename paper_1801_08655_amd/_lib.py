"""ctypes binding of ``libhelm.so`` (argument marshalling only).

Every step of the solver runs in the HIP library; this module converts
arguments (NumPy arrays, torch device tensors) into the plain pointers and
sizes of the C ABI declared in ``include/helm.h``.  Loading fails loudly if
the library has not been built: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelm.so")

HELM_OK, HELM_EINVAL, HELM_ENOMEM, HELM_EZEROPIVOT, HELM_ENOCONV, HELM_EHIP = range(6)
HELM_FP64, HELM_MIXED = 0, 1

EXPORTED = [
    "helm_default_options", "helm_plan", "helm_plan_lane", "helm_factorize",
    "helm_factorize_dev",
    "helm_solve", "helm_solve_dev", "helm_solve_points", "helm_free",
    "helm_strerror", "helm_last_error", "helm_layer_info", "helm_layer_solve_dev",
    "helm_apply_operator_dev", "helm_polarized_op_dev", "helm_kernel_stats",
    "helm_set_solve_options", "helm_tile_choices", "helm_device_peaks",
    "helm_get_factor_info", "helm_layer_solve_noalloc_dev",
    # include/helm_serve.h
    "helm_server_default_options", "helm_server_create", "helm_server_add_model",
    "helm_server_submit", "helm_server_wait", "helm_server_poll", "helm_server_get_stats",
    "helm_server_free", "helm_server_remove_model",
    # include/helm_batch.h
    "helm_batch_default_options", "helm_solve_batch",
]
HELM_FLAG_PROFILE = 1
HELM_FLAG_NO_GRAPHS = 2
HELM_FLAG_AUTOTUNE = 4
HELM_FLAG_FULL_KRYLOV = 16
HELM_FLAG_PROFILE_FWD = 8
HELM_FLAG_TEST_ZERO_FRONT = 32
HELM_FLAG_BICGSTAB = 64
HELM_FLAG_UNPOLARIZED = 128
HELM_FLAG_NO_PRUNE = 256
HELM_FLAG_GEMM_4M = 512
HELM_FLAG_FACTOR_4M = 1024
HELM_FLAG_NO_NARROW = 2048
HELM_NOALLOC_SCRATCH_BYTES = 128 << 20


class helm_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double)]


class helm_options(ctypes.Structure):
    _fields_ = [
        ("pml_local", ctypes.c_int),
        ("pml_C", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("gmres_tol", ctypes.c_double),
        ("gmres_max_iter", ctypes.c_int),
        ("ir_tol", ctypes.c_double),
        ("ir_max_steps", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("inner_tol_refine", ctypes.c_double),
        ("err_target", ctypes.c_double),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("max_rhs", ctypes.c_int),
        ("leaf_size", ctypes.c_int),
        ("flags", ctypes.c_int),
        ("gmres_restart", ctypes.c_int),
        ("inner_tol_final", ctypes.c_double),
    ]


class helm_solve_info(ctypes.Structure):
    _fields_ = [
        ("n_rhs", ctypes.c_int),
        ("gmres_iters", ctypes.c_int),
        ("ir_steps", ctypes.c_int),
        ("rel_residual_max", ctypes.c_double),
        ("t_setup_ms", ctypes.c_double),
        ("t_gmres_ms", ctypes.c_double),
        ("t_reconstruct_ms", ctypes.c_double),
        ("t_residual_ms", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("layer_solves", ctypes.c_longlong),
        ("factor_bytes_read", ctypes.c_double),
        ("ir_residual", ctypes.c_double * 8),
        ("est_error_max", ctypes.c_double),
        ("ir_gmres_iters", ctypes.c_int * 8),
        ("rhs_rel_residual", ctypes.c_void_p),
        ("rhs_est_error", ctypes.c_void_p),
        ("rhs_ir_steps", ctypes.c_void_p),
        ("rhs_gmres_iters", ctypes.c_void_p),
        ("krylov_bytes", ctypes.c_double),
        ("ir_width", ctypes.c_int * 8),
        ("narrow_products", ctypes.c_int),
    ]
    PER_RHS = ("rhs_rel_residual", "rhs_est_error", "rhs_ir_steps", "rhs_gmres_iters")

    def attach(self, n):
        """Per-right-hand-side output arrays for n columns (kept alive here)."""
        import numpy as np
        self._arrays = {"rhs_rel_residual": np.zeros(n), "rhs_est_error": np.zeros(n),
                        "rhs_ir_steps": np.zeros(n, dtype=np.int32),
                        "rhs_gmres_iters": np.zeros(n, dtype=np.int32)}
        for name, a in self._arrays.items():
            setattr(self, name, a.ctypes.data if n else None)
        return self

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_
             if name not in self.PER_RHS}
        n = max(1, min(8, self.ir_steps))
        d["ir_residual"] = list(self.ir_residual[:n])
        d["ir_gmres_iters"] = list(self.ir_gmres_iters[:n])
        d["ir_width"] = list(self.ir_width[:n])
        for name, a in getattr(self, "_arrays", {}).items():
            d[name] = a.tolist()
        return d


class helm_factor_info(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("lu_flops", ctypes.c_double),
                ("gj_flops", ctypes.c_double), ("pivot_min", ctypes.c_double),
                ("pivot_max", ctypes.c_double), ("diag_max", ctypes.c_double),
                ("factor_bytes", ctypes.c_size_t), ("n_fronts", ctypes.c_longlong),
                ("max_front", ctypes.c_longlong), ("symbolic_seconds", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("lists_seconds", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class helm_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_longlong),
                ("total_ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class helm_tile_choice(ctypes.Structure):
    _fields_ = [("set_layers", ctypes.c_int), ("k", ctypes.c_int), ("depth", ctypes.c_int),
                ("fronts", ctypes.c_int), ("mean_s", ctypes.c_double),
                ("mean_b", ctypes.c_double), ("fwd_bn", ctypes.c_int),
                ("bwd_bn", ctypes.c_int), ("bwd_bm", ctypes.c_int), ("tuned", ctypes.c_int),
                ("t_fwd_us", ctypes.c_double * 4), ("t_bwd_us", ctypes.c_double * 4),
                ("fwd_elems", ctypes.c_double), ("bwd_elems", ctypes.c_double)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["t_fwd_us"] = list(self.t_fwd_us)
        d["t_bwd_us"] = list(self.t_bwd_us)
        return d


class helm_server_options(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int),
                ("device", ctypes.c_int)]


class helm_request_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("n_rhs", ctypes.c_int),
        ("model", ctypes.c_int),
        ("ir_steps_max", ctypes.c_int),
        ("rel_residual_max", ctypes.c_double),
        ("est_error_max", ctypes.c_double),
        ("t_submit_ms", ctypes.c_double),
        ("t_first_ms", ctypes.c_double),
        ("t_done_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class helm_server_summary(ctypes.Structure):
    _fields_ = [
        ("requests_done", ctypes.c_longlong),
        ("columns_done", ctypes.c_longlong),
        ("steps", ctypes.c_longlong),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
        ("mean_active_slots", ctypes.c_double),
        ("elapsed_s", ctypes.c_double),
        ("columns_per_s", ctypes.c_double),
        ("bytes_reserved", ctypes.c_size_t),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class helm_problem(ctypes.Structure):
    _fields_ = [("grid", helm_grid), ("m", ctypes.c_void_p), ("omega", ctypes.c_double),
                ("pml_width", ctypes.c_int), ("n_layers", ctypes.c_int),
                ("n_rhs", ctypes.c_int), ("node_index", ctypes.c_void_p),
                ("amplitude", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class helm_batch_options(ctypes.Structure):
    _fields_ = [("opt", helm_options), ("hbm_budget_bytes", ctypes.c_size_t),
                ("slots", ctypes.c_int), ("max_resident", ctypes.c_int)]


class helm_problem_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("slots", ctypes.c_int),
                ("planned_bytes", ctypes.c_size_t), ("t_admit_ms", ctypes.c_double),
                ("t_factored_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("factor_ms", ctypes.c_double), ("ir_steps_max", ctypes.c_int),
                ("rel_residual_max", ctypes.c_double), ("est_error_max", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class helm_batch_summary(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("factor_s", ctypes.c_double),
                ("columns", ctypes.c_longlong), ("rhs_per_s", ctypes.c_double),
                ("max_resident", ctypes.c_int), ("peak_planned_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """The loaded library; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` or "
            "`python paper_1801_08655_amd/build.py`")
    # PyTorch ships its own HIP runtime with the same SONAME as the system one;
    # loading torch first makes the library bind to that runtime, so that one
    # process never holds two HIP runtimes (device memory and streams are
    # shared with torch).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    H = ctypes.c_void_p
    L.helm_default_options.argtypes = [ctypes.POINTER(helm_options)]
    L.helm_default_options.restype = None
    L.helm_plan.argtypes = [ctypes.POINTER(helm_grid), I, I, ctypes.POINTER(helm_options),
                            ctypes.POINTER(S), ctypes.POINTER(S), ctypes.POINTER(S)]
    L.helm_plan.restype = I
    L.helm_plan_lane.argtypes = [ctypes.POINTER(helm_grid), I, I, ctypes.POINTER(helm_options),
                                 ctypes.POINTER(S)]
    L.helm_plan_lane.restype = I
    for fn in (L.helm_factorize, L.helm_factorize_dev):
        fn.argtypes = [ctypes.POINTER(helm_grid), P, D, I, I,
                       ctypes.POINTER(helm_options), ctypes.POINTER(H)]
        fn.restype = I
    for fn in (L.helm_solve, L.helm_solve_dev):
        fn.argtypes = [H, I, P, P, ctypes.POINTER(helm_solve_info)]
        fn.restype = I
    L.helm_solve_points.argtypes = [H, I, P, P, P, ctypes.POINTER(helm_solve_info)]
    L.helm_solve_points.restype = I
    L.helm_free.argtypes = [H]
    L.helm_free.restype = I
    L.helm_strerror.argtypes = [I]
    L.helm_strerror.restype = ctypes.c_char_p
    L.helm_last_error.argtypes = []
    L.helm_last_error.restype = ctypes.c_char_p
    L.helm_layer_info.argtypes = [H, I] + [ctypes.POINTER(I)] * 4
    L.helm_layer_info.restype = I
    L.helm_layer_solve_dev.argtypes = [H, I, I, P, P]
    L.helm_layer_solve_dev.restype = I
    L.helm_layer_solve_noalloc_dev.argtypes = [H, I, I, P, P]
    L.helm_layer_solve_noalloc_dev.restype = I
    L.helm_apply_operator_dev.argtypes = [H, I, P, P, P]
    L.helm_apply_operator_dev.restype = I
    L.helm_polarized_op_dev.argtypes = [H, I, I, P, P]
    L.helm_polarized_op_dev.restype = I
    L.helm_kernel_stats.argtypes = [H, ctypes.POINTER(helm_kernel_stat), I,
                                    ctypes.POINTER(I), I]
    L.helm_kernel_stats.restype = I
    L.helm_set_solve_options.argtypes = [H, ctypes.POINTER(helm_options)]
    L.helm_set_solve_options.restype = I
    L.helm_tile_choices.argtypes = [H, ctypes.POINTER(helm_tile_choice), I, ctypes.POINTER(I)]
    L.helm_tile_choices.restype = I
    L.helm_device_peaks.argtypes = [I] + [ctypes.POINTER(D)] * 4
    L.helm_device_peaks.restype = I
    L.helm_get_factor_info.argtypes = [H, ctypes.POINTER(helm_factor_info)]
    L.helm_get_factor_info.restype = I
    SV = ctypes.c_void_p
    L.helm_server_default_options.argtypes = [ctypes.POINTER(helm_server_options)]
    L.helm_server_default_options.restype = None
    L.helm_server_create.argtypes = [ctypes.POINTER(helm_server_options), ctypes.POINTER(SV)]
    L.helm_server_create.restype = I
    L.helm_server_add_model.argtypes = [SV, H, ctypes.POINTER(I), ctypes.POINTER(I)]
    L.helm_server_add_model.restype = I
    L.helm_server_submit.argtypes = [SV, I, I, P, P, P, ctypes.POINTER(ctypes.c_int64)]
    L.helm_server_submit.restype = I
    L.helm_server_wait.argtypes = [SV, ctypes.c_int64, ctypes.POINTER(helm_request_info)]
    L.helm_server_wait.restype = I
    L.helm_server_poll.argtypes = [SV, ctypes.c_int64, ctypes.POINTER(I)]
    L.helm_server_poll.restype = I
    L.helm_server_get_stats.argtypes = [SV, ctypes.POINTER(helm_server_summary)]
    L.helm_server_get_stats.restype = I
    L.helm_server_free.argtypes = [SV]
    L.helm_server_free.restype = I
    L.helm_server_remove_model.argtypes = [SV, I]
    L.helm_server_remove_model.restype = I
    L.helm_batch_default_options.argtypes = [ctypes.POINTER(helm_batch_options)]
    L.helm_batch_default_options.restype = None
    L.helm_solve_batch.argtypes = [I, ctypes.POINTER(helm_problem),
                                   ctypes.POINTER(helm_batch_options),
                                   ctypes.POINTER(helm_problem_info),
                                   ctypes.POINTER(helm_batch_summary)]
    L.helm_solve_batch.restype = I
    _lib = L
    return L


class HelmError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.helm_strerror(status).decode()
        detail = L.helm_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")
        self.status = status


def check(status, where):
    if status not in (HELM_OK,):
        raise HelmError(status, where)
