"""ctypes declarations of libscdg.so (C ABI in include/scdg.h).

Argument marshalling only: every step of the solve runs inside the library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscdg.so")

SCDG_OK = 0
STATUS = {0: "SCDG_OK", -1: "SCDG_ERR_ARG", -2: "SCDG_ERR_STATE", -3: "SCDG_ERR_HIP",
          -4: "SCDG_ERR_NOMEM", -5: "SCDG_ERR_SINGULAR", -6: "SCDG_ERR_NOCONV",
          -7: "SCDG_ERR_NONFINITE", -8: "SCDG_ERR_UNSUPPORTED"}
SCDG_FP64, SCDG_FP32 = 0, 1
SCDG_COPY, SCDG_BORROW = 0, 1          # scdg_assemble flags
SOLVER_AUTO, SOLVER_DENSE, SOLVER_GMRES = 0, 1, 2
EXPORT_AII_INV, EXPORT_SCHUR, EXPORT_X = 1, 2, 3

EXPORTED = [
    "scdg_plan_create", "scdg_plan_destroy", "scdg_set_stream", "scdg_plan_sizes",
    "scdg_assemble", "scdg_factor", "scdg_factor_info", "scdg_condense", "scdg_condense_rhs",
    "scdg_solve_condensed", "scdg_backsolve", "scdg_solve", "scdg_residual",
    "scdg_schur_apply", "scdg_export", "scdg_status_string", "scdg_last_error",
    "scdg_enable_timing", "scdg_phase_times", "scdg_autotune", "scdg_set_gemm_config",
    "scdg_get_gemm_config", "scdg_plan_fold_counts", "scdg_set_inverse_mode", "scdg_get_inverse_mode",
    "scdg_set_krylov_mode", "scdg_set_schur_mode", "scdg_get_schur_mode", "scdg_newton_step",
    "scdg_dg_create", "scdg_dg_destroy", "scdg_dg_residual", "scdg_dg_gradient", "scdg_dg_set_geometry",
    "scdg_dg_jacobian_apply",
    "scdg_dg_jacobian_apply_noalloc", "scdg_dg_jacobian_blocks", "scdg_schur_apply_transpose",
    "scdg_guess_schur_loss",
    "scdg_mlp_create", "scdg_mlp_destroy", "scdg_mlp_param_count", "scdg_mlp_set_compute", "scdg_mlp_forward",
    "scdg_mlp_backward", "scdg_mlp_adam", "scdg_mlp_mse", "scdg_mlp_gather", "scdg_guess_stats",
    "scdg_guess_features", "scdg_guess_target", "scdg_guess_apply",
    "scdg_probe_mfma", "scdg_probe_hbm_read",
]
GEMM_CONFIGS = ["64x64", "64x128", "128x128", "128x128w8", "128x64", "240x80", "80x80", "256x128", "128x256"]
PHASES = ["inverse", "gemm_x", "gemm_s", "rhs", "schur_apply", "condensed_solve", "backsolve",
          "residual"]


class Structure(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("order", C.c_void_p), ("c_ptr", C.c_void_p),
                ("c_node", C.c_void_p), ("bb_rowptr", C.c_void_p), ("bb_col", C.c_void_p),
                ("phys_faces", C.c_void_p)]


class DgParams(C.Structure):
    _fields_ = [("k_elem", C.c_int32), ("order", C.c_int32), ("length", C.c_double),
                ("mach", C.c_double), ("reynolds", C.c_double), ("gamma", C.c_double),
                ("prandtl", C.c_double), ("sutherland_ratio", C.c_double), ("viscous_flux", C.c_int32),
                ("sipg_eta", C.c_double)]


class MlpShape(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_layers", C.c_int32),
                ("n_out", C.c_int32), ("max_batch", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("restart", C.c_int32), ("max_iters", C.c_int32),
                ("tol", C.c_double), ("precond", C.c_int32), ("ir_max", C.c_int32),
                ("ir_tol", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("ir_sweeps", C.c_int32),
                ("solver_used", C.c_int32), ("rel_res_S", C.c_double), ("rel_res_full", C.c_double),
                ("guess_rejected", C.c_int32), ("rel_res_guess", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class NewtonOpts(C.Structure):
    _fields_ = [("newton_tol", C.c_double), ("lin_tol", C.c_double), ("forcing", C.c_double),
                ("eta_max", C.c_double), ("restart", C.c_int32), ("cycles", C.c_int32),
                ("precond", C.c_int32), ("max_newton", C.c_int32)]


class NewtonInfo(C.Structure):
    _fields_ = [("newton", C.c_int32), ("gmres", C.c_int32), ("first_gmres", C.c_int32),
                ("lin_unconverged", C.c_int32), ("start_rejected", C.c_int32), ("converged", C.c_int32),
                ("r0", C.c_double), ("rel_res", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ScdgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} {detail}".strip())


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1911_02366_amd/build.py "
                          "(the solver has no fallback path)")
    lib = C.CDLL(path)
    vp, i32, i64, d, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "scdg_plan_create": (i32, [C.POINTER(vp), C.POINTER(Structure), vp, i32]),
        "scdg_plan_destroy": (i32, [vp]),
        "scdg_set_stream": (i32, [vp, vp]),
        "scdg_plan_sizes": (i32, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
        "scdg_assemble": (i32, [vp, vp, vp, vp, vp, i32]),
        "scdg_factor": (i32, [vp, i32]),
        "scdg_factor_info": (i32, [vp, C.POINTER(i64), C.POINTER(i32)]),
        "scdg_condense": (i32, [vp]),
        "scdg_condense_rhs": (i32, [vp, vp, vp]),
        "scdg_solve_condensed": (i32, [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
        "scdg_backsolve": (i32, [vp, vp, vp, vp]),
        "scdg_solve": (i32, [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
        "scdg_residual": (i32, [vp, vp, vp, vp, C.POINTER(d)]),
        "scdg_schur_apply": (i32, [vp, vp, vp]),
        "scdg_export": (i32, [vp, i32, vp, sz]),
        "scdg_status_string": (C.c_char_p, [i32]),
        "scdg_last_error": (i32, [vp, C.c_char_p, sz]),
        "scdg_enable_timing": (i32, [vp, i32]),
        "scdg_phase_times": (i32, [vp, C.POINTER(d), C.POINTER(i32), i32]),
        "scdg_autotune": (i32, [vp, C.POINTER(d), C.POINTER(d), i32]),
        "scdg_set_gemm_config": (i32, [vp, i32, i32]),
        "scdg_get_gemm_config": (i32, [vp, C.POINTER(i32), C.POINTER(i32)]),
        "scdg_plan_fold_counts": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
        "scdg_set_inverse_mode": (i32, [vp, i32]),
        "scdg_set_krylov_mode": (i32, [vp, i32]),
        "scdg_set_schur_mode": (i32, [vp, i32]),
        "scdg_get_schur_mode": (i32, [vp, C.POINTER(i32)]),
        "scdg_get_inverse_mode": (i32, [vp, C.POINTER(i32)]),
        "scdg_newton_step": (i32, [vp, vp, vp, d, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonInfo)]),
        "scdg_dg_create": (i32, [C.POINTER(vp), C.POINTER(DgParams), vp]),
        "scdg_dg_destroy": (i32, [vp]),
        "scdg_dg_residual": (i32, [vp, vp, vp, d, vp]),
        "scdg_dg_gradient": (i32, [vp, vp]),
        "scdg_dg_jacobian_apply": (i32, [vp, vp, vp, d, vp]),
        "scdg_dg_jacobian_apply_noalloc": (i32, [vp, vp, vp, d, vp]),
        "scdg_dg_jacobian_blocks": (i32, [vp, vp, vp, d, vp, vp, vp, vp]),
        "scdg_schur_apply_transpose": (i32, [vp, vp, vp]),
        "scdg_guess_schur_loss": (i32, [vp, vp, vp, vp, d, vp, vp]),
        "scdg_dg_set_geometry": (i32, [vp, vp]),
        "scdg_mlp_create": (i32, [C.POINTER(vp), C.POINTER(MlpShape), vp]),
        "scdg_mlp_destroy": (i32, [vp]),
        "scdg_mlp_param_count": (i32, [vp, C.POINTER(i64)]),
        "scdg_mlp_set_compute": (i32, [vp, i32]),
        "scdg_mlp_forward": (i32, [vp, vp, vp, i32, vp]),
        "scdg_mlp_backward": (i32, [vp, vp, vp, vp, i32, vp, vp]),
        "scdg_mlp_adam": (i32, [vp, vp, vp, vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, i32]),
        "scdg_mlp_mse": (i32, [vp, vp, vp, i64, vp, vp]),
        "scdg_mlp_gather": (i32, [vp, vp, i32, vp, i32, vp]),
        "scdg_guess_stats": (i32, [vp, vp, vp, vp, vp, i64, vp]),
        "scdg_guess_features": (i32, [vp, vp, vp, vp, vp, i32, vp]),
        "scdg_guess_target": (i32, [vp, vp, vp, vp, i32, vp]),
        "scdg_guess_apply": (i32, [vp, vp, vp, vp, i32, vp]),
        "scdg_probe_mfma": (i32, [i32, i32, vp, C.POINTER(d)]),
        "scdg_probe_hbm_read": (i32, [i64, vp, C.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error(plan_handle) -> str:
    lib = load()
    buf = C.create_string_buffer(1024)
    lib.scdg_last_error(plan_handle, buf, 1024)
    return buf.value.decode(errors="replace")
