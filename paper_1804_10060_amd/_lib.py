"""ctypes declarations of the C ABI in include/te.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libte_amd.so")

TE_OK, TE_ENOTCONV = 0, 1
TE_EINVAL, TE_ENOMEM, TE_EHIP, TE_EINDEF, TE_ENAN, TE_ERANK, TE_ECHOL = -1, -2, -3, -4, -5, -6, -7
TE_PREC_FP64, TE_PREC_MIXED = 0, 1
TE_AGG_GREEDY, TE_AGG_MIS2 = 0, 1
TE_OP_A, TE_OP_P, TE_OP_R, TE_OP_SMOOTH, TE_OP_VCYCLE = 0, 1, 2, 3, 4
KERNEL_CLASSES = ["Ap", "pre_smooth", "residual", "restrict", "prolong", "post_init", "post_smooth", "coarse_levels",
                  "vector"]

CODE_NAMES = {TE_ENOTCONV: "TE_ENOTCONV", TE_EINVAL: "TE_EINVAL", TE_ENOMEM: "TE_ENOMEM", TE_EHIP: "TE_EHIP",
              TE_EINDEF: "TE_EINDEF", TE_ENAN: "TE_ENAN", TE_ERANK: "TE_ERANK", TE_ECHOL: "TE_ECHOL"}

# exported names declared in include/te.h
EXPORTS = ["te_version", "te_last_error", "fe_assemble_pattern", "fe_assemble_thermoelastic", "fe_assemble_load",
           "fe_assemble_thermoelastic_materials",
           "amg_options_default", "amg_setup", "amg_setup_with_aggregates", "amg_get_info", "amg_get_aggregates",
           "amg_get_level_matrix", "amg_apply", "pcg_options_default", "amg_pcg_solve", "amg_pcg_solve_multi", "te_autotune_multi", "amg_energy_scale",
           "te_autotune", "amg_destroy",
           "amg_set_operator", "te_timestep", "te_timestep_noalloc",
           "mpnn_param_count", "mpnn_create", "mpnn_destroy", "mpnn_features", "mpnn_forward", "mpnn_backward", "mpnn_backward_from", "mpnn_energy_grad",
           "mpnn_adam_step", "mpnn_guess",
           "fe_assemble_thermal", "camg_options_default", "camg_setup", "camg_destroy", "camg_get_info",
           "camg_get_splitting", "camg_get_level_matrix", "camg_apply", "camg_pcg_solve", "newton_options_default",
           "thermal_create", "thermal_set_exterior", "thermal_newton", "thermal_reset_preconditioner",
           "thermal_destroy"]
TE_CAMG_A, TE_CAMG_P, TE_CAMG_R, TE_CAMG_VCYCLE, TE_CAMG_SWEEP_FWD, TE_CAMG_SWEEP_BWD = 0, 1, 2, 3, 4, 5


class TeMesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_cells", C.c_int64), ("degree", C.c_int32),
                ("coords", C.c_void_p), ("cells", C.c_void_p)]


class TeMaterial(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("alpha", C.c_double), ("T_ref", C.c_double)]


class TeMaterialTables(C.Structure):
    _fields_ = [("n_materials", C.c_int32), ("n_points", C.c_int32), ("T", C.c_void_p), ("E", C.c_void_p),
                ("nu", C.c_void_p), ("alpha", C.c_void_p), ("T_ref", C.c_double)]


class TePressure(C.Structure):
    _fields_ = [("n_faces", C.c_int64), ("faces", C.c_void_p), ("p", C.c_void_p)]


class TeBsr(C.Structure):
    _fields_ = [("n_brows", C.c_int64), ("nnzb", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("val", C.c_void_p)]


class TeCsr(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("val", C.c_void_p)]


class TeThermalTables(C.Structure):
    _fields_ = [("n_materials", C.c_int32), ("n_points", C.c_int32), ("T", C.c_void_p), ("kappa", C.c_void_p),
                ("cv", C.c_void_p), ("rho", C.c_void_p)]


class TeRobin(C.Structure):
    _fields_ = [("n_faces", C.c_int64), ("faces", C.c_void_p), ("h", C.c_void_p), ("T_bc", C.c_void_p)]


class CamgOptions(C.Structure):
    _fields_ = [("theta", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("max_coarse_ratio", C.c_double), ("block", C.c_int32)]


class CamgInfo(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_rows", C.c_int64 * 16), ("nnz", C.c_int64 * 16),
                ("p_nnz", C.c_int64 * 16), ("setup_ms", C.c_double)]


class NewtonOptions(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("lin_rtol", C.c_double), ("maxit", C.c_int32),
                ("rebuild_factor", C.c_double), ("amg", CamgOptions)]


class NewtonReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rebuilds", C.c_int32),
                ("lin_iters_total", C.c_int32), ("res0", C.c_double), ("res", C.c_double),
                ("res_hist", C.c_double * 33), ("lin_iters", C.c_int32 * 32), ("time_ms", C.c_double),
                ("assembly_ms", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


class AmgOptions(C.Structure):
    _fields_ = [("theta0", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("lanczos_steps", C.c_int32), ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
                ("cheb_safety", C.c_double), ("max_coarse_ratio", C.c_double), ("build_fp32", C.c_int32),
                ("host_threads", C.c_int32), ("max_nrhs", C.c_int32), ("coarse_sym", C.c_int32),
                ("aggregation", C.c_int32), ("smooth_filtered", C.c_int32)]


class AmgInfo(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_dof", C.c_int64 * 16), ("nnzb", C.c_int64 * 16),
                ("bs", C.c_int32 * 16), ("lambda_hat", C.c_double * 16), ("p_nnzb", C.c_int64 * 16),
                ("setup_ms", C.c_double), ("bytes_device", C.c_int64)]


class PcgOptions(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("precision", C.c_int32), ("max_replace", C.c_int32),
                ("profile", C.c_int32), ("block", C.c_int32)]


class PcgReport(C.Structure):
    _fields_ = [("iters", C.c_void_p), ("converged", C.c_void_p), ("relres_true", C.c_void_p),
                ("history", C.c_void_p), ("max_iters", C.c_int32), ("time_ms", C.c_double),
                ("kernel_ms", C.c_double * 9), ("kernel_launches", C.c_int32 * 9)]


_lib = None


def load():
    """Load libte_amd.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1804_10060_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "te_version": ([], C.c_int),
        "te_last_error": ([], C.c_char_p),
        "fe_assemble_pattern": ([C.POINTER(TeMesh), vp, C.POINTER(i64), vp], C.c_int),
        "fe_assemble_thermoelastic": ([C.POINTER(TeMesh), C.POINTER(TeMaterial), vp, vp, vp, vp, C.POINTER(TeBsr),
                                       vp, vp], C.c_int),
        "fe_assemble_load": ([C.POINTER(TeMesh), C.POINTER(TeMaterial), vp, vp, vp, i32, vp, vp], C.c_int),
        "fe_assemble_thermoelastic_materials": ([C.POINTER(TeMesh), C.POINTER(TeMaterialTables), vp, vp, vp,
                                                 C.POINTER(TePressure), vp, vp, C.POINTER(TeBsr), vp, vp], C.c_int),
        "amg_options_default": ([C.POINTER(AmgOptions)], None),
        "amg_setup": ([C.POINTER(TeBsr), vp, vp, C.POINTER(AmgOptions), C.POINTER(vp), vp], C.c_int),
        "amg_setup_with_aggregates": ([C.POINTER(TeBsr), vp, vp, C.POINTER(AmgOptions), C.POINTER(vp), i32,
                                       C.POINTER(vp), vp], C.c_int),
        "amg_get_info": ([vp, C.POINTER(AmgInfo)], C.c_int),
        "amg_get_aggregates": ([vp, i32, vp], C.c_int),
        "amg_get_level_matrix": ([vp, i32, C.POINTER(i64), C.POINTER(i64), vp, vp, vp], C.c_int),
        "amg_apply": ([vp, i32, i32, i32, vp, vp, vp], C.c_int),
        "pcg_options_default": ([C.POINTER(PcgOptions)], None),
        "amg_pcg_solve": ([vp, vp, vp, i32, C.POINTER(PcgOptions), C.POINTER(PcgReport), vp], C.c_int),
        "amg_pcg_solve_multi": ([C.POINTER(vp), i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(PcgOptions),
                                 C.POINTER(PcgReport), vp], C.c_int),
        "te_autotune_multi": ([C.POINTER(vp), i32, C.c_char_p, i64, vp], C.c_int),
        "amg_energy_scale": ([vp, vp, vp, C.POINTER(C.c_double), vp], C.c_int),
        "te_autotune": ([vp, C.c_char_p, i32, C.c_char_p, i64, vp], C.c_int),
        "amg_destroy": ([vp], C.c_int),
        "amg_set_operator": ([vp, C.POINTER(TeBsr), vp], C.c_int),
        "te_timestep": ([vp, vp, i64, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double),
                         C.POINTER(C.c_int32), C.POINTER(C.c_double), vp], C.c_int),
        "te_timestep_noalloc": ([vp, vp, i64, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double), vp], C.c_int),
        "mpnn_param_count": ([], i64),
        "mpnn_create": ([i64, vp, vp, vp, C.POINTER(vp), vp], C.c_int),
        "mpnn_destroy": ([vp], C.c_int),
        "mpnn_features": ([vp, vp, C.c_double, vp, vp, vp, vp], C.c_int),
        "mpnn_forward": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "mpnn_backward": ([vp, vp, vp, vp, C.POINTER(C.c_double), vp], C.c_int),
        "mpnn_backward_from": ([vp, vp, vp, vp, vp], C.c_int),
        "mpnn_energy_grad": ([vp, vp, vp, vp, C.POINTER(C.c_double), vp], C.c_int),
        "mpnn_adam_step": ([i64, vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp], C.c_int),
        "mpnn_guess": ([vp, vp, vp], C.c_int),
        "fe_assemble_thermal": ([C.POINTER(TeMesh), C.POINTER(TeThermalTables), vp, C.POINTER(TeRobin), vp, vp,
                                 C.c_double, C.POINTER(TeCsr), vp, vp], C.c_int),
        "camg_options_default": ([C.POINTER(CamgOptions)], None),
        "camg_setup": ([C.POINTER(TeCsr), C.POINTER(CamgOptions), C.POINTER(vp), vp], C.c_int),
        "camg_destroy": ([vp], C.c_int),
        "camg_get_info": ([vp, C.POINTER(CamgInfo)], C.c_int),
        "camg_get_splitting": ([vp, i32, vp], C.c_int),
        "camg_get_level_matrix": ([vp, i32, i32, C.POINTER(i64), C.POINTER(i64), vp, vp, vp], C.c_int),
        "camg_apply": ([vp, i32, i32, vp, vp, vp], C.c_int),
        "camg_pcg_solve": ([vp, C.POINTER(TeCsr), vp, vp, C.c_double, i32, C.POINTER(C.c_int32),
                            C.POINTER(C.c_double), vp], C.c_int),
        "newton_options_default": ([C.POINTER(NewtonOptions)], None),
        "thermal_create": ([C.POINTER(TeMesh), C.POINTER(TeThermalTables), vp, C.POINTER(TeRobin), C.POINTER(vp),
                            vp], C.c_int),
        "thermal_set_exterior": ([vp, vp, vp], C.c_int),
        "thermal_newton": ([vp, vp, vp, C.c_double, C.POINTER(NewtonOptions), C.POINTER(NewtonReport), vp],
                           C.c_int),
        "thermal_reset_preconditioner": ([vp], C.c_int),
        "thermal_destroy": ([vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class TeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, allow=(TE_OK,)):
    if code in allow:
        return code
    msg = load().te_last_error().decode(errors="replace")
    raise TeError(code, msg)
