"""ctypes view of include/dg.h (argument marshalling only).

Loading fails loudly: there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdg.so")

DG_OK, DG_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "DG_OK", 1: "DG_NOT_CONVERGED", -1: "DG_ERR_ARG", -2: "DG_ERR_HIP", -3: "DG_ERR_OOM",
                -4: "DG_ERR_STATE", -5: "DG_ERR_SINGULAR_BLOCK", -6: "DG_ERR_NONFINITE"}
DG_BASIS_PK, DG_BASIS_QK = 0, 1
DG_FLUX_LF, DG_FLUX_ROE = 0, 1
DG_JVP_EXACT, DG_JVP_FD, DG_JVP_EXACT_FP32, DG_JVP_STAB, DG_JVP_EXACT_BF16 = 0, 1, 2, 3, 4
DG_FP64, DG_FP32, DG_BF16 = 0, 1, 2
DG_PREC_NONE, DG_PREC_BJ, DG_PREC_MG, DG_PREC_MLP = 0, 1, 2, 3
DG_MG_V, DG_MG_FULL = 0, 1
DG_ORTH_CGS2, DG_ORTH_MGS = 0, 1
DG_MLP_DIRECT, DG_MLP_CORRECT_BJ = 0, 1
DG_PHYS_COMPRESSIBLE, DG_PHYS_INCOMPRESSIBLE, DG_PHYS_DIFFUSION = 0, 1, 2
DG_TUNE_FIXED, DG_TUNE_AUTO = 0, 1
DG_PROBE_AUTO, DG_PROBE_COLOURED = 0, 1

EXPORTED = ["dg_create", "dg_destroy", "dg_ndof", "dg_nbasis", "dg_nvar", "dg_nq", "dg_volume_points",
            "dg_project", "dg_residual", "dg_residual_fp32", "dg_residual_bf16", "dg_jvp", "dg_jvp_noalloc", "dg_jvp_noalloc_scratch_bytes",
            "dg_block_precond_setup", "dg_set_block_probing", "dg_block_precond_apply",
            "dg_fgmres_solve", "dg_rosenbrock_step", "dg_mg_setup", "dg_mg_update_fine", "dg_mg_apply", "dg_mg_level_apply", "dg_mlp_nparams", "dg_mlp_set_mode",
            "dg_mlp_set_weights", "dg_mlp_get_weights", "dg_mlp_features", "dg_mlp_forward", "dg_mlp_grad",
            "dg_mlp_train_step", "dg_mlp_apply", "dg_max_wave_speed",
            "dg_set_tuning", "dg_autotune", "dg_tuning_report", "dg_set_fine_shape", "dg_set_apply_shape",
            "dg_set_bsr_shape",
            "dg_set_profiling", "dg_kernel_time", "dg_last_error", "dg_sync"]


class DGParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order", ctypes.c_int), ("basis", ctypes.c_int), ("nq1d", ctypes.c_int),
                ("flux", ctypes.c_int), ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("mu", ctypes.c_double), ("eta_br2", ctypes.c_double), ("entropy_fix", ctypes.c_double),
                ("physics", ctypes.c_int), ("ac_beta", ctypes.c_double)]


class DGMesh(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int64), ("elem_xyz", ctypes.POINTER(ctypes.c_double)),
                ("elem_nbr", ctypes.POINTER(ctypes.c_int64))]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double),
                ("precond", ctypes.c_int), ("jvp_mode", ctypes.c_int), ("rho_ref", ctypes.c_double),
                ("judge_after", ctypes.c_int), ("orth", ctypes.c_int), ("check_every", ctypes.c_int)]


ROS_MAX_STAGES = 6


class RosCoeffs(ctypes.Structure):
    _fields_ = [("n_stages", ctypes.c_int), ("gamma", ctypes.c_double),
                ("a", (ctypes.c_double * ROS_MAX_STAGES) * ROS_MAX_STAGES),
                ("c", (ctypes.c_double * ROS_MAX_STAGES) * ROS_MAX_STAGES), ("m", ctypes.c_double * ROS_MAX_STAGES)]


class MgOpts(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("orders", ctypes.c_int * 3), ("smooth_iters", ctypes.c_int * 3),
                ("storage", ctypes.c_int), ("use_graph", ctypes.c_int), ("fine_precision", ctypes.c_int),
                ("cycle", ctypes.c_int), ("rescale", ctypes.c_int), ("coarse_ilu", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_res_est", ctypes.c_double), ("rel_res_true", ctypes.c_double), ("rho", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("fallbacks", ctypes.c_int), ("ms_setup", ctypes.c_double)]


_lib = None


def load():
    """Load libdg.so and declare signatures; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_00866_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
    ctx = ctypes.c_void_p
    sig = {
        "dg_create": (i, [ctypes.POINTER(DGParams), ctypes.POINTER(DGMesh), ctypes.POINTER(ctypes.c_void_p)]),
        "dg_destroy": (None, [ctx]),
        "dg_ndof": (i64, [ctx]),
        "dg_nbasis": (i, [ctx]),
        "dg_nvar": (i, [ctx]),
        "dg_nq": (i, [ctx]),
        "dg_volume_points": (i, [ctx, vp, vp]),
        "dg_project": (i, [ctx, vp, vp, vp]),
        "dg_residual": (i, [ctx, vp, vp, vp]),
        "dg_residual_fp32": (i, [ctx, vp, vp, vp]),
        "dg_residual_bf16": (i, [ctx, vp, vp, vp]),
        "dg_jvp": (i, [ctx, vp, vp, vp, d, i, vp, vp]),
        "dg_jvp_noalloc": (i, [ctx, vp, vp, d, vp, vp]),
        "dg_jvp_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "dg_block_precond_setup": (i, [ctx, vp, d, i, vp]),
        "dg_block_precond_apply": (i, [ctx, vp, vp, vp]),
        "dg_fgmres_solve": (i, [ctx, vp, d, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]),
        "dg_rosenbrock_step": (i, [ctx, vp, d, ctypes.POINTER(RosCoeffs), ctypes.POINTER(SolveOpts), vp,
                                   ctypes.POINTER(SolveStats), vp]),
        "dg_mg_setup": (i, [ctx, vp, d, ctypes.POINTER(MgOpts), vp]),
        "dg_mg_update_fine": (i, [ctx, vp, d, i, vp]),
        "dg_mg_apply": (i, [ctx, vp, vp, vp]),
        "dg_mg_level_apply": (i, [ctx, i, vp, vp, vp]),
        "dg_mlp_nparams": (i64, [ctx]),
        "dg_mlp_set_mode": (i, [ctx, i]),
        "dg_mlp_set_weights": (i, [ctx, vp, vp]),
        "dg_mlp_get_weights": (i, [ctx, vp, vp]),
        "dg_mlp_features": (i, [ctx, vp, vp, vp, vp, vp, vp, vp]),
        "dg_mlp_forward": (i, [ctx, vp, i64, vp, vp]),
        "dg_mlp_grad": (i, [ctx, vp, vp, vp, i64, vp, vp, vp]),
        "dg_mlp_train_step": (i, [ctx, vp, vp, vp, i64, ctypes.c_float, vp, vp]),
        "dg_mlp_apply": (i, [ctx, vp, vp, vp, vp]),
        "dg_max_wave_speed": (i, [ctx, vp, ctypes.POINTER(ctypes.c_double), vp]),
        "dg_set_tuning": (i, [ctx, i]),
        "dg_set_block_probing": (i, [ctx, i]),
        "dg_autotune": (i, [ctx, vp, vp]),
        "dg_tuning_report": (i, [ctx, ctypes.c_char_p, ctypes.c_size_t]),
        "dg_set_fine_shape": (i, [ctx, i, i, i, i]),
        "dg_set_apply_shape": (i, [ctx, i, i, i, i]),
        "dg_set_bsr_shape": (i, [ctx, i, i, i, i]),
        "dg_set_profiling": (i, [ctx, i]),
        "dg_kernel_time": (i, [ctx, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
        "dg_last_error": (ctypes.c_char_p, []),
        "dg_sync": (i, [ctx]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class DGError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.dg_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, where, allow_not_converged=False):
    if status == DG_OK or (allow_not_converged and status == DG_NOT_CONVERGED):
        return status
    raise DGError(status, where)
