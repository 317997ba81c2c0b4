"""ctypes binding of libstokesmg (include/stokesmg.h): argument marshalling
only.  Every computation happens in the HIP library; if the library is not
built this module raises at import."""
import ctypes
import os

try:
    # torch ships its own HIP runtime; it must be the process's only one, so it is
    # loaded before libstokesmg (whose libamdhip64 dependency then resolves to it)
    import torch  # noqa: F401
except ImportError:
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstokesmg.so")

OK, EINVAL, EHIP, ENOMEM, ENOTCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
F64, F32 = 0, 1


class Config(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int), ("k", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("penalty_factor", ctypes.c_double), ("cg_rtol", ctypes.c_double), ("cg_max_it", ctypes.c_int)]


MAX_HISTORY = 512


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("nu", ctypes.c_double), ("history", ctypes.c_double * MAX_HISTORY),
                ("cg_iterations", ctypes.c_longlong), ("local_solves", ctypes.c_longlong),
                ("seconds", ctypes.c_double), ("fallback_iteration", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2410_09497_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p, szp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "stokesmg_create": (i32, [ctypes.POINTER(Config), ctypes.POINTER(vp)]),
        "stokesmg_destroy": (None, [vp]),
        "stokesmg_last_error": (ctypes.c_char_p, [vp]),
        "stokesmg_num_levels": (i32, [vp]),
        "stokesmg_sizes": (i32, [vp, i32, i64p, i64p, i64p]),
        "stokesmg_workspace_size": (i32, [vp, szp]),
        "stokesmg_set_workspace": (i32, [vp, vp, ctypes.c_size_t, vp]),
        "stokes_apply": (i32, [vp, i32, i32, vp, vp, vp]),
        "stokes_residual": (i32, [vp, i32, i32, vp, vp, vp, vp]),
        "patch_smooth": (i32, [vp, i32, i32, vp, vp, i32, vp]),
        "stokesmg_cg_stats": (i32, [vp, i64p, i64p, i32, vp]),
        "patch_smooth_noalloc": (i32, [vp, i32, i32, vp, vp, i32, i64p, vp]),
        "stokesmg_noalloc_scratch_size": (i32, [szp]),
        "vcycle": (i32, [vp, i32, vp, vp, vp]),
        "stokesmg_solve_workspace_size": (i32, [vp, i32, i32, szp]),
        "solve": (i32, [vp, vp, vp, ctypes.c_double, i32, i32, i32, vp, ctypes.c_size_t, ctypes.POINTER(Info), vp]),
        "stokesmg_rhs_manufactured": (i32, [vp, i32, i32, vp, vp]),
        "stokesmg_rhs_fourier": (i32, [vp, i32, i32, vp, vp, vp, vp, vp]),
        "mlp_dims": (i32, [vp, i64p, i64p]),
        "mlp_workspace_size": (i32, [vp, ctypes.c_int64, szp]),
        "mlp_set_workspace": (i32, [vp, vp, ctypes.c_size_t, ctypes.c_int64]),
        "mlp_init": (i32, [vp, ctypes.c_uint64, vp]),
        "mlp_get_state": (i32, [vp, vp, i64p, vp]),
        "mlp_set_state": (i32, [vp, vp, ctypes.c_int64, vp]),
        "mlp_forward": (i32, [vp, i32, vp, vp, ctypes.c_int64, vp]),
        "mlp_backward": (i32, [vp, i32, vp, vp, ctypes.c_int64, vp, vp, vp]),
        "mlp_adam_step": (i32, [vp, vp, ctypes.c_float, vp]),
        "mlp_collect_pairs": (i32, [vp, vp, vp, vp, vp, ctypes.c_int64, i64p, vp]),
        "mlp_train": (i32, [vp, i32, vp, vp, ctypes.c_int64, i32, i32, ctypes.c_float, ctypes.c_uint64,
                            ctypes.POINTER(ctypes.c_float), vp]),
        "stokesmg_set_local_solver": (i32, [vp, i32, i32, ctypes.c_double]),
        "stokesmg_set_fallback": (i32, [vp, ctypes.c_double]),
        "stokesmg_set_smoothing": (i32, [vp, i32, i32]),
        "stokesmg_direct_matrix": (i32, [vp, i32, vp]),
        "stokesmg_l2_error": (i32, [vp, i32, i32, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    vp]),
        "stokesmg_direct_setup": (i32, [vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

EXPORTED = ["stokesmg_create", "stokesmg_destroy", "stokesmg_last_error", "stokesmg_num_levels",
            "stokesmg_sizes", "stokesmg_workspace_size", "stokesmg_set_workspace", "stokes_apply",
            "stokes_residual", "patch_smooth", "stokesmg_cg_stats", "vcycle", "stokesmg_solve_workspace_size",
            "solve", "stokesmg_rhs_manufactured", "stokesmg_rhs_fourier", "mlp_dims", "mlp_workspace_size", "mlp_set_workspace", "mlp_init",
            "mlp_get_state", "mlp_set_state", "mlp_forward", "mlp_backward", "mlp_adam_step", "mlp_collect_pairs",
            "mlp_train", "stokesmg_set_local_solver", "stokesmg_set_fallback", "stokesmg_set_smoothing"]
