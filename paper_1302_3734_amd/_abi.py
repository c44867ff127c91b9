"""ctypes declarations of the C ABI in include/wmcao.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwmcao.so")

WMCAO_F32, WMCAO_F64 = 0, 1
WMCAO_FRAME_OK, WMCAO_FRAME_CONVERGED, WMCAO_FRAME_BREAKDOWN = 0, 1, -7
KERNELS = ["idwt_coarse", "idwt_tile", "sensor", "fdwt_tile", "fdwt_coarse", "init", "update_r",
           "update_p", "replace_r", "project", "adjoint", "weights"]
ERRORS = {-1: "INVALID_ARG", -2: "SIZE", -3: "FOOTPRINT", -4: "UNSUPPORTED", -5: "OOM",
          -6: "HIP", -7: "BREAKDOWN"}


class Pupil(C.Structure):
    _fields_ = [("diameter_m", C.c_double), ("obstruction_ratio", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("altitude_m", C.c_double), ("cn2_weight", C.c_double),
                ("spacing_m", C.c_double), ("n", C.c_int)]


class Wfs(C.Structure):
    _fields_ = [("is_lgs", C.c_int), ("theta_x", C.c_double), ("theta_y", C.c_double),
                ("lgs_height_m", C.c_double), ("n_sub", C.c_int), ("tt_aggregate", C.c_int),
                ("remove_tt", C.c_int), ("in_precond", C.c_int), ("sigma", C.c_double),
                ("cinv_blocks", C.POINTER(C.c_double)), ("kind", C.c_int)]


class Wavelet(C.Structure):
    _fields_ = [("family", C.c_int), ("order", C.c_int)]


class Options(C.Structure):
    _fields_ = [("alpha", C.c_double), ("r0_m", C.c_double), ("L0_m", C.c_double),
                ("dtype", C.c_int), ("max_batch", C.c_int), ("resid_replace_every", C.c_int),
                ("precond", C.c_int), ("tile", C.c_int), ("lds_budget", C.c_int),
                ("streams", C.c_int), ("op_precision", C.c_int), ("op_fp64_stages", C.c_int),
                ("proj_rows", C.c_int), ("vec_chunk", C.c_int), ("adj_lds", C.c_int)]


class WmcaoError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code}): {msg}")
        self.code = code


_lib = None


def lib():
    """Load libwmcao.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
        L.wmcao_plan.argtypes = [C.POINTER(Pupil), C.POINTER(Layer), C.c_int, C.POINTER(Wfs),
                                 C.c_int, Wavelet, C.c_int, C.POINTER(Options), C.POINTER(vp)]
        L.wmcao_sizes.argtypes = [vp, i64p, i64p, i64p, i64p]
        for name in ("wmcao_coeffs_to_layers", "wmcao_layers_to_coeffs", "wmcao_forward_layers",
                     "wmcao_rhs", "wmcao_apply_A"):
            getattr(L, name).argtypes = [vp, vp, vp, C.c_int, vp]
        L.wmcao_precond_diag.argtypes = [vp, vp, vp]
        L.wmcao_solve.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
        L.wmcao_solve_graph.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
        L.wmcao_solve_noalloc.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
        L.wmcao_solve_noalloc.restype = C.c_int
        for name in ("wmcao_solve_multi", "wmcao_solve_multi_graph"):
            getattr(L, name).argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                         C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int, vp]
        L.wmcao_profile_enable.argtypes = [vp, C.c_int]
        L.wmcao_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int),
                                         C.POINTER(C.c_double)]
        L.wmcao_serve_launch.argtypes = [vp, vp, vp, C.c_int, C.POINTER(vp), C.POINTER(vp), C.c_int,
                                         C.POINTER(C.c_int), C.POINTER(vp), C.c_int, vp]
        L.wmcao_serve_launch.restype = C.c_int
        L.wmcao_axpby.argtypes = [C.c_int, C.c_int64, C.c_double, vp, C.c_double, vp, vp, vp]
        L.wmcao_axpby.restype = C.c_int
        L.wmcao_plan_destroy.argtypes = [vp]
        L.wmcao_plan_destroy.restype = None
        L.wmcao_strerror.restype = C.c_char_p
        L.wmcao_strerror.argtypes = [C.c_int]
        L.wmcao_last_error.restype = C.c_char_p
        for name in ("wmcao_plan", "wmcao_sizes", "wmcao_coeffs_to_layers",
                     "wmcao_layers_to_coeffs", "wmcao_forward_layers", "wmcao_rhs",
                     "wmcao_apply_A", "wmcao_precond_diag", "wmcao_solve", "wmcao_solve_graph",
                     "wmcao_solve_multi", "wmcao_solve_multi_graph", "wmcao_profile_enable",
                     "wmcao_profile_read"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc, where):
    if rc != 0:
        msg = lib().wmcao_last_error().decode()
        raise WmcaoError(rc, where, msg)


EXPORTED = ("wmcao_plan", "wmcao_sizes", "wmcao_coeffs_to_layers", "wmcao_layers_to_coeffs",
            "wmcao_forward_layers", "wmcao_rhs", "wmcao_apply_A", "wmcao_precond_diag",
            "wmcao_solve", "wmcao_solve_noalloc", "wmcao_solve_multi", "wmcao_solve_multi_graph",
            "wmcao_solve_graph", "wmcao_serve_launch",
            "wmcao_profile_enable",
            "wmcao_profile_read", "wmcao_axpby", "wmcao_plan_destroy",
            "wmcao_strerror", "wmcao_last_error")
