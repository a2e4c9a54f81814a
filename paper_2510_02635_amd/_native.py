"""ctypes binding of libfbsde.so (the C ABI of include/fbsde.h).  Argument marshalling only."""
import ctypes
import os

# FBSDE_LIB_PATH selects another build of the same library (the host-sanitized one, for instance)
_LIB_PATH = os.environ.get("FBSDE_LIB_PATH") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib",
                                                             "libfbsde.so")

F64, F32C = 0, 1
F_ZERO, F_ALLEN_CAHN, F_HJB, F_BURGERS, F_HJ_SINK, F_LOG_POT = 0, 1, 2, 3, 4, 5
G_QUAD, G_AC, G_HJB_LOG, G_AFFINE, G_LOGISTIC, G_HJ_GAUSS, G_CASE2 = 0, 1, 2, 3, 4, 5, 6
OK, EINVAL, ENOSPC, EHIP, ESTATE = 0, -1, -2, -3, -4
ST_CG_MAXIT, ST_NEWTON_FLAT, ST_NONFINITE, ST_WAIT_LIMIT = 1, 2, 4, 8
WS_TAPE = 1

EXPORTED = ("fbsde_state_ld", "fbsde_workspace_size", "fbsde_terminal", "fbsde_solve_step", "fbsde_solve",
            "fbsde_solve_backward", "fbsde_normals", "fbsde_box_muller", "fbsde_time_kernel", "fbsde_gemm", "fbsde_cholesky_workspace",
            "fbsde_cholesky_solve", "fbsde_batched_workspace_size", "fbsde_solve_batched",
            "fbsde_solve_batched_backward", "fbsde_graph_capture", "fbsde_graph_launch", "fbsde_graph_destroy",
            "fbsde_graph_capture_batched", "fbsde_autotune", "fbsde_autotune_reset", "fbsde_launch_timer", "fbsde_launch_timer_read", "fbsde_launch_timer_kinds",
            "fbsde_workspace_cg_rows", "fbsde_solve_noalloc", "fbsde_batched_cg_bytes",
            "fbsde_literal_workspace_size", "fbsde_literal_workspace_size_stored", "fbsde_literal_coef_workspace_size",
            "fbsde_solve_literal_coef", "fbsde_coef_workspace_size", "fbsde_solve_coef",
            "fbsde_sigma_workspace_size", "fbsde_solve_sigma", "fbsde_solve_sigma_backward",
            "fbsde_solve_coef_backward", "fbsde_solve_literal", "fbsde_strerror")


BATCH_TILED, BATCH_PERSISTENT = 0, 1
SOLVER_AUTO, SOLVER_CG = 0, 1


class CBatchOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("streams", ctypes.c_int32), ("tile_bytes", ctypes.c_int64),
                ("max_slots", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CTuneResult(ctypes.Structure):
    _fields_ = [("team", ctypes.c_int32), ("q", ctypes.c_int32), ("nchunk", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float)]


COEF_GEOMETRIC, COEF_AFFINE_DIAG = 1, 2


class CCoef(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mu0", ctypes.c_double),
                ("sigma0", ctypes.c_double), ("mu1", ctypes.c_double), ("sigma1", ctypes.c_double)]


class CProblem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int64), ("M", ctypes.c_int64), ("N", ctypes.c_int64),
        ("T", ctypes.c_double), ("s", ctypes.c_double),
        ("mu", ctypes.c_void_p),
        ("f_kind", ctypes.c_int32), ("g_kind", ctypes.c_int32),
        ("fp", ctypes.c_double * 4), ("gp", ctypes.c_double * 4),
        ("gvec", ctypes.c_void_p),
        ("eps_h", ctypes.c_double), ("ridge_rel", ctypes.c_double),
        ("newton_iters", ctypes.c_int32), ("cg_maxit", ctypes.c_int32),
        ("cg_rtol", ctypes.c_double),
        ("cg_fixed_iters", ctypes.c_int32), ("shared_dw", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("instance", ctypes.c_uint32), ("point_base", ctypes.c_uint32),
        ("prec", ctypes.c_int32), ("solver", ctypes.c_int32),
    ]


class FbsdeError(RuntimeError):
    pass


_lib = None


def lib_path():
    return _LIB_PATH


def load():
    """Load libfbsde.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise FbsdeError(f"{_LIB_PATH} is missing: build it with `python -m paper_2510_02635_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    pb = P(CProblem)
    lib.fbsde_state_ld.argtypes = [pb]
    lib.fbsde_state_ld.restype = i64
    lib.fbsde_workspace_size.argtypes = [pb, i64, i32, P(sz)]
    lib.fbsde_terminal.argtypes = [pb, i64, vp, vp, i64, vp, vp, vp]
    lib.fbsde_solve_step.argtypes = [pb, i64, i32, vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fbsde_solve.argtypes = [pb, i64, vp, vp, vp, vp, vp, sz, i32, vp, vp]
    lib.fbsde_solve_backward.argtypes = [pb, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp, vp]
    lib.fbsde_normals.argtypes = [pb, i64, i32, i64, i64, vp, vp, vp]
    lib.fbsde_time_kernel.argtypes = [pb, i64, i32, i32, vp, sz, P(ctypes.c_float), vp]
    lib.fbsde_box_muller.argtypes = [i32, i64, vp, vp, vp]
    lib.fbsde_launch_timer.argtypes = [i32]
    lib.fbsde_launch_timer_read.argtypes = [vp, vp, i64, P(i64)]
    lib.fbsde_launch_timer_kinds.argtypes = [vp, i64, P(i64)]
    lib.fbsde_workspace_cg_rows.argtypes = [vp, P(i64), vp]
    lib.fbsde_solve_noalloc.argtypes = [pb, i64, vp, vp, vp, vp, vp]
    lib.fbsde_batched_cg_bytes.argtypes = [pb, i64, vp, vp, i32, vp, P(ctypes.c_double), vp]
    lib.fbsde_gemm.argtypes = [i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, ctypes.c_double,
                               ctypes.c_double, vp]
    lib.fbsde_cholesky_workspace.argtypes = [i32, i64, i64]
    lib.fbsde_cholesky_workspace.restype = sz
    lib.fbsde_cholesky_solve.argtypes = [i32, i64, vp, i64, i64, vp, i64, vp, sz, P(i32), vp]
    lib.fbsde_batched_workspace_size.argtypes = [pb, i64, vp, vp, i32, P(sz)]
    lib.fbsde_solve_batched.argtypes = [pb, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fbsde_solve_batched_backward.argtypes = [pb, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fbsde_graph_capture.argtypes = [pb, i64, vp, vp, vp, vp, vp, sz, i32, P(vp), vp]
    lib.fbsde_graph_capture_batched.argtypes = [pb, i64, vp, vp, vp, vp, vp, vp, vp, sz, P(vp), vp]
    lib.fbsde_graph_launch.argtypes = [vp, vp]
    lib.fbsde_graph_destroy.argtypes = [vp]
    lib.fbsde_autotune.argtypes = [pb, i64, vp, vp, sz, P(CTuneResult), vp]
    lib.fbsde_autotune_reset.argtypes = []
    lib.fbsde_literal_workspace_size.argtypes = [pb, i64, P(sz)]
    lib.fbsde_literal_workspace_size_stored.argtypes = [pb, i64, P(sz)]
    lib.fbsde_solve_literal.argtypes = [pb, i64, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fbsde_literal_coef_workspace_size.argtypes = [pb, P(CCoef), i64, P(sz)]
    lib.fbsde_solve_literal_coef.argtypes = [pb, P(CCoef), i64, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fbsde_coef_workspace_size.argtypes = [pb, P(CCoef), i64, i32, P(sz)]
    lib.fbsde_sigma_workspace_size.argtypes = [pb, i64, i32, P(sz)]
    lib.fbsde_solve_sigma.argtypes = [pb, vp, i64, vp, vp, vp, vp, vp, sz, i32, vp, vp]
    lib.fbsde_solve_sigma_backward.argtypes = [pb, vp, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp, vp]
    lib.fbsde_solve_coef.argtypes = [pb, P(CCoef), i64, vp, vp, vp, vp, vp, sz, i32, vp, vp]
    lib.fbsde_solve_coef_backward.argtypes = [pb, P(CCoef), i64, vp, vp, vp, vp, vp, vp, vp, sz, vp, vp]
    lib.fbsde_strerror.argtypes = [ctypes.c_int]
    lib.fbsde_strerror.restype = ctypes.c_char_p
    for name in ("fbsde_workspace_size", "fbsde_terminal", "fbsde_solve_step", "fbsde_solve",
                 "fbsde_solve_backward", "fbsde_normals", "fbsde_box_muller", "fbsde_time_kernel", "fbsde_gemm",
                 "fbsde_cholesky_solve", "fbsde_batched_workspace_size", "fbsde_solve_batched",
                 "fbsde_solve_batched_backward", "fbsde_graph_capture", "fbsde_graph_capture_batched",
                 "fbsde_graph_launch",
                 "fbsde_graph_destroy", "fbsde_autotune", "fbsde_autotune_reset", "fbsde_literal_workspace_size",
                 "fbsde_launch_timer_read", "fbsde_launch_timer_kinds", "fbsde_literal_coef_workspace_size",
                 "fbsde_workspace_cg_rows", "fbsde_solve_noalloc", "fbsde_batched_cg_bytes",
                 "fbsde_literal_workspace_size_stored",
                 "fbsde_solve_literal_coef", "fbsde_coef_workspace_size", "fbsde_solve_coef",
                 "fbsde_sigma_workspace_size", "fbsde_solve_sigma", "fbsde_solve_sigma_backward",
                 "fbsde_solve_coef_backward",
                 "fbsde_solve_literal"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc):
    if rc != OK:
        raise FbsdeError(f"libfbsde: {load().fbsde_strerror(rc).decode()} (code {rc})")
    return rc
