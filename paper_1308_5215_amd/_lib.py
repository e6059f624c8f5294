"""ctypes binding of ``libadr.so`` (include/adr.h).  Argument marshalling
only: every step of the solver runs in the library's HIP kernels.  There is
no fallback: if the library is missing or does not load, importing this
module raises."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadr.so")

# Names and numbering of include/adr.h
OK, ERR_ARG, ERR_NOMEM, ERR_DEVICE, ERR_STATE = 0, -1, -2, -3, -4
MAXIT, BREAKDOWN_RHO, OMEGA_ZERO, ZERO_PIVOT, NONFINITE, INACCURATE = 1, 2, 3, 4, 5, 6
UPWIND, CENTERED = 0, 1
DIRICHLET, NEUMANN_XY = 0, 1
FP64, FP32_FACTORS, FP32_SWEEPS = 0, 1, 2

EXPORTS = [
    "adr_assemble", "adr_ilu0", "adr_bicgstab_solve", "adr_destroy", "adr_get_dia", "adr_set_dia",
    "adr_get_factors", "adr_spmv", "adr_precond", "adr_lsolve", "adr_usolve", "adr_dot", "adr_device_bytes",
    "adr_set_sweep_rows", "adr_status_str", "adr_last_error", "adr_batch_assemble", "adr_batch_layout",
    "adr_batch_ilu0", "adr_batch_solve", "adr_autotune", "adr_use_stencil_tables", "adr_stencil_tables",
    "adr_last_call_ms", "adr_workspace_bytes", "adr_bind_workspace", "adr_set_sweep_ring", "adr_sweep_ring",
    "adr_set_max_restarts", "adr_assemble_data", "adr_batch_assemble_data", "adr_max_error", "adr_classify",
    "adr_stream_copy", "adr_dot_noalloc",
    # include/adr_cnn.h
    "adr_cnn_param_count", "adr_cnn_create", "adr_cnn_destroy", "adr_cnn_set_params", "adr_cnn_get_params",
    "adr_cnn_forward", "adr_cnn_gradient", "adr_cnn_adam", "adr_cnn_train_step", "adr_cnn_features",
    "adr_batch_warm_start",
]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("hist_len", ctypes.c_int32),
                ("half_step", ctypes.c_int32), ("bnorm", ctypes.c_double),
                ("true_relres", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("restarts", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ProblemData(ctypes.Structure):
    """adr_problem_data: the caller's forcing and boundary data."""
    _fields_ = [("f", ctypes.c_void_p), ("f_len", ctypes.c_int64),
                ("u_x0", ctypes.c_void_p), ("u_x0_len", ctypes.c_int64),
                ("u_xX", ctypes.c_void_p), ("u_xX_len", ctypes.c_int64),
                ("u_y0", ctypes.c_void_p), ("u_y0_len", ctypes.c_int64),
                ("u_yY", ctypes.c_void_p), ("u_yY_len", ctypes.c_int64),
                ("f_on_device", ctypes.c_int32), ("pad", ctypes.c_int32)]


class InstanceClass(ctypes.Structure):
    """adr_instance_class."""
    _fields_ = [("pe_x", ctypes.c_double), ("pe_y", ctypes.c_double), ("g_y", ctypes.c_double),
                ("neg_offdiag", ctypes.c_int64), ("nonneg_diag", ctypes.c_int64),
                ("expect_fail", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


def load():
    """Load the HIP library (raises OSError if it is absent or broken)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError("libadr.so is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1308_5215_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    D = ctypes.POINTER(ctypes.c_double)
    L.adr_assemble.restype = ctypes.c_int
    L.adr_assemble.argtypes = [f64, f64, f64, i32, i32, i32, i32, P, f64, P, ctypes.POINTER(P)]
    L.adr_ilu0.restype = ctypes.c_int
    L.adr_ilu0.argtypes = [P, i32, ctypes.POINTER(i64)]
    L.adr_bicgstab_solve.restype = ctypes.c_int
    L.adr_bicgstab_solve.argtypes = [P, f64, i32, P, P, D, D, ctypes.POINTER(SolveInfo)]
    L.adr_destroy.restype = None
    L.adr_destroy.argtypes = [P]
    L.adr_get_dia.restype = ctypes.c_int
    L.adr_get_dia.argtypes = [P] + [D] * 6
    L.adr_set_dia.restype = ctypes.c_int
    L.adr_set_dia.argtypes = [P] + [D] * 6
    L.adr_get_factors.restype = ctypes.c_int
    L.adr_get_factors.argtypes = [P] + [D] * 3
    L.adr_spmv.restype = ctypes.c_int
    L.adr_spmv.argtypes = [P, P, P]
    L.adr_precond.restype = ctypes.c_int
    L.adr_precond.argtypes = [P, P, P]
    for nm in ("adr_lsolve", "adr_usolve"):
        getattr(L, nm).restype = ctypes.c_int
        getattr(L, nm).argtypes = [P, P, P]
    L.adr_dot.restype = ctypes.c_int
    L.adr_dot.argtypes = [P, P, i64, P, D]
    L.adr_device_bytes.restype = ctypes.c_size_t
    L.adr_device_bytes.argtypes = [P]
    L.adr_set_sweep_rows.restype = ctypes.c_int
    L.adr_set_sweep_rows.argtypes = [P, i32]
    L.adr_set_sweep_ring.restype = ctypes.c_int
    L.adr_set_sweep_ring.argtypes = [P, i32]
    L.adr_sweep_ring.restype = ctypes.c_int32
    L.adr_sweep_ring.argtypes = [P]
    L.adr_use_stencil_tables.restype = ctypes.c_int
    L.adr_use_stencil_tables.argtypes = [P, i32]
    L.adr_stencil_tables.restype = ctypes.c_int32
    L.adr_stencil_tables.argtypes = [P]
    L.adr_last_call_ms.restype = ctypes.c_double
    L.adr_last_call_ms.argtypes = [P]
    L.adr_workspace_bytes.restype = ctypes.c_size_t
    L.adr_workspace_bytes.argtypes = [P, i32]
    L.adr_bind_workspace.restype = ctypes.c_int
    L.adr_bind_workspace.argtypes = [P, P, ctypes.c_size_t]
    I32P = ctypes.POINTER(ctypes.c_int32)
    I64P = ctypes.POINTER(ctypes.c_int64)
    L.adr_batch_assemble.restype = ctypes.c_int
    L.adr_batch_assemble.argtypes = [i32, D, D, D, I32P, I32P, I32P, I32P, P, f64, P, ctypes.POINTER(P)]
    L.adr_batch_layout.restype = ctypes.c_int
    L.adr_batch_layout.argtypes = [P, I32P, I64P]
    L.adr_batch_ilu0.restype = ctypes.c_int
    L.adr_batch_ilu0.argtypes = [P, i32, I64P]
    L.adr_batch_solve.restype = ctypes.c_int
    L.adr_batch_solve.argtypes = [P, f64, i32, P, P, D, D, ctypes.POINTER(SolveInfo)]
    L.adr_autotune.restype = ctypes.c_int
    L.adr_autotune.argtypes = [P, I32P, D]
    F32P = ctypes.POINTER(ctypes.c_float)
    f32 = ctypes.c_float
    L.adr_cnn_param_count.restype = i64
    L.adr_cnn_param_count.argtypes = []
    L.adr_cnn_create.restype = ctypes.c_int
    L.adr_cnn_create.argtypes = [i32, i32, i32, P, ctypes.POINTER(P)]
    L.adr_cnn_destroy.restype = None
    L.adr_cnn_destroy.argtypes = [P]
    L.adr_cnn_set_params.restype = ctypes.c_int
    L.adr_cnn_set_params.argtypes = [P, F32P]
    L.adr_cnn_get_params.restype = ctypes.c_int
    L.adr_cnn_get_params.argtypes = [P, F32P]
    L.adr_cnn_forward.restype = ctypes.c_int
    L.adr_cnn_forward.argtypes = [P, P, i32, P]
    L.adr_cnn_gradient.restype = ctypes.c_int
    L.adr_cnn_gradient.argtypes = [P, P, P, i32, P, F32P, D]
    L.adr_cnn_adam.restype = ctypes.c_int
    L.adr_cnn_adam.argtypes = [P, f32, f32, f32, f32]
    L.adr_cnn_train_step.restype = ctypes.c_int
    L.adr_cnn_train_step.argtypes = [P, P, P, i32, f32, D]
    L.adr_cnn_features.restype = ctypes.c_int
    L.adr_cnn_features.argtypes = [P, i32, i32, P]
    L.adr_batch_warm_start.restype = ctypes.c_int
    L.adr_batch_warm_start.argtypes = [P, P, P, I32P]
    L.adr_set_max_restarts.restype = ctypes.c_int
    L.adr_set_max_restarts.argtypes = [P, i32]
    L.adr_assemble_data.restype = ctypes.c_int
    L.adr_assemble_data.argtypes = [f64, f64, f64, i32, i32, i32, i32, ctypes.POINTER(ProblemData), P,
                                    ctypes.POINTER(P)]
    L.adr_batch_assemble_data.restype = ctypes.c_int
    L.adr_batch_assemble_data.argtypes = [i32, D, D, D, I32P, I32P, I32P, I32P, ctypes.POINTER(ProblemData), P,
                                          ctypes.POINTER(P)]
    L.adr_max_error.restype = ctypes.c_int
    L.adr_max_error.argtypes = [P, P, D]
    L.adr_classify.restype = ctypes.c_int
    L.adr_classify.argtypes = [f64, f64, f64, i32, i32, i32, i32, f64, ctypes.POINTER(InstanceClass)]
    L.adr_stream_copy.restype = ctypes.c_int
    L.adr_stream_copy.argtypes = [P, P, i64, P]
    L.adr_dot_noalloc.restype = ctypes.c_int
    L.adr_dot_noalloc.argtypes = [P, P, i64, P, P]
    L.adr_status_str.restype = ctypes.c_char_p
    L.adr_status_str.argtypes = [i32]
    L.adr_last_error.restype = ctypes.c_char_p
    L.adr_last_error.argtypes = []
    _lib = L
    return L


class AdrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (load().adr_status_str(status).decode(), status, msg))
        self.status = status


def check(status):
    """Raise AdrError on a call error (negative status); return outcomes."""
    if status < 0:
        raise AdrError(status, load().adr_last_error().decode())
    return status
