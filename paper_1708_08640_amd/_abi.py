"""ctypes view of the C ABI in include/s3cmtf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libs3cmtf.so")

MAX_ORDER = 4
MAX_MATRICES = 4

S3_OK = 0
S3_ERR_INVALID_ARG = -1
S3_ERR_INDEX_RANGE = -2
S3_ERR_UNSUPPORTED = -3
S3_ERR_NONFINITE = -4
S3_ERR_HIP = -5
S3_ERR_WORKSPACE = -6
S3_ERR_STATE = -7

S3_F64, S3_F32, S3_BF16 = 0, 1, 2
S3_DET_MINIBATCH, S3_LOCKFREE = 0, 1
S3_DAMP_NONE, S3_DAMP_CURVATURE = 0, 1
S3_CONTRACT_REUSE, S3_CONTRACT_NAIVE, S3_CONTRACT_MATRIX = 0, 1, 2
S3_CORE_TUCKER, S3_CORE_CP = 0, 1

# every function the header declares
EXPORTS = [
    "s3_status_string", "s3_last_error", "s3_plan_create", "s3_plan_destroy", "s3_workspace_size",
    "s3_bind", "s3_epoch", "s3_det_batches", "s3_loss", "s3_rmse", "s3_predict", "s3_predict_noalloc", "s3_predict_matrix",
    "s3_backward", "s3_export", "s3_import", "s3_orthogonalize", "s3_init_params", "s3_set_profiling",
    "s3_last_epoch_profile",
]


class S3Desc(C.Structure):
    _fields_ = [
        ("order", C.c_int32), ("n_mat", C.c_int32),
        ("dims", C.c_int64 * MAX_ORDER), ("rank", C.c_int32 * MAX_ORDER),
        ("mat_mode", C.c_int32 * MAX_MATRICES), ("mat_cols", C.c_int64 * MAX_MATRICES),
        ("dtype", C.c_int32), ("damping", C.c_int32),
        ("eta0", C.c_double), ("mu", C.c_double), ("lambda_reg", C.c_double), ("lambda_m", C.c_double),
        ("batch", C.c_int64), ("round_items", C.c_int64), ("seed", C.c_uint64),
        ("hot_rows", C.c_int32), ("contraction", C.c_int32), ("core_kind", C.c_int32),
    ]


class S3Buffers(C.Structure):
    _fields_ = [
        ("x_idx", C.c_void_p), ("x_val", C.c_void_p), ("x_nnz", C.c_int64),
        ("t_idx", C.c_void_p), ("t_val", C.c_void_p), ("t_nnz", C.c_int64),
        ("y_row", C.c_void_p * MAX_MATRICES), ("y_col", C.c_void_p * MAX_MATRICES),
        ("y_val", C.c_void_p * MAX_MATRICES), ("y_nnz", C.c_int64 * MAX_MATRICES),
        ("U", C.c_void_p * MAX_ORDER), ("G", C.c_void_p), ("V", C.c_void_p * MAX_MATRICES),
        ("order", C.c_void_p),
    ]


class S3Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"s3cmtf status {status}: {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Load the in-tree HIP library; raise loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} is missing: build it with `python -m paper_1708_08640_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "s3_status_string": ([i32], C.c_char_p),
        "s3_last_error": ([vp, C.c_char_p, C.c_size_t], i32),
        "s3_plan_create": ([C.POINTER(S3Desc), C.POINTER(vp)], i32),
        "s3_plan_destroy": ([vp], i32),
        "s3_workspace_size": ([vp, i64, i64, C.POINTER(i64), C.POINTER(C.c_size_t)], i32),
        "s3_bind": ([vp, C.POINTER(S3Buffers), vp, C.c_size_t, vp], i32),
        "s3_epoch": ([vp, i32, i32, vp], i32),
        "s3_det_batches": ([vp, i64, i64, dbl, vp], i32),
        "s3_loss": ([vp, C.POINTER(dbl), vp], i32),
        "s3_rmse": ([vp, C.POINTER(dbl), vp], i32),
        "s3_predict": ([vp, vp, i64, vp, vp], i32),
        "s3_predict_noalloc": ([vp, vp, i64, vp, vp], i32),
        "s3_predict_matrix": ([vp, i32, vp, vp, i64, vp, vp], i32),
        "s3_backward": ([vp, vp, C.POINTER(vp), C.POINTER(vp), vp, C.POINTER(vp), vp], i32),
        "s3_export": ([vp, i32, i32, C.POINTER(dbl), C.c_size_t, vp], i32),
        "s3_import": ([vp, i32, i32, C.POINTER(dbl), C.c_size_t, vp], i32),
        "s3_orthogonalize": ([vp, vp], i32),
        "s3_init_params": ([vp, C.c_uint64, dbl, vp], i32),
        "s3_set_profiling": ([vp, i32], i32),
        "s3_last_epoch_profile": ([vp, C.POINTER(dbl), C.POINTER(i64)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return load().s3_status_string(st).decode()


def check(st: int, plan=None) -> None:
    if st == S3_OK:
        return
    msg = status_string(st)
    if plan:
        buf = C.create_string_buffer(512)
        load().s3_last_error(plan, buf, 512)
        if buf.value:
            msg += ": " + buf.value.decode()
    raise S3Error(st, msg)
