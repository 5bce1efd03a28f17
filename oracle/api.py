"""ctypes marshalling for the FP64 oracle in ``s3_oracle.c`` (test infrastructure)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "s3_oracle.c")
_LIB = os.path.join(_HERE, "libs3oracle.so")
MAXN = 8
MAXM = 8

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


class _Model(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("M", C.c_int32),
        ("dims", C.c_int64 * MAXN), ("J", C.c_int32 * MAXN),
        ("U", _dp * MAXN), ("G", _dp),
        ("mode", C.c_int32 * MAXM), ("cols", C.c_int64 * MAXM),
        ("V", _dp * MAXM), ("cp", C.c_int32),
    ]


class _Tensor(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("idx", _i32p), ("val", _dp)]


class _Matrix(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("row", _i32p), ("col", _i32p), ("val", _dp)]


class _Counts(C.Structure):
    _fields_ = [("nX", C.c_int64), ("cnt", _i64p * MAXN), ("cntV", _i64p * MAXM)]


class _Hyper(C.Structure):
    _fields_ = [("lambda_reg", C.c_double), ("lambda_m", C.c_double)]


def _sanitized() -> bool:
    # S3_ORACLE_SANITIZE=1: load a build instrumented with AddressSanitizer and
    # UndefinedBehaviorSanitizer (the process must preload gcc's libasan)
    return os.environ.get("S3_ORACLE_SANITIZE") == "1"


def lib_path() -> str:
    """The oracle library this process loads (the sanitized build when
    S3_ORACLE_SANITIZE=1)."""
    return os.path.join(_HERE, "libs3oracle_san.so") if _sanitized() else _LIB


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math; with
    S3_ORACLE_SANITIZE=1 a separate ASan/UBSan build, stopping at the first
    report)."""
    lib, flags = lib_path(), ["-O2"]
    if _sanitized():
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=all"]
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *flags, "-std=c11", "-fPIC", "-shared", "-Wall", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        M, T, Y, Cn, H = (C.POINTER(_Model), C.POINTER(_Tensor), C.POINTER(_Matrix),
                          C.POINTER(_Counts), C.POINTER(_Hyper))
        lib.or_counts_build.argtypes = [M, T, C.c_int32, Y, Cn]
        lib.or_predict_one.argtypes = [M, _i32p]
        lib.or_predict_one.restype = C.c_double
        lib.or_predict.argtypes = [M, T, _dp]
        lib.or_tensor_item_grad.argtypes = [M, _i32p, C.c_double, _dp, C.c_double, _dp, _dp]
        lib.or_tensor_item_grad.restype = C.c_double
        lib.or_tensor_item_grad_opt.argtypes = [M, _i32p, C.c_double, _dp, C.c_double, _dp, _dp, _dp]
        lib.or_tensor_item_grad_opt.restype = C.c_double
        lib.or_matrix_item_grad.argtypes = [_dp, _dp, C.c_int32, C.c_double, C.c_double,
                                            C.c_double, _dp, _dp]
        lib.or_matrix_item_grad.restype = C.c_double
        lib.or_sgd_epoch.argtypes = [M, T, C.c_int32, Y, Cn, H, _i64p, C.c_int64, C.c_double]
        lib.or_sgd_epoch.restype = C.c_int64
        lib.or_minibatch_epoch.argtypes = [M, T, C.c_int32, Y, Cn, H, _i64p, C.c_int64,
                                           C.c_int64, C.c_double, C.c_int64, C.c_int64, C.c_int32]
        lib.or_minibatch_epoch_mt.argtypes = [M, T, C.c_int32, Y, Cn, H, _i64p, C.c_int64,
                                              C.c_int64, C.c_double, C.c_int64, C.c_int64, C.c_int32,
                                              C.c_int32]
        lib.or_minibatch_epoch_mt.restype = C.c_int64
        lib.or_tensor_item_w.argtypes = [M, _i32p, _dp]
        lib.or_minibatch_epoch.restype = C.c_int64
        lib.or_loss.argtypes = [M, T, C.c_int32, Y, Cn, H, _dp]
        lib.or_rmse.argtypes = [M, T]
        lib.or_rmse.restype = C.c_double
        lib.or_full_grad.argtypes = [M, T, C.c_int32, Y, Cn, H, C.POINTER(_dp), _dp, C.POINTER(_dp)]
        lib.or_adjoint.argtypes = [M, T, _dp, C.c_int32, Y, C.POINTER(_dp), C.POINTER(_dp), _dp,
                                   C.POINTER(_dp)]
        lib.or_matrix_predict.argtypes = [M, C.c_int32, Y, _dp]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


@dataclass
class Params:
    """Model parameters in float64: U[n] (I_n x J_n), G (J_1 x .. x J_N, C order),
    V[m] (K_m x J_{c_m}); ``modes[m]`` is the tensor mode matrix m couples to.
    cp: hyper-diagonal core (every J_n = J, G holds the J diagonal values)."""
    U: List[np.ndarray]
    G: np.ndarray
    V: List[np.ndarray]
    modes: List[int]
    cp: bool = False

    @classmethod
    def from_arrays(cls, U, G, V, modes, cp: bool = False):
        return cls([_f64(u).copy() for u in U], _f64(G).copy(), [_f64(v).copy() for v in V],
                   [int(c) for c in modes], bool(cp))

    def copy(self) -> "Params":
        return Params.from_arrays(self.U, self.G, self.V, self.modes, self.cp)

    def _model(self) -> _Model:
        md = _Model()
        md.N = len(self.U)
        md.M = len(self.V)
        for n, u in enumerate(self.U):
            assert u.dtype == np.float64 and u.flags.c_contiguous
            md.dims[n] = u.shape[0]
            md.J[n] = u.shape[1]
            md.U[n] = _ptr(u, _dp)
        if self.cp:
            J = self.U[0].shape[1]
            assert all(u.shape[1] == J for u in self.U) and tuple(self.G.shape) == (J,)
            md.cp = 1
        else:
            assert tuple(self.G.shape) == tuple(u.shape[1] for u in self.U)
        assert self.G.dtype == np.float64 and self.G.flags.c_contiguous
        md.G = _ptr(self.G, _dp)
        for m, v in enumerate(self.V):
            assert v.dtype == np.float64 and v.flags.c_contiguous
            md.mode[m] = self.modes[m]
            md.cols[m] = v.shape[0]
            md.V[m] = _ptr(v, _dp)
        return md


class _Data:
    """Keeps the C structs and the arrays they point into alive together."""

    def __init__(self, idx, val, mats):
        self.idx = _i32(idx)
        self.val = _f64(val)
        self.X = _Tensor(self.val.shape[0], _ptr(self.idx, _i32p), _ptr(self.val, _dp))
        self.keep = []
        Ys = (_Matrix * max(1, len(mats)))()
        for m, (r, c, v) in enumerate(mats):
            r, c, v = _i32(r), _i32(c), _f64(v)
            self.keep += [r, c, v]
            Ys[m] = _Matrix(v.shape[0], _ptr(r, _i32p), _ptr(c, _i32p), _ptr(v, _dp))
        self.Y = Ys
        self.M = len(mats)


def _mats(problem):
    return [(problem.mat_row[m], problem.mat_col[m], problem.mat_val[m])
            for m in range(len(problem.mat_val))]


class _CountsHolder:
    def __init__(self, params: Params, data: _Data):
        md = params._model()
        self.cnt = [np.zeros(u.shape[0], dtype=np.int64) for u in params.U]
        self.cntV = [np.zeros(v.shape[0], dtype=np.int64) for v in params.V]
        self.c = _Counts()
        for n, a in enumerate(self.cnt):
            self.c.cnt[n] = _ptr(a, _i64p)
        for m, a in enumerate(self.cntV):
            self.c.cntV[m] = _ptr(a, _i64p)
        _L().or_counts_build(C.byref(md), C.byref(data.X), data.M, data.Y, C.byref(self.c))


def counts(params: Params, problem):
    """|Omega_X^{n,i}| per mode and |Omega_Y^{2,k}| per matrix, over the training split."""
    d = _Data(problem.train_idx, problem.train_val, _mats(problem))
    ch = _CountsHolder(params, d)
    return ch.cnt, ch.cntV


def predict(params: Params, idx) -> np.ndarray:
    """Eq (4) for every entry of ``idx`` (int [N, nnz])."""
    idx = _i32(idx)
    d = _Data(idx, np.zeros(idx.shape[1]), [])
    out = np.empty(idx.shape[1])
    md = params._model()
    _L().or_predict(C.byref(md), C.byref(d.X), _ptr(out, _dp))
    return out


def matrix_predict(params: Params, m: int, row, col) -> np.ndarray:
    row, col = _i32(row), _i32(col)
    val = np.zeros(row.shape[0])
    y = _Matrix(row.shape[0], _ptr(row, _i32p), _ptr(col, _i32p), _ptr(val, _dp))
    out = np.empty(row.shape[0])
    md = params._model()
    _L().or_matrix_predict(C.byref(md), m, C.byref(y), _ptr(out, _dp))
    return out


def tensor_item_grad(params: Params, rows, x, reg_row, reg_core):
    """Eq (8) for one tensor entry: returns (e, [dU_n rows], dG)."""
    md = params._model()
    rows = _i32(rows)
    reg_row = _f64(reg_row)
    Js = [u.shape[1] for u in params.U]
    gU = np.empty(sum(Js))
    gG = np.empty(params.G.size)
    e = _L().or_tensor_item_grad(C.byref(md), _ptr(rows, _i32p), float(x), _ptr(reg_row, _dp),
                                 float(reg_core), _ptr(gU, _dp), _ptr(gG, _dp))
    return e, np.split(gU, np.cumsum(Js)[:-1]), gG.reshape(params.G.shape)


def tensor_item_grad_opt(params: Params, rows, x, reg_row, reg_core):
    """Algorithm 3 (intermediate tensor S, Collapse, elementwise division)."""
    md = params._model()
    rows = _i32(rows)
    reg_row = _f64(reg_row)
    Js = [u.shape[1] for u in params.U]
    gU = np.empty(sum(Js))
    gG = np.empty(params.G.size)
    S = np.empty(params.G.size)
    e = _L().or_tensor_item_grad_opt(C.byref(md), _ptr(rows, _i32p), float(x), _ptr(reg_row, _dp),
                                     float(reg_core), _ptr(gU, _dp), _ptr(gG, _dp), _ptr(S, _dp))
    return e, np.split(gU, np.cumsum(Js)[:-1]), gG.reshape(params.G.shape), S.reshape(params.G.shape)


def tensor_item_w(params: Params, rows):
    """Leave-one-out contractions G x_{-n} {u} of one entry (Eq 3 / Eq 8)."""
    md = params._model()
    rows = _i32(rows)
    Js = [u.shape[1] for u in params.U]
    w = np.empty(sum(Js))
    _L().or_tensor_item_w(C.byref(md), _ptr(rows, _i32p), _ptr(w, _dp))
    return np.split(w, np.cumsum(Js)[:-1])


def matrix_item_grad(u, v, y, lambda_m, reg_v):
    u, v = _f64(u), _f64(v)
    gu, gv = np.empty_like(u), np.empty_like(v)
    e = _L().or_matrix_item_grad(_ptr(u, _dp), _ptr(v, _dp), u.shape[0], float(y), float(lambda_m),
                                 float(reg_v), _ptr(gu, _dp), _ptr(gv, _dp))
    return e, gu, gv


def eta_at(eta0: float, mu: float, epoch: int) -> float:
    """Learning-rate decay of Algorithm 1: eta_t = eta0 / (1 + mu t), epoch t = 0, 1, ..."""
    return eta0 / (1.0 + mu * epoch)


class _Run:
    def __init__(self, params: Params, problem, lambda_reg, lambda_m):
        self.d = _Data(problem.train_idx, problem.train_val, _mats(problem))
        self.ch = _CountsHolder(params, self.d)
        self.h = _Hyper(float(lambda_reg), float(lambda_m))
        self.md = params._model()


def _hyper(problem, lambda_reg, lambda_m):
    cfg = problem.cfg
    return (cfg.lambda_reg if lambda_reg is None else lambda_reg,
            cfg.lambda_m if lambda_m is None else lambda_m)


def sgd_epoch(params: Params, problem, order, eta: float, lambda_reg=None, lambda_m=None) -> None:
    """Algorithm 1, one pass over ``order`` (item ids), one worker. In place."""
    lr, lm = _hyper(problem, lambda_reg, lambda_m)
    r = _Run(params, problem, lr, lm)
    order = np.ascontiguousarray(order, dtype=np.int64)
    _L().or_sgd_epoch(C.byref(r.md), C.byref(r.d.X), r.d.M, r.d.Y, C.byref(r.ch.c), C.byref(r.h),
                      _ptr(order, _i64p), order.shape[0], float(eta))


def minibatch_epoch(params: Params, problem, order, batch: int, eta: float, first_batch: int = 0,
                    n_batches: int = -1, lambda_reg=None, lambda_m=None, damping: bool = False,
                    threads: int = 1) -> int:
    """Deterministic mini-batch pass (batch-start gradients summed, then applied,
    optionally with the curvature damping of each block's step). In place.
    threads > 1: the items' gradients are evaluated by that many threads and
    summed in the same order (bitwise the same result)."""
    lr, lm = _hyper(problem, lambda_reg, lambda_m)
    r = _Run(params, problem, lr, lm)
    order = np.ascontiguousarray(order, dtype=np.int64)
    args = (C.byref(r.md), C.byref(r.d.X), r.d.M, r.d.Y, C.byref(r.ch.c), C.byref(r.h), _ptr(order, _i64p),
            order.shape[0], int(batch), float(eta), int(first_batch), int(n_batches), int(bool(damping)))
    if threads > 1:
        return int(_L().or_minibatch_epoch_mt(*args, int(threads)))
    return int(_L().or_minibatch_epoch(*args))


def loss(params: Params, problem, lambda_reg=None, lambda_m=None):
    """Eq (7): returns (f, f_t, f_m)."""
    lr, lm = _hyper(problem, lambda_reg, lambda_m)
    r = _Run(params, problem, lr, lm)
    out = np.empty(3)
    _L().or_loss(C.byref(r.md), C.byref(r.d.X), r.d.M, r.d.Y, C.byref(r.ch.c), C.byref(r.h),
                 _ptr(out, _dp))
    return float(out[0]), float(out[1]), float(out[2])


def rmse(params: Params, idx, val) -> float:
    """Held-out RMSE over the entries (idx, val)."""
    d = _Data(idx, val, [])
    md = params._model()
    return float(_L().or_rmse(C.byref(md), C.byref(d.X)))


def full_grad(params: Params, problem, lambda_reg=None, lambda_m=None):
    """Sum of all per-entry gradients: returns (dU list, dG, dV list)."""
    lr, lm = _hyper(problem, lambda_reg, lambda_m)
    r = _Run(params, problem, lr, lm)
    dU = [np.zeros_like(u) for u in params.U]
    dV = [np.zeros_like(v) for v in params.V]
    dG = np.zeros_like(params.G)
    pU = (_dp * MAXN)(*[_ptr(a, _dp) for a in dU])
    pV = (_dp * MAXM)(*[_ptr(a, _dp) for a in dV])
    _L().or_full_grad(C.byref(r.md), C.byref(r.d.X), r.d.M, r.d.Y, C.byref(r.ch.c), C.byref(r.h),
                      pU, _ptr(dG, _dp), pV)
    return dU, dG, dV


def adjoint(params: Params, idx, gx, mats: Sequence, gy: Sequence):
    """Transpose of the prediction map: returns (dU list, dG, dV list).

    ``mats`` is a list of (row, col) per coupled matrix, ``gy`` the matching
    upstream sensitivities."""
    idx = _i32(idx)
    gx = _f64(gx)
    d = _Data(idx, np.zeros(idx.shape[1]), [(r, c, np.zeros(len(r))) for (r, c) in mats])
    gys = [_f64(g) for g in gy]
    pgy = (_dp * MAXM)(*[_ptr(a, _dp) for a in gys])
    dU = [np.zeros_like(u) for u in params.U]
    dV = [np.zeros_like(v) for v in params.V]
    dG = np.zeros_like(params.G)
    pU = (_dp * MAXN)(*[_ptr(a, _dp) for a in dU])
    pV = (_dp * MAXM)(*[_ptr(a, _dp) for a in dV])
    md = params._model()
    _L().or_adjoint(C.byref(md), C.byref(d.X), _ptr(gx, _dp), d.M, d.Y, pgy, pU, _ptr(dG, _dp), pV)
    return dU, dG, dV


def qr_orthogonalize(params: Params) -> Params:
    """Algorithm 1's closing step: U^(n) = Q R, U^(n) <- Q, G <- G x_n R, and for
    every coupled matrix on mode c, V <- V R^(c)T.  numpy's Householder QR serves
    as the factorisation primitive.  Returns a new Params."""
    if params.cp:
        raise ValueError("the QR step transforms the core densely; it does not apply to a hyper-diagonal core")
    out = params.copy()
    Rs = []
    for n, u in enumerate(params.U):
        q, r = np.linalg.qr(u, mode="reduced")
        out.U[n] = np.ascontiguousarray(q)
        Rs.append(r)
    G = params.G.copy()
    for n, r in enumerate(Rs):
        # mode-n product G x_n R: contract the n-th core index with R's columns
        G = np.moveaxis(np.tensordot(r, G, axes=([1], [n])), 0, n)
    out.G = np.ascontiguousarray(G)
    for m, v in enumerate(params.V):
        out.V[m] = np.ascontiguousarray(v @ Rs[params.modes[m]].T)
    return out
