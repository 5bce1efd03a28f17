"""Python front end of the C ABI: device buffers come from torch, every step
of the computation runs in the HIP library."""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import check, load

# bf16: FP32 values and parameters (the master copies), BF16 contraction
# operands on the matrix cores
_DTYPES = {"f64": (_abi.S3_F64, torch.float64), "f32": (_abi.S3_F32, torch.float32),
           "bf16": (_abi.S3_BF16, torch.float32)}
_CONTRACTIONS = {"reuse": _abi.S3_CONTRACT_REUSE, "naive": _abi.S3_CONTRACT_NAIVE,
                 "matrix": _abi.S3_CONTRACT_MATRIX}
_MODES = {"det": _abi.S3_DET_MINIBATCH, "lockfree": _abi.S3_LOCKFREE}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class S3Plan:
    """One bound factorisation problem on one GPU.

    Parameters (``U``, ``G``, ``V``) are torch tensors on the device, updated
    in place by :meth:`epoch`; inputs are copied to the device once.
    """

    def __init__(self, dims: Sequence[int], ranks: Sequence[int], matrices: Sequence[Tuple[int, int]] = (),
                 dtype: str = "f32", eta0: float = 0.01, mu: float = 0.1, lambda_reg: float = 0.01,
                 lambda_m: float = 10.0, batch: int = 65536, round_items: int = 65536, damping: bool = False,
                 seed: int = 0, device: str = "cuda", hot_rows: int = 0, contraction: str = "reuse",
                 core: str = "tucker"):
        self.lib = load()
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be one of {list(_DTYPES)}")
        self.dtype_code, self.tdtype = _DTYPES[dtype]
        self.dtype = dtype
        self.device = torch.device(device)
        self.dims = [int(d) for d in dims]
        self.ranks = [int(r) for r in ranks]
        self.matrices = [(int(c), int(k)) for c, k in matrices]
        d = _abi.S3Desc()
        d.order = len(self.dims)
        d.n_mat = len(self.matrices)
        for n, (I, J) in enumerate(zip(self.dims, self.ranks)):
            d.dims[n] = I
            d.rank[n] = J
        for m, (c, k) in enumerate(self.matrices):
            d.mat_mode[m] = c
            d.mat_cols[m] = k
        d.dtype = self.dtype_code
        d.damping = _abi.S3_DAMP_CURVATURE if damping else _abi.S3_DAMP_NONE
        d.eta0, d.mu, d.lambda_reg, d.lambda_m = eta0, mu, lambda_reg, lambda_m
        d.batch = int(batch)
        d.round_items = int(round_items)
        d.seed = int(seed)
        d.hot_rows = int(hot_rows)
        if contraction not in _CONTRACTIONS:
            raise ValueError(f"contraction must be one of {list(_CONTRACTIONS)}")
        d.contraction = _CONTRACTIONS[contraction]
        if core not in ("tucker", "cp"):
            raise ValueError("core must be 'tucker' or 'cp'")
        d.core_kind = _abi.S3_CORE_CP if core == "cp" else _abi.S3_CORE_TUCKER
        self.core = core
        self.desc = d
        h = C.c_void_p()
        check(self.lib.s3_plan_create(C.byref(d), C.byref(h)))
        self.h = h
        self.bound = False
        self._keep = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                self.lib.s3_plan_destroy(h)
            except Exception:
                pass
            self.h = None

    # ------------------------------------------------------------ binding

    def workspace_bytes(self, x_nnz: int, t_nnz: int, y_nnz: Sequence[int]) -> int:
        arr = (C.c_int64 * max(1, len(y_nnz)))(*y_nnz)
        out = C.c_size_t()
        check(self.lib.s3_workspace_size(self.h, int(x_nnz), int(t_nnz), arr, C.byref(out)), self.h)
        return int(out.value)

    def _dev(self, a, dtype) -> torch.Tensor:
        t = torch.as_tensor(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else torch.as_tensor(a)
        return t.to(device=self.device, dtype=dtype).contiguous()

    def bind(self, train_idx, train_val, test_idx, test_val, mats: Sequence, U, G, V, order=None) -> None:
        """Copy the entries to the device, take the parameters (copied to the device
        in the compute dtype) and bind everything plus a workspace to the plan."""
        f = self.tdtype
        self.x_idx = self._dev(train_idx, torch.int32)
        self.x_val = self._dev(train_val, f)
        self.t_idx = self._dev(test_idx, torch.int32)
        self.t_val = self._dev(test_val, f)
        self.y = [(self._dev(r, torch.int32), self._dev(c, torch.int32), self._dev(v, f)) for (r, c, v) in mats]
        self.U = [self._dev(u, f) for u in U]
        self.G = self._dev(G, f)
        self.V = [self._dev(v, f) for v in V]
        self.order = None if order is None else self._dev(order, torch.int32)
        b = _abi.S3Buffers()
        b.x_idx, b.x_val, b.x_nnz = self.x_idx.data_ptr(), self.x_val.data_ptr(), self.x_val.numel()
        b.t_idx = self.t_idx.data_ptr() if self.t_val.numel() else None
        b.t_val = self.t_val.data_ptr() if self.t_val.numel() else None
        b.t_nnz = self.t_val.numel()
        for m, (r, c, v) in enumerate(self.y):
            b.y_row[m] = r.data_ptr() if v.numel() else None
            b.y_col[m] = c.data_ptr() if v.numel() else None
            b.y_val[m] = v.data_ptr() if v.numel() else None
            b.y_nnz[m] = v.numel()
        for n, u in enumerate(self.U):
            b.U[n] = u.data_ptr()
        b.G = self.G.data_ptr()
        for m, v in enumerate(self.V):
            b.V[m] = v.data_ptr()
        b.order = None if self.order is None else self.order.data_ptr()
        nbytes = self.workspace_bytes(b.x_nnz, b.t_nnz, [v.numel() for (_, _, v) in self.y])
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.buffers = b
        check(self.lib.s3_bind(self.h, C.byref(b), C.c_void_p(self.ws.data_ptr()), nbytes, _stream()), self.h)
        self.bound = True
        self.n_items = b.x_nnz + sum(v.numel() for (_, _, v) in self.y)

    @classmethod
    def from_problem(cls, problem, params, dtype: str = "f32", batch: int = 65536, order=None,
                     damping: bool = False, round_items: int = 65536, seed: int = 0, device: str = "cuda",
                     hot_rows: int = 0, contraction: str = "reuse", core: str = "tucker", **hyper) -> "S3Plan":
        """Plan for a generated problem (see ``synth``) with initial (U, G, V)."""
        cfg = problem.cfg
        U, G, V = params
        kw = dict(eta0=cfg.eta0, mu=cfg.mu, lambda_reg=cfg.lambda_reg, lambda_m=cfg.lambda_m)
        kw.update(hyper)
        p = cls(cfg.dims, cfg.ranks, [(s.mode, s.cols) for s in cfg.matrices], dtype=dtype, batch=batch,
                round_items=round_items, damping=damping, seed=seed, device=device, hot_rows=hot_rows,
                contraction=contraction, core=core, **kw)
        mats = [(problem.mat_row[m], problem.mat_col[m], problem.mat_val[m]) for m in range(len(problem.mat_val))]
        p.bind(problem.train_idx, problem.train_val, problem.test_idx, problem.test_val, mats, U, G, V, order)
        return p

    # ------------------------------------------------------------ training

    def epoch(self, epoch: int, mode: str = "det") -> None:
        check(self.lib.s3_epoch(self.h, int(epoch), _MODES[mode], _stream()), self.h)

    def det_batches(self, first: int, count: int, eta: float) -> None:
        check(self.lib.s3_det_batches(self.h, int(first), int(count), float(eta), _stream()), self.h)

    def n_batches(self) -> int:
        return (self.n_items + self.desc.batch - 1) // self.desc.batch

    def set_profiling(self, on: bool) -> None:
        check(self.lib.s3_set_profiling(self.h, 1 if on else 0), self.h)

    def last_epoch_profile(self):
        ms = C.c_double()
        n = C.c_int64()
        check(self.lib.s3_last_epoch_profile(self.h, C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value

    # ------------------------------------------------------------ evaluation

    def loss(self):
        out = (C.c_double * 3)()
        check(self.lib.s3_loss(self.h, out, _stream()), self.h)
        return out[0], out[1], out[2]

    def rmse(self) -> float:
        out = C.c_double()
        check(self.lib.s3_rmse(self.h, C.byref(out), _stream()), self.h)
        return out.value

    def predict(self, idx) -> torch.Tensor:
        idx = self._dev(idx, torch.int32)
        out = torch.empty(idx.shape[1], dtype=self.tdtype, device=self.device)
        check(self.lib.s3_predict(self.h, _ptr(idx), idx.shape[1], _ptr(out), _stream()), self.h)
        return out

    def predict_noalloc(self, idx: torch.Tensor, out: torch.Tensor) -> None:
        """s3_predict_noalloc: predictions of the device entries idx (int32
        [N, nnz]) into out, with no device memory taken from the workspace or
        allocated (the library's static scratch array instead)."""
        check(self.lib.s3_predict_noalloc(self.h, _ptr(idx), idx.shape[1], _ptr(out), _stream()), self.h)

    def predict_matrix(self, m: int, row, col) -> torch.Tensor:
        row = self._dev(row, torch.int32)
        col = self._dev(col, torch.int32)
        out = torch.empty(row.numel(), dtype=self.tdtype, device=self.device)
        check(self.lib.s3_predict_matrix(self.h, int(m), _ptr(row), _ptr(col), row.numel(), _ptr(out), _stream()),
              self.h)
        return out

    def backward(self, gx: Optional[torch.Tensor], gy: Sequence[Optional[torch.Tensor]] = ()):
        """Adjoint of (x~ over training entries, y^ over each matrix's entries)."""
        dU = [torch.empty_like(u) for u in self.U]
        dG = torch.empty_like(self.G)
        dV = [torch.empty_like(v) for v in self.V]
        gx_c = None if gx is None else gx.to(self.tdtype).contiguous()
        gy_c = [None if (g is None) else g.to(self.tdtype).contiguous() for g in gy]
        gy_c += [None] * (len(self.V) - len(gy_c))
        pU = (C.c_void_p * _abi.MAX_ORDER)(*[u.data_ptr() for u in dU])
        pV = (C.c_void_p * _abi.MAX_MATRICES)(*[v.data_ptr() for v in dV])
        pgy = (C.c_void_p * _abi.MAX_MATRICES)(*[(g.data_ptr() if g is not None else None) for g in gy_c])
        check(self.lib.s3_backward(self.h, _ptr(gx_c), pgy, pU, _ptr(dG), pV, _stream()), self.h)
        return dU, dG, dV

    def export(self, which: str, index: int = 0) -> np.ndarray:
        code = {"U": 0, "G": 1, "V": 2}[which]
        t = {"U": lambda: self.U[index], "G": lambda: self.G, "V": lambda: self.V[index]}[which]()
        out = np.empty(t.shape, dtype=np.float64)
        check(self.lib.s3_export(self.h, code, int(index), out.ctypes.data_as(C.POINTER(C.c_double)),
                                 out.nbytes, _stream()), self.h)
        return out

    def import_(self, which: str, index: int, values) -> None:
        """Write host float64 values into parameter U[index], G or V[index]
        (the inverse of export)."""
        code = {"U": 0, "G": 1, "V": 2}[which]
        a = np.ascontiguousarray(values, dtype=np.float64)
        check(self.lib.s3_import(self.h, code, int(index), a.ctypes.data_as(C.POINTER(C.c_double)),
                                 a.nbytes, _stream()), self.h)

    def orthogonalize(self) -> None:
        """Algorithm 1's closing step on the device: U <- Q, G <- G x_n R,
        V <- V R^T (predictions unchanged)."""
        check(self.lib.s3_orthogonalize(self.h, _stream()), self.h)

    def init_params(self, seed: int, sigma: float = 0.1) -> None:
        """Fill U, G and V with N(0, sigma^2) values on the device
        (counter-based; see s3_init_params)."""
        check(self.lib.s3_init_params(self.h, C.c_uint64(int(seed) & (2 ** 64 - 1)), float(sigma), _stream()),
              self.h)

    def params_numpy(self):
        return ([self.export("U", n) for n in range(len(self.U))], self.export("G"),
                [self.export("V", m) for m in range(len(self.V))])
