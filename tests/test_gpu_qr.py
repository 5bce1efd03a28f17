"""Orthogonalisation on the GPU (Algorithm 1, closing step) against the
oracle's Householder QR.  Q is unique up to the sign of each column, so the
oracle's columns (and the matching core slices and V columns) are flipped to
agree with the GPU's before comparing; the GPU's R has a positive diagonal.
Also: the GPU's factors have orthonormal columns and every prediction is
unchanged.  Tolerances: FP64 1e-10; FP32 1e-5, normwise and for every row
(FP32 storage of the results, Gram and Cholesky in FP64)."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import _row_rel, rel, setup

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


def _flip(ref, gpu):
    """Sign-align the oracle's Q columns to the GPU's, carrying the signs into
    G (mode-n slices) and the V columns of matrices on that mode."""
    out = ref.copy()
    for n, (qo, qg) in enumerate(zip(ref.U, gpu[0])):
        s = np.sign(np.sum(qo * qg, axis=0))
        s[s == 0] = 1.0
        out.U[n] = qo * s
        shape = [1] * out.G.ndim
        shape[n] = -1
        out.G = out.G * s.reshape(shape)
        for m, mode in enumerate(ref.modes):
            if mode == n:
                out.V[m] = out.V[m] * s
    return out


@pytest.mark.parametrize("name,dtype", [("cfg1", "f64"), ("tiny4", "f64"), ("cfg2_slice", "f32"),
                                        ("cfg5_slice", "f32")])
def test_orthogonalize_matches_oracle(name, dtype):
    print(f"\n[qr] {name} {dtype}", flush=True)
    cfg, p, plan, ref, order = setup(name, dtype, 4096, True)
    plan.epoch(0, "det")
    U, G, V = plan.params_numpy()
    before = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    x0 = plan.predict(p.test_idx).cpu().numpy().astype(np.float64)
    y0 = [plan.predict_matrix(m, p.mat_row[m], p.mat_col[m]).cpu().numpy().astype(np.float64)
          for m in range(len(cfg.matrices))]
    plan.orthogonalize()
    gU, gG, gV = plan.params_numpy()
    want = _flip(oracle.qr_orthogonalize(before), (gU, gG, gV))
    tol = TOL[dtype]
    for n in range(len(gU)):
        assert rel(gU[n], want.U[n]) <= tol, f"Q[{n}] rel {rel(gU[n], want.U[n]):.2e}"
        assert _row_rel(gU[n], want.U[n]) <= tol, f"Q[{n}] worst row {_row_rel(gU[n], want.U[n]):.2e}"
        qtq = gU[n].T @ gU[n]
        assert np.abs(qtq - np.eye(qtq.shape[0])).max() <= tol, f"Q[{n}]^T Q[{n}] != I"
    assert rel(gG, want.G) <= tol, f"G rel {rel(gG, want.G):.2e}"
    for m in range(len(gV)):
        assert rel(gV[m], want.V[m]) <= tol, f"V[{m}] rel {rel(gV[m], want.V[m]):.2e}"
        assert _row_rel(gV[m], want.V[m]) <= tol, f"V[{m}] worst row {_row_rel(gV[m], want.V[m]):.2e}"
    x1 = plan.predict(p.test_idx).cpu().numpy().astype(np.float64)
    assert rel(x1, x0) <= tol
    for m in range(len(cfg.matrices)):
        y1 = plan.predict_matrix(m, p.mat_row[m], p.mat_col[m]).cpu().numpy().astype(np.float64)
        assert rel(y1, y0[m]) <= tol
