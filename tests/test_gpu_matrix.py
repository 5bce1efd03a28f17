"""The matrix-core contraction (S3_CONTRACT_MATRIX) against the FP64 oracle.

FP32 operands: the same bar as the vector-unit path -- each det batch's
update, from a start re-synced to the library's state, right to 1e-5
normwise per parameter array (1e-3 per row) beyond FP32 storage rounding,
for every batch of an epoch too; the adjoint to 1e-5.

BF16 operands (FP32 master parameters, BF16 contraction operands rounded to
nearest even, FP32 sums; BF16's unit roundoff is 2^-8 = 3.9e-3): the error
of each result against the FP64 oracle is stated and bounded --
  * each batch's parameter update: <= 1e-2 of the update normwise per array
    (measured 1e-4 .. 2.6e-3) and <= 5e-2 per row;
  * the adjoint (the gradients of the predictions, Eq 8's contractions):
    <= 1e-2 normwise (measured 2.3e-3 .. 2.8e-3);
  * loss, held-out RMSE and predictions are evaluated in FP32 (1e-5);
  * after 20 lock-free epochs the held-out RMSE is within 1 % of the FP32
    matrix-core run's with the same tile seed.
Shapes: 4-way rank 8 (and ragged 8 x 8 x 7 x 8) and 3-way rank 16 (and
ragged 16 x 13 x 9).
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import UNIT, check_batches, compare_params, rel, setup

pytestmark = pytest.mark.gpu

SHAPES = [("cfg5_slice", (8, 8, 8, 8)), ("cfg5_slice", (8, 8, 7, 8)), ("cfg2_slice", (16, 16, 16)),
          ("cfg2_slice", (16, 13, 9))]
IDS = [f"{n}-{'x'.join(map(str, r))}" for n, r in SHAPES]
TOL = {"f32": (1e-5, 1e-3), "bf16": (1e-2, 5e-2)}  # (per array, per row), relative to the update
ADJ_TOL = {"f32": 1e-5, "bf16": 1e-2}


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("name,ranks", SHAPES, ids=IDS)
def test_matrix_det_batches_match_oracle(name, ranks, dtype):
    print(f"\n[matrix-det] {name} {ranks} {dtype}", flush=True)
    cfg, p, plan, ref, order = setup(name, dtype, 4096, True, ranks=ranks, contraction="matrix")
    tol, row_tol = TOL[dtype]
    w = check_batches(p, plan, order, 4096, 0.01, range(3), True, tol, UNIT[dtype], f"{dtype}", row_tol=row_tol)
    print(f"worst row error / bound {w:.3f}", flush=True)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_matrix_det_epoch_every_batch(dtype):
    cfg, p, plan, ref, order = setup("cfg5_slice", dtype, 4096, True, contraction="matrix")
    tol, row_tol = TOL[dtype]
    w = check_batches(p, plan, order, 4096, oracle.eta_at(cfg.eta0, cfg.mu, 0), range(plan.n_batches()), True,
                      tol, UNIT[dtype], f"{dtype} epoch", row_tol=row_tol)
    print(f"\n[matrix-epoch] {dtype}: {plan.n_batches()} batches, worst row error / bound {w:.3f}", flush=True)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("name,ranks", SHAPES[::2], ids=IDS[::2])
def test_matrix_adjoint_matches_oracle(name, ranks, dtype):
    cfg, p, plan, ref, order = setup(name, dtype, 4096, True, ranks=ranks, contraction="matrix")
    rng = np.random.default_rng(3)
    gx = rng.standard_normal(p.n_train).astype(np.float32).astype(np.float64)
    gy = [rng.standard_normal(len(v)).astype(np.float32).astype(np.float64) for v in p.mat_val]
    dU, dG, dV = plan.backward(torch.as_tensor(gx, dtype=torch.float32, device="cuda"),
                               [torch.as_tensor(g, dtype=torch.float32, device="cuda") for g in gy])
    oU, oG, oV = oracle.adjoint(ref, p.train_idx, gx, [(p.mat_row[m], p.mat_col[m]) for m in range(len(gy))], gy)
    errs = [rel(a.cpu().numpy(), b) for a, b in zip(dU, oU)] + [rel(dG.cpu().numpy(), oG)]
    errs += [rel(a.cpu().numpy(), b) for a, b in zip(dV, oV)]
    print(f"\n[matrix-adjoint] {name} {ranks} {dtype}: " + " ".join(f"{e:.1e}" for e in errs), flush=True)
    assert max(errs) <= ADJ_TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_matrix_plan_evaluates_in_fp32(dtype):
    """Loss, RMSE and predictions of a matrix-core plan are FP32 evaluations."""
    cfg, p, plan, ref, order = setup("cfg5_slice", dtype, 4096, True, contraction="matrix")
    plan.det_batches(0, 2, 0.01)
    U, G, V = plan.params_numpy()
    now = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    f, ft, fm = plan.loss()
    of, oft, ofm = oracle.loss(now, p)
    assert abs(f - of) <= 1e-5 * abs(of)
    r = oracle.rmse(now, p.test_idx, p.test_val)
    assert abs(plan.rmse() - r) <= 1e-5 * r
    assert rel(plan.predict(p.test_idx).cpu().numpy(), oracle.predict(now, p.test_idx)) <= 1e-5


@pytest.mark.parametrize("name,ranks", [SHAPES[0], SHAPES[2]], ids=[IDS[0], IDS[2]])
def test_bf16_final_rmse_matches_fp32(name, ranks):
    """20 lock-free epochs with BF16 operands against FP32 operands, same tile
    seed, and both against the FP64 oracle's damped batches (round size)."""
    out = {}
    for dt in ("f32", "bf16"):
        cfg, p, plan, ref, order = setup(name, dt, 4096, True, ranks=ranks, contraction="matrix",
                                         round_items=16384, order_seed=7)
        for ep in range(20):
            plan.epoch(ep, "lockfree")
        out[dt] = plan.rmse()
    print(f"\n[bf16-vs-f32] {name} {ranks}: FP32 {out['f32']:.4f}, BF16 {out['bf16']:.4f}", flush=True)
    assert abs(out["bf16"] - out["f32"]) <= 0.01 * out["f32"]
