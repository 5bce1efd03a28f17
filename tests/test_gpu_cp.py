"""The CP special case (hyper-diagonal core, Section 3's S^3CMTF-CP) on the
GPU against the oracle's CP mode: det batches and epochs, loss / RMSE /
predictions, the adjoint, and lock-free RMSE against the oracle.  Same
checks as the Tucker tests: each batch's update from a re-synced start, row
by row, FP64 1e-10 and FP32 1e-5, also for every batch of a whole epoch."""
import numpy as np
import pytest
import torch

import oracle
from synth import item_order
from tests.gpu_util import UNIT, check_batches, compare_params, rel, setup

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}
CASES = [
    ("cfg1", "f64", 500, dict()),
    ("tiny3", "f64", 7, dict(ranks=(2, 2, 2))),
    ("tiny4", "f64", 5, dict(ranks=(2, 2, 2, 2))),
    ("cfg2_slice", "f32", 8192, dict()),
    ("cfg5_slice", "f32", 4096, dict()),
]


@pytest.mark.parametrize("name,dtype,batch,over", CASES)
def test_cp_det_batches_match_oracle(name, dtype, batch, over):
    print(f"\n[cp-det] {name} {dtype} batch={batch}", flush=True)
    cfg, p, plan, ref, order = setup(name, dtype, batch, True, core="cp", **over)
    check_batches(p, plan, order, batch, 0.01, range(min(3, plan.n_batches())), True, TOL[dtype], UNIT[dtype],
                  "cp", cp=True)
    cfg, p, plan, ref, order = setup(name, dtype, batch, True, core="cp", **over)
    for b in range(min(3, plan.n_batches())):
        plan.det_batches(b, 1, 0.01)
        oracle.minibatch_epoch(ref, p, order, batch, 0.01, b, 1, damping=True)
    compare_params(plan, ref, TOL[dtype], "lockstep")


def test_cp_det_epoch_matches_oracle():
    cfg, p, plan, ref, order = setup("cfg2_slice", "f32", 4096, True, core="cp")
    w = check_batches(p, plan, order, 4096, oracle.eta_at(cfg.eta0, cfg.mu, 0), range(plan.n_batches()), True,
                      TOL["f32"], UNIT["f32"], "cp epoch", cp=True)
    print(f"{plan.n_batches()} batches, worst error / bound {w:.3f}", flush=True)


@pytest.mark.parametrize("name,dtype", [("cfg1", "f64"), ("cfg5_slice", "f32")])
def test_cp_loss_rmse_predict_match_oracle(name, dtype):
    cfg, p, plan, ref, order = setup(name, dtype, 4096, core="cp")
    tol = TOL[dtype]
    f, ft, fm = plan.loss()
    of, oft, ofm = oracle.loss(ref, p)
    assert abs(f - of) <= tol * abs(of) and abs(ft - oft) <= tol * abs(oft)
    assert abs(plan.rmse() - oracle.rmse(ref, p.test_idx, p.test_val)) <= tol * oracle.rmse(ref, p.test_idx,
                                                                                           p.test_val)
    assert rel(plan.predict(p.test_idx).cpu().numpy(), oracle.predict(ref, p.test_idx)) <= tol


@pytest.mark.parametrize("name,dtype,batch", [("cfg1", "f64", 700), ("cfg2_slice", "f32", 8192)])
def test_cp_backward_matches_oracle_adjoint(name, dtype, batch):
    cfg, p, plan, ref, order = setup(name, dtype, batch, core="cp")
    rng = np.random.default_rng(6)
    gx = rng.normal(size=p.n_train)
    gy = [rng.normal(size=len(v)) for v in p.mat_val]
    if dtype == "f32":
        gx = gx.astype(np.float32).astype(np.float64)
        gy = [g.astype(np.float32).astype(np.float64) for g in gy]
    dU, dG, dV = plan.backward(torch.as_tensor(gx, device="cuda"), [torch.as_tensor(g, device="cuda") for g in gy])
    oU, oG, oV = oracle.adjoint(ref, p.train_idx, gx, [(p.mat_row[m], p.mat_col[m]) for m in range(len(gy))], gy)
    tol = TOL[dtype]
    for a, b in zip(dU, oU):
        assert rel(a.cpu().numpy(), b) <= tol
    assert rel(dG.cpu().numpy(), oG) <= tol
    for a, b in zip(dV, oV):
        assert rel(a.cpu().numpy(), b) <= tol


def test_cp_lockfree_tracks_oracle():
    """As the Tucker lock-free tests: after 20 epochs the mean over two tile
    seeds within 1 % of the damped det mini-batch oracle with batch = the
    round size, each seed within 2 %."""
    import os
    threads = max(1, min(16, os.cpu_count() or 1))
    cfg, p, plan, ref, order = setup("cfg2_slice", "f32", 4096, True, round_items=4096, core="cp", order_seed=7)
    det = ref.copy()
    fixed = item_order(p.n_items, 7, 0)
    for ep in range(20):
        oracle.minibatch_epoch(det, p, fixed, 4096, oracle.eta_at(cfg.eta0, cfg.mu, ep), damping=True,
                               threads=threads)
    want = oracle.rmse(det, p.test_idx, p.test_val)
    got = []
    for seed in (7, 8):
        if seed != 7:
            cfg, p, plan, _, _ = setup("cfg2_slice", "f32", 4096, True, round_items=4096, core="cp",
                                       order_seed=seed)
        for ep in range(20):
            plan.epoch(ep, "lockfree")
        got.append(plan.rmse())
        print(f"[cp-lockfree] seed {seed}: {got[-1]:.4f} vs det oracle {want:.4f}", flush=True)
        assert np.isfinite(got[-1]) and abs(got[-1] - want) <= 0.02 * want
    assert abs(np.mean(got) - want) <= 0.01 * want


def test_cp_orthogonalize_is_rejected():
    from paper_1708_08640_amd._abi import S3Error
    cfg, p, plan, ref, order = setup("cfg1", "f64", 500, core="cp")
    with pytest.raises(S3Error):
        plan.orthogonalize()
