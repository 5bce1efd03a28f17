"""Adjoint (backward) kernel and the autograd.Function against the oracle's
transpose of the prediction map."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import rel, setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,dtype,batch", [("cfg1", "f64", 700), ("tiny4", "f64", 4),
                                              ("cfg2_slice", "f32", 8192), ("cfg5_slice", "f32", 8192)])
def test_backward_matches_oracle_adjoint(name, dtype, batch):
    print(f"\n[adjoint] {name} {dtype}", flush=True)
    cfg, p, plan, ref, order = setup(name, dtype, batch)
    rng = np.random.default_rng(5)
    gx = rng.normal(size=p.n_train)
    gy = [rng.normal(size=len(v)) for v in p.mat_val]
    if dtype == "f32":
        gx = gx.astype(np.float32).astype(np.float64)
        gy = [g.astype(np.float32).astype(np.float64) for g in gy]
    dU, dG, dV = plan.backward(torch.as_tensor(gx, device="cuda"), [torch.as_tensor(g, device="cuda") for g in gy])
    mats = [(p.mat_row[m], p.mat_col[m]) for m in range(len(p.mat_val))]
    oU, oG, oV = oracle.adjoint(ref, p.train_idx, gx, mats, gy)
    tol = 1e-10 if dtype == "f64" else 1e-5
    for a, b in zip(dU, oU):
        assert rel(a.cpu().numpy(), b) <= tol
    assert rel(dG.cpu().numpy(), oG) <= tol
    for a, b in zip(dV, oV):
        assert rel(a.cpu().numpy(), b) <= tol


def _oracle_adjoint(p, ref, gx, gy):
    mats = [(p.mat_row[m], p.mat_col[m]) for m in range(len(p.mat_val))]
    return oracle.adjoint(ref, p.train_idx, gx, mats, gy)


@pytest.mark.parametrize("name,dtype,batch", [("cfg1", "f64", 700), ("tiny4", "f64", 4),
                                              ("cfg5_slice", "f32", 8192)])
def test_backward_without_item_order(name, dtype, batch):
    """A plan bound without an item order sums in the storage order: the
    first call builds that order's reduction structures; results match the
    oracle's adjoint, repeat bitwise, and survive a lock-free epoch and a
    workspace query (the structures overlap nothing else)."""
    from paper_1708_08640_amd import S3Error
    print(f"\n[adjoint, no order] {name} {dtype} batch {batch}", flush=True)
    cfg, p, plan, ref, _ = setup(name, dtype, batch, with_order=False)
    rng = np.random.default_rng(6)
    gx = rng.normal(size=p.n_train)
    gy = [rng.normal(size=len(v)) for v in p.mat_val]
    if dtype == "f32":
        gx = gx.astype(np.float32).astype(np.float64)
        gy = [g.astype(np.float32).astype(np.float64) for g in gy]
    tgx = torch.as_tensor(gx, device="cuda")
    tgy = [torch.as_tensor(g, device="cuda") for g in gy]
    tol = 1e-10 if dtype == "f64" else 1e-5

    def check_against_oracle(dU, dG, dV, ref):
        oU, oG, oV = _oracle_adjoint(p, ref, gx, gy)
        for a, b in zip(dU, oU):
            assert rel(a.cpu().numpy(), b) <= tol
        assert rel(dG.cpu().numpy(), oG) <= tol
        for a, b in zip(dV, oV):
            assert rel(a.cpu().numpy(), b) <= tol

    first = plan.backward(tgx, tgy)
    check_against_oracle(*first, ref)
    plan.workspace_bytes(p.n_train, len(p.test_val), [len(v) for v in p.mat_val])
    second = plan.backward(tgx, tgy)
    for a, b in zip(first[0] + [first[1]] + first[2], second[0] + [second[1]] + second[2]):
        assert torch.equal(a, b)
    with pytest.raises(S3Error) as ei:  # det epochs still need an item order
        plan.epoch(0, "det")
    assert ei.value.status == -7
    plan.epoch(0, "lockfree")
    torch.cuda.synchronize()
    U, G, V = plan.params_numpy()
    moved = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    check_against_oracle(*plan.backward(tgx, tgy), moved)


def test_autograd_function_gradients():
    from paper_1708_08640_amd import predictions
    cfg, p, plan, ref, order = setup("cfg1", "f64", 1000)
    for t in plan.U + [plan.G] + plan.V:
        t.requires_grad_(True)
    xhat, yhat = predictions(plan)
    # the data part of Eq (7): 1/2 sum (x - x~)^2 + lambda_m/2 sum (y - y^)^2
    loss = 0.5 * ((plan.x_val - xhat) ** 2).sum() + 0.5 * cfg.lambda_m * sum(
        ((v - yh) ** 2).sum() for (_, _, v), yh in zip(plan.y, yhat))
    loss.backward()
    xo = oracle.predict(ref, p.train_idx)
    gx = -(p.train_val - xo)
    gy = [-cfg.lambda_m * (p.mat_val[m] - oracle.matrix_predict(ref, m, p.mat_row[m], p.mat_col[m]))
          for m in range(len(p.mat_val))]
    oU, oG, oV = oracle.adjoint(ref, p.train_idx, gx, [(p.mat_row[m], p.mat_col[m]) for m in range(len(gy))], gy)
    for t, b in zip(plan.U, oU):
        assert rel(t.grad.cpu().numpy(), b) <= 1e-10
    assert rel(plan.G.grad.cpu().numpy(), oG) <= 1e-10
    for t, b in zip(plan.V, oV):
        assert rel(t.grad.cpu().numpy(), b) <= 1e-10


def test_autograd_gradcheck_tiny():
    from paper_1708_08640_amd import SparseTuckerCMTF
    cfg, p, plan, ref, order = setup("tiny3", "f64", 4)
    params = [t.detach().requires_grad_(True) for t in plan.U + [plan.G] + plan.V]
    # rebind the plan's views so the Function sees the tensors it is bound to
    plan.U = params[:len(plan.U)]
    plan.G = params[len(plan.U)]
    plan.V = params[len(plan.U) + 1:]

    def f(*ps):
        return SparseTuckerCMTF.apply(plan, *ps)

    assert torch.autograd.gradcheck(f, tuple(params), eps=1e-6, atol=1e-7, rtol=1e-5)
