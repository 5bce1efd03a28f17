"""The three larger workloads at full size:

* 3-way 2M x 2M x 500, 50M Zipf(1.1) entries, core 10^3, coupled 2M x 2M
  (20M) and 2M x 200 (10M) matrices: FP32, vector-unit contraction; also the
  adjoint, checked by finite differences on a 1,000-entry subsample;
* the same shape with 100M entries and core 16^3: the matrix-core
  contraction, FP32 and BF16 operands;
* 4-way 1M x 500K x 1000 x 24, 200M entries, core 8^4, three coupled
  matrices (one of them dense): the matrix-core contraction, FP32 and BF16;
  also two whole det epochs (batches of 524,288) against the stored FP64 det
  oracle trajectory.

Each is checked on outputs the oracle can compute at full size: the first
det batch (65,536 items) as an update from the same start (the bounds of
tests/gpu_util.check_update: FP32 1e-5 per array and 1e-3 per row, BF16
1e-2 and 5e-2), sampled held-out predictions, and one lock-free epoch at the
benchmark's settings through properties (finite, unobserved rows unchanged,
held-out RMSE below its untrained value); on the 4-way workload three
lock-free epochs in the benchmark's configuration (rounds of 786,432) end at
or below the benchmark's target, 1.01 times the stored sequential-SGD
oracle's held-out RMSE.
"""
import os
import time

import numpy as np
import pytest
import torch

import oracle
from synth import get_config, init_params, item_order, make_problem
from tests.gpu_util import UNIT, check_update, rel, rounded_problem

pytestmark = pytest.mark.gpu

BATCH, ROUND, HOT, SEED = 65536, 524288, 64, 7
ROUNDS = {"cfg5_4way_200m": 786432}  # the benchmark's round size on the 4-way workload
THREADS = max(1, min(16, os.cpu_count() or 1))
TOL = {"f32": (1e-5, 1e-3), "bf16": (1e-2, 5e-2)}


def _gen(name):
    t = time.time()
    print(f"\n[large] generating {name}", flush=True)
    cfg = get_config(name)
    p = rounded_problem(make_problem(cfg), "f32")
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    U, G, V = init_params(cfg)
    print(f"[large] {cfg.description}: {p.n_train:,} train, {p.n_items - p.n_train:,} matrix entries "
          f"({time.time() - t:.0f} s)", flush=True)
    return cfg, p, ([r(u) for u in U], r(G), [r(v) for v in V])


def _plan(p, params, dtype="f32", contraction="reuse", **kw):
    from paper_1708_08640_amd import S3Plan
    return S3Plan.from_problem(p, params, dtype=dtype, damping=True, seed=SEED,
                               round_items=ROUNDS.get(p.cfg.name, ROUND), hot_rows=HOT,
                               batch=BATCH, contraction=contraction, **kw)


def _det_first_batch(cfg, p, params, order, dtype, contraction):
    t = time.time()
    plan = _plan(p, params, dtype, contraction, order=order)
    eta = oracle.eta_at(cfg.eta0, cfg.mu, 0)
    plan.det_batches(0, 1, eta)
    got = plan.params_numpy()
    del plan
    torch.cuda.empty_cache()
    U, G, V = params
    ref = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    oracle.minibatch_epoch(ref, p, order, BATCH, eta, 0, 1, damping=True, threads=THREADS)
    tol, row_tol = TOL[dtype]
    w = check_update(got, ref, params, tol, UNIT[dtype], f"{cfg.name} {dtype} {contraction} det batch 0", row_tol)
    print(f"[large] {cfg.name} det batch 0 ({dtype}, {contraction}): worst row error / bound {w:.3f} "
          f"({time.time() - t:.0f} s)", flush=True)


def _lockfree_epoch(cfg, p, params, dtype, contraction, epochs=1, target=None):
    U = params[0]
    plan = _plan(p, params, dtype, contraction, order=None)
    r0 = plan.rmse()
    t = time.time()
    traj = []
    for e in range(epochs):
        plan.epoch(e, "lockfree")
        traj.append(plan.rmse())
    r1 = traj[-1]
    if target is not None:
        print(f"[large] {cfg.name} lock-free RMSE after epochs 1..{epochs}: {traj}; target {target:.4f}", flush=True)
        assert r1 <= target
    print(f"[large] {cfg.name} lock-free epoch ({dtype}, {contraction}): RMSE {r0:.4f} -> {r1:.4f} "
          f"({time.time() - t:.2f} s incl. RMSE)", flush=True)
    lU, lG, lV = plan.params_numpy()
    seen = [np.zeros(d, dtype=bool) for d in cfg.dims]
    for n in range(len(cfg.dims)):
        seen[n][p.train_idx[n]] = True
    for m, s in enumerate(cfg.matrices):
        seen[s.mode][p.mat_row[m]] = True
    for n in range(len(lU)):
        assert np.all(np.isfinite(lU[n]))
        assert np.array_equal(lU[n][~seen[n]], U[n][~seen[n]]), f"unobserved rows of U[{n}] changed"
    assert np.all(np.isfinite(lG)) and all(np.all(np.isfinite(v)) for v in lV)
    assert r1 < r0
    # sampled held-out predictions on the trained parameters
    rng = np.random.default_rng(9)
    sel = np.sort(rng.choice(p.test_idx.shape[1], 4000, replace=False))
    idx = np.ascontiguousarray(p.test_idx[:, sel])
    got = plan.predict(idx).cpu().numpy().astype(np.float64)
    want = oracle.predict(oracle.Params.from_arrays(lU, lG, lV, [s.mode for s in cfg.matrices]), idx)
    assert rel(got, want) <= 1e-5
    del plan
    torch.cuda.empty_cache()


def test_large_cfg3_fp32_and_adjoint():
    cfg, p, params = _gen("cfg3")
    order = item_order(p.n_items, SEED, 0)
    _det_first_batch(cfg, p, params, order, "f32", "reuse")
    # the adjoint with an upstream gradient on 1,000 sampled training entries,
    # at the initial parameters: against the oracle's adjoint on those entries
    # and against central finite differences of sum_e gx_e x~_e (FP64)
    U, G, V = params
    modes = [s.mode for s in cfg.matrices]
    plan = _plan(p, params, "f32", "reuse", order=order)
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(p.n_train, 1000, replace=False))
    gx = np.zeros(p.n_train)
    gx[sel] = rng.standard_normal(sel.size)
    gx = gx.astype(np.float32).astype(np.float64)
    dU, dG, dV = plan.backward(torch.as_tensor(gx, dtype=torch.float32, device="cuda"))
    dU = [d.cpu().numpy().astype(np.float64) for d in dU]
    dG = dG.cpu().numpy().astype(np.float64).reshape(G.shape)
    del plan
    torch.cuda.empty_cache()
    sub_idx = np.ascontiguousarray(p.train_idx[:, sel])
    ref = oracle.Params.from_arrays(U, G, V, modes)
    wU, wG, wV = oracle.adjoint(ref, sub_idx, gx[sel], [], [])
    for n in range(len(dU)):
        rows = np.unique(sub_idx[n])
        assert rel(dU[n][rows], wU[n][rows]) <= 1e-5, f"adjoint U[{n}]"
        mask = np.ones(dU[n].shape[0], dtype=bool)
        mask[rows] = False
        assert not np.any(dU[n][mask]), f"adjoint U[{n}] touched rows outside the sample"
    assert rel(dG, wG) <= 1e-5, "adjoint G"

    def L():
        return float(np.dot(gx[sel], oracle.predict(ref, sub_idx)))

    checked = 0
    for n in range(len(U)):
        rows = np.unique(sub_idx[n])
        for r in rng.choice(rows, 4, replace=False):
            for k in (0, cfg.ranks[n] - 1):
                old = ref.U[n][r, k]
                h = 1e-6 * max(1.0, abs(old))
                ref.U[n][r, k] = old + h
                fp = L()
                ref.U[n][r, k] = old - h
                fm = L()
                ref.U[n][r, k] = old
                fd = (fp - fm) / (2 * h)
                assert abs(dU[n][r, k] - fd) <= 1e-4 * abs(fd) + 1e-6, f"FD U[{n}][{r},{k}]: {dU[n][r, k]} vs {fd}"
                checked += 1
    flat = ref.G.reshape(-1)
    for j in rng.choice(flat.size, 12, replace=False):
        old = flat[j]
        h = 1e-6 * max(1.0, abs(old))
        flat[j] = old + h
        fp = L()
        flat[j] = old - h
        fm = L()
        flat[j] = old
        fd = (fp - fm) / (2 * h)
        assert abs(dG.reshape(-1)[j] - fd) <= 1e-4 * abs(fd) + 1e-6, f"FD G[{j}]"
        checked += 1
    print(f"[large] cfg3 adjoint: oracle rows <= 1e-5, {checked} coordinates against finite differences",
          flush=True)
    _lockfree_epoch(cfg, p, params, "f32", "reuse")


@pytest.mark.parametrize("name", ["cfg4", "cfg5"])
def test_large_matrix_core(name):
    cfg, p, params = _gen(name)
    order = item_order(p.n_items, SEED, 0)
    for dtype in ("f32", "bf16"):
        _det_first_batch(cfg, p, params, order, dtype, "matrix")
    if name == "cfg5":
        # the benchmark's configuration: after 3 epochs at most 1.01 times the
        # stored sequential-SGD oracle's held-out RMSE (the fixed-RMSE target)
        _lockfree_epoch(cfg, p, params, "bf16", "matrix", epochs=3, target=1.01 * _sgd_mean("cfg5", 3))
        _det_epochs_against_stored_oracle(cfg, p, params, order)
    else:
        _lockfree_epoch(cfg, p, params, "bf16", "matrix")


def _sgd_mean(config, epoch):
    import glob
    import json
    vals = []
    for f in glob.glob(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{config}_sgd_s*.json")):
        with open(f) as fh:
            r = json.load(fh)["rmse"]
        if len(r) >= epoch:
            vals.append(r[epoch - 1])
    assert vals, f"no stored SGD trajectory for {config}"
    return float(np.mean(vals))


def _det_epochs_against_stored_oracle(cfg, p, params, order):
    """Two whole det epochs (batches of 524,288, damped, BF16 operands) on all
    230M items: the held-out RMSE after each against the stored FP64 det
    oracle trajectory with the same item order and FP32-rounded inputs
    (tests/golden/cfg5_det524288_s7.json), to 1e-4 relative."""
    import json
    from paper_1708_08640_amd import S3Plan
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg5_det524288_s7.json")) as f:
        ref = json.load(f)["rmse"]
    plan = S3Plan.from_problem(p, params, dtype="bf16", damping=True, seed=SEED, batch=524288, order=order,
                               contraction="matrix")
    got = []
    for e in range(min(2, len(ref))):
        plan.epoch(e, "det")
        got.append(plan.rmse())
    del plan
    torch.cuda.empty_cache()
    print(f"[large] cfg5 det epochs (BF16, batches of 524,288): RMSE {got} against the oracle's {ref[:len(got)]}",
          flush=True)
    assert got, "no stored det oracle epochs"
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-4 * r
