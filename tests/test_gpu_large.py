"""The three larger workloads at full size, FP32:

* 3-way 2M x 2M x 500, 50M Zipf(1.1) entries, core 10^3, coupled 2M x 2M
  (20M) and 2M x 200 (10M) matrices -- also the adjoint;
* the same shape with 100M entries and core 16^3;
* 4-way 1M x 500K x 1000 x 24, 200M entries, core 8^4, three coupled
  matrices (one of them dense).

Each is checked on outputs the oracle can compute one by one at full size:
the first det batch (65,536 items) on the touched rows and their updates
(bounds as in test_gpu_fullsize.py), sampled held-out predictions, and one
lock-free epoch at the benchmark's settings through properties (finite,
unobserved rows unchanged, held-out RMSE below its untrained value).  The
adjoint is checked with an upstream gradient that is non-zero on 2,000
sampled training entries only, which the oracle evaluates exactly.

Generating these inputs takes minutes on a host core (the redraw rule that
keeps Omega a set is sequential per round), so the module runs only with
S3_LARGE=1 in the environment.
"""
import os
import time

import numpy as np
import pytest

import oracle
from synth import get_config, init_params, item_order, make_problem
from tests.gpu_util import rel, rounded_problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(os.environ.get("S3_LARGE") != "1",
                                                  reason="full-size 50M-200M entry inputs: set S3_LARGE=1")]

BATCH, ROUND, HOT, SEED = 65536, 524288, 64, 7


def _gen(name):
    t = time.time()
    print(f"\n[large] generating {name}", flush=True)
    cfg = get_config(name)
    p = rounded_problem(make_problem(cfg, progress=True), "f32")
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    U, G, V = init_params(cfg)
    print(f"[large] {cfg.description}: {p.n_train:,} train, {p.n_items - p.n_train:,} matrix entries "
          f"({time.time() - t:.0f} s)", flush=True)
    return cfg, p, ([r(u) for u in U], r(G), [r(v) for v in V])


def _plan(p, params, **kw):
    from paper_1708_08640_amd import S3Plan
    return S3Plan.from_problem(p, params, dtype="f32", damping=True, seed=SEED, round_items=ROUND, hot_rows=HOT,
                               batch=BATCH, **kw)


def _touched(cfg, p, items):
    nt = p.n_train
    t = items[items < nt]
    rows_u = [set(p.train_idx[n][t].tolist()) for n in range(len(cfg.dims))]
    rows_v = []
    off = nt
    for m, s in enumerate(cfg.matrices):
        k = items[(items >= off) & (items < off + len(p.mat_val[m]))] - off
        rows_u[s.mode] |= set(p.mat_row[m][k].tolist())
        rows_v.append(set(p.mat_col[m][k].tolist()))
        off += len(p.mat_val[m])
    return ([np.array(sorted(r), dtype=np.int64) for r in rows_u],
            [np.array(sorted(r), dtype=np.int64) for r in rows_v])


@pytest.mark.parametrize("name", ["cfg3", "cfg4", "cfg5"])
def test_large_workload(name):
    cfg, p, (U, G, V) = _gen(name)
    modes = [s.mode for s in cfg.matrices]

    # det: first batch against the oracle
    order = item_order(p.n_items, SEED, 0)
    plan = _plan(p, (U, G, V), order=order)
    # adjoint (it runs on the det structures) with an upstream gradient on
    # 2,000 sampled training entries, at the initial parameters
    if name == "cfg3":
        import torch
        rng = np.random.default_rng(11)
        sel = np.sort(rng.choice(p.n_train, 2000, replace=False))
        gx = np.zeros(p.n_train)
        gx[sel] = rng.standard_normal(sel.size)
        gx = gx.astype(np.float32).astype(np.float64)
        dU, dG, dV = plan.backward(torch.as_tensor(gx, dtype=torch.float32, device="cuda"))
        sub_idx = np.ascontiguousarray(p.train_idx[:, sel])
        wU, wG, wV = oracle.adjoint(oracle.Params.from_arrays(U, G, V, modes), sub_idx, gx[sel], [], [])
        for n in range(len(dU)):
            d = dU[n].cpu().numpy().astype(np.float64)
            rows = np.unique(sub_idx[n])
            print(f"[large] adjoint U[{n}] rel {rel(d[rows], wU[n][rows]):.2e}", flush=True)
            assert rel(d[rows], wU[n][rows]) <= 1e-5, f"adjoint U[{n}]"
            mask = np.ones(d.shape[0], dtype=bool)
            mask[rows] = False
            assert not np.any(d[mask]), f"adjoint U[{n}] touched rows outside the sample"
        assert rel(dG.cpu().numpy().astype(np.float64), wG) <= 1e-5, "adjoint G"
        for m in range(len(dV)):
            assert not np.any(dV[m].cpu().numpy()), f"adjoint V[{m}] without matrix gradients"
        del dU, dG, dV

    eta = oracle.eta_at(cfg.eta0, cfg.mu, 0)
    plan.det_batches(0, 1, eta)
    gU, gG, gV = plan.params_numpy()
    del plan
    ref = oracle.Params.from_arrays(U, G, V, modes)
    oracle.minibatch_epoch(ref, p, order, BATCH, eta, 0, 1, damping=True)
    ru, rv = _touched(cfg, p, np.asarray(order[:BATCH], dtype=np.int64))
    pairs = [(f"U[{n}]", gU[n][ru[n]], ref.U[n][ru[n]], U[n][ru[n]]) for n in range(len(U))]
    pairs += [("G", gG, ref.G, G)]
    pairs += [(f"V[{m}]", gV[m][rv[m]], ref.V[m][rv[m]], V[m][rv[m]]) for m in range(len(V))]
    for what, a, b, a0 in pairs:
        r = rel(a, b)
        err = np.linalg.norm((a - a0) - (b - a0))
        bound = 2.0 ** -24 * np.linalg.norm(b) + 1e-5 * np.linalg.norm(b - a0)
        print(f"[large] {name} det {what}: rows rel {r:.2e}, update err {err:.2e} (bound {bound:.2e})", flush=True)
        assert np.all(np.isfinite(a)) and r <= 1e-5 and err <= bound, what
    del gU, gG, gV, ref

    # lock-free epoch at the benchmark's settings
    plan = _plan(p, (U, G, V), order=None)
    r0 = plan.rmse()
    t = time.time()
    plan.epoch(0, "lockfree")
    r1 = plan.rmse()
    print(f"[large] {name} lock-free epoch: RMSE {r0:.4f} -> {r1:.4f} ({time.time() - t:.2f} s incl. RMSE)",
          flush=True)
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

    # sampled predictions
    rng = np.random.default_rng(9)
    sel = np.sort(rng.choice(p.test_idx.shape[1], 4000, replace=False))
    idx = np.ascontiguousarray(p.test_idx[:, sel])
    got = plan.predict(idx).cpu().numpy().astype(np.float64)
    want = oracle.predict(oracle.Params.from_arrays(lU, lG, lV, modes), idx)
    assert rel(got, want) <= 1e-5

