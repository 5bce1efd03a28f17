"""Full-size checks on the 10M-entry workload (3-way 1M x 100K x 100 tensor,
Zipf(1.2) indices, core 10^3, coupled 1M x 1M matrix with 5M entries), in
the launch configurations the benchmark times.

* Det mode, batches of 65,536: the first batch against the FP64 oracle's same
  batch on the same full problem.  Compared normwise over the rows the batch
  touches (1e-5, the FP32 precision target), and over the updates themselves
  with a bound derived from FP32 storage: each stored parameter carries a
  rounding error of at most 2^-24 of its magnitude, so
  ||d_gpu - d_ref|| <= 2^-24 ||theta_new|| + 1e-5 ||d_ref||.
* Predictions at sampled held-out entries, against the oracle evaluating the
  exported parameters entry by entry.
* Lock-free mode, rounds of 524,288 items and 64 hot rows: racy by design, so
  checked through properties that hold at any size -- rows no training entry
  touches stay bitwise unchanged, everything stays finite -- and through the
  held-out RMSE against the stored FP64 oracle trajectories
  (tests/golden/, written by make_oracle_rmse.py): after 3 epochs below
  1.01 times sequential SGD's (Algorithm 1, one worker; mean of five item
  orders), the benchmark's fixed-RMSE target; after 25 epochs, over three
  tile-shuffle seeds, the mean within 1 % of the damped det mini-batch
  oracle's at the round size (each seed within 2 %) and below 1.01 times
  sequential SGD's.
* The planted variant (values with a learnable signal) at the same size:
  after 10 lock-free epochs the held-out RMSE lies between the two oracle
  readings, above 0.99 times the damped det oracle's at the round size and
  below 1.01 times sequential SGD's.  Here the lock-free runs lag the det
  oracle by about 2 % at 10 epochs and 1.5 % at 25 (0.7314 / 0.7337 against
  about 0.721): concurrent read-modify-writes of a cold row in one round
  lose updates, and on this data the rows just below the 64 hot ones (the
  100-row mode has 36 of them) carry many entries per round; with 256 hot
  rows the gap narrows (0.7264 / 0.7299 at 25 epochs).  Sequential SGD
  lags both after its first epochs (0.7648 at 10).
"""
import json
import os

import numpy as np
import pytest

import oracle
from synth import get_config, init_params, item_order, make_problem
from tests.gpu_util import rel, rounded_problem

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BATCH, ROUND, HOT, SEED = 65536, 524288, 64, 7


@pytest.fixture(scope="module")
def full():
    print("\n[fullsize] generating the 10M-entry workload", flush=True)
    cfg = get_config("cfg2")
    p = rounded_problem(make_problem(cfg), "f32")
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    U, G, V = init_params(cfg)
    return cfg, p, ([r(u) for u in U], r(G), [r(v) for v in V])


def _plan(p, params, **kw):
    from paper_1708_08640_amd import S3Plan
    return S3Plan.from_problem(p, params, dtype="f32", damping=True, seed=SEED, round_items=ROUND, hot_rows=HOT,
                               batch=BATCH, **kw)


def _touched(cfg, p, items):
    """Rows of every factor touched by the given item ids."""
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
    return [np.array(sorted(r), dtype=np.int64) for r in rows_u], [np.array(sorted(r), dtype=np.int64)
                                                                   for r in rows_v]


def test_det_first_batch_full_size(full):
    cfg, p, (U, G, V) = full
    order = item_order(p.n_items, SEED, 0)
    print("[fullsize] det bind + first batch", flush=True)
    plan = _plan(p, (U, G, V), order=order)
    eta = oracle.eta_at(cfg.eta0, cfg.mu, 0)
    plan.det_batches(0, 1, eta)
    gU, gG, gV = plan.params_numpy()
    print("[fullsize] oracle batch", flush=True)
    ref = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    oracle.minibatch_epoch(ref, p, order, BATCH, eta, 0, 1, damping=True)
    ru, rv = _touched(cfg, p, np.asarray(order[:BATCH], dtype=np.int64))
    pairs = [(f"U[{n}]", gU[n][ru[n]], ref.U[n][ru[n]], U[n][ru[n]]) for n in range(len(U))]
    pairs += [("G", gG, ref.G, G)]
    pairs += [(f"V[{m}]", gV[m][rv[m]], ref.V[m][rv[m]], V[m][rv[m]]) for m in range(len(V))]
    for name, a, b, a0 in pairs:
        assert np.all(np.isfinite(a)), name
        r = rel(a, b)
        assert r <= 1e-5, f"{name}: touched rows rel {r:.3e}"
        d_gpu, d_ref = a - a0, b - a0
        bound = 2.0 ** -24 * np.linalg.norm(b) + 1e-5 * np.linalg.norm(d_ref)
        err = np.linalg.norm(d_gpu - d_ref)
        print(f"[fullsize] {name}: rows rel {r:.2e}, update err {err:.3e} (bound {bound:.3e}, "
              f"|d| {np.linalg.norm(d_ref):.3e})", flush=True)
        assert err <= bound, f"{name}: update error {err:.3e} > {bound:.3e}"
    # every untouched row is bitwise the initial value
    for n in range(len(U)):
        mask = np.ones(U[n].shape[0], dtype=bool)
        mask[ru[n]] = False
        assert np.array_equal(gU[n][mask], U[n][mask]), f"untouched rows of U[{n}] changed"


def test_predictions_full_size(full):
    cfg, p, params = full
    plan = _plan(p, params, order=None)
    plan.epoch(0, "lockfree")
    gU, gG, gV = plan.params_numpy()
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(p.test_idx.shape[1], 4000, replace=False))
    idx = np.ascontiguousarray(p.test_idx[:, sel])
    got = plan.predict(idx).cpu().numpy().astype(np.float64)
    want = oracle.predict(oracle.Params.from_arrays(gU, gG, gV, [s.mode for s in cfg.matrices]), idx)
    r = rel(got, want)
    print(f"[fullsize] predictions rel {r:.2e}", flush=True)
    assert r <= 1e-5


def _gold(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)["rmse"]


def _mean_at(names, epoch):
    return float(np.mean([_gold(n)[epoch - 1] for n in names]))


SGD = [f"cfg2_sgd_s{s}.json" for s in (7, 8, 10, 11, 12)]
DET = [f"cfg2_det524288_s{s}.json" for s in (7, 8)]


def test_lockfree_full_size_properties(full):
    cfg, p, params = full
    U0 = params[0]
    plan = _plan(p, params, order=None)
    seen = [np.zeros(d, dtype=bool) for d in cfg.dims]
    for n in range(len(cfg.dims)):
        seen[n][p.train_idx[n]] = True
    for m, s in enumerate(cfg.matrices):
        seen[s.mode][p.mat_row[m]] = True
    rmse = []
    for e in range(3):
        plan.epoch(e, "lockfree")
        rmse.append(plan.rmse())
    print(f"[fullsize] lock-free RMSE {rmse}", flush=True)
    gU, gG, gV = plan.params_numpy()
    for n in range(len(gU)):
        assert np.all(np.isfinite(gU[n])), f"U[{n}] not finite"
        assert np.array_equal(gU[n][~seen[n]], U0[n][~seen[n]]), f"unobserved rows of U[{n}] changed"
    assert np.all(np.isfinite(gG)) and all(np.all(np.isfinite(v)) for v in gV)
    target = 1.01 * _mean_at(SGD, 3)
    assert rmse[0] < plan_init_rmse(p, params) and rmse[2] < rmse[0]
    assert rmse[2] <= target, f"epoch-3 RMSE {rmse[2]:.4f} > 1.01 x sequential SGD {target / 1.01:.4f}"


def plan_init_rmse(p, params):
    return oracle.rmse(oracle.Params.from_arrays(params[0], params[1], params[2], [s.mode for s in p.cfg.matrices]),
                       p.test_idx, p.test_val)


def test_lockfree_full_size_tracks_oracle(full):
    """25 epochs, three tile-shuffle seeds, against the stored oracles."""
    cfg, p, params = full
    from paper_1708_08640_amd import S3Plan
    got = []
    for seed in (7, 8, 9):
        plan = S3Plan.from_problem(p, params, dtype="f32", damping=True, seed=seed, round_items=ROUND,
                                   hot_rows=HOT, batch=BATCH, order=None)
        for e in range(25):
            plan.epoch(e, "lockfree")
        got.append(plan.rmse())
        del plan
    det, sgd = _mean_at(DET, 25), _mean_at(SGD, 25)
    print(f"[fullsize] lock-free RMSE after 25 epochs, seeds 7/8/9: {got}; det oracle {det:.4f}, "
          f"sequential SGD {sgd:.4f}", flush=True)
    assert all(abs(g - det) <= 0.02 * det for g in got)
    assert abs(float(np.mean(got)) - det) <= 0.01 * det
    assert max(got) <= 1.01 * sgd


def test_lockfree_planted_full_size():
    """The planted variant: a held-out RMSE with real signal to learn."""
    print("\n[fullsize] generating the planted 10M-entry workload", flush=True)
    cfg = get_config("cfg2_planted")
    p = rounded_problem(make_problem(cfg), "f32")
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    U, G, V = init_params(cfg)
    params = ([r(u) for u in U], r(G), [r(v) for v in V])
    det = _gold("cfg2_planted_det524288_s7.json")
    sgd = _gold("cfg2_planted_sgd_s7.json")
    epochs = min(len(det), len(sgd), 10)
    from paper_1708_08640_amd import S3Plan
    got = []
    for seed in (7, 8):
        plan = S3Plan.from_problem(p, params, dtype="f32", damping=True, seed=seed, round_items=ROUND,
                                   hot_rows=HOT, batch=BATCH, order=None)
        for e in range(epochs):
            plan.epoch(e, "lockfree")
        got.append(plan.rmse())
        del plan
    d, s_ = det[epochs - 1], sgd[epochs - 1]
    print(f"[fullsize] planted: lock-free RMSE after {epochs} epochs {got}, det oracle {d:.4f}, sequential SGD "
          f"{s_:.4f} (untrained {plan_init_rmse(p, params):.4f})", flush=True)
    assert all(0.99 * d <= g <= 1.01 * s_ for g in got)
