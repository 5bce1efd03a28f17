"""Edge cases of the method on the GPU, against the oracle: a tensor with no
coupled matrix, a coupled matrix with no entries, rank-one cores (every
padded lane of the contraction is zero), one batch holding every item (a
full gradient step), training entries that fill whole 256-entry tiles (no
ragged tail), an empty held-out set and empty prediction requests.
Tolerances as in the det tests (FP64 1e-10)."""
import numpy as np
import pytest

import oracle
from synth.gen import MatrixSpec
from tests.gpu_util import UNIT, check_batches, compare_params, setup

pytestmark = pytest.mark.gpu

CASES = [
    ("tensor only", "cfg1", 500, dict(matrices=()), "tucker"),
    ("empty coupled matrix", "cfg1", 500, dict(matrices=(MatrixSpec(mode=0, cols=100, nnz=0),)), "tucker"),
    ("rank-one core", "tiny3", 5, dict(ranks=(1, 1, 1)), "tucker"),
    ("4-way, rank-one modes", "tiny4", 3, dict(ranks=(1, 2, 1, 2)), "tucker"),
    ("CP, J = 1", "tiny3", 5, dict(ranks=(1, 1, 1)), "cp"),
    ("one batch = every item", "cfg1", 10 ** 6, dict(), "tucker"),
    ("whole tiles, no ragged tail", "cfg1", 256, dict(nnz=569), "tucker"),
]


@pytest.mark.parametrize("what,name,batch,over,core", CASES, ids=[c[0] for c in CASES])
def test_edge_det_matches_oracle(what, name, batch, over, core):
    print(f"\n[edge] {what}", flush=True)
    cfg, p, plan, ref, order = setup(name, "f64", batch, True, core=core, **over)
    if what.startswith("whole tiles"):
        assert p.n_train % 256 == 0
    check_batches(p, plan, order, batch, 0.01, range(min(3, plan.n_batches())), True, 1e-10, UNIT["f64"], what,
                  cp=(core == "cp"))
    U, G, V = plan.params_numpy()
    ref = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices], cp=(core == "cp"))
    f, _, _ = plan.loss()
    assert abs(f - oracle.loss(ref, p)[0]) <= 1e-10 * abs(f)


@pytest.mark.parametrize("what,name,batch,over,core", CASES, ids=[c[0] for c in CASES])
def test_edge_lockfree_epoch(what, name, batch, over, core):
    cfg, p, plan, ref, order = setup(name, "f64", batch, True, core=core, round_items=256, **over)
    U0 = [u.copy() for u in ref.U]
    plan.epoch(0, "lockfree")
    U, G, V = plan.params_numpy()
    seen = [np.zeros(d, dtype=bool) for d in cfg.dims]
    for n in range(cfg.order):
        seen[n][p.train_idx[n]] = True
    for m, s in enumerate(cfg.matrices):
        seen[s.mode][p.mat_row[m]] = True
    for n in range(cfg.order):
        assert np.all(np.isfinite(U[n]))
        assert np.array_equal(U[n][~seen[n]], U0[n][~seen[n]])
    assert np.all(np.isfinite(G)) and all(np.all(np.isfinite(v)) for v in V)
    assert np.isfinite(plan.rmse())


def test_empty_heldout_set_and_empty_requests():
    cfg, p, plan, ref, order = setup("cfg1", "f64", 500, test_frac=0.0)
    assert p.test_idx.shape[1] == 0
    assert plan.rmse() == 0.0  # no held-out entry: defined as 0
    f, ft, fm = plan.loss()
    of, oft, ofm = oracle.loss(ref, p)
    assert abs(f - of) <= 1e-10 * abs(of)
    assert plan.predict(np.zeros((3, 0), dtype=np.int32)).numel() == 0
    assert plan.predict_matrix(0, np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.int32)).numel() == 0
