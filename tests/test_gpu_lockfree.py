"""Lock-free mode: many entries in flight, racy row updates.  The write order
differs from run to run, so it is judged statistically: held-out RMSE after
the same number of epochs as the sequential FP64 oracle (Algorithm 1, one
worker) must be within the stated relative tolerance."""
import numpy as np
import pytest

import oracle
from synth import item_order
from tests.gpu_util import setup

pytestmark = pytest.mark.gpu


def _oracle_rmse(cfg, p, ref, epochs, seed=7):
    out = []
    for ep in range(epochs):
        oracle.sgd_epoch(ref, p, item_order(p.n_items, seed, ep), oracle.eta_at(cfg.eta0, cfg.mu, ep))
        out.append(oracle.rmse(ref, p.test_idx, p.test_val))
    return out


@pytest.mark.parametrize("name,dtype,round_items,epochs,over", [
    ("cfg1", "f64", 256, 40, dict(planted=True)),
    ("cfg2_slice", "f32", 4096, 3, dict()),
])
def test_lockfree_rmse_tracks_sequential_sgd(name, dtype, round_items, epochs, over):
    print(f"\n[lockfree] {name} {dtype} round={round_items} epochs={epochs}", flush=True)
    cfg, p, plan, ref, order = setup(name, dtype, 4096, True, round_items=round_items, **over)
    want = _oracle_rmse(cfg, p, ref, epochs)
    got = []
    for ep in range(epochs):
        plan.epoch(ep, "lockfree")
        got.append(plan.rmse())
    print("oracle  ", " ".join(f"{v:.4f}" for v in want), flush=True)
    print("lockfree", " ".join(f"{v:.4f}" for v in got), flush=True)
    assert np.isfinite(got[-1])
    assert abs(got[-1] - want[-1]) <= 0.05 * want[-1]


# The other FP32 kernel shapes (every padded rank of 3-way tensors with
# Zipf data, ragged ranks that take the predicated row loads, and 4-way
# tensors), judged by properties that hold for any interleaving: everything
# stays finite, rows no training entry touches stay bitwise unchanged, and
# three epochs bring the held-out RMSE below its untrained value.
SHAPES = [
    ("cfg2_slice", (4, 4, 4)), ("cfg2_slice", (8, 7, 8)), ("cfg2_slice", (12, 12, 12)),
    ("cfg2_slice", (16, 16, 16)), ("cfg2_slice", (16, 13, 9)),
    ("cfg5_slice", (4, 4, 4, 4)), ("cfg5_slice", (8, 8, 7, 8)),
]


@pytest.mark.parametrize("name,ranks", SHAPES, ids=[f"{c[0]}-{'x'.join(map(str, c[1]))}" for c in SHAPES])
def test_lockfree_shapes_properties(name, ranks):
    print(f"\n[lockfree-shape] {name} ranks={ranks}", flush=True)
    cfg, p, plan, ref, order = setup(name, "f32", 4096, True, round_items=16384, ranks=ranks)
    U0 = [u.copy() for u in ref.U]
    r0 = plan.rmse()
    for ep in range(3):
        plan.epoch(ep, "lockfree")
    r3 = plan.rmse()
    print(f"RMSE {r0:.4f} -> {r3:.4f}", flush=True)
    U, G, V = plan.params_numpy()
    seen = [np.zeros(d, dtype=bool) for d in cfg.dims]
    for n in range(cfg.order):
        seen[n][p.train_idx[n]] = True
    for m, s in enumerate(cfg.matrices):
        seen[s.mode][p.mat_row[m]] = True
    for n in range(cfg.order):
        assert np.all(np.isfinite(U[n])), f"U[{n}] not finite"
        assert np.array_equal(U[n][~seen[n]], U0[n][~seen[n]]), f"unobserved rows of U[{n}] changed"
    assert np.all(np.isfinite(G)) and all(np.all(np.isfinite(v)) for v in V)
    assert np.isfinite(r3) and r3 < r0
