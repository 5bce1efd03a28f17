"""Lock-free mode against the oracle.

The lock-free write order differs from run to run, so the mode is judged by
its held-out RMSE at equal epochs.  A round moves the hot rows and the core
once, by their damped summed gradient, and every other row at once, without
locks; the oracle's deterministic reading of a round is the damped det
mini-batch epoch with batch = the round size (FP64).  After 20 epochs the
lock-free RMSE, averaged over two tile-shuffle seeds, is within 1 % of that
oracle's (two-sided), and each seed within 2 % (the seed-to-seed spread of
the racy runs reaches about 1 %), on every kernel shape: the vector-unit contraction at
the padded ranks (3-way 4, 8, 10, 12, 16 and ragged; 4-way 4 and 8 and
ragged) and the matrix-core contraction (FP32 and BF16 operands) at its two
shapes.  Sequential SGD (Algorithm 1, one worker) is the other reading: it
moves every row at once and is slower per epoch here; for the default shape
the lock-free RMSE is also checked to be below 1.01 times its value.  In the
first epochs large rounds on these small inputs lag both oracles (few
rounds per epoch), so the check is made once the runs have settled.
Properties that hold for any interleaving are checked as well: finite
parameters, and rows no training entry touches bitwise unchanged.
"""
import os

import numpy as np
import pytest

import oracle
from synth import item_order
from tests.gpu_util import setup

pytestmark = pytest.mark.gpu

EPOCHS = 20
THREADS = max(1, min(16, os.cpu_count() or 1))

# name, ranks (None: the configuration's), round items, contraction, dtype
SHAPES = [
    ("cfg2_slice", None, 4096, "reuse", "f32"),
    ("cfg2_slice", (4, 4, 4), 16384, "reuse", "f32"),
    ("cfg2_slice", (8, 7, 8), 16384, "reuse", "f32"),
    ("cfg2_slice", (12, 12, 12), 16384, "reuse", "f32"),
    ("cfg2_slice", (16, 16, 16), 16384, "reuse", "f32"),
    ("cfg2_slice", (16, 13, 9), 16384, "reuse", "f32"),
    ("cfg5_slice", (4, 4, 4, 4), 16384, "reuse", "f32"),
    ("cfg5_slice", (8, 8, 7, 8), 16384, "reuse", "f32"),
    ("cfg5_slice", None, 16384, "matrix", "f32"),
    ("cfg5_slice", None, 16384, "matrix", "bf16"),
    ("cfg5_slice", (8, 8, 7, 8), 16384, "matrix", "bf16"),
    ("cfg2_slice", (16, 16, 16), 16384, "matrix", "f32"),
    ("cfg2_slice", (16, 13, 9), 16384, "matrix", "bf16"),
]


def _ids(c):
    r = "x".join(map(str, c[1])) if c[1] else "cfg"
    return f"{c[0]}-{r}-r{c[2]}-{c[3]}-{c[4]}"


def _det_oracle(cfg, p, ref, rnd, epochs):
    order = item_order(p.n_items, 7, 0)
    out = []
    for ep in range(epochs):
        oracle.minibatch_epoch(ref, p, order, rnd, oracle.eta_at(cfg.eta0, cfg.mu, ep), damping=True,
                               threads=THREADS)
        out.append(oracle.rmse(ref, p.test_idx, p.test_val))
    return out


@pytest.mark.parametrize("name,ranks,rnd,contraction,dtype", SHAPES, ids=[_ids(c) for c in SHAPES])
def test_lockfree_tracks_oracle(name, ranks, rnd, contraction, dtype):
    over = {} if ranks is None else dict(ranks=ranks)
    print(f"\n[lockfree] {_ids((name, ranks, rnd, contraction, dtype))}", flush=True)
    cfg, p, plan, ref, order = setup(name, dtype, 4096, True, round_items=rnd, order_seed=7,
                                     contraction=contraction, **over)
    det = _det_oracle(cfg, p, ref.copy(), rnd, EPOCHS)
    U0 = [u.copy() for u in ref.U]
    seen = [np.zeros(d, dtype=bool) for d in cfg.dims]
    for n in range(cfg.order):
        seen[n][p.train_idx[n]] = True
    for m, s in enumerate(cfg.matrices):
        seen[s.mode][p.mat_row[m]] = True
    got = []
    for seed in (7, 8):
        if seed != 7:
            cfg, p, plan, _, _ = setup(name, dtype, 4096, True, round_items=rnd, order_seed=seed,
                                       contraction=contraction, **over)
        r = []
        for ep in range(EPOCHS):
            plan.epoch(ep, "lockfree")
            r.append(plan.rmse())
        U, G, V = plan.params_numpy()
        for n in range(cfg.order):
            assert np.all(np.isfinite(U[n])), f"U[{n}] not finite"
            assert np.array_equal(U[n][~seen[n]], U0[n][~seen[n]]), f"unobserved rows of U[{n}] changed"
        assert np.all(np.isfinite(G)) and all(np.all(np.isfinite(v)) for v in V)
        got.append(r)
    print("det oracle", " ".join(f"{v:.4f}" for v in det[::4]), f"... {det[-1]:.4f}", flush=True)
    for r in got:
        print("lock-free ", " ".join(f"{v:.4f}" for v in r[::4]), f"... {r[-1]:.4f}", flush=True)
        assert abs(r[-1] - det[-1]) <= 0.02 * det[-1], f"epoch {EPOCHS}: {r[-1]:.4f} vs oracle {det[-1]:.4f}"
    mean = float(np.mean([r[-1] for r in got]))
    assert abs(mean - det[-1]) <= 0.01 * det[-1], f"epoch {EPOCHS}: mean {mean:.4f} vs oracle {det[-1]:.4f}"
    if name == "cfg2_slice" and ranks is None:
        sgd = ref.copy()
        for ep in range(EPOCHS):
            oracle.sgd_epoch(sgd, p, item_order(p.n_items, 7, ep), oracle.eta_at(cfg.eta0, cfg.mu, ep))
        s = oracle.rmse(sgd, p.test_idx, p.test_val)
        print(f"sequential SGD after {EPOCHS} epochs: {s:.4f}", flush=True)
        assert max(r[-1] for r in got) <= 1.01 * s
