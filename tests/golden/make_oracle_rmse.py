"""Write an FP64 oracle's held-out RMSE trajectory for a configuration.

Two readings of the training loop, both from the seeded start:

* sgd: sequential SGD (Algorithm 1, one worker) with the per-epoch item
  orders item_order(n_items, seed, epoch);
* det: the damped deterministic mini-batch epoch with one fixed item order
  item_order(n_items, seed, 0) cut into batches of `batch` items (the
  library's det mode; with batch = the lock-free round size it is the
  deterministic counterpart of a lock-free round), evaluated by `threads`
  threads (bitwise the same as one).

--f32-inputs rounds the values and initial parameters to FP32 first, as the
library receives them.  Records the held-out RMSE after every epoch; the
JSON file is rewritten after every epoch, so a long run leaves its finished
epochs behind.  Calls only the oracle and the input generator.  Usage:
    python tests/golden/make_oracle_rmse.py cfg2 25 7 tests/golden/cfg2_sgd_s7.json
    python tests/golden/make_oracle_rmse.py cfg2 25 7 tests/golden/cfg2_det524288_s7.json \\
        --det 524288 --threads 4 --f32-inputs
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import get_config, init_params, item_order, make_problem  # noqa: E402


def _write(out, path):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    os.replace(tmp, path)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config")
    ap.add_argument("epochs", type=int)
    ap.add_argument("seed", type=int)
    ap.add_argument("out")
    ap.add_argument("--det", type=int, default=0, metavar="BATCH", help="det mini-batch epochs of BATCH items")
    ap.add_argument("--threads", type=int, default=1)
    ap.add_argument("--f32-inputs", action="store_true")
    a = ap.parse_args()
    t0 = time.time()
    cfg = get_config(a.config)
    p = make_problem(cfg, progress=True)
    U, G, V = init_params(cfg)
    if a.f32_inputs:
        p = dataclasses.replace(p, train_val=_f32(p.train_val), test_val=_f32(p.test_val),
                                mat_val=[_f32(v) for v in p.mat_val])
        U, G, V = [_f32(u) for u in U], _f32(G), [_f32(v) for v in V]
    params = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    mode = f"det{a.det}" if a.det else "sgd"
    out = {"config": a.config, "description": cfg.description, "mode": mode, "order_seed": a.seed,
           "batch": a.det or None, "damping": bool(a.det), "f32_inputs": a.f32_inputs,
           "n_train": p.n_train, "n_items": p.n_items, "n_test": int(p.test_val.shape[0]),
           "generate_seconds": time.time() - t0,
           "rmse_init": oracle.rmse(params, p.test_idx, p.test_val), "rmse": [], "epoch_seconds": []}
    _write(out, a.out)
    fixed = item_order(p.n_items, a.seed, 0) if a.det else None
    for ep in range(a.epochs):
        t = time.time()
        eta = oracle.eta_at(cfg.eta0, cfg.mu, ep)
        if a.det:
            oracle.minibatch_epoch(params, p, fixed, a.det, eta, damping=True, threads=a.threads)
        else:
            oracle.sgd_epoch(params, p, item_order(p.n_items, a.seed, ep), eta)
        out["epoch_seconds"].append(time.time() - t)
        out["rmse"].append(oracle.rmse(params, p.test_idx, p.test_val))
        _write(out, a.out)
        print(f"[{a.config} {mode} seed {a.seed}] epoch {ep}: rmse {out['rmse'][-1]:.6f} "
              f"({out['epoch_seconds'][-1]:.0f} s)", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
