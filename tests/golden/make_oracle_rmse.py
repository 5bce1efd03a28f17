"""Write the FP64 oracle's held-out RMSE trajectory for a configuration.

Runs sequential SGD (Algorithm 1, one worker) from the seeded start with the
per-epoch item orders item_order(n_items, seed, epoch), and records the
held-out RMSE after every epoch.  Calls only the oracle and the input
generator.  The JSON file is rewritten after every epoch, so a long run
leaves its finished epochs behind.  Usage:
    python tests/golden/make_oracle_rmse.py cfg2 25 7 tests/golden/cfg2_oracle_rmse_s7.json
"""
import json
import os
import sys
import time

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


def main(name, epochs, seed, path):
    t0 = time.time()
    cfg = get_config(name)
    p = make_problem(cfg, progress=True)
    U, G, V = init_params(cfg)
    params = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    out = {"config": name, "description": cfg.description, "order_seed": seed,
           "n_train": p.n_train, "n_items": p.n_items, "n_test": int(p.test_val.shape[0]),
           "generate_seconds": time.time() - t0,
           "rmse_init": oracle.rmse(params, p.test_idx, p.test_val), "rmse": [], "epoch_seconds": []}
    _write(out, path)
    for ep in range(epochs):
        t = time.time()
        oracle.sgd_epoch(params, p, item_order(p.n_items, seed, ep), oracle.eta_at(cfg.eta0, cfg.mu, ep))
        out["epoch_seconds"].append(time.time() - t)
        out["rmse"].append(oracle.rmse(params, p.test_idx, p.test_val))
        _write(out, path)
        print(f"[{name} seed {seed}] epoch {ep}: rmse {out['rmse'][-1]:.6f} ({out['epoch_seconds'][-1]:.0f} s)",
              file=sys.stderr, flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]), sys.argv[4])
