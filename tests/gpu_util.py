"""Shared set-up for the GPU parity tests: the same seeded inputs feed the
oracle and the library (the library's FP32 runs start from FP32-rounded
inputs, and the oracle is given those same rounded values)."""
import dataclasses

import numpy as np

import oracle
from synth import get_config, init_params, item_order, make_problem


def rounded_problem(p, dtype):
    if dtype == "f64":
        return p
    f = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    return dataclasses.replace(p, train_val=f(p.train_val), test_val=f(p.test_val),
                               mat_val=[f(v) for v in p.mat_val])


def setup(name, dtype="f64", batch=512, damping=False, order_seed=123, round_items=65536, contraction="reuse",
          core="tucker", **over):
    from paper_1708_08640_amd import S3Plan
    cfg = get_config(name, **over)
    p = rounded_problem(make_problem(cfg), dtype)
    U, G, V = init_params(cfg)
    if core == "cp":  # the hyper-diagonal part of the same seeded core
        G = np.array([G[(r,) * cfg.order] for r in range(cfg.ranks[0])])
    if dtype in ("f32", "bf16"):  # bf16 plans keep FP32 parameters (the master copies)
        r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
        U, G, V = [r(u) for u in U], r(G), [r(v) for v in V]
    order = item_order(p.n_items, order_seed, 0)
    plan = S3Plan.from_problem(p, (U, G, V), dtype=dtype, batch=batch, order=order, damping=damping,
                               round_items=round_items, seed=order_seed, contraction=contraction, core=core)
    ref = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices], cp=(core == "cp"))
    return cfg, p, plan, ref, order


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def compare_params(plan, ref, tol, what=""):
    U, G, V = plan.params_numpy()
    worst = 0.0
    for n, (a, b) in enumerate(zip(U, ref.U)):
        r = rel(a, b)
        worst = max(worst, r)
        assert r <= tol, f"{what} U[{n}] rel {r:.3e} > {tol:g}"
    r = rel(G, ref.G)
    worst = max(worst, r)
    assert r <= tol, f"{what} G rel {r:.3e} > {tol:g}"
    for m, (a, b) in enumerate(zip(V, ref.V)):
        r = rel(a, b)
        worst = max(worst, r)
        assert r <= tol, f"{what} V[{m}] rel {r:.3e} > {tol:g}"
    return worst
