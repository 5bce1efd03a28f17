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
          core="tucker", with_order=True, **over):
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
    plan = S3Plan.from_problem(p, (U, G, V), dtype=dtype, batch=batch, order=order if with_order else None,
                               damping=damping,
                               round_items=round_items, seed=order_seed, contraction=contraction, core=core)
    ref = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices], cp=(core == "cp"))
    return cfg, p, plan, ref, order


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _row_rel(a, b):
    """Largest row-wise relative error (rows with a tiny reference norm are
    measured against 1e-3 of the array's root-mean-square row norm)."""
    A, B = _rows(a), _rows(b)
    nb = np.linalg.norm(B, axis=1)
    floor = 1e-3 * float(np.sqrt(np.mean(nb ** 2))) if nb.size else 0.0
    den = np.maximum(nb, max(floor, 1e-300))
    return float(np.max(np.linalg.norm(A - B, axis=1) / den)) if nb.size else 0.0


def compare_params(plan, ref, tol, what=""):
    """Every parameter array against the oracle's, normwise and row by row."""
    U, G, V = plan.params_numpy()
    worst = 0.0
    for name, a, b in ([(f"U[{n}]", a, b) for n, (a, b) in enumerate(zip(U, ref.U))] + [("G", G, ref.G)] +
                       [(f"V[{m}]", a, b) for m, (a, b) in enumerate(zip(V, ref.V))]):
        r = rel(a, b)
        rr = _row_rel(a, b)
        worst = max(worst, r, rr)
        assert r <= tol, f"{what} {name} rel {r:.3e} > {tol:g}"
        assert rr <= tol, f"{what} {name} worst row rel {rr:.3e} > {tol:g}"
    return worst


# FP32 and FP64 storage rounding: a stored value is within UNIT of its exact
# value, relatively
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -24}


def _rows(a):
    a = np.asarray(a, dtype=np.float64)
    return a.reshape(1, -1) if a.ndim != 2 else a


def check_update(got, ref, start, tol, unit, what="", row_tol=None):
    """One step's parameters against the oracle's from the same start.

    Every parameter array, normwise: ||got - ref|| <= unit ||ref|| + tol
    ||ref - start||, i.e. the update is right to `tol` relative and the stored
    result carries at most its own rounding.  Every row (the core counts as
    one): the same with row_tol (default 100 tol), which still catches a
    dropped or wrong row update (error ~ 1) but allows for a row whose summed
    contributions cancel (the sum's rounding is relative to the sum of their
    magnitudes, not to the net update).  Untouched rows must match exactly.
    Returns the largest ratio error / bound over the rows."""
    row_tol = 100 * tol if row_tol is None else row_tol
    worst = 0.0
    names = [f"U[{n}]" for n in range(len(got[0]))] + ["G"] + [f"V[{m}]" for m in range(len(got[2]))]
    for name, a, b, a0 in zip(names, list(got[0]) + [got[1]] + list(got[2]),
                              list(ref.U) + [ref.G] + list(ref.V), list(start[0]) + [start[1]] + list(start[2])):
        A, B, A0 = _rows(a), _rows(b), _rows(a0)
        assert np.all(np.isfinite(A)), f"{what} {name}: not finite"
        err = np.linalg.norm(A - B, axis=1)
        bound = unit * np.linalg.norm(B, axis=1) + row_tol * np.linalg.norm(B - A0, axis=1)
        bad = err > bound
        if np.any(bad):
            r = int(np.flatnonzero(bad)[0])
            raise AssertionError(f"{what} {name} row {r}: error {err[r]:.3e} > bound {bound[r]:.3e} "
                                 f"(|ref| {np.linalg.norm(B[r]):.3e}, |update| {np.linalg.norm(B[r] - A0[r]):.3e}); "
                                 f"{int(bad.sum())} rows over")
        moved = bound > 0
        if np.any(moved):
            worst = max(worst, float(np.max(err[moved] / bound[moved])))
        # normwise over the array as well
        dn = np.linalg.norm(B - A0)
        assert np.linalg.norm(A - B) <= unit * np.linalg.norm(B) + tol * dn, f"{what} {name}: normwise"
    return worst


def check_batches(p, plan, order, batch, eta, batches, damping, tol, unit, what="", cp=False, modes=None,
                  row_tol=None):
    """Det batches one at a time, the oracle re-synced to the plan's exported
    state before each, so each batch's update is checked on its own
    (check_update).  Returns the worst ratio over the batches."""
    modes = [s.mode for s in p.cfg.matrices] if modes is None else modes
    worst = 0.0
    for b in batches:
        start = plan.params_numpy()
        ref = oracle.Params.from_arrays(start[0], start[1], start[2], modes, cp=cp)
        plan.det_batches(b, 1, eta)
        oracle.minibatch_epoch(ref, p, order, batch, eta, b, 1, damping=damping)
        worst = max(worst, check_update(plan.params_numpy(), ref, start, tol, unit, f"{what} batch {b}", row_tol))
    return worst
