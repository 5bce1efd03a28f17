"""Per-launch timing of the dominant kernel (s3_set_profiling /
s3_last_epoch_profile), the numbers bench.py's roofline is built on: one
dispatch-stamped event pair per tensor-entry launch, durations that fit in
the epoch, and no effect on the results (det mode is bitwise reproducible,
so a profiled and an unprofiled epoch must agree exactly)."""
import time

import numpy as np
import pytest
import torch

from tests.gpu_util import setup

pytestmark = pytest.mark.gpu


def _flat(plan):
    U, G, V = plan.params_numpy()
    return np.concatenate([u.ravel() for u in U] + [G.ravel()] + [v.ravel() for v in V])


def test_det_profile_counts_batches_and_leaves_results_unchanged():
    cfg, p, plan, ref, order = setup("cfg2_slice", "f32", 4096, True)
    plan.set_profiling(True)
    t = time.perf_counter()
    plan.epoch(0, "det")
    ms, n = plan.last_epoch_profile()
    wall = (time.perf_counter() - t) * 1e3
    print(f"\n[profile] det: {n} launches, {ms:.3f} ms of {wall:.3f} ms", flush=True)
    assert n == plan.n_batches()
    assert 0.0 < ms <= wall
    profiled = _flat(plan)
    cfg, p, plain, ref, order = setup("cfg2_slice", "f32", 4096, True)
    plain.epoch(0, "det")
    assert np.array_equal(profiled, _flat(plain))
    # profiling off: the whole epoch and its batch count
    plain.epoch(1, "det")
    ms_off, n_off = plain.last_epoch_profile()
    assert n_off == plain.n_batches() and ms_off > 0.0


def test_lockfree_profile_one_pair_per_round():
    cfg, p, plan, ref, order = setup("cfg2_slice", "f32", 4096, True, round_items=8192)
    rounds = (p.n_items + 8192 - 1) // 8192
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.epoch(0, "lockfree")
    ms, n = plan.last_epoch_profile()
    wall = (time.perf_counter() - t) * 1e3
    print(f"\n[profile] lock-free: {n} launches over {rounds} rounds, {ms:.3f} ms of {wall:.3f} ms", flush=True)
    assert 1 <= n <= rounds
    assert 0.0 < ms <= wall
    plan.set_profiling(False)
    plan.epoch(1, "lockfree")
    ms_off, n_off = plan.last_epoch_profile()
    assert ms_off > 0.0 and n_off == rounds
    assert np.isfinite(plan.rmse())
