"""The data-scalability claims (Figure 5; the per-entry cost does not depend
on the dimensionality, Lemma 5) measured on the GPU with the benchmark's
reduced sweep: lock-free epochs on uniform 3-way tensors, core 10^3, one
coupled matrix.  Epoch time may grow with I only through cache effects
(bound: 2x from I = 10^3 to 10^6 at 1M entries; measured about 1.2x) and
grows in proportion to the entry count once rounds are full (10x the entries
at I = 10^4 takes 4x..16x the time; measured about 9x)."""
import argparse
import math

import pytest

pytestmark = pytest.mark.gpu


def test_epoch_time_flat_in_dims_and_linear_in_entries():
    import bench
    args = argparse.Namespace(round_items=None, hot_rows=64, seed=7)
    sw = bench.small_sweep(args)
    for pt in sw["dims"] + sw["nnz"]:
        assert pt["ms_per_epoch"] > 0 and math.isfinite(pt["heldout_rmse"])
    assert [p["I"] for p in sw["dims"]] == [1_000, 10_000, 100_000, 1_000_000]
    assert sw["time_ratio_I_1e6_over_1e3"] < 2.0, sw
    r = sw["entries_ratio_nnz_1e7_over_1e6"]
    assert 9.5 < r < 10.5
    assert 0.4 * r < sw["time_ratio_nnz_1e7_over_1e6"] < 1.6 * r, sw
