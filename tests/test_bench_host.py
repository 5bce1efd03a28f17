"""Host-side logic of bench.py (no GPU): the algorithmic work per entry behind
the roofline, the fixed-RMSE target from the stored oracle trajectories, and
the counter-summary lookup."""
import json
import os

import numpy as np

import bench

HERE = os.path.dirname(os.path.abspath(__file__))


def test_work_per_entry():
    # VALU single pass: 4K contraction + 2K core gradient + 10 per row element
    assert bench.tensor_entry_flops((10, 10, 10)) == 6 * 1000 + 10 * 30
    # matrix cores: two dense products (2 J^N multiply-adds each, in flops)
    # and the core gradient; VALU: Khatri-Rao columns, four contractions of
    # J^2 values, x~, and the row updates
    mx, valu = bench.mx_entry_work((8, 8, 8, 8))
    assert mx == 6 * 8 ** 4
    assert valu == (64 + 64) + 4 * (64 + 64) + 2 * 8 + 10 * 32
    mx3, valu3 = bench.mx_entry_work((16, 16, 16))
    assert mx3 == 6 * 16 ** 3 and valu3 == 6 * 256 + 10 * 48
    assert bench.matrix_entry_flops(8) == 80


def test_rmse_target_is_1_01_times_the_stored_sgd_mean():
    def finite_at(name, epoch):
        with open(os.path.join(HERE, "golden", name)) as f:
            r = json.load(f)["rmse"]
        return r[epoch - 1] if len(r) >= epoch and np.all(np.isfinite(r[:epoch])) else None

    for config in ("cfg2", "cfg5"):  # trajectories shorter than E* (a stopped run) do not count
        names = [n for n in os.listdir(os.path.join(HERE, "golden")) if n.startswith(f"{config}_sgd_s")]
        vals = [v for v in (finite_at(n, 3) for n in names) if v is not None]
        target, sgd, det = bench.oracle_target(config, 3)
        assert vals and abs(sgd - np.mean(vals)) < 1e-12 and abs(target - 1.01 * sgd) < 1e-12
        assert det is not None and det < sgd
    traj = bench.oracle_det_trajectory("cfg5", 524288, 2)
    assert all(t is not None for t in traj) and traj[1] < traj[0]
    assert bench.oracle_target("no_such_workload", 3) == (None, None, None)


def test_traffic_lookup_follows_the_kernel_code():
    h = bench.kernel_source_hash()
    assert len(h) == 16
    # a committed summary is used only while its hash matches the sources
    for kernel, workload in (("k_lf_tensor_mx", "cfg5_bf16"), ("k_lf_tensor", "cfg2_f32")):
        path = os.path.join(bench.ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
        with open(path) as f:
            text = f.read()
        fields = dict(line.split(":", 1) for line in text.splitlines()
                      if ":" in line and not line.startswith(("#", " ", "|")))
        stored = fields["source_sha256_16"].strip()
        expect = int(fields["traffic_bytes_per_launch"]) if stored == h else None
        assert bench.profiled_traffic(kernel, workload) == expect
    assert bench.profiled_traffic("k_lf_tensor_mx", "no_such_workload") is None


def test_epoch_log_lines(tmp_path):
    from synth import get_config
    cfg = get_config("cfg2")
    bench.EpochLog(None).write(cfg, "lockfree", "f32", "timed", 0, 2.0, 100)  # no path: nothing
    path = tmp_path / "epochs.jsonl"
    log = bench.EpochLog(str(path))
    log.write(cfg, "lockfree", "f32", "warmup", 0, 4.0, 1000, (3.0, 2.0, 1.0), 1.5)
    log.write(cfg, "lockfree", "f32", "timed", 2, 2.0, 1000)
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(recs) == 2
    a, b = recs
    assert a["epoch"] == 1 and a["eta"] == cfg.eta0 and a["updates_per_s"] == 250000.0
    assert (a["f"], a["f_t"], a["f_m"], a["heldout_rmse"]) == (3.0, 2.0, 1.0, 1.5)
    # the rate of epoch e (0-based) is eta0 / (1 + mu e)
    assert b["epoch"] == 3 and abs(b["eta"] - cfg.eta0 / (1 + 2 * cfg.mu)) < 1e-15
    assert b["f"] is None and b["heldout_rmse"] is None and b["phase"] == "timed"


def test_small_sweep_points_and_ratios(monkeypatch):
    calls = []

    def fake_point(I, nnz, round_items, hot_rows, seed, warmup=1, steps=2):
        calls.append((I, nnz))
        n_train = int(nnz * 0.9)
        return {"I": I, "nnz_tensor_train": n_train, "nnz_matrix": nnz // 10,
                "ms_per_epoch": 1.0 + I / 1e6 + nnz / 1e6, "updates_per_s": 1.0, "heldout_rmse": 3.3}

    monkeypatch.setattr(bench, "scaling_point", fake_point)
    import argparse
    sw = bench.small_sweep(argparse.Namespace(round_items=None, hot_rows=64, seed=7))
    assert calls == [(1_000, 1_000_000), (10_000, 1_000_000), (100_000, 1_000_000), (1_000_000, 1_000_000),
                     (10_000, 100_000), (10_000, 10_000_000)]
    # the 1M-entry point at I = 10^4 is shared by both sweeps
    assert [p["nnz_tensor_train"] + p["nnz_matrix"] for p in sw["nnz"]] == [100_000, 1_000_000, 10_000_000]
    assert sw["nnz"][1] is sw["dims"][1]
    assert abs(sw["time_ratio_I_1e6_over_1e3"] - (1.0 + 1.0 + 1.0) / (1.0 + 0.001 + 1.0)) < 1e-12
    assert abs(sw["time_ratio_nnz_1e7_over_1e6"] - (1.0 + 0.01 + 10.0) / (1.0 + 0.01 + 1.0)) < 1e-12
    assert sw["entries_ratio_nnz_1e7_over_1e6"] == 10.0


def test_cp_entry_bytes():
    # 3-way rank 10 FP32: 12 B of indices + 4 B value + 3 rows of 40 B read and written
    assert bench.cp_entry_bytes(3, 10, "f32") == (16 + 240, 12 + 160)
    # FP64 doubles the value and row bytes, not the 4-byte indices
    assert bench.cp_entry_bytes(4, 8, "f64") == (16 + 8 + 2 * 8 * 8 * 4, 8 + 8 + 4 * 8 * 8)
