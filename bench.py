#!/usr/bin/env python3
"""Benchmark: tensor + coupled-matrix nonzero updates per second per epoch, at
a fixed held-out RMSE, on one MI355X.

Workload (default): the 3-way 1M x 100K x 100 tensor with 10M Zipf(1.2)
entries (9M train / 1M held out), Tucker core 10x10x10, one coupled 1M x 1M
matrix with 5M entries on mode 1; FP32; lock-free mode.  One "step" is one
epoch: every training tensor entry and every matrix entry updated once.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tensor+matrix nonzero updates/sec per epoch at fixed held-out RMSE, 1 GPU"
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def tensor_entry_flops(ranks):
    """Algorithmic FP operations of one tensor entry: 4K for the single-pass
    contraction (x~ and every leave-one-out vector), 2K for its share of the
    core gradient, and 10 per factor-row element for gradients, curvatures
    and the update (K = prod J)."""
    K = 1
    for j in ranks:
        K *= j
    return 6 * K + 10 * sum(ranks)


def matrix_entry_flops(rank):
    """Prediction, error, both row gradients, curvatures and updates of one
    coupled-matrix entry: about 10 flops per factor-row element."""
    return 10 * rank


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("common.hpp", "contract.hpp", "kernels.hpp", "lockfree.hpp"):
        with open(os.path.join(ROOT, "paper_1708_08640_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel sources changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_lf_tensor_cfg2_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", " ", "|")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256_16") != kernel_source_hash() or kernel not in fields.get("kernel", ""):
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_baseline(cfg, p, U, G, V, sample, seed):
    import oracle
    from synth import item_order
    params = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    order = item_order(p.n_items, seed, 0)[:sample]
    t = time.perf_counter()
    oracle.sgd_epoch(params, p, order, cfg.eta0)
    dt = time.perf_counter() - t
    return {"value": sample / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential FP64 SGD (Algorithm 1, one worker) over the first {sample:,} items of an "
                      f"epoch order of the same workload ({dt:.1f} s)"}


def scaling_sweep(args):
    """The paper's data-scalability experiment on synthetic tensors: 3-way,
    uniform indices, integer values 1..5, core 10^3, one coupled matrix on
    mode 1 with a tenth as many entries; lock-free epochs at the benchmark's
    round and hot-row settings."""
    import numpy as np
    import torch
    from paper_1708_08640_amd import S3Plan
    from synth import init_params, make_problem
    from synth.gen import UNIFORM15, Config, MatrixSpec
    if args.scaling == "dims":
        points = [(i, 1_000_000) for i in (1_000, 10_000, 100_000, 1_000_000, 10_000_000)]
    else:
        points = [(10_000, n) for n in (10_000, 100_000, 1_000_000, 10_000_000, 30_000_000)]
    for I, nnz in points:
        cfg = Config(name=f"uniform_I{I}_nnz{nnz}", dims=(I, I, I), ranks=(10, 10, 10), nnz=nnz,
                     index_law=("uniform",) * 3, value_law=UNIFORM15,
                     matrices=(MatrixSpec(mode=0, cols=I, nnz=max(nnz // 10, 1)),), dtype="f32",
                     description=f"3-way {I}^3 uniform, {nnz} nnz, core 10^3, coupled {I}x{I} on mode 1")
        log(f"scaling point I={I:,} nnz={nnz:,}: generating")
        p = make_problem(cfg)
        U, G, V = init_params(cfg)
        plan = S3Plan.from_problem(p, (U, G, V), dtype="f32", damping=True, round_items=args.round_items,
                                   seed=args.seed, hot_rows=args.hot_rows)
        for e in range(args.warmup):
            plan.epoch(e, "lockfree")
        torch.cuda.synchronize()
        steps = max(args.steps, 2)
        t0 = time.perf_counter()
        for e in range(args.warmup, args.warmup + steps):
            plan.epoch(e, "lockfree")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        print(json.dumps({"sweep": args.scaling, "I": I, "nnz_tensor_train": p.n_train,
                          "nnz_matrix": p.n_items - p.n_train, "ms_per_epoch": ms,
                          "updates_per_s": p.n_items / (ms / 1e3), "heldout_rmse": plan.rmse()}), flush=True)
        del plan
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed epochs before the timed ones")
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--mode", default="lockfree", choices=["lockfree", "det"])
    ap.add_argument("--round-items", type=int, default=524288)
    ap.add_argument("--hot-rows", type=int, default=64)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--core", default="tucker", choices=["tucker", "cp"],
                    help="cp: the hyper-diagonal core (the CP special case), measured against the HBM roof")
    ap.add_argument("--contraction", default="reuse", choices=["reuse", "naive", "matrix"],
                    help="naive: the per-entry contraction without reuse of partial products (ablation); "
                         "matrix: the dense part on the matrix cores")
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16"],
                    help="bf16: FP32 master parameters, BF16 operands on the matrix cores (needs --contraction "
                         "matrix)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="profiling runs only: entry counts of the tensor and of the sparse matrices times this "
                         "(same dimensions, ranks and rounds)")
    ap.add_argument("--cpu-sample", type=int, default=300_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--scaling", choices=["dims", "nnz"], default=None,
                    help="data-scalability sweep instead of the benchmark: epoch time of uniform 3-way tensors "
                         "against the dimensionality I (1M entries) or the entry count (I = 10K); one JSON line "
                         "per point")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times), to calibrate the HBM "
                         "byte counters of a profiler run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "copies": 3}), flush=True)
        return

    from paper_1708_08640_amd import S3Plan
    from synth import get_config, init_params, item_order, make_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.scaling:
        scaling_sweep(args)
        return
    cfg = get_config(args.config)
    if args.scale != 1.0:
        import dataclasses
        mats = tuple(m if m.nnz == cfg.dims[m.mode] * m.cols else dataclasses.replace(m, nnz=int(m.nnz * args.scale))
                     for m in cfg.matrices)
        cfg = cfg.scaled(name=f"{cfg.name}_x{args.scale:g}", nnz=int(cfg.nnz * args.scale), matrices=mats,
                         description=cfg.description + f"; entry counts x {args.scale:g} (profiling)")
    log(f"generating {cfg.name}: {cfg.description}")
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    if args.core == "cp":  # the hyper-diagonal part of the same seeded core
        G = np.array([G[(r,) * cfg.order] for r in range(cfg.ranks[0])])
    n_updates = p.n_items
    log(f"{p.n_train:,} train entries, {p.test_val.shape[0]:,} held out, {n_updates - p.n_train:,} matrix entries")
    order = item_order(p.n_items, args.seed, 0) if args.mode == "det" else None
    plan = S3Plan.from_problem(p, (U, G, V), dtype=args.dtype, batch=args.batch, order=order, damping=True,
                               round_items=args.round_items, seed=args.seed, hot_rows=args.hot_rows,
                               contraction=args.contraction, core=args.core)
    torch.cuda.synchronize()
    rmse0 = plan.rmse()
    log(f"bound; initial held-out RMSE {rmse0:.4f}")

    for e in range(args.warmup):
        plan.epoch(e, args.mode)
        torch.cuda.synchronize()
        log(f"warmup epoch {e}: RMSE {plan.rmse():.4f}")

    plan.set_profiling(True)
    kernel_ms, launches, epoch_ms = 0.0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(args.warmup, args.warmup + args.steps):
        te = time.perf_counter()
        plan.epoch(e, args.mode)
        ms, n = plan.last_epoch_profile()  # waits for the epoch
        kernel_ms += ms
        launches += n
        epoch_ms.append((time.perf_counter() - te) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_profiling(False)
    rmse = plan.rmse()
    E = args.warmup + args.steps
    log(f"timed {args.steps} epochs: {(t1 - t0) * 1e3 / args.steps:.3f} ms/epoch; RMSE after {E} epochs {rmse:.4f}")

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n_updates / (ms_per_step / 1e3)

    # held-out RMSE target from the oracle's trajectory (sequential FP64 SGD)
    target = None
    gold = os.path.join(ROOT, "tests", "golden", f"{args.config}_oracle_rmse.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        if len(g["rmse"]) >= E:
            target = 1.01 * g["rmse"][E - 1]

    mat_flops = sum(matrix_entry_flops(cfg.ranks[s.mode]) * len(p.mat_val[m]) for m, s in enumerate(cfg.matrices))
    # the timed launch (lock-free: k_lf_tensor; det: k_det_entries) also runs
    # the matrix entries
    flops = (tensor_entry_flops(cfg.ranks) * p.n_train + mat_flops) * args.steps
    achieved = flops / (kernel_ms / 1e3) / 1e12 if kernel_ms > 0 else None
    roofline = {
        "bound": "alu", "kernel": "k_lf_tensor" if args.mode == "lockfree" else "k_det_entries",
        "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
        "frac": (achieved / PEAK_FP32_VECTOR_TFLOPS) if achieved else None,
        # counters were taken for the default launch only (lock-free, reuse
        # contraction, Tucker core, 10M-entry workload, rounds of 524,288
        # items, 64 hot rows)
        "traffic": profiled_traffic("k_lf_tensor") if (args.mode == "lockfree" and cfg.name == "cfg2_zipf_10m"
                                                       and args.contraction == "reuse" and args.core == "tucker"
                                                       and args.round_items == 524288 and args.hot_rows == 64)
        else None,
        "flops_per_tensor_entry": tensor_entry_flops(cfg.ranks),
        "flops_per_matrix_entry": matrix_entry_flops(cfg.ranks[cfg.matrices[0].mode]) if cfg.matrices else None,
        "launches": launches,
        "avg_launch_ms": kernel_ms / max(launches, 1), "kernel_share_of_epoch": kernel_ms / (t1 - t0) / 1e3,
    }

    if args.core == "cp":
        # CP: O(NJ) flops per entry, so the bound is HBM: algorithmic bytes =
        # index + value stream and every touched row read and written once
        J = cfg.ranks[0]
        t_bytes = 4 * cfg.order + 4 + 2 * 4 * J * cfg.order
        m_bytes = 12 + 2 * 2 * 4 * J
        nbytes = (t_bytes * p.n_train + m_bytes * (n_updates - p.n_train)) * args.steps
        gbs = nbytes / (kernel_ms / 1e3) / 1e9 if kernel_ms > 0 else None
        roofline.update({"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": (gbs / PEAK_HBM_GBS) if gbs else None, "traffic": None,
                         "bytes_per_tensor_entry": t_bytes, "bytes_per_matrix_entry": m_bytes})
    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the FP64 oracle on {args.cpu_sample:,} items (CPU baseline)")
        cpu = cpu_baseline(cfg, p, U, G, V, args.cpu_sample, args.seed)
        log(f"oracle: {cpu['value']:.0f} updates/s")

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description}", "mode": args.mode,
                   "round_items": args.round_items if args.mode == "lockfree" else None,
                   "hot_rows": args.hot_rows if args.mode == "lockfree" else None,
                   "batch": args.batch if args.mode == "det" else None, "damping": "curvature",
                   "contraction": args.contraction, "core": args.core,
                   "updates_per_epoch": n_updates, "parallelism": "single GPU"},
        "heldout_rmse": rmse, "heldout_rmse_init": rmse0, "rmse_epochs": E, "rmse_target": target,
        "rmse_ok": (rmse <= target) if target is not None else None,
        "epoch_ms": epoch_ms,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
