#!/usr/bin/env python3
"""Benchmark: tensor + coupled-matrix nonzero updates per second per epoch, at
a fixed held-out RMSE, on one MI355X.

Workload (default, the largest configuration): the 4-way 1M x 500K x 1000 x
24 tensor with 200M Zipf(1.2) entries (180M train / 20M held out), Tucker
core 8^4, three coupled matrices (1M x 1M with 30M entries, 500K x 300 with
20M, a dense 1000 x 50); lock-free mode; the dense part of the contraction on
the matrix cores with BF16 operands, FP32 master parameters.  One "step" is
one epoch: every training tensor entry and every matrix entry updated once.
The 10M-entry 3-way workload (FP32, vector-unit contraction) is measured
after it and reported as secondary keys.

Fixed held-out RMSE: after the timed epochs the parameters are reset to
their initial values and E* epochs are run again; the held-out RMSE after
epoch E* must be at most 1.01 times the FP64 oracle's sequential SGD
(Algorithm 1, one worker) at E* (tests/golden/).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tensor+matrix nonzero updates/sec per epoch at fixed held-out RMSE, 1 GPU"
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
E_STAR = {"cfg2": 3, "cfg5": 3}
# lock-free round size per workload (items per round): the 10M-entry
# workload's held-out RMSE after 3 epochs worsens with larger rounds (1 %
# margin left at 1,048,576), the 4-way workload's does not (1.3261-1.3311 over
# 393,216-1,048,576), where 786,432 items (2,403 tensor tiles, 5 per
# persistent workgroup) gave the shortest epoch
ROUND_ITEMS = {"cfg5": 786432}
DEFAULT_ROUND = 524288
# det-mode batch per workload: on the 4-way workload the batch of the stored
# det oracle trajectory (larger batches: fewer launches and a lower RMSE per
# epoch there), 65,536 otherwise
DET_BATCH = {"cfg5": 524288}
DEFAULT_BATCH = 65536


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


class EpochLog:
    """One JSON line per epoch appended to a file (nothing without a path):
    workload, mode, operand type, phase (warmup, timed, quality), epoch, the
    epoch's learning rate eta0 / (1 + mu e), its wall time and update rate,
    and where they are evaluated (not inside the timed region) the loss terms
    f, f_t, f_m of Eq (7) and the held-out RMSE."""

    def __init__(self, path):
        self.path = path

    def write(self, cfg, mode, dtype, phase, epoch, ms, updates, loss=None, rmse=None):
        if not self.path:
            return
        rec = {"workload": cfg.name, "mode": mode, "dtype": dtype, "phase": phase, "epoch": epoch + 1,
               "eta": cfg.eta0 / (1.0 + cfg.mu * epoch), "epoch_ms": ms,
               "updates_per_s": updates / (ms / 1e3) if ms > 0 else None,
               "f": None if loss is None else loss[0], "f_t": None if loss is None else loss[1],
               "f_m": None if loss is None else loss[2], "heldout_rmse": rmse}
        with open(self.path, "a") as f:
            f.write(json.dumps(rec) + "\n")


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


def cp_entry_bytes(order, J, dtype):
    """Algorithmic HBM bytes of one entry with the CP core, as (tensor,
    matrix): the index and value stream, and every factor row the entry
    touches read and written once (values and parameters of 8 bytes in FP64,
    4 otherwise)."""
    es = 8 if dtype == "f64" else 4
    return 4 * order + es + 2 * es * J * order, 8 + es + 2 * 2 * es * J


def kernel_source_hash():
    """Hash of the kernel sources' code (comments and blank space removed, so
    that editing a comment does not orphan the committed counter summaries)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("common.hpp", "contract.hpp", "kernels.hpp", "lockfree.hpp", "mfma.hpp", "plan.hpp"):
        with open(os.path.join(ROOT, "paper_1708_08640_amd", "csrc", f)) as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary, or None when there is none or the kernel sources changed
    since those counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", " ", "|")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256_16") != kernel_source_hash() or fields.get("kernel", "") != kernel:
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(cfg, p, U, G, V, sample, seed, batch):
    """The FP64 oracle on the host cores, on the first `sample` items of an
    item order of the same workload: the deterministic mini-batch epoch
    evaluated by one thread per core (the value), and sequential SGD on one
    core (Algorithm 1 with one worker, reported beside it)."""
    import oracle
    from synth import item_order
    nproc, model = cpu_info()
    threads = min(nproc, 16)
    order = item_order(p.n_items, seed, 0)[:sample]
    params = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    t = time.perf_counter()
    oracle.minibatch_epoch(params, p, order, min(batch, sample), cfg.eta0, damping=True, threads=threads)
    dt_det = time.perf_counter() - t
    n_seq = max(1, sample // 8)
    params = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    t = time.perf_counter()
    oracle.sgd_epoch(params, p, order[:n_seq], cfg.eta0)
    dt_seq = time.perf_counter() - t
    return {"value": sample / dt_det, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 det mini-batch oracle (damped, batches of {min(batch, sample):,}, {threads} threads, "
                      f"bitwise the one-thread result) over the first {sample:,} items of an epoch order of the "
                      f"same workload ({dt_det:.1f} s); host: {nproc} logical CPUs, {model}",
            "sequential_sgd_value": n_seq / dt_seq,
            "sequential_sgd_sample": f"sequential FP64 SGD (Algorithm 1, one worker, 1 core) over the first "
                                     f"{n_seq:,} of those items ({dt_seq:.1f} s)",
            "nproc": nproc, "cpu_model": model}


def oracle_target(config, epoch):
    """1.01 x the mean over item orders of the stored sequential-SGD oracle
    RMSE after `epoch` epochs, and the det oracle's (round size) beside it."""
    import glob
    sgd, det = [], []
    for f in glob.glob(os.path.join(ROOT, "tests", "golden", f"{config}_sgd_s*.json")):
        with open(f) as fh:
            r = json.load(fh)["rmse"]
        if len(r) >= epoch and all(np.isfinite(r[:epoch])):
            sgd.append(r[epoch - 1])
    for f in glob.glob(os.path.join(ROOT, "tests", "golden", f"{config}_det524288_s*.json")):
        with open(f) as fh:
            r = json.load(fh)["rmse"]
        if len(r) >= epoch:
            det.append(r[epoch - 1])
    return (1.01 * float(np.mean(sgd)) if sgd else None, float(np.mean(sgd)) if sgd else None,
            float(np.mean(det)) if det else None)


def scaling_point(I, nnz, round_items, hot_rows, seed, warmup=1, steps=2):
    """One point of the paper's data-scalability experiment (Figure 5) on a
    synthetic tensor: 3-way I x I x I, uniform indices, integer values 1..5,
    core 10^3, one coupled I x I matrix on mode 1 with a tenth as many
    entries; lock-free epochs.  Returns its epoch time and update rate."""
    import torch
    from paper_1708_08640_amd import S3Plan
    from synth import init_params, make_problem
    from synth.gen import UNIFORM15, Config, MatrixSpec
    cfg = Config(name=f"uniform_I{I}_nnz{nnz}", dims=(I, I, I), ranks=(10, 10, 10), nnz=nnz,
                 index_law=("uniform",) * 3, value_law=UNIFORM15,
                 matrices=(MatrixSpec(mode=0, cols=I, nnz=max(nnz // 10, 1)),), dtype="f32",
                 description=f"3-way {I}^3 uniform, {nnz} nnz, core 10^3, coupled {I}x{I} on mode 1")
    log(f"scaling point I={I:,} nnz={nnz:,}: generating")
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    plan = S3Plan.from_problem(p, (U, G, V), dtype="f32", damping=True, round_items=round_items, seed=seed,
                               hot_rows=hot_rows)
    for e in range(warmup):
        plan.epoch(e, "lockfree")
    torch.cuda.synchronize()
    steps = max(steps, 2)
    t0 = time.perf_counter()
    for e in range(warmup, warmup + steps):
        plan.epoch(e, "lockfree")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = {"I": I, "nnz_tensor_train": p.n_train, "nnz_matrix": p.n_items - p.n_train, "ms_per_epoch": ms,
           "updates_per_s": p.n_items / (ms / 1e3), "heldout_rmse": plan.rmse()}
    del plan
    torch.cuda.empty_cache()
    return out


def scaling_sweep(args):
    """The data-scalability sweeps, one JSON line per point: the dimensionality
    I at 1M entries, or the entry count at I = 10K."""
    if args.scaling == "dims":
        points = [(i, 1_000_000) for i in (1_000, 10_000, 100_000, 1_000_000, 10_000_000)]
    else:
        points = [(10_000, n) for n in (10_000, 100_000, 1_000_000, 10_000_000, 30_000_000)]
    for I, nnz in points:
        pt = scaling_point(I, nnz, args.round_items or DEFAULT_ROUND, args.hot_rows, args.seed, args.warmup,
                           args.steps)
        print(json.dumps({"sweep": args.scaling, **pt}), flush=True)


def small_sweep(args):
    """A reduced sweep reported beside the headline: epoch time against I
    (10^3 .. 10^6 at 1M entries) and against the entry count (10^5 .. 10^7
    at I = 10^4), with the two ratios the paper's claims are about: time
    flat in I, linear in the entry count."""
    rnd = args.round_items or DEFAULT_ROUND
    dims = [scaling_point(i, 1_000_000, rnd, args.hot_rows, args.seed, 1, 3) for i in (1_000, 10_000, 100_000,
                                                                                       1_000_000)]
    nnz = [scaling_point(10_000, n, rnd, args.hot_rows, args.seed, 1, 3) for n in (100_000, 10_000_000)]
    nnz.insert(1, dims[1])
    return {"dims": dims, "nnz": nnz,
            "time_ratio_I_1e6_over_1e3": dims[-1]["ms_per_epoch"] / dims[0]["ms_per_epoch"],
            "time_ratio_nnz_1e7_over_1e6": nnz[-1]["ms_per_epoch"] / nnz[1]["ms_per_epoch"],
            "entries_ratio_nnz_1e7_over_1e6": (nnz[-1]["nnz_tensor_train"] + nnz[-1]["nnz_matrix"]) /
                                              (nnz[1]["nnz_tensor_train"] + nnz[1]["nnz_matrix"])}


def mx_entry_work(ranks):
    """Algorithmic work of one tensor entry in the matrix-core contraction,
    as (matrix-core flops, VALU flops).  Matrix cores: the two dense products
    (2 J^N multiply-adds each) and the entry's share of the core gradient
    (J^N), 6 J^N flops in all.  VALU, 4-way: the two Khatri-Rao columns
    (J1 J2 + J3 J4 products), the four leave-one-out contractions of the
    products' outputs (2 (J1 J2 + J3 J4) multiply-adds) and x~ (J4); 3-way:
    the contractions of the two mode products' tails (3 J2 J3 multiply-adds).
    Both: 10 flops per row element for gradients, curvatures and updates."""
    K = 1
    for j in ranks:
        K *= j
    if len(ranks) == 4:
        kr = ranks[0] * ranks[1] + ranks[2] * ranks[3]
        valu = kr + 4 * kr + 2 * ranks[3]
    else:
        valu = 6 * (K // ranks[0])
    return 6 * K, valu + 10 * sum(ranks)


def generate(args, config):
    from synth import get_config, init_params, make_problem
    cfg = get_config(config)
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
    log(f"{p.n_train:,} train entries, {p.test_val.shape[0]:,} held out, {p.n_items - p.n_train:,} matrix entries")
    return cfg, p, U, G, V


def round_items(args, config):
    return args.round_items or ROUND_ITEMS.get(config, DEFAULT_ROUND)


def det_batch(args, config):
    return args.batch or DET_BATCH.get(config, DEFAULT_BATCH)


def oracle_det_trajectory(config, batch, epochs):
    """Mean over item orders of the stored det oracle RMSE after epochs
    1..epochs at this batch size (None where not stored)."""
    import glob
    runs = []
    for f in glob.glob(os.path.join(ROOT, "tests", "golden", f"{config}_det{batch}_s*.json")):
        with open(f) as fh:
            runs.append(json.load(fh)["rmse"])
    return [float(np.mean([r[e] for r in runs if len(r) > e])) if any(len(r) > e for r in runs) else None
            for e in range(epochs)]


def run(args, data, config, contraction, dtype, mode, steps, warmup, cpu=False):
    import torch
    from paper_1708_08640_amd import S3Plan
    from synth import item_order
    cfg, p, U, G, V = data
    n_updates = p.n_items
    order = item_order(p.n_items, args.seed, 0) if mode == "det" else None
    plan = S3Plan.from_problem(p, (U, G, V), dtype=dtype, batch=det_batch(args, config), order=order, damping=True,
                               round_items=round_items(args, config), seed=args.seed, hot_rows=args.hot_rows,
                               contraction=contraction, core=args.core)
    torch.cuda.synchronize()
    rmse0 = plan.rmse()
    log(f"bound; initial held-out RMSE {rmse0:.4f}")
    elog = EpochLog(args.epoch_log)
    for e in range(warmup):
        te = time.perf_counter()
        plan.epoch(e, mode)
        torch.cuda.synchronize()
        wms = (time.perf_counter() - te) * 1e3
        r = plan.rmse()
        log(f"warmup epoch {e}: RMSE {r:.4f}")
        elog.write(cfg, mode, dtype, "warmup", e, wms, n_updates, plan.loss() if elog.path else None, r)

    plan.set_profiling(True)
    kernel_ms, launches, epoch_ms = 0.0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(warmup, warmup + steps):
        te = time.perf_counter()
        plan.epoch(e, mode)
        ms, n = plan.last_epoch_profile()  # waits for the epoch
        kernel_ms += ms
        launches += n
        epoch_ms.append((time.perf_counter() - te) * 1e3)
        elog.write(cfg, mode, dtype, "timed", e, epoch_ms[-1], n_updates)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_profiling(False)
    E = warmup + steps
    rmse = plan.rmse()
    ms_per_step = (t1 - t0) * 1e3 / steps
    log(f"timed {steps} epochs: {ms_per_step:.3f} ms/epoch; RMSE after {E} epochs {rmse:.4f}")

    # fixed held-out RMSE: E* epochs again from the initial parameters
    estar = E_STAR.get(config, 3)
    with torch.no_grad():
        for dst, src in zip(plan.U + [plan.G] + plan.V, U + [G] + V):
            dst.copy_(torch.as_tensor(np.asarray(src), dtype=dst.dtype))
    traj = []
    for e in range(estar):
        te = time.perf_counter()
        plan.epoch(e, mode)
        traj.append(plan.rmse())
        if elog.path:
            elog.write(cfg, mode, dtype, "quality", e, (time.perf_counter() - te) * 1e3, n_updates, plan.loss(),
                       traj[-1])
    target, sgd_mean, det_mean = oracle_target(config, estar) if args.scale == 1.0 else (None, None, None)
    log(f"quality pass: RMSE after epochs 1..{estar}: {' '.join(f'{v:.4f}' for v in traj)}; target "
        f"{target if target is None else round(target, 4)}")

    # roofline of the dominant kernel (the round kernel, or the det entries kernel)
    mat_flops = sum(matrix_entry_flops(cfg.ranks[s.mode]) * len(p.mat_val[m]) for m, s in enumerate(cfg.matrices))
    secs = kernel_ms / 1e3
    kname = ("k_lf_tensor_mx" if contraction == "matrix" else "k_lf_tensor") if mode == "lockfree" else "k_det_entries"
    default_shape = (args.scale == 1.0 and args.core == "tucker" and args.round_items is None
                     and args.hot_rows == 64 and mode == "lockfree")
    traffic = profiled_traffic(kname, f"{config}_{dtype}") if default_shape else None
    if contraction == "matrix":
        # the bound is whichever share takes longer at its peak: the
        # matrix-core flops (BF16 or FP32 rate) or the VALU flops
        mx, valu = mx_entry_work(cfg.ranks)
        peak = PEAK_BF16_MFMA_TFLOPS if dtype == "bf16" else PEAK_FP32_MFMA_TFLOPS
        mx_flops = mx * p.n_train * steps
        valu_flops = (valu * p.n_train + mat_flops) * steps
        mx_t = mx_flops / secs / 1e12 if secs > 0 else None
        valu_t = valu_flops / secs / 1e12 if secs > 0 else None
        mx_roof = mx_flops / (peak * 1e12)
        valu_roof = valu_flops / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
        mfma = {"achieved": mx_t, "peak": peak, "unit": "TFLOP/s", "frac": (mx_t / peak) if mx_t else None,
                "flops_per_tensor_entry": mx, "dtype": dtype}
        valu_d = {"achieved": valu_t, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                  "frac": (valu_t / PEAK_FP32_VECTOR_TFLOPS) if valu_t else None, "flops_per_tensor_entry": valu}
        main_, other, bound = (mfma, valu_d, "mfma") if mx_roof >= valu_roof else (valu_d, mfma, "alu")
        roofline = {"bound": bound, "kernel": kname, "achieved": main_["achieved"], "peak": main_["peak"],
                    "unit": "TFLOP/s", "frac": main_["frac"], "traffic": traffic,
                    "flops_per_tensor_entry": main_["flops_per_tensor_entry"],
                    ("valu" if bound == "mfma" else "mfma"): other,
                    "time_at_roof_fraction": (mx_roof + valu_roof) / secs if secs > 0 else None}
    else:
        flops = (tensor_entry_flops(cfg.ranks) * p.n_train + mat_flops) * steps
        achieved = flops / secs / 1e12 if secs > 0 else None
        vpeak = PEAK_FP64_VECTOR_TFLOPS if dtype == "f64" else PEAK_FP32_VECTOR_TFLOPS
        roofline = {"bound": "alu", "kernel": kname,
                    "achieved": achieved, "peak": vpeak, "unit": "TFLOP/s",
                    "frac": (achieved / vpeak) if achieved else None,
                    "traffic": traffic,
                    "flops_per_tensor_entry": tensor_entry_flops(cfg.ranks)}
    roofline.update({"launches": launches, "avg_launch_ms": kernel_ms / max(launches, 1),
                     "kernel_share_of_epoch": kernel_ms / (t1 - t0) / 1e3,
                     "flops_per_matrix_entry": matrix_entry_flops(cfg.ranks[cfg.matrices[0].mode]) if cfg.matrices
                     else None})
    if args.core == "cp":
        # CP: O(NJ) flops per entry, so the bound is HBM: algorithmic bytes =
        # index + value stream and every touched row read and written once
        t_bytes, m_bytes = cp_entry_bytes(cfg.order, cfg.ranks[0], dtype)
        nbytes = (t_bytes * p.n_train + m_bytes * (n_updates - p.n_train)) * steps
        gbs = nbytes / secs / 1e9 if secs > 0 else None
        roofline.update({"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": (gbs / PEAK_HBM_GBS) if gbs else None, "traffic": None,
                         "bytes_per_tensor_entry": t_bytes, "bytes_per_matrix_entry": m_bytes})
    out = {"cfg": cfg, "ms_per_step": ms_per_step, "value": n_updates / (ms_per_step / 1e3),
           "updates_per_epoch": n_updates, "heldout_rmse": rmse, "heldout_rmse_init": rmse0, "rmse_epochs": E,
           "epoch_ms": epoch_ms, "roofline": roofline, "rmse_estar": estar, "rmse_trajectory": traj,
           "rmse_target": target, "rmse_ok": (traj[-1] <= target) if target is not None else None,
           "oracle_sgd_rmse": sgd_mean, "oracle_det_rmse": det_mean}
    del plan
    torch.cuda.empty_cache()
    if cpu:
        log(f"timing the FP64 oracle on {args.cpu_sample:,} items (CPU baseline)")
        out["cpu"] = cpu_baseline(cfg, p, U, G, V, args.cpu_sample, args.seed, DEFAULT_BATCH)
        log(f"oracle: {out['cpu']['value']:.0f} updates/s ({out['cpu']['cores']} threads), sequential "
            f"{out['cpu']['sequential_sgd_value']:.0f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed epochs before the timed ones")
    ap.add_argument("--config", default="cfg5")
    ap.add_argument("--mode", default="lockfree", choices=["lockfree", "det"])
    ap.add_argument("--round-items", type=int, default=None,
                    help="lock-free items per round (default: 786,432 for cfg5, 524,288 otherwise)")
    ap.add_argument("--hot-rows", type=int, default=64)
    ap.add_argument("--batch", type=int, default=None,
                    help="det-mode items per batch (default: 524,288 for cfg5, 65,536 otherwise)")
    ap.add_argument("--core", default="tucker", choices=["tucker", "cp"],
                    help="cp: the hyper-diagonal core (the CP special case), measured against the HBM roof")
    ap.add_argument("--contraction", default=None, choices=["reuse", "naive", "matrix"],
                    help="reuse: the single pass on the vector units; naive: without reuse of partial products "
                         "(ablation); matrix: the dense part on the matrix cores (default where it is built)")
    ap.add_argument("--dtype", default=None, choices=["f64", "f32", "bf16"],
                    help="bf16: FP32 master parameters, BF16 operands on the matrix cores (default with the "
                         "matrix contraction); f64: FP64 throughout, on the vector units")
    ap.add_argument("--no-f32-compare", action="store_true",
                    help="skip the FP32-operand run of the same workload that follows a BF16 headline")
    ap.add_argument("--no-det-compare", action="store_true",
                    help="skip the det mini-batch run of the same workload that follows a lock-free headline")
    ap.add_argument("--secondary", default="cfg2", help="second workload reported as extra keys ('none' for none)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="profiling runs only: entry counts of the tensor and of the sparse matrices times this "
                         "(same dimensions, ranks and rounds)")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the reduced data-scalability sweep reported beside the headline")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--epoch-log", default=None, metavar="PATH",
                    help="append one JSON line per epoch (warmup, timed, quality pass) to PATH")
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

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.scaling:
        scaling_sweep(args)
        return

    def defaults(config):
        from synth import get_config
        c = get_config(config)
        jp = max(c.ranks)
        built = (c.order == 4 and 5 <= jp <= 8) or (c.order == 3 and 13 <= jp <= 16)
        ct = args.contraction or ("matrix" if (built and args.core == "tucker" and args.dtype != "f64")
                                  else "reuse")
        dt = args.dtype or ("bf16" if ct == "matrix" else "f32")
        return ct, dt

    ct, dt = defaults(args.config)
    if dt == "f64" and args.mode == "lockfree":
        # FP64 staging of a tile's rows alone exceeds the 64 KB LDS budget of
        # the round kernel at 3-way rank 10 and 4-way rank 8
        print("bench.py: FP64 runs in det mode only on these workloads (--mode det)", file=sys.stderr)
        sys.exit(2)
    data = generate(args, args.config)
    head = run(args, data, args.config, ct, dt, args.mode, args.steps, args.warmup, cpu=not args.no_cpu_baseline)
    cfg = head["cfg"]
    extra = {}
    if dt == "bf16" and not args.no_f32_compare:
        # the same workload, plan settings and tile seed with FP32 operands
        f = run(args, data, args.config, ct, "f32", args.mode, args.steps, args.warmup)
        extra["fp32_same_gpu"] = {
            "dtype": "f32", "contraction": ct, "value": f["value"], "unit": "updates/s",
            "ms_per_step": f["ms_per_step"], "heldout_rmse": f["heldout_rmse"], "rmse_epochs": f["rmse_epochs"],
            "rmse_trajectory": f["rmse_trajectory"], "rmse_ok": f["rmse_ok"],
            "bf16_speedup": head["value"] / f["value"],
            "bf16_minus_fp32_final_rmse": head["rmse_trajectory"][-1] - f["rmse_trajectory"][-1],
            "roofline": f["roofline"]}
    if args.mode == "lockfree" and not args.no_det_compare:
        # the deterministic mini-batch mode on the same workload and operands
        d = run(args, data, args.config, ct, dt, "det", args.steps, args.warmup)
        extra["det_mode"] = {
            "dtype": dt, "contraction": ct, "batch": det_batch(args, args.config), "damping": "curvature",
            "value": d["value"],
            "oracle_det_rmse_trajectory": oracle_det_trajectory(args.config, det_batch(args, args.config),
                                                                len(d["rmse_trajectory"])),
            "unit": "updates/s", "ms_per_step": d["ms_per_step"], "heldout_rmse": d["heldout_rmse"],
            "rmse_epochs": d["rmse_epochs"], "rmse_trajectory": d["rmse_trajectory"], "rmse_ok": d["rmse_ok"],
            "roofline": d["roofline"]}
    del data
    if args.secondary not in ("", "none") and args.secondary != args.config:
        sct, sdt = defaults(args.secondary)
        sec = run(args, generate(args, args.secondary), args.secondary, sct, sdt, args.mode, args.steps,
                  args.warmup)
        extra["secondary"] = {
            "workload": f"{sec['cfg'].name}: {sec['cfg'].description}", "contraction": sct, "dtype": sdt,
            "value": sec["value"], "unit": "updates/s", "ms_per_step": sec["ms_per_step"],
            "heldout_rmse": sec["heldout_rmse"], "rmse_epochs": sec["rmse_epochs"],
            "rmse_estar": sec["rmse_estar"], "rmse_trajectory": sec["rmse_trajectory"],
            "rmse_target": sec["rmse_target"], "rmse_ok": sec["rmse_ok"],
            "oracle_sgd_rmse": sec["oracle_sgd_rmse"], "oracle_det_rmse": sec["oracle_det_rmse"],
            "roofline": sec["roofline"]}
    if not args.no_sweep:
        # the data-scalability sweep, reduced; a failure here leaves the
        # headline intact and is reported in its place
        try:
            extra["scaling_sweep"] = small_sweep(args)
        except Exception as exc:  # noqa: BLE001
            log(f"scaling sweep failed: {exc!r}")
            extra["scaling_sweep"] = {"error": repr(exc)}
    out = {
        "metric": METRIC, "value": head["value"], "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description}", "mode": args.mode,
                   "round_items": round_items(args, args.config) if args.mode == "lockfree" else None,
                   "hot_rows": args.hot_rows if args.mode == "lockfree" else None,
                   "batch": det_batch(args, args.config) if args.mode == "det" else None, "damping": "curvature",
                   "contraction": ct, "core": args.core, "master_dtype": "f32",
                   "updates_per_epoch": head["updates_per_epoch"], "parallelism": "single GPU"},
        "heldout_rmse": head["heldout_rmse"], "heldout_rmse_init": head["heldout_rmse_init"],
        "rmse_epochs": head["rmse_epochs"], "rmse_estar": head["rmse_estar"],
        "rmse_trajectory": head["rmse_trajectory"], "rmse_target": head["rmse_target"],
        "rmse_ok": head["rmse_ok"], "oracle_sgd_rmse": head["oracle_sgd_rmse"],
        "oracle_det_rmse": head["oracle_det_rmse"], "epoch_ms": head["epoch_ms"],
        "roofline": head["roofline"], "cpu_baseline": head.get("cpu"),
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
