"""Synthetic COO tensors and coupled matrices shaped like the paper's workloads.

The paper evaluates on rating tensors (user, item, time; rating) coupled to
side-information matrices (Table 4) and on synthetic 3-mode tensors whose
dimensionality and entry count it sweeps (Section 4.1, "Data"). Those
datasets are not available here; the configurations below stand in for them
with the same kind of structure: power-law (bounded Zipf) mode indices,
integer ratings 1-5, coupled matrices sharing one tensor mode.

Recipe:

* Mode indices: bounded Zipf, P(rank r) proportional to r^-s for r = 1..I,
  sampled by inverse CDF, then mapped rank -> index through a seeded
  permutation of the mode (so hot rows are scattered, not index 0). A matrix
  coupled to mode c maps its row ranks through mode c's permutation, so the
  hot rows of the matrix and of the tensor mode coincide; its column ranks
  use a permutation of their own. "uniform" draws indices uniformly.
* Entries form a set (the paper's index set Omega): duplicates are removed
  and redrawn until the requested count of distinct coordinates is reached.
  A matrix whose requested count equals its size is enumerated densely.
* Values: integers 1..5, uniform or with p = (.1, .1, .2, .3, .3); matrix
  values U[0, 1) or the constant 1.0.
* A "planted" variant adds a learnable signal: x = clip(round(3 + a_i1 +
  b_i2 + ... + noise), 1, 5) with per-index offsets a, b, ... ~ N(0, 0.5) and
  noise ~ N(0, 0.5). An additive signal is exactly representable by a Tucker
  model of rank >= 2 per mode, so held-out RMSE well below the value spread
  is reachable.
* Split: a seeded 90/10 train/test split of the tensor entries; matrices are
  all training data.
* Initial parameters: every factor, coupled factor and core entry i.i.d.
  N(0, sigma), sigma = 0.1.
* Item orders: a permutation of all training items (tensor entries first,
  then each matrix's entries), drawn from (seed, epoch).

Randomness is numpy's PCG64 seeded with [seed, stream-id] so that each
component has its own reproducible stream.
"""
from __future__ import annotations

import dataclasses
import functools
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# value-law names
UNIFORM15 = "int15_uniform"
SKEWED15 = "int15_skewed"  # p = (.1, .1, .2, .3, .3)
U01 = "u01"
ONE = "one"

_SKEW_P = np.array([0.1, 0.1, 0.2, 0.3, 0.3])

# stream ids for the per-component generators
_S_PERM = 1
_S_IDX = 2
_S_VAL = 3
_S_SPLIT = 4
_S_INIT = 5
_S_ORDER = 6
_S_MAT = 100
_S_PLANT = 7


@dataclass(frozen=True)
class MatrixSpec:
    mode: int  # coupled tensor mode (0-based)
    cols: int  # K: number of columns (rows of the coupled factor V)
    nnz: int
    col_law: object = "uniform"  # "uniform" or Zipf exponent (float)
    value_law: str = U01


@dataclass(frozen=True)
class Config:
    name: str
    dims: Tuple[int, ...]
    ranks: Tuple[int, ...]
    nnz: int  # tensor entries before the train/test split
    index_law: Tuple[object, ...]  # per mode: "uniform" or Zipf exponent
    value_law: str
    matrices: Tuple[MatrixSpec, ...] = ()
    eta0: float = 0.01
    mu: float = 0.1
    lambda_reg: float = 0.01
    lambda_m: float = 10.0
    init_sigma: float = 0.1
    test_frac: float = 0.1
    seed_data: int = 1
    seed_split: int = 2
    seed_init: int = 3
    dtype: str = "f32"
    planted: bool = False
    description: str = ""

    @property
    def order(self) -> int:
        return len(self.dims)

    def scaled(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


@dataclass
class Problem:
    cfg: Config
    train_idx: np.ndarray  # int32 [N, n_train] (SoA)
    train_val: np.ndarray  # float64 [n_train]
    test_idx: np.ndarray  # int32 [N, n_test]
    test_val: np.ndarray  # float64 [n_test]
    mat_row: List[np.ndarray] = field(default_factory=list)  # int32 [nnz_m]
    mat_col: List[np.ndarray] = field(default_factory=list)
    mat_val: List[np.ndarray] = field(default_factory=list)  # float64

    @property
    def n_train(self) -> int:
        return int(self.train_val.shape[0])

    @property
    def n_items(self) -> int:
        return self.n_train + sum(int(v.shape[0]) for v in self.mat_val)


def _rng(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream), int(sub)]))


@functools.lru_cache(maxsize=16)
def _zipf_cdf(I: int, s: float) -> np.ndarray:
    w = np.arange(1, I + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf.setflags(write=False)  # shared by every draw of this law
    return cdf


# worker threads for the large array steps (numpy's searches and sorts run
# without the interpreter lock); results do not depend on the thread count
_THREADS = max(1, min(16, os.cpu_count() or 1))
_pool = None


def _map(fn, items):
    global _pool
    if _pool is None:
        _pool = ThreadPoolExecutor(_THREADS)
    return list(_pool.map(fn, items))


_GUIDE = 1 << 20  # cells of the inverse-CDF guide table


@functools.lru_cache(maxsize=16)
def _zipf_guide(I: int, s: float) -> np.ndarray:
    """guide[g] = #{i : cdf[i] <= g / _GUIDE} for g = 0 .. _GUIDE (exact
    fractions: _GUIDE is a power of two)."""
    cdf = _zipf_cdf(I, s)
    g = np.searchsorted(cdf, np.arange(_GUIDE + 1, dtype=np.float64) / _GUIDE, side="right")
    g.setflags(write=False)
    return g


def _inverse_cdf(cdf: np.ndarray, guide: np.ndarray, u: np.ndarray) -> np.ndarray:
    """#{i : cdf[i] <= u} per element of u in [0, 1), the result of
    searchsorted(cdf, u, side="right"), found from the guide cell of u and a
    search between its bounds (the count is monotone in u, so it lies in
    [guide[g], guide[g + 1]] for g = floor(u * _GUIDE))."""
    g = (u * _GUIDE).astype(np.int64)
    r = guide[g]
    hi = guide[g + 1]
    amb = np.flatnonzero(r < hi)
    lo, hi, uu = r[amb], hi[amb], u[amb]
    while amb.size:
        mid = (lo + hi) >> 1
        le = cdf[mid] <= uu           # mid < hi <= len(cdf)
        lo = np.where(le, mid + 1, lo)
        hi = np.where(le, hi, mid)
        open_ = lo < hi
        if not open_.all():
            r[amb[~open_]] = lo[~open_]
            amb, lo, hi, uu = amb[open_], lo[open_], hi[open_], uu[open_]
    return r


def zipf_ranks(rng: np.random.Generator, I: int, s: float, n: int) -> np.ndarray:
    """Draw n ranks in [0, I) with P(r) proportional to (r+1)^-s (bounded Zipf)."""
    cdf = _zipf_cdf(int(I), float(s))
    guide = _zipf_guide(int(I), float(s))
    u = rng.random(n)
    # inverse CDF, looked up in chunks by the worker threads
    nch = max(1, min(4 * _THREADS, n // 65536 + 1))
    edges = [n * k // nch for k in range(nch + 1)]
    r = np.empty(n, dtype=np.int64)

    def look(k):
        a, b = edges[k], edges[k + 1]
        np.minimum(_inverse_cdf(cdf, guide, u[a:b]), I - 1, out=r[a:b])

    _map(look, range(nch))
    return r


def _draw_ranks(rng, I, law, n):
    if law == "uniform":
        return rng.integers(0, I, size=n, dtype=np.int64)
    return zipf_ranks(rng, I, float(law), n)


def _mode_perm(seed: int, mode_tag: int, I: int) -> np.ndarray:
    return _rng(seed, _S_PERM, mode_tag).permutation(I).astype(np.int32)


def _draw_values(rng, law, n):
    if law == UNIFORM15:
        return rng.integers(1, 6, size=n).astype(np.float64)
    if law == SKEWED15:
        return (rng.choice(5, size=n, p=_SKEW_P) + 1).astype(np.float64)
    if law == U01:
        return rng.random(n)
    if law == ONE:
        return np.ones(n, dtype=np.float64)
    raise ValueError(f"unknown value law {law!r}")


# set by make_problem(progress=True): a line per redraw round on stderr
_progress = None


def _bucket_of(keys: np.ndarray, nbucket: int) -> np.ndarray:
    """A hash bucket per key (Fibonacci hashing of the 64-bit key)."""
    if nbucket == 1:
        return np.zeros(keys.size, dtype=np.uint8)
    return ((keys.view(np.uint64) * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(56)).astype(np.uint8)


def _fresh_positions(keys: np.ndarray, runs: List[List[np.ndarray]]) -> np.ndarray:
    """Positions of the keys of one draw that occur there for the first time
    and are not in the kept set (runs: per hash bucket, 1 or 256 of them,
    sorted disjoint runs of kept keys), which they join; increasing positions."""
    nbucket = len(runs)
    b = _bucket_of(keys, nbucket)
    perm = np.argsort(b, kind="stable")  # draw order kept within a bucket
    bounds = np.concatenate([[0], np.cumsum(np.bincount(b, minlength=nbucket))])

    def work(j):
        idx = perm[bounds[j]:bounds[j + 1]]
        if idx.size == 0:
            return idx
        sub = keys[idx]
        o = np.argsort(sub)  # not stable: a run of equal keys takes its smallest position below
        srt = sub[o]
        first = np.ones(srt.size, dtype=bool)
        first[1:] = srt[1:] != srt[:-1]
        starts = np.flatnonzero(first)
        cand, pos = srt[starts], np.minimum.reduceat(idx[o], starts)  # idx increases: draw order
        seen = np.zeros(cand.size, dtype=bool)
        for r in runs[j]:
            at = np.minimum(np.searchsorted(r, cand), r.size - 1)
            seen |= r[at] == cand
        keep = ~seen
        if keep.any():
            rs = runs[j]
            rs.append(cand[keep])
            # merge runs of similar size (sizes at least halve from the
            # first run on), so a bucket holds O(log n) runs
            while len(rs) > 1 and 2 * rs[-1].size >= rs[-2].size:
                top = rs.pop()
                rs[-1] = np.sort(np.concatenate([rs[-1], top]))
        return pos[keep]

    if nbucket > 1 and keys.size >= 65536:
        parts = _map(work, range(nbucket))
    else:  # small draws: the thread hand-offs would cost more than the work
        parts = [work(j) for j in range(nbucket) if bounds[j + 1] > bounds[j]]
    pos = np.concatenate(parts) if parts else np.empty(0, dtype=np.int64)
    pos.sort()
    return pos


# coordinate spaces up to this size keep their set as a byte map (one byte
# per possible coordinate) instead of sorted runs of keys
_MAP_LIMIT = 1 << 29


def _fresh_positions_map(keys: np.ndarray, seen: np.ndarray) -> np.ndarray:
    """_fresh_positions for a byte map of the kept set (same result)."""
    idx = np.flatnonzero(seen[keys] == 0)
    if idx.size == 0:
        return idx
    _, first = np.unique(keys[idx], return_index=True)  # first occurrence in the draw
    pos = np.sort(idx[first])
    seen[keys[pos]] = 1
    return pos


def _distinct_coords(draw, dims: Sequence[int], n: int, max_rounds: int = 2000) -> np.ndarray:
    """Draw n distinct coordinate tuples; draw(k) returns int32 [len(dims), k].

    Duplicates of an already-kept coordinate are discarded and redrawn, so the
    result is a set, in first-drawn order.
    """
    strides = np.ones(len(dims), dtype=np.int64)
    for d in range(len(dims) - 2, -1, -1):
        strides[d] = strides[d + 1] * int(dims[d + 1])
    total = int(strides[0]) * int(dims[0])
    if n > total:
        raise ValueError(f"{n} distinct entries requested from a space of {total}")
    if total <= _MAP_LIMIT:
        seen = np.zeros(total, dtype=np.uint8)
        fresh = lambda keys: _fresh_positions_map(keys, seen)  # noqa: E731
    else:
        # hash buckets (searched by the worker threads) for large sets
        runs: List[List[np.ndarray]] = [[] for _ in range(256 if n >= (1 << 20) else 1)]
        fresh = lambda keys: _fresh_positions(keys, runs)  # noqa: E731
    n_kept = 0
    kept = []
    need = n
    for _ in range(max_rounds):
        c = draw(need)
        keys = c[-1].astype(np.int64)
        for d in range(len(dims) - 1):
            keys += c[d] * strides[d]  # int32 times an int64 scalar: int64
        pos = fresh(keys)
        kept.append(c[:, pos])
        n_kept += pos.size
        need = n - n_kept
        if _progress:
            _progress(f"{n_kept:,} of {n:,} distinct coordinates")
        if need == 0:
            return np.concatenate(kept, axis=1)
    raise RuntimeError("could not draw enough distinct coordinates")


def _tensor(cfg: Config):
    N = cfg.order
    perms = [_mode_perm(cfg.seed_data, n, cfg.dims[n]) for n in range(N)]
    rng = _rng(cfg.seed_data, _S_IDX)

    def draw(k):
        out = np.empty((N, k), dtype=np.int32)
        for n in range(N):
            out[n] = perms[n][_draw_ranks(rng, cfg.dims[n], cfg.index_law[n], k)]
        return out

    coords = _distinct_coords(draw, cfg.dims, cfg.nnz)
    vals = _draw_values(_rng(cfg.seed_data, _S_VAL), cfg.value_law, cfg.nnz)
    if cfg.planted:
        prng = _rng(cfg.seed_data, _S_PLANT)
        x = np.full(cfg.nnz, 3.0)
        for n in range(N):
            off = prng.normal(0.0, 0.5, size=cfg.dims[n])
            x += off[coords[n]]
        x += prng.normal(0.0, 0.5, size=cfg.nnz)
        vals = np.clip(np.rint(x), 1.0, 5.0)
    return coords, vals, perms


def _matrix(cfg: Config, m: int, spec: MatrixSpec, row_perm: np.ndarray):
    I = cfg.dims[spec.mode]
    K = spec.cols
    rng = _rng(cfg.seed_data, _S_MAT + m)
    vrng = _rng(cfg.seed_data, _S_MAT + m, 1)
    if spec.nnz == I * K:  # fully observed: enumerate
        r, c = np.meshgrid(np.arange(I), np.arange(K), indexing="ij")
        coords = np.stack([r.ravel(), c.ravel()]).astype(np.int32)
        order = rng.permutation(coords.shape[1])
        coords = coords[:, order]
    else:
        col_perm = _mode_perm(cfg.seed_data, 1000 + m, K)
        row_law = cfg.index_law[spec.mode]

        def draw(k):
            rows = row_perm[_draw_ranks(rng, I, row_law, k)]
            cols = col_perm[_draw_ranks(rng, K, spec.col_law, k)]
            return np.stack([rows, cols])

        coords = _distinct_coords(draw, (I, K), spec.nnz)
    vals = _draw_values(vrng, spec.value_law, spec.nnz)
    return coords[0].astype(np.int32), coords[1].astype(np.int32), vals


def make_problem(cfg: Config, progress: bool = False) -> Problem:
    """Draw the tensor, its train/test split and every coupled matrix.
    progress: report each redraw round on stderr (large inputs)."""
    global _progress
    if progress:
        import sys
        _progress = lambda msg: print(f"[synth {cfg.name}] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    try:
        return _make_problem(cfg)
    finally:
        _progress = None


def _make_problem(cfg: Config) -> Problem:
    coords, vals, perms = _tensor(cfg)
    n = cfg.nnz
    n_test = int(round(cfg.test_frac * n))
    sp = _rng(cfg.seed_split, _S_SPLIT).permutation(n)
    is_test = np.zeros(n, dtype=bool)
    is_test[sp[:n_test]] = True
    test_sel = np.flatnonzero(is_test)   # increasing, as a sort of sp[:n_test]
    train_sel = np.flatnonzero(~is_test)
    N = coords.shape[0]
    train_idx = np.empty((N, train_sel.size), dtype=np.int32)
    test_idx = np.empty((N, test_sel.size), dtype=np.int32)
    train_val = np.empty(train_sel.size, dtype=vals.dtype)
    test_val = np.empty(test_sel.size, dtype=vals.dtype)
    jobs = [(coords[d], sel, dst[d]) for d in range(N) for sel, dst in ((train_sel, train_idx), (test_sel, test_idx))]
    jobs += [(vals, train_sel, train_val), (vals, test_sel, test_val)]
    _map(lambda j: np.take(j[0], j[1], out=j[2]), jobs)  # the split's gathers, by the worker threads
    p = Problem(cfg=cfg, train_idx=train_idx, train_val=train_val, test_idx=test_idx, test_val=test_val)
    for m, spec in enumerate(cfg.matrices):
        r, c, v = _matrix(cfg, m, spec, perms[spec.mode])
        p.mat_row.append(r)
        p.mat_col.append(c)
        p.mat_val.append(v)
    return p


def init_params(cfg: Config, seed: Optional[int] = None):
    """Initial factors U[n] (I_n x J_n), core G (J_1 x ... x J_N, C order) and
    coupled factors V[m] (K_m x J_c), all i.i.d. N(0, sigma), float64."""
    seed = cfg.seed_init if seed is None else seed
    U = [
        _rng(seed, _S_INIT, n).normal(0.0, cfg.init_sigma, size=(cfg.dims[n], cfg.ranks[n]))
        for n in range(cfg.order)
    ]
    G = _rng(seed, _S_INIT, 99).normal(0.0, cfg.init_sigma, size=tuple(cfg.ranks))
    V = [
        _rng(seed, _S_INIT, 200 + m).normal(0.0, cfg.init_sigma, size=(spec.cols, cfg.ranks[spec.mode]))
        for m, spec in enumerate(cfg.matrices)
    ]
    return U, G, V


def item_order(n_items: int, seed: int, epoch: int = 0) -> np.ndarray:
    """A permutation of the item ids 0..n_items-1 for (seed, epoch), int64."""
    return _rng(seed, _S_ORDER, epoch).permutation(n_items).astype(np.int64)


# ---------------------------------------------------------------------------
# configurations

def _cfg1():
    return Config(
        name="cfg1_small_fp64",
        dims=(200, 150, 50), ranks=(3, 3, 3), nnz=5000,
        index_law=("uniform",) * 3, value_law=UNIFORM15,
        matrices=(MatrixSpec(mode=0, cols=100, nnz=2000, col_law="uniform", value_law=U01),),
        eta0=0.01, lambda_reg=0.01, seed_data=1, seed_split=2, seed_init=3, dtype="f64",
        description="3-way 200x150x50, 5,000 nnz uniform, core 3^3, one 200x100 coupled matrix "
                    "(2,000 nnz) on mode 1; FP64",
    )


def _cfg2():
    return Config(
        name="cfg2_zipf_10m",
        dims=(1_000_000, 100_000, 100), ranks=(10, 10, 10), nnz=10_000_000,
        index_law=(1.2, 1.2, 1.2), value_law=SKEWED15,
        matrices=(MatrixSpec(mode=0, cols=1_000_000, nnz=5_000_000, col_law=1.2, value_law=ONE),),
        eta0=0.01, lambda_reg=0.01, seed_data=11, seed_split=12, seed_init=13, dtype="f32",
        description="3-way 1Mx100Kx100, 10M nnz Zipf(1.2), core 10^3, coupled 1Mx1M (5M nnz, "
                    "value 1.0) on mode 1; FP32",
    )


def _cfg3():
    return Config(
        name="cfg3_diff_50m",
        dims=(2_000_000, 2_000_000, 500), ranks=(10, 10, 10), nnz=50_000_000,
        index_law=(1.1, 1.1, 1.1), value_law=SKEWED15,
        matrices=(MatrixSpec(mode=0, cols=2_000_000, nnz=20_000_000, col_law=1.1, value_law=ONE),
                  MatrixSpec(mode=1, cols=200, nnz=10_000_000, col_law=1.1, value_law=U01)),
        eta0=0.01, lambda_reg=0.01, seed_data=21, seed_split=22, seed_init=23, dtype="f32",
        description="3-way 2Mx2Mx500, 50M nnz Zipf(1.1), core 10^3, coupled 2Mx2M (20M) on mode 1 "
                    "and 2Mx200 (10M) on mode 2",
    )


def _cfg4():
    return _cfg3().scaled(
        name="cfg4_bf16_100m", ranks=(16, 16, 16), nnz=100_000_000,
        seed_data=31, seed_split=32, seed_init=33, dtype="bf16",
        description="as cfg3 with core 16^3 and 100M tensor nnz (BF16 matrix-core operands, FP32 masters)",
    )


def _cfg5():
    return Config(
        name="cfg5_4way_200m",
        dims=(1_000_000, 500_000, 1000, 24), ranks=(8, 8, 8, 8), nnz=200_000_000,
        index_law=(1.2, 1.2, 1.2, 1.2), value_law=SKEWED15,
        matrices=(MatrixSpec(mode=0, cols=1_000_000, nnz=30_000_000, col_law=1.2, value_law=U01),
                  MatrixSpec(mode=1, cols=300, nnz=20_000_000, col_law=1.2, value_law=U01),
                  MatrixSpec(mode=2, cols=50, nnz=50_000, col_law="uniform", value_law=U01)),
        eta0=0.01, lambda_reg=0.01, seed_data=41, seed_split=42, seed_init=43, dtype="bf16",
        description="4-way 1Mx500Kx1000x24, 200M nnz Zipf(1.2), core 8^4, three coupled matrices (BF16 matrix-core operands, FP32 masters)",
    )


def _tiny3():
    return Config(
        name="tiny3", dims=(4, 3, 5), ranks=(2, 3, 2), nnz=40,
        index_law=("uniform",) * 3, value_law=UNIFORM15,
        matrices=(MatrixSpec(mode=1, cols=4, nnz=9, value_law=U01),),
        seed_data=5, seed_split=6, seed_init=7, dtype="f64",
    )


def _tiny4():
    return Config(
        name="tiny4", dims=(3, 2, 2, 3), ranks=(2, 2, 1, 2), nnz=25,
        index_law=("uniform",) * 4, value_law=UNIFORM15,
        matrices=(MatrixSpec(mode=0, cols=3, nnz=6, value_law=U01),
                  MatrixSpec(mode=3, cols=2, nnz=6, value_law=U01)),
        seed_data=8, seed_split=9, seed_init=10, dtype="f64",
    )


def _cfg2_slice():
    return _cfg2().scaled(name="cfg2_slice_100k", nnz=100_000,
                          matrices=(MatrixSpec(mode=0, cols=1_000_000, nnz=50_000,
                                               col_law=1.2, value_law=ONE),))


def _cfg5_slice():
    return _cfg5().scaled(
        name="cfg5_slice_50k", nnz=50_000, dtype="f32",
        matrices=(MatrixSpec(mode=0, cols=1_000_000, nnz=7_500, col_law=1.2, value_law=U01),
                  MatrixSpec(mode=1, cols=300, nnz=5_000, col_law=1.2, value_law=U01),
                  MatrixSpec(mode=2, cols=50, nnz=50_000, col_law="uniform", value_law=U01)))


def _cfg2_planted():
    return _cfg2().scaled(name="cfg2_planted_10m", planted=True,
                          description="as cfg2 with planted values: clip(round(3 + per-index offsets + noise), 1, 5)")


CONFIGS = {
    "cfg1": _cfg1,
    "cfg2": _cfg2,
    "cfg2_planted": _cfg2_planted,
    "cfg3": _cfg3,
    "cfg4": _cfg4,
    "cfg5": _cfg5,
    "tiny3": _tiny3,
    "tiny4": _tiny4,
    "cfg2_slice": _cfg2_slice,
    "cfg5_slice": _cfg5_slice,
}


def get_config(name: str, **overrides) -> Config:
    cfg = CONFIGS[name]()
    return cfg.scaled(**overrides) if overrides else cfg
