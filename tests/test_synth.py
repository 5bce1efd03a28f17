"""The synthetic input generator (host only): the inverse-CDF lookup of the
bounded Zipf law, distinct coordinate sets on both deduplication paths, and
the split of a generated problem."""
import numpy as np
import pytest

from synth import gen, get_config, make_problem


@pytest.mark.parametrize("I,s", [(1_000_000, 1.2), (1000, 1.2), (24, 1.2), (300, 1.1), (2, 0.5), (1, 1.2)])
def test_guide_lookup_equals_a_plain_search(I, s):
    cdf = gen._zipf_cdf(I, s)
    rng = np.random.default_rng(11)
    below_one = np.nextafter(1.0, 0.0)
    u = np.concatenate([
        rng.random(200_000),
        np.minimum(cdf[:2000], below_one),                  # on the CDF's steps
        np.nextafter(np.minimum(cdf[:2000], 1.0), 0.0),     # just below them
        np.arange(0, gen._GUIDE, 997) / gen._GUIDE,          # on guide cell edges
        [0.0, below_one],
    ])
    got = gen._inverse_cdf(cdf, gen._zipf_guide(I, s), u)
    assert np.array_equal(got, np.searchsorted(cdf, u, side="right"))


def test_zipf_head_frequency():
    """P(rank 0) = 1 / sum_r (r+1)^-s for the bounded law."""
    I, s, n = 10_000, 1.2, 2_000_000
    r = gen.zipf_ranks(np.random.default_rng(5), I, s, n)
    assert r.min() >= 0 and r.max() < I
    p0 = 1.0 / np.sum(np.arange(1, I + 1, dtype=np.float64) ** -s)
    sd = np.sqrt(p0 * (1 - p0) / n)
    assert abs(np.mean(r == 0) - p0) < 5 * sd


@pytest.mark.parametrize("dims,n", [((300, 200, 40), 200_000),            # byte map
                                    ((40_000, 40_000), 1_100_000)])     # hash buckets (space above 2^29)
def test_distinct_coordinates(dims, n):
    rng = np.random.default_rng(9)

    def draw(k):
        return np.stack([gen.zipf_ranks(rng, d, 1.2, k).astype(np.int32) for d in dims])

    c = gen._distinct_coords(draw, dims, n)
    assert c.shape == (len(dims), n)
    for d, size in enumerate(dims):
        assert c[d].min() >= 0 and c[d].max() < size
    keys = np.zeros(n, dtype=np.int64)
    for d, size in enumerate(dims):
        keys = keys * size + c[d]
    assert np.unique(keys).size == n


def test_generated_problem_split():
    cfg = get_config("cfg1")
    p = make_problem(cfg)
    n_test = int(round(cfg.test_frac * cfg.nnz))
    assert p.test_val.size == n_test and p.train_val.size == cfg.nnz - n_test
    both = np.concatenate([p.train_idx, p.test_idx], axis=1).astype(np.int64)
    keys = np.zeros(both.shape[1], dtype=np.int64)
    for d, size in enumerate(cfg.dims):
        assert both[d].max() < size
        keys = keys * size + both[d]
    assert np.unique(keys).size == cfg.nnz  # a set, split without overlap
    for m, spec in enumerate(cfg.matrices):
        k = p.mat_row[m].astype(np.int64) * spec.cols + p.mat_col[m]
        assert np.unique(k).size == spec.nnz == p.mat_val[m].size
