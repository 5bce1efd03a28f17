"""Device initialisation (s3_init_params) against an independent numpy
implementation of the same counter-based definition: SplitMix64's output
function (Steele, Lea and Flood 2014, Vigna's constants) on the counters
key_q + 2i and key_q + 2i + 1, 53-bit uniforms, Box-Muller in FP64.  The
transcendental functions of the two sides may differ in the last bits, so
FP64 values agree to 1e-12 of sigma and FP32 values to FP32 rounding.  Also:
the sample moments, determinism per seed, and a det batch trained from the
device-drawn values matching the oracle started from the same values."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import UNIT, check_batches, setup

pytestmark = pytest.mark.gpu

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def _mix(z):
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = z.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _normal(seed, q, n, sigma):
    key = int(_mix(np.array([(seed + GAMMA * (q + 1)) & MASK], dtype=np.uint64))[0])
    pairs = (n + 1) // 2
    i = np.arange(pairs, dtype=np.uint64)
    with np.errstate(over="ignore"):
        a = _mix(np.uint64(key) + np.uint64(2) * i)
        b = _mix(np.uint64(key) + np.uint64(2) * i + np.uint64(1))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = sigma * np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * pairs)
    out[0::2] = r * np.cos(2.0 * np.pi * u2)
    out[1::2] = r * np.sin(2.0 * np.pi * u2)
    return out[:n]


def _reference(cfg, seed, sigma):
    N = cfg.order
    U = [_normal(seed, n, d * r, sigma).reshape(d, r) for n, (d, r) in enumerate(zip(cfg.dims, cfg.ranks))]
    G = _normal(seed, N, int(np.prod(cfg.ranks)), sigma).reshape(cfg.ranks)
    V = [_normal(seed, N + 1 + m, s.cols * cfg.ranks[s.mode], sigma).reshape(s.cols, cfg.ranks[s.mode])
         for m, s in enumerate(cfg.matrices)]
    return U, G, V


@pytest.mark.parametrize("dtype,name", [("f64", "cfg1"), ("f32", "cfg1"), ("f32", "tiny4")])
def test_init_params_matches_reference(dtype, name):
    cfg, p, plan, ref, order = setup(name, dtype, 500, True)
    seed, sigma = 12345, 0.1
    plan.init_params(seed, sigma)
    gU, gG, gV = plan.params_numpy()
    wU, wG, wV = _reference(cfg, seed, sigma)
    for what, a, b in [(f"U[{n}]", gU[n], wU[n]) for n in range(len(wU))] + [("G", gG, wG)] + \
            [(f"V[{m}]", gV[m], wV[m]) for m in range(len(wV))]:
        assert a.shape == b.shape, what
        if dtype == "f64":
            err = np.max(np.abs(a - b))
            assert err <= 1e-12 * sigma, f"{what}: {err:.3e}"
        else:
            want = b.astype(np.float32).astype(np.float64)
            err = np.max(np.abs(a - want) / np.maximum(np.abs(want), 1e-30))
            assert err <= 2 ** -23, f"{what}: {err:.3e}"


def test_init_params_moments_and_determinism():
    cfg, p, plan, ref, order = setup("cfg2_slice", "f32", 4096, True)
    plan.init_params(7, 0.25)
    U1, G1, V1 = plan.params_numpy()
    plan.init_params(7, 0.25)
    U2, G2, V2 = plan.params_numpy()
    assert all(np.array_equal(a, b) for a, b in zip(U1 + [G1] + V1, U2 + [G2] + V2))
    plan.init_params(8, 0.25)
    U3, _, _ = plan.params_numpy()
    assert not np.array_equal(U1[0], U3[0])
    x = U1[0].ravel()  # 1M x 10 values
    assert abs(x.mean()) <= 5 * 0.25 / np.sqrt(x.size)
    assert abs(x.std() / 0.25 - 1.0) <= 0.01
    # the modes are drawn from different keys
    assert not np.array_equal(U1[0].ravel()[:100], V1[0].ravel()[:100])


def test_det_batch_from_device_init_matches_oracle():
    cfg, p, plan, ref, order = setup("cfg1", "f64", 500, True)
    plan.init_params(99, 0.1)
    check_batches(p, plan, order, 500, 0.01, range(2), True, 1e-10, UNIT["f64"], "device init")
