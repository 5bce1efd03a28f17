"""CPU pins of the numpy reference behind tests/test_gpu_init.py: its
SplitMix64 output function reproduces the generator's published first
outputs for seed 0 (the state advanced by the golden gamma, then mixed), and
its Box-Muller values have the moments of N(0, sigma^2)."""
import numpy as np

from tests.test_gpu_init import GAMMA, MASK, _mix, _normal


def test_splitmix64_published_sequence_seed0():
    got = [int(_mix(np.array([(k * GAMMA) & MASK], dtype=np.uint64))[0]) for k in (1, 2, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_box_muller_moments():
    x = _normal(3, 0, 1_000_000, 0.5)
    assert abs(x.mean()) <= 5 * 0.5 / np.sqrt(x.size)
    assert abs(x.std() / 0.5 - 1.0) <= 0.005
    # fourth moment of a normal: 3 sigma^4
    assert abs(np.mean(x ** 4) / 0.5 ** 4 - 3.0) <= 0.05
