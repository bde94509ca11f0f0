"""Integer identities the library's kernels rely on (no GPU)."""
import numpy as np


def test_division_by_multiplication_is_exact():
    """x // d equals the high 64 bits of ceil(2^64 / d) * x for every 32-bit
    x and every divisor d >= 2 (Lemire, Kaser and Kurz 2019); the bin index of
    the counting sort is computed this way."""
    rng = np.random.default_rng(0)
    ds = [2, 3, 5, 7, 8, 131072, 204800, 262144, 409600, 1 << 20, 3 << 20, (1 << 31) - 1, 999983]
    ds += [int(v) for v in rng.integers(2, 1 << 31, 40)]
    xs = [0, 1, (1 << 31) - 1, (1 << 32) - 1] + [int(v) for v in rng.integers(0, 1 << 32, 2000)]
    for d in ds:
        c = (2 ** 64 - 1) // d + 1
        for x in xs:
            assert (c * x) >> 64 == x // d, (d, x)
        for k in range(1, 50):   # around multiples of d
            for x in (k * d - 1, k * d, k * d + 1):
                if 0 <= x < 1 << 32:
                    assert (c * x) >> 64 == x // d, (d, x)
