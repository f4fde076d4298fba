"""The kernels divide by workgroup-uniform divisors through a float reciprocal:
q = trunc((e + 1/2) * fl(1/n)) in IEEE single precision with round-to-nearest.
The claim is that q = floor(e / n) for every divisor n >= 1 and every e < 2^22.
Checked here exhaustively for e < 2^16 and every divisor up to 8192 (the largest
a tile uses), and near the top of the range for small and large divisors, with
numpy's float32 arithmetic (the same IEEE operations as the GPU's)."""
import numpy as np


def _q(e: np.ndarray, n: int) -> np.ndarray:
    inv = np.float32(1.0) / np.float32(n)
    return ((e.astype(np.float32) + np.float32(0.5)) * inv).astype(np.uint32)


def test_float_reciprocal_division_exhaustive_small_dividends():
    e = np.arange(0, 1 << 16, dtype=np.uint32)
    for n in range(1, 8193):
        assert np.array_equal(_q(e, n), e // n), n


def test_float_reciprocal_division_near_the_bound():
    e = np.arange((1 << 22) - 65536, 1 << 22, dtype=np.uint32)
    for n in list(range(1, 257)) + list(range(7936, 8193)) + [1000, 4097, 6300, 6720]:
        assert np.array_equal(_q(e, n), e // n), n
