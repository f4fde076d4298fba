"""Periodic solves on extents with prime factors above 7 (Bluestein's chirp-z DFT
on those axes, complex transforms on the others) against the loop oracle.
Tolerances as for the 7-smooth path (relative L2 against the FP64 oracle)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_periodic, rel_l2, rounded_input

pytestmark = pytest.mark.gpu

CASES = [
    ((11,), 1, 7), ((97,), 2, 300), ((1009,), 1, 1000), ((8191,), 1, 2000), ((10007,), 1, 50),
    ((13, 17), 1, 40), ((11, 64), 1, 100), ((64, 11), 2, 100), ((101, 60), 1, 250), ((1021, 1031), 1, 20),
    ((9, 11, 13), 1, 30), ((16, 13, 8), 1, 60), ((7, 32, 23), 2, 12),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dims,r,T", CASES)
def test_non_smooth_extents_match_oracle(dims, r, T, dtype):
    c = wl.box_random_coeffs(50 + len(dims) + r, len(dims), r)
    a = wl.uniform(50 + sum(dims), "grid", int(np.prod(dims))).reshape(dims)
    got = gpu_periodic(a, c, T, dtype)
    want = oracle.periodic(rounded_input(a, dtype), c, T)
    assert_close(got, want, TOL[dtype])


def test_non_smooth_complex_stencil_long_T():
    # a non-symmetric stencil (complex symbol) over many steps on a prime torus
    c = np.zeros(5)
    c[[0, 1, 2, 3, 4]] = [0.05, 0.3, 0.4, 0.15, 0.1]
    a = wl.uniform(60, "grid", 4093)
    got = gpu_periodic(a, c, 5000, "f64")
    assert_close(got, oracle.periodic(a, c, 5000), 1e-12)


def test_pure_shift_on_a_prime_torus():
    # c = delta at offset +1: after T steps the grid is rolled by -T (exact data movement)
    n, T = 127, 1000
    c = np.array([0.0, 0.0, 1.0])
    a = wl.uniform(61, "grid", n)
    got = gpu_periodic(a, c, T, "f64")
    assert np.allclose(got, np.roll(a, -T), rtol=0, atol=1e-12)
