"""Whole-spectrum parity at full sizes.

Diffusive stencils at large T leave only the modes near the zero frequency above
the tolerance, so they cannot see the upper half of a spectrum, where the
split-axis twiddles, the digit-reversed position -> frequency map and the
real-data untangling act.  These cases keep every mode visible:

* T = 1 (and T = 3) with asymmetric box stencils: every mode's lambda is O(1);
  compared with the FP64 loop oracle on the dtype-rounded input;
* pure shifts (a single weight 1 at a corner offset): every mode has |lambda| = 1,
  and the exact answer is a cyclic roll of the input, ``a_T[i] = a_0[i + T o]``
  (Sec. 3: the shift matrix X and S^T).  Unit-modulus symbols lose about T
  ulps in FP64 whatever the method, so the FP64 tolerance is max(1e-12, 8 T eps).

Shapes: the workloads' full sizes (8192^2, 512^3, the 1-D heat grid), the split
shapes of long axes (1-D 2^16 and 2^20 on the complex row middle pass, (1024, 24)),
and every length class of the generic mixed-radix kernels (5- and 7-smooth rows,
columns, split axes, 3-D), plus chirp-z extents.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_periodic, rounded_input

pytestmark = pytest.mark.gpu

EPS64 = 2.220446049250313e-16


def _t1(dims, r, T, dtype, seed):
    c = wl.box_random_coeffs(seed, len(dims), r)
    a0 = wl.uniform(seed, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    got = gpu_periodic(a0, c, T, dtype)
    assert_close(got, ref, TOL[dtype], (dims, r, T, dtype))


def _shift(dims, offs, T, dtype, seed):
    d = len(dims)
    r = max(abs(o) for o in offs)
    c = np.zeros((2 * r + 1,) * d)
    c[tuple(o + r for o in offs)] = 1.0
    a0 = wl.uniform(seed, "grid", int(np.prod(dims))).reshape(dims)
    want = np.roll(rounded_input(a0, dtype), tuple(-T * o for o in offs), axis=tuple(range(d)))
    tol = TOL["f32"] if dtype == "f32" else max(1e-12, 8 * T * EPS64)
    assert_close(gpu_periodic(a0, c, T, dtype), want, tol, (dims, offs, T, dtype))


# ------------------------------------------------------------------ full sizes

@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_jacobi_size_8192sq_T1_asymmetric(dtype):
    """The exact kernels of the 8192^2 workload (R2C rows, split column passes, the
    fused middle pass, C2R rows) against the oracle with every mode visible."""
    _t1((8192, 8192), 1, 1, dtype, 61)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_jacobi_size_8192sq_pure_shift(dtype):
    _shift((8192, 8192), (1, -1), 4097, dtype, 62)


@pytest.mark.slow
def test_star_size_512cube_T1_asymmetric():
    _t1((512, 512, 512), 1, 1, "f32", 63)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_star_size_512cube_pure_shift(dtype):
    _shift((512, 512, 512), (1, 1, -1), 1001, dtype, 64)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims", [(16384,), (65536,), (1 << 20,), (1024, 24), (24, 1024), (4096, 4096)])
def test_split_and_long_axes_T1(dims, dtype):
    _t1(dims, 1, 1, dtype, 65 + len(dims))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims,offs,T", [((65536,), (1,), 1025), ((1 << 20,), (-2,), 123457),
                                          ((1024, 24), (1, 1), 99), ((16384,), (1,), 40000)])
def test_split_and_long_axes_pure_shift(dims, offs, T, dtype):
    _shift(dims, offs, T, dtype, 66)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_r2_T3_asymmetric_full_spectrum(dtype):
    """Radius 2 at T = 3: the squared and multiplied symbol of every mode."""
    _t1((2048, 1024), 2, 3, dtype, 67)
    _t1((64, 128, 32), 2, 3, dtype, 68)


# ------------------------------------------------- generic mixed-radix kernels

GENERIC = [
    (3000,), (6720,), (4374,), (15625,), (16807,), (59049,), (75,), (84,),
    (800, 800), (3000, 2800), (6300, 6720), (343, 625), (2, 3000), (5, 7),
    (120, 126, 100), (200, 210, 240), (49, 45, 50),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims", GENERIC)
def test_generic_lengths_T1(dims, dtype):
    _t1(dims, 1, 1, dtype, 70 + sum(dims) % 17)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims", [(15625,), (3000, 2800), (200, 210, 240)])
def test_generic_lengths_pure_shift(dims, dtype):
    _shift(dims, (1,) * len(dims), 1777, dtype, 71)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_paper_size_8000sq_T1_and_shift(dtype):
    """The paper's 2-D extent (8000 = 2^6 5^3) on the generic kernels."""
    _t1((8000, 8000), 1, 1, dtype, 72)
    _shift((8000, 8000), (1, 1), 4097, dtype, 73)


# ------------------------------------------------------------- chirp-z extents

@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims", [(10007,), (1009, 2003), (8191, 64), (37, 41, 43)])
def test_chirp_z_T1_and_shift(dims, dtype):
    _t1(dims, 1, 1, dtype, 74)
    _shift(dims, (1,) * len(dims), 333, dtype, 75)
