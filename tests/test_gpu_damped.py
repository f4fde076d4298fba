"""Stencils whose symbol does not reach 1: damped (sum of coefficients below 1),
growing, and mixed-sign stencils, on every kind of middle pass.

For such stencils lambda^T is small for every mode, so a power kept only to
absolute accuracy (a deviation 1 - lambda^T rounded near 1) would lose the whole
result.  Each case compares the library with the FP64 loop oracle on the same
(dtype-rounded) input under both gates (relative L2 and largest cell error
relative to max |ref|): 1e-5 for the FP32 path, 1e-12 for the FP64 path.

The shapes pick the kernel families: power-of-two fused 1-D rows, split 1-D axes
(complex row middle pass), strided-axis middle passes in 2-D and 3-D, the
generic mixed-radix kernels (7-smooth extents) and the chirp-z path (a prime
factor above 7).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_aperiodic, gpu_periodic, rounded_input, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(4096,), (32768,), (256, 128), (16, 32, 64), (3000,), (60, 90), (6, 10, 14), (1009,), (31, 37)]


def damped(seed, d, r, total):
    """Nonnegative box weights scaled to sum `total` (one sign: lambda(0) is the largest |lambda|)."""
    return wl.box_random_coeffs(seed, d, r) * total


def mixed(seed, d, r, total):
    """Box weights with the first (corner) weight negated and cut to a tenth, rescaled
    to sum `total` (sum |c| stays within 1.2 of it, so no mode outgrows FP32 at T = 200)."""
    c = wl.box_random_coeffs(seed, d, r)
    c.flat[0] = -0.1 * c.flat[0]
    return c * (total / c.sum())


STENCILS = {
    "damped_095": lambda seed, d: damped(seed, d, 1, 0.95),
    "mixed_090": lambda seed, d: mixed(seed, d, 1, 0.90),
    "growing_101": lambda seed, d: damped(seed, d, 1, 1.01),
    "mixed_100": lambda seed, d: mixed(seed, d, 1, 1.0),
}


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("kind", list(STENCILS))
@pytest.mark.parametrize("dims", SHAPES)
def test_damped_and_mixed_sign_every_kernel(dims, kind, dtype):
    seed = 300 + sum(dims) % 97
    c = STENCILS[kind](seed, len(dims))
    T = 500 if kind == "damped_095" else 200
    a0 = wl.uniform(seed, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype], (dims, kind))


@pytest.mark.parametrize("dims", [(64, 48), (4096,), (32768,), (16, 8, 32), (60, 90), (1009,)])
@pytest.mark.parametrize("T", [200, 1000])
def test_pointwise_decay_r0(dims, T):
    """c = 0.9 alone: a_T = 0.9^T a_0 exactly (0.9^1000 ~ 1.7e-46, far below 1e-16)."""
    c = np.full((1,) * len(dims), 0.9)
    a0 = wl.uniform(17, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(a0, c, T)
    assert_close(gpu_periodic(a0, c, T, "f64"), ref, 1e-12, dims)
    np.testing.assert_allclose(ref, 0.9 ** T * a0, rtol=1e-13)
    if T == 200:
        assert_close(gpu_periodic(a0, c, T, "f32"), oracle.periodic(rounded_input(a0, "f32"), c, T), 1e-5)


def test_gaussian_input_damped():
    """Zero-mean input: the surviving modes are not the zero mode."""
    dims = (128, 96)
    c = damped(5, 2, 1, 0.97)
    a0 = wl.gaussian(5, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(a0, c, 300)
    assert_close(gpu_periodic(a0, c, 300, "f64"), ref, 1e-12)


def test_all_negative_coefficients():
    """All weights negative: lambda(0) = sum c < 0 is still the largest |lambda|; odd T flips the sign."""
    dims = (64, 64)
    c = -damped(6, 2, 1, 0.98)
    a0 = wl.uniform(6, "grid", int(np.prod(dims))).reshape(dims)
    for T in (301, 300):
        ref = oracle.periodic(a0, c, T)
        assert_close(gpu_periodic(a0, c, T, "f64"), ref, 1e-12, T)


def test_damped_batch_matches_oracle():
    import torch
    import paper_2105_06676_amd as sfft
    cases = [((256, 128), damped(1, 2, 1, 0.95), 500, "f64"), ((4096,), mixed(2, 1, 1, 0.9), 200, "f32"),
             ((60, 90), damped(3, 2, 2, 0.99), 700, "f64"), ((16, 32, 64), mixed(4, 3, 1, 0.9), 150, "f64")]
    grids, refs = [], []
    for dims, c, T, dt in cases:
        a0 = wl.uniform(40 + len(grids), "grid", int(np.prod(dims))).reshape(dims)
        grids.append(to_dev(a0, dt))
        refs.append(oracle.periodic(rounded_input(a0, dt), c, T))
    sfft.batch([(g, c, T) for g, (dims, c, T, dt) in zip(grids, cases)])
    torch.cuda.synchronize()
    for g, ref, (dims, c, T, dt) in zip(grids, refs, cases):
        assert_close(g.cpu().numpy().astype(np.float64), ref, TOL[dt], dims)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["damped_095", "mixed_090"])
def test_damped_aperiodic(kind, dtype):
    dims = (70, 90)
    c = STENCILS[kind](9, 2)
    a = wl.uniform(9, "grid", (dims[0] + 2) * (dims[1] + 2)).reshape(dims[0] + 2, dims[1] + 2)
    ref = oracle.aperiodic(rounded_input(a, dtype), c, 40)
    assert_close(gpu_aperiodic(a, c, 40, dtype), ref, TOL[dtype])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_damped_fields(dtype):
    """Two coupled damped diffusions: every mode's symbol matrix has spectral radius below 1."""
    import torch
    import paper_2105_06676_amd as sfft
    dims = (64, 48)
    c = np.zeros((2, 2, 3, 3))
    c[0, 0] = damped(1, 2, 1, 0.85)
    c[1, 1] = damped(2, 2, 1, 0.80)
    c[0, 1, 1, 1] = 0.05
    c[1, 0, 1, 1] = 0.10
    a = wl.uniform(3, "grid", 2 * 64 * 48).reshape((2,) + dims)
    T = 300
    g = to_dev(a, dtype)
    sfft.periodic_fields(g, c, T)
    torch.cuda.synchronize()
    want = oracle.periodic_fields(rounded_input(a, dtype), c, T)
    assert_close(g.cpu().numpy().astype(np.float64), want, TOL[dtype])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_damped_implicit(dtype):
    """Backward Euler with a reaction term: Q = (1 + 0.02) I - k Laplacian, S = I."""
    import torch
    import paper_2105_06676_amd as sfft
    dims = (48, 40)
    q = np.zeros((3, 3))
    k = 0.7
    q[1, 1] = 1.02 + 4 * k
    q[0, 1] = q[2, 1] = q[1, 0] = q[1, 2] = -k
    s = np.zeros((3, 3))
    s[1, 1] = 1.0
    a = wl.uniform(4, "grid", 48 * 40).reshape(dims)
    T = 600
    g = to_dev(a, dtype)
    sfft.periodic_implicit(g, q, s, T)
    torch.cuda.synchronize()
    want = oracle.implicit_periodic(rounded_input(a, dtype), q, s, T)
    assert_close(g.cpu().numpy().astype(np.float64), want, TOL[dtype])
