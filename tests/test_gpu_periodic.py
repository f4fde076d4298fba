"""Parity of the HIP periodic solver (StencilFFT-P) with the FP64 loop oracle.

Every case runs the library through its C ABI on seeded inputs and compares with
``oracle.periodic`` on the same (dtype-rounded) input, element by element via the
relative L2 error: <= 1e-5 for the FP32 path, <= 1e-12 for the FP64 path.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_periodic, rel_l2, rounded_input

pytestmark = pytest.mark.gpu


def _coeffs(d, r, symmetric, seed):
    c = wl.box_random_coeffs(seed, d, r)
    if symmetric:
        c = 0.5 * (c + c[tuple(slice(None, None, -1) for _ in range(d))])
    return c


CASES = []
for dtype in ("f32", "f64"):
    for dims in [(1,), (2,), (3,), (5,), (7,), (16,), (30,), (63,), (64,), (1000,),
                 (1, 1), (2, 3), (7, 9), (16, 16), (25, 12), (64, 50), (3, 64), (48, 1),
                 (2, 2, 2), (5, 6, 7), (16, 8, 4), (9, 1, 12), (32, 32, 32)]:
        for r in (0, 1, 2):
            if len(dims) == 3 and r == 2 and max(dims) > 16:
                continue
            for T in (1, 7, 64):
                for sym in (True, False):
                    if (sum(dims) + r + T + sym) % 3:  # thin the cross product deterministically
                        continue
                    CASES.append((dtype, dims, r, T, sym))


@pytest.mark.parametrize("dtype,dims,r,T,sym", CASES)
def test_periodic_small_grids(dtype, dims, r, T, sym):
    seed = 100 + sum(dims) * 7 + r * 3 + T
    c = _coeffs(len(dims), r, sym, seed)
    a0 = wl.uniform(seed, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    got = gpu_periodic(a0, c, T, dtype)
    assert_close(got, ref, TOL[dtype], (dims, r, T, sym))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("T", [2, 3, 1023, 1024, 4096])
def test_periodic_long_T(dtype, T):
    dims = (24, 40)
    c = _coeffs(2, 1, False, 7)
    a0 = wl.uniform(7, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims", [(4096,), (8192,), (16384,), (20000,), (65536,), (3 * 5 * 7 * 64,),
                                  (1024, 24), (24, 2048), (600, 40), (2, 3000), (40, 30, 36), (128, 6, 10)])
def test_periodic_multi_tile_and_split_axes(dtype, dims):
    """Shapes that span many tiles, split long axes into sub-transforms, and
    leave ragged last tiles."""
    c = _coeffs(len(dims), 1, False, 11)
    a0 = wl.uniform(11, "grid", int(np.prod(dims))).reshape(dims)
    T = 37
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("dims", [(2048,), (32768,), (128, 96), (512, 40), (16, 32, 24)])
def test_fused_symbol_every_radius(dtype, r, sym, dims):
    """The fused middle passes evaluate the symbol with code specialised on the
    radius (0, 1, 2) and on whether lambda is real: every combination, on a fused
    1-D row, a split 1-D axis, and strided-axis middle passes of 2-D and 3-D grids."""
    seed = 900 + r * 10 + sym + len(dims)
    c = _coeffs(len(dims), r, sym, seed)
    a0 = wl.uniform(seed, "grid", int(np.prod(dims))).reshape(dims)
    T = 45
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype], (dims, r, sym))


def test_T_zero_is_identity_and_r0_is_pointwise():
    a0 = wl.uniform(3, "grid", 12 * 10).reshape(12, 10)
    c = _coeffs(2, 1, False, 3)
    got = gpu_periodic(a0, c, 0, "f64")
    assert np.array_equal(got, a0)
    c0 = np.array([[0.9]])
    got = gpu_periodic(a0, c0, 11, "f64")
    np.testing.assert_allclose(got, 0.9 ** 11 * a0, rtol=1e-13)


def test_printed_matrix_example():
    """The appendix's 4-cell example: a_{t+1}[i] = -2 a[i-1] + a[i] + 3 a[i+1]."""
    c = np.array([-2.0, 1.0, 3.0])
    x = np.array([1.0, 2.0, 3.0, 4.0])
    np.testing.assert_allclose(gpu_periodic(x, c, 1, "f64"), [-1.0, 9.0, 11.0, 1.0], atol=1e-13)
    np.testing.assert_allclose(gpu_periodic(x, c, 2, "f64"), [24.0, 44.0, -4.0, -24.0], atol=1e-12)


def test_pure_shift_large_T():
    n, T = 1000, 123457
    c = np.array([0.0, 0.0, 1.0])
    a0 = wl.uniform(4, "grid", n)
    got = gpu_periodic(a0, c, T, "f64")
    np.testing.assert_allclose(got, np.roll(a0, -(T % n)), atol=T * 4e-16)


def test_single_mode_full_jacobi2d_8192():
    """cos mode k of the 8192^2 Jacobi grid scales by exactly lambda(k)^T (symmetric stencil)."""
    w = wl.config("jacobi2d_8192")
    n0, n1 = w.dims
    k0, k1 = 3, 5
    m0 = np.arange(n0)[:, None]
    m1 = np.arange(n1)[None, :]
    a0 = np.cos(2 * np.pi * (k0 * m0 / n0 + k1 * m1 / n1))
    lam = 0.2 * (1 + 2 * np.cos(2 * np.pi * k0 / n0) + 2 * np.cos(2 * np.pi * k1 / n1))
    got = gpu_periodic(a0, w.coeffs, w.T, "f64")
    assert_close(got, lam ** w.T * a0, 1e-12)


def test_semigroup_and_translation():
    dims = (30, 42)
    c = _coeffs(2, 2, False, 8)
    a0 = wl.uniform(8, "grid", int(np.prod(dims))).reshape(dims)
    whole = gpu_periodic(a0, c, 300, "f64")
    parts = gpu_periodic(gpu_periodic(a0, c, 123, "f64"), c, 177, "f64")
    assert_close(parts, whole, 1e-13)
    sh = gpu_periodic(np.roll(a0, (5, -7), axis=(0, 1)), c, 300, "f64")
    assert_close(sh, np.roll(whole, (5, -7), axis=(0, 1)), 1e-13)


def test_symbol_power_matches_definition():
    """lambda(k)^T from the library against Step 1(i) written literally (DFT of the
    first column) and Step 2 in 60-digit arithmetic."""
    import torch
    import paper_2105_06676_amd as sfft
    for dims, r, T, seed in [((12,), 1, 1000, 1), ((6, 10), 1, 77, 2), ((4, 3, 5), 1, 33, 3),
                             ((8, 6), 2, 4096, 4), ((5,), 2, 100000, 5), ((7, 4), 0, 9, 6)]:
        c = wl.box_random_coeffs(seed, len(dims), r)
        if T < 5000:
            c.flat[0] += 0.05  # not summing to 1 (kept exact-sum at large T: 1.05^T overflows)
        out = torch.zeros(dims, dtype=torch.complex128, device="cuda:0")
        sfft.symbol_power(out, dims, c, T)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        lam = oracle.symbol(c, dims)
        ref = oracle.symbol_power(lam, T)
        big = np.abs(ref) > 1e-250
        rel = np.abs(got - ref)[big] / np.abs(ref)[big]
        # lambda itself carries an absolute rounding error ~ eps * sum|c| (from either
        # side), which the power magnifies T-fold relative to |lambda|
        bound = 16 * 2.3e-16 * (1.0 + T * np.abs(c).sum() / np.abs(lam)[big])
        assert np.all(rel <= bound), (dims, r, T, float((rel / bound).max()))
        assert np.all(np.abs(got[~big]) <= 1e-240)


@pytest.mark.slow
def test_heat1d_65536_full_against_oracle_and_binomial():
    w = wl.config("heat1d_65536")
    a0 = w.grid()
    got = gpu_periodic(a0, w.coeffs, w.T, "f64")
    ref = oracle.periodic(a0, w.coeffs, w.T)
    assert_close(got, ref, 1e-12)
    from fractions import Fraction
    from math import comb
    T = w.T
    expect = np.zeros_like(a0)
    for m in range(2 * T + 1):
        expect += float(Fraction(comb(2 * T, m), 4 ** T)) * np.roll(a0, -(m - T))
    assert_close(got, expect, 1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_jacobi2d_crop_instance(dtype):
    """The 256x256 periodic instance with the 8192^2 Jacobi workload's stencil and T, initial data = the
    top-left crop of the seeded 8192^2 grid."""
    w = wl.config("jacobi2d_8192")
    a0 = wl.crop_grid(w, 256)
    ref = oracle.periodic(rounded_input(a0, dtype), w.coeffs, w.T)
    assert_close(gpu_periodic(a0, w.coeffs, w.T, dtype), ref, TOL[dtype])


@pytest.mark.slow
def test_jacobi2d_8192_full_invariants():
    """Full 8192^2, T = 4096: the sum is conserved (coefficients sum to 1 up to the
    rounding of 0.2) and the FP32 path agrees with the FP64 path."""
    w = wl.config("jacobi2d_8192")
    a0 = w.grid()
    g64 = gpu_periodic(a0, w.coeffs, w.T, "f64")
    g32 = gpu_periodic(a0, w.coeffs, w.T, "f32")
    s0 = a0.sum()
    assert abs(g64.sum() - s0) <= 1e-12 * abs(s0)
    assert_close(g32, g64, 1e-5)


@pytest.mark.slow
def test_star3d_instance_and_full_size():
    w = wl.config("star3d_512")
    a0 = wl.crop_grid(w, 64)
    ref = oracle.periodic(rounded_input(a0, "f32"), w.coeffs, w.T)
    assert_close(gpu_periodic(a0, w.coeffs, w.T, "f32"), ref, TOL["f32"])
    full = w.grid()
    g32 = gpu_periodic(full, w.coeffs, w.T, "f32")
    g64 = gpu_periodic(rounded_input(full, "f32"), w.coeffs, w.T, "f64")
    assert_close(g32, g64, TOL["f32"])


@pytest.mark.slow
def test_largest_1d_extent():
    n = 1 << 24
    c = _coeffs(1, 2, False, 12)
    a0 = wl.uniform(12, "grid", n)
    T = 3
    for dtype in ("f32", "f64"):
        ref = oracle.periodic(rounded_input(a0, dtype), c, T)
        assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype])
