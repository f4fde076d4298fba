"""The periodic entry point that allocates no device memory, through the C ABI:
its results against the allocating entry point's on the same inputs (the same
passes run, so they agree bit for bit) and, for the smaller shapes, against the
FP64 loop oracle; two calls in a row with the second on a smaller input (the
fixed device array keeps the first call's contents); a shape too large for the
array is rejected before anything runs."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rounded_input, to_dev

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2105_06676_amd as sfft
    return sfft


def _inputs(dims, r, seed):
    c = wl.box_random_coeffs(seed, len(dims), r)
    a0 = wl.uniform(seed, "grid", int(np.prod(dims))).reshape(dims)
    return a0, c


# (larger shape, smaller shape) pairs run back to back
SEQUENCES = [
    (((1536, 1280), 1, 37), ((96, 80), 2, 5)),        # 2-D: power-of-two register kernels, then small
    (((1000, 1200), 2, 11), ((60, 84), 1, 3)),        # 2-D 5-/7-smooth: generic kernels
    (((64, 48, 40), 1, 9), ((16, 12, 10), 1, 4)),     # 3-D
    (((1 << 20,), 1, 64), ((1000,), 2, 17)),          # 1-D split axis, then one row
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("seq", range(len(SEQUENCES)))
def test_noalloc_matches_allocating_entry_point_twice(dtype, seq):
    """Two no-allocation calls back to back (the second on a smaller grid), then
    the allocating entry point on copies of the same inputs."""
    torch = pytest.importorskip("torch")
    sfft = _lib()
    cases = []
    for i, (dims, r, T) in enumerate(SEQUENCES[seq]):
        a0, c = _inputs(dims, r, 700 + 10 * seq + i)
        g = to_dev(a0, dtype)
        cases.append((dims, r, T, a0, c, g, g.clone()))
    for i, (dims, r, T, a0, c, g, _) in enumerate(cases):
        print(f"noalloc call {i}: seq={seq} dims={dims} r={r} T={T} {dtype}", flush=True)
        sfft.periodic_noalloc(g, c, T)
    torch.cuda.synchronize()
    for dims, r, T, a0, c, _, g2 in cases:
        sfft.periodic(g2, c, T)
    torch.cuda.synchronize()
    for dims, r, T, a0, c, g, g2 in cases:
        got = g.cpu().numpy().astype(np.float64)
        want = g2.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, want, err_msg=f"{dims} {dtype}")
        if np.prod(dims) * T <= 2e7:
            ref = oracle.periodic(rounded_input(a0, dtype), c, T)
            assert_close(got, ref, TOL[dtype], (dims, r, T, dtype))


def test_noalloc_rejects_a_shape_larger_than_its_array():
    torch = pytest.importorskip("torch")
    sfft = _lib()
    g = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda:0")
    g[0, 0] = 1.0
    c = np.zeros((3, 3))
    c[1, 1] = 0.5
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_noalloc(g, c, 3)
    assert e.value.code == -3 and "fixed" in str(e.value)
    torch.cuda.synchronize()
    assert float(g[0, 0]) == 1.0 and float(g.abs().sum()) == 1.0  # untouched


def test_noalloc_rejects_non_smooth_extents():
    torch = pytest.importorskip("torch")
    sfft = _lib()
    g = torch.zeros((11, 16), dtype=torch.float32, device="cuda:0")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_noalloc(g, np.ones((3, 3)) / 9, 3)
    assert e.value.code == -2


def test_noalloc_c_abi_symbol_and_limit():
    sfft = _lib()
    f = sfft.lib.stencil_fft_periodic_noalloc
    f.restype = ctypes.c_int
    dims = (ctypes.c_int64 * 2)(8, 8)
    c = np.ones((3, 3)) / 9
    assert f(None, 0, 2, dims, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1, 5, None) == -1
