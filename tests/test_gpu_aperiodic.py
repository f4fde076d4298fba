"""Parity of the HIP aperiodic solver (StencilFFT-A with RecursiveBoundary) with the
FP64 aperiodic loop oracle (fixed r-wide frame), on the same seeded inputs."""
import contextlib

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_aperiodic, rel_l2, rounded_input

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def cutoff(value):
    import paper_2105_06676_amd as sfft
    sfft.set_option("aperiodic_cutoff", value)
    try:
        yield
    finally:
        sfft.set_option("aperiodic_cutoff", 0)


def _case(dims, r, seed):
    d = len(dims)
    c = wl.box_random_coeffs(seed, d, r)
    store = tuple(n + 2 * r for n in dims)
    a = wl.uniform(seed, "grid", int(np.prod(store))).reshape(store)
    return c, a


CASES = []
for dtype in ("f64", "f32"):
    for dims in [(10,), (37,), (64,), (300,), (8, 8), (13, 29), (40, 40), (64, 50), (100, 7), (33, 1),
                 (6, 7, 8), (12, 12, 12), (20, 16, 10)]:
        for r in (1, 2):
            for T in (1, 2, 5, 17, 40):
                for cut in (0, 1, 3):
                    if (sum(dims) + r * 7 + T + cut) % 4:
                        continue
                    CASES.append((dtype, dims, r, T, cut))


@pytest.mark.parametrize("dtype,dims,r,T,cut", CASES)
def test_aperiodic_small(dtype, dims, r, T, cut):
    c, a = _case(dims, r, 1000 + sum(dims) + T)
    ref = oracle.aperiodic(rounded_input(a, dtype), c, T)
    with cutoff(cut):
        got = gpu_aperiodic(a, c, T, dtype)
    assert_close(got, ref, TOL[dtype], (dims, r, T, cut))
    # the frame is read-only
    inner = tuple(slice(r, r + n) for n in dims)
    mask = np.ones(got.shape, bool)
    mask[inner] = False
    assert np.array_equal(got[mask], rounded_input(a, dtype)[mask])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dims,T,cut", [((200, 180), 37, 4), ((96, 96), 64, 2), ((128, 130), 100, 0),
                                        ((1000,), 300, 16), ((50, 60, 40), 12, 1)])
def test_aperiodic_deep_recursion(dtype, dims, T, cut):
    """Several recursion levels, odd splits, bands wider than half the grid."""
    c, a = _case(dims, 1, 77 + T)
    ref = oracle.aperiodic(rounded_input(a, dtype), c, T)
    with cutoff(cut):
        got = gpu_aperiodic(a, c, T, dtype)
    assert_close(got, ref, TOL[dtype])


def test_aperiodic_non_smooth_extents_and_r0():
    c, a = _case((41, 43), 1, 5)
    ref = oracle.aperiodic(a, c, 9)
    assert_close(gpu_aperiodic(a, c, 9, "f64"), ref, 1e-12)
    c0 = np.array([[0.5]])
    b = wl.uniform(6, "grid", 11 * 13).reshape(11, 13)
    np.testing.assert_allclose(gpu_aperiodic(b, c0, 5, "f64"), 0.5 ** 5 * b, rtol=1e-13)


def test_aperiodic_interior_matches_periodic_far_cells():
    """Cells with dist > r*T equal the periodic solve of the interior (Sec. 4)."""
    from gpu_util import gpu_periodic
    dims, r, T = (64, 48), 1, 10
    c, a = _case(dims, r, 9)
    ap = gpu_aperiodic(a, c, T, "f64")
    inner = tuple(slice(r, r + n) for n in dims)
    per = gpu_periodic(a[inner], c, T, "f64")
    far = oracle.dist(dims) > r * T
    np.testing.assert_allclose(ap[inner][far], per[far], rtol=0, atol=1e-13)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_box2d_aperiodic_reduced_sizes(dtype):
    """The 4096^2 aperiodic workload's stencil (9-point box, r = 1) on 512^2 with T = 512 (the band covers the
    whole grid) and 1024^2 with T = 128, against the full aperiodic oracle."""
    w = wl.config("box2d_aperiodic_4096")
    for n, T in ((512, 512), (1024, 128)):
        store = (n + 2, n + 2)
        a = wl.uniform(w.seed, "grid", store[0] * store[1]).reshape(store)
        ref = oracle.aperiodic(rounded_input(a, dtype), w.coeffs, T)
        got = gpu_aperiodic(a, w.coeffs, T, dtype)
        assert_close(got, ref, TOL[dtype], (n, T))


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_box2d_aperiodic_4096_full_size_sampled(dtype):
    """Full 4096^2, T = 512: cells near two corners and a far interior block are
    checked against the oracle run on sub-boxes of the stored array that contain
    each cell's whole r*T dependency cone (cells whose cone stays inside a box do
    not see the box's cut edges; Sec. 4)."""
    w = wl.config("box2d_aperiodic_4096")
    a = w.grid()
    got = gpu_aperiodic(a, w.coeffs, w.T, dtype)
    src = rounded_input(a, dtype)
    s, K = w.radius * w.T, 128
    n = w.dims[0]
    # top-left corner: interior cells [0, K)^2 (stored [1, K+1)); box up to K + s beyond
    box = src[: K + s + 2, : K + s + 2]
    ref = oracle.aperiodic(box, w.coeffs, w.T)
    assert_close(got[1:K + 1, 1:K + 1], ref[1:K + 1, 1:K + 1], TOL[dtype])
    # bottom-right corner
    box = src[-(K + s + 2):, -(K + s + 2):]
    ref = oracle.aperiodic(box, w.coeffs, w.T)
    assert_close(got[-(K + 1):-1, -(K + 1):-1], ref[-(K + 1):-1, -(K + 1):-1], TOL[dtype])
    # an edge strip straddling the band boundary (depth r*T from the top face),
    # away from corners; the box reaches r*T + 1 cells beyond every checked cell
    # except at the real frame
    c0, h = n // 2, K // 2
    box = src[: 2 * s + h + 2, c0 - h - s: c0 + h + s + 2]
    ref = oracle.aperiodic(box, w.coeffs, w.T)
    rows = slice(1, 1 + s + h)
    assert_close(got[rows, c0 - h + 1: c0 + h + 1], ref[rows, s + 1: s + 1 + K], TOL[dtype])


def _biased(shape_offsets, seed):
    """Coefficients on a (2r+1)^d box that are non-zero only at the listed offsets
    (positive weights of sum 1): asymmetric reach per face."""
    offs, r, d = shape_offsets
    c = np.zeros((2 * r + 1,) * d)
    w = wl.uniform(seed, "coef", len(offs)) + 0.1
    for o, x in zip(offs, w / w.sum()):
        c[tuple(oi + r for oi in o)] = x
    return c


# (name, dims, (offsets, r, d), T, cutoff)
BIASED = [
    ("upwind_1d", (300,), ([(-1,), (0,)], 1, 1), 150, 8),
    ("upwind_1d_r2", (257,), ([(-2,), (-1,), (0,)], 2, 1), 90, 4),
    ("upwind_2d", (120, 100), ([(-1, 0), (0, -1), (0, 0)], 1, 2), 60, 0),
    ("downwind_2d", (90, 110), ([(1, 0), (0, 1), (0, 0), (1, 1)], 1, 2), 45, 3),
    ("axis0_only_2d", (96, 80), ([(-2, 0), (-1, 0), (0, 0), (1, 0), (2, 0)], 2, 2), 40, 0),
    ("biased_axis0_2d", (100, 90), ([(-2, 0), (-1, -1), (0, 0), (1, 1), (0, 1)], 2, 2), 33, 2),
    ("radius2_reach1_2d", (70, 60), ([(-1, 0), (1, 0), (0, -1), (0, 1), (0, 0)], 2, 2), 50, 0),
    ("upwind_3d", (20, 18, 16), ([(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0)], 1, 3), 24, 0),
    ("axis2_only_3d", (12, 10, 40), ([(0, 0, -1), (0, 0, 1), (0, 0, 0)], 1, 3), 30, 2),
    # reach differs between axes: per-axis entry times (2 cells per step along one axis)
    ("reach2_axis0_reach1_axis1", (150, 130), ([(-2, 0), (2, 0), (0, -1), (0, 1), (0, 0)], 2, 2), 70, 0),
    ("reach1_axis0_reach2_axis1", (90, 160), ([(-1, 0), (1, 0), (0, -2), (0, 2), (0, 0), (1, 1)], 2, 2), 45, 3),
    ("reach_2_1_1_3d", (30, 24, 20), ([(-2, 0, 0), (2, 0, 0), (0, -1, 0), (0, 0, 1), (0, 0, 0)], 2, 3), 14, 1),
    ("upwind_reach2_axis1_2d", (64, 120), ([(0, -2), (0, -1), (-1, 0), (0, 0)], 2, 2), 40, 2),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,dims,spec,T,cut", BIASED, ids=[b[0] for b in BIASED])
def test_aperiodic_biased_stencils(name, dims, spec, T, cut, dtype):
    """Stencils that reach unevenly (or not at all) toward some faces: entry-time
    bookkeeping (appendix on l-shells) drops the slabs and base-case strips of faces
    the stencil never reads toward and scales the others by the reach of their axis."""
    c = _biased(spec, 70 + len(dims))
    r = spec[1]
    store = tuple(n + 2 * r for n in dims)
    a = wl.uniform(71 + sum(dims), "grid", int(np.prod(store))).reshape(store)
    ref = oracle.aperiodic(rounded_input(a, dtype), c, T)
    with cutoff(cut):
        got = gpu_aperiodic(a, c, T, dtype)
    assert_close(got, ref, TOL[dtype], name)
