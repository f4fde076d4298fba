"""Parity of the aperiodic solver with a reflecting (zero-flux, Neumann) boundary
against the FP64 loop oracle with the same boundary (Sec. 4: the base case of
RecursiveBoundary applies the boundary condition; the FFT parts only keep cells
the boundary cannot reach)."""
import contextlib

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rounded_input, to_dev, torch_mod

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def cutoff(value):
    import paper_2105_06676_amd as sfft
    sfft.set_option("aperiodic_cutoff", value)
    try:
        yield
    finally:
        sfft.set_option("aperiodic_cutoff", 0)


def _inner(a, r):
    return a[tuple(slice(r, s - r) for s in a.shape)]


def gpu_reflect(a, c, T, dtype):
    import paper_2105_06676_amd as sfft
    g = to_dev(a, dtype)
    sfft.aperiodic(g, c, T, bc="reflect")
    torch_mod().cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


def _check(a, c, T, dtype, what):
    r = (c.shape[0] - 1) // 2
    src = rounded_input(a, dtype)
    ref = oracle.aperiodic(src, c, T, bc="reflect")
    got = gpu_reflect(a, c, T, dtype)
    assert_close(_inner(got, r), _inner(ref, r), TOL[dtype], what)
    # the frame is neither read nor written
    mask = np.ones(got.shape, bool)
    mask[tuple(slice(r, s - r) for s in got.shape)] = False
    assert np.array_equal(got[mask], src[mask]), what


def _case(dims, r, seed):
    c = wl.box_random_coeffs(seed, len(dims), r)
    store = tuple(n + 2 * r for n in dims)
    a = wl.uniform(seed, "grid", int(np.prod(store))).reshape(store)
    return c, a


CASES = []
for dtype in ("f64", "f32"):
    for dims in [(10,), (37,), (300,), (8, 8), (13, 29), (64, 50), (100, 7), (33, 2),
                 (6, 7, 8), (12, 12, 12), (20, 16, 10)]:
        for r in (1, 2):
            for T in (1, 3, 17, 40):
                for cut in (0, 1, 3):
                    if (sum(dims) + 3 * r + T + cut) % 5:
                        continue
                    CASES.append((dtype, dims, r, T, cut))


@pytest.mark.parametrize("dtype,dims,r,T,cut", CASES)
def test_reflect_small(dtype, dims, r, T, cut):
    """Random full-box stencils (asymmetric), recursion depth set by the cutoff."""
    c, a = _case(dims, r, 2000 + sum(dims) + T)
    with cutoff(cut):
        _check(a, c, T, dtype, (dims, r, T, cut))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dims,T,cut", [((200, 180), 37, 4), ((96, 96), 64, 2), ((1000,), 300, 16),
                                        ((50, 60, 40), 12, 1)])
def test_reflect_deep_recursion(dtype, dims, T, cut):
    c, a = _case(dims, 1, 91 + T)
    with cutoff(cut):
        _check(a, c, T, dtype, (dims, T, cut))


def _biased(offs, r, d, seed):
    c = np.zeros((2 * r + 1,) * d)
    w = wl.uniform(seed, "coef", len(offs)) + 0.1
    for o, x in zip(offs, w / w.sum()):
        c[tuple(oi + r for oi in o)] = x
    return c


BIASED = [
    ("upwind_1d", (300,), [(-1,), (0,)], 1, 150, 8),
    ("upwind_2d", (120, 100), [(-1, 0), (0, -1), (0, 0)], 1, 60, 0),
    ("downwind_2d", (90, 110), [(1, 0), (0, 1), (0, 0), (1, 1)], 1, 45, 3),
    ("radius2_reach1_2d", (70, 60), [(-1, 0), (1, 0), (0, -1), (0, 1), (0, 0)], 2, 50, 0),
    ("axis2_only_3d", (12, 10, 40), [(0, 0, -1), (0, 0, 1), (0, 0, 0)], 1, 30, 2),
    ("reach2_axis0_reach1_axis1", (150, 130), [(-2, 0), (2, 0), (0, -1), (0, 1), (0, 0)], 2, 70, 0),
    ("reach_2_1_1_3d", (30, 24, 20), [(-2, 0, 0), (2, 0, 0), (0, -1, 0), (0, 0, 1), (0, 0, 0)], 2, 14, 1),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,dims,offs,r,T,cut", BIASED, ids=[b[0] for b in BIASED])
def test_reflect_biased_stencils(name, dims, offs, r, T, cut, dtype):
    """Faces the stencil never reads toward are dropped: the reflection there is never seen."""
    c = _biased(offs, r, len(dims), 40 + len(dims))
    store = tuple(n + 2 * r for n in dims)
    a = wl.uniform(41 + sum(dims), "grid", int(np.prod(store))).reshape(store)
    with cutoff(cut):
        _check(a, c, T, dtype, name)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_reflect_half_sample_cosine_at_size(dtype):
    """1500 x 1300, T = 700, heat stencil: the half-sample cosine mode evolves by its
    eigenvalue (closed form of the reflecting boundary, no oracle run needed)."""
    r = 1
    c = np.array([[0.0, 0.2, 0.0], [0.2, 0.2, 0.2], [0.0, 0.2, 0.0]])
    dims, ks, T = (1500, 1300), (3, 2), 700
    mode = np.cos(np.pi * ks[0] * (np.arange(dims[0]) + 0.5) / dims[0])[:, None] * \
        np.cos(np.pi * ks[1] * (np.arange(dims[1]) + 0.5) / dims[1])[None, :]
    lam = 0.2 + 0.4 * np.cos(np.pi * ks[0] / dims[0]) + 0.4 * np.cos(np.pi * ks[1] / dims[1])
    a = np.pad(mode, r, mode="constant", constant_values=5.0)
    got = _inner(gpu_reflect(a, c, T, dtype), r)
    assert_close(got, lam ** T * mode, TOL[dtype], (dims, T))


def test_reflect_conserves_mass_large():
    """Symmetric stencil of sum 1: the interior sum is conserved (FP64, 700^2, T = 900)."""
    c = wl.box_random_coeffs(5, 2, 1)
    c = (c + c[::-1, :] + c[:, ::-1] + c[::-1, ::-1]) / 4
    c /= c.sum()
    a = np.pad(wl.uniform(6, "grid", 700 * 700).reshape(700, 700), 1)
    got = _inner(gpu_reflect(a, c, 900, "f64"), 1)
    assert abs(got.sum() - a.sum()) <= 1e-11 * a.sum()


def test_reflect_batch_and_server_equal_single_solve():
    import paper_2105_06676_amd as sfft
    torch = torch_mod()
    probs = []
    for i, (dims, r, T) in enumerate([((40, 30), 1, 9), ((257,), 2, 70), ((9, 10, 11), 1, 5), ((64, 64), 2, 33)]):
        c, a = _case(dims, r, 300 + i)
        probs.append((a, c, T))
    alone = [gpu_reflect(a, c, T, "f64") for a, c, T in probs]
    grids = [to_dev(a, "f64") for a, _, _ in probs]
    sfft.batch([(g, c, T, "reflect") for g, (_, c, T) in zip(grids, probs)])
    torch.cuda.synchronize()
    for g, ref in zip(grids, alone):
        assert np.array_equal(g.cpu().numpy(), ref)
    srv = sfft.Server(0)
    try:
        grids = [to_dev(a, "f64") for a, _, _ in probs]
        tickets = [srv.submit(g, c, T, "reflect") for g, (_, c, T) in zip(grids, probs)]
        for t in tickets:
            srv.wait(t)
        torch.cuda.synchronize()
        for g, ref in zip(grids, alone):
            assert np.array_equal(g.cpu().numpy(), ref)
    finally:
        srv.close()
    # and the fixed-frame kind is a different problem
    c, a = _case((40, 30), 1, 300)
    fixed = to_dev(a, "f64")
    sfft.aperiodic(fixed, c, 9)
    torch.cuda.synchronize()
    assert not np.array_equal(fixed.cpu().numpy(), alone[0])


def test_reflect_rejects_bad_arguments():
    import paper_2105_06676_amd as sfft
    c = np.ones((5,)) / 5
    g = to_dev(np.zeros(1 + 4), "f64")   # interior 1 < radius 2
    with pytest.raises(RuntimeError, match="EINVAL"):
        sfft.aperiodic(g, c, 3, bc="reflect")
    with pytest.raises(ValueError):
        sfft.aperiodic(to_dev(np.zeros(9), "f64"), c, 3, bc="mirror")


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_reflect_4096_full_size_sampled(dtype):
    """Full 4096^2, T = 512, reflecting frame: two corners and an edge strip against
    the oracle run on sub-boxes of the stored array that hold each checked cell's
    whole r*T dependency cone (a box's cut edges, reflecting in the oracle run, lie
    more than r*T cells from every checked cell; Sec. 4)."""
    w = wl.config("box2d_reflect_4096")
    a = w.grid()
    got = gpu_reflect(a, w.coeffs, w.T, dtype)
    src = rounded_input(a, dtype)
    s, K, n = w.radius * w.T, 128, w.dims[0]
    box = src[: K + s + 2, : K + s + 2]
    ref = oracle.aperiodic(box, w.coeffs, w.T, bc="reflect")
    assert_close(got[1:K + 1, 1:K + 1], ref[1:K + 1, 1:K + 1], TOL[dtype])
    box = src[-(K + s + 2):, -(K + s + 2):]
    ref = oracle.aperiodic(box, w.coeffs, w.T, bc="reflect")
    assert_close(got[-(K + 1):-1, -(K + 1):-1], ref[-(K + 1):-1, -(K + 1):-1], TOL[dtype])
    c0, h = n // 2, K // 2
    box = src[: 2 * s + h + 2, c0 - h - s: c0 + h + s + 2]
    ref = oracle.aperiodic(box, w.coeffs, w.T, bc="reflect")
    rows = slice(1, 1 + s + h)
    assert_close(got[rows, c0 - h + 1: c0 + h + 1], ref[rows, s + 1: s + 1 + K], TOL[dtype])
