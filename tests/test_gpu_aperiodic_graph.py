"""Repeated aperiodic solves replayed from captured graphs.

The second identical call (same grid address, shape, coefficients, T, stream)
captures the RecursiveBoundary enqueue into a graph and later identical calls
replay it.  Every replay must reproduce the directly enqueued solve bit for bit,
also with unrelated eager work and synchronisations between replays, and a call
that differs in T or in the coefficients must not pick up another call's graph.
"""
import contextlib

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rel_l2, rounded_input, to_dev

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def graphs(enabled):
    import paper_2105_06676_amd as sfft
    sfft.set_option("aperiodic_graphs", 1 if enabled else 0)
    try:
        yield
    finally:
        sfft.set_option("aperiodic_graphs", 1)


def _direct(a0, c, T):
    import torch
    import paper_2105_06676_amd as sfft
    g = a0.clone()
    with graphs(False):
        sfft.aperiodic(g, c, T)
    torch.cuda.synchronize()
    return g


def _other_work():
    import torch
    import paper_2105_06676_amd as sfft
    x = to_dev(wl.uniform(99, "grid", 64 * 64).reshape(64, 64), "f32")
    sfft.periodic(x, wl.jacobi5_coeffs(), 7)
    y = to_dev(wl.uniform(98, "grid", 50 * 46).reshape(50, 46), "f64")
    sfft.aperiodic(y, wl.box_random_coeffs(98, 2, 1), 40)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dims,r,T", [((300, 260), 1, 100), ((130, 100), 2, 37), ((40, 36, 30), 1, 20),
                                      ((5000,), 1, 900)])
def test_replays_match_direct(dims, r, T, dtype):
    import torch
    import paper_2105_06676_amd as sfft
    d = len(dims)
    c = wl.box_random_coeffs(41 + d + r, d, r)
    store = tuple(n + 2 * r for n in dims)
    host = wl.uniform(41, "grid", int(np.prod(store))).reshape(store)
    a0 = to_dev(host, dtype)
    ref = _direct(a0, c, T)
    g = a0.clone()
    for rep in range(5):
        g.copy_(a0)
        torch.cuda.synchronize()
        sfft.aperiodic(g, c, T)
        torch.cuda.synchronize()
        assert torch.equal(g, ref), rep
        _other_work()
    want = oracle.aperiodic(rounded_input(host, dtype), c, T)
    assert_close(g.cpu().numpy().astype(np.float64), want, TOL[dtype])


def test_changed_key_is_not_replayed():
    import torch
    import paper_2105_06676_amd as sfft
    dims, r = (200, 180), 1
    store = tuple(n + 2 * r for n in dims)
    a0 = to_dev(wl.uniform(43, "grid", int(np.prod(store))).reshape(store), "f64")
    c1 = wl.box_random_coeffs(43, 2, 1)
    c2 = c1.copy()
    c2.flat[0] += 2.0 ** -20
    cases = [(c1, 64), (c1, 65), (c2, 64), (c1, 64), (c2, 65), (c1, 65), (c2, 64)]
    refs = {(id(c), T): _direct(a0, c, T) for c, T in cases}
    g = a0.clone()
    for _ in range(2):
        for c, T in cases:
            g.copy_(a0)
            sfft.aperiodic(g, c, T)
            torch.cuda.synchronize()
            assert torch.equal(g, refs[(id(c), T)]), T
    assert not torch.equal(refs[(id(c1), 64)], refs[(id(c2), 64)])


def test_graphs_follow_buffer_growth():
    """A larger solve between replays regrows shared scratch buffers; the
    smaller solve's graph must then not be replayed with stale addresses."""
    import torch
    import paper_2105_06676_amd as sfft
    r = 1
    c = wl.box_random_coeffs(44, 2, 1)
    small = to_dev(wl.uniform(44, "grid", 122 * 102).reshape(122, 102), "f64")
    ref = _direct(small, c, 50)
    g = small.clone()
    for rep in range(4):
        g.copy_(small)
        sfft.aperiodic(g, c, 50)
        torch.cuda.synchronize()
        assert torch.equal(g, ref), rep
        big = to_dev(np.ones((300 + 40 * rep, 280 + 2 * r)), "f64")
        sfft.aperiodic(big, c, 60)
        torch.cuda.synchronize()
