"""Stencils of radius 3..8 (the general-radius path: forward passes, the symbol
power of any radius on the half spectrum, inverse passes) against the FP64 loop
oracle, through the single-problem entry point, the batch and the server; and
problems the batched launches cannot hold (extents with a prime factor above 7,
radius above 2) mixed into a batch and a serving stream."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_periodic, rounded_input, to_dev

pytestmark = pytest.mark.gpu


def _coeffs(kind, d, r, seed):
    if kind == "box":  # nonnegative, sum 1
        return wl.box_random_coeffs(seed, d, r)
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1.0, 1.0, size=(2 * r + 1,) * d)
    if kind == "mixed":  # mixed signs, |lambda| <= 1 bound by sum |c| = 1
        return c / np.abs(c).sum()
    if kind == "damped":  # one sign, sum 0.95
        c = np.abs(c)
        return 0.95 * c / c.sum()
    raise ValueError(kind)


CASES = [
    ((4096,), 3, 50, "box"), ((1000,), 4, 17, "mixed"), ((120,), 8, 9, "box"),
    ((96, 80), 3, 21, "box"), ((64, 60), 4, 200, "damped"), ((50, 48), 5, 3, "mixed"), ((32, 30), 8, 2, "box"),
    ((24, 20, 18), 3, 9, "box"), ((16, 12, 10), 4, 4, "mixed"), ((512, 512), 3, 1, "mixed"),
    ((7, 5), 3, 5, "box"),  # extents shorter than 2r + 1: offsets alias
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_general_radius_against_oracle(case, dtype):
    dims, r, T, kind = CASES[case]
    c = _coeffs(kind, len(dims), r, 300 + case)
    a0 = wl.uniform(300 + case, "grid", int(np.prod(dims))).reshape(dims)
    print(f"general radius: dims={dims} r={r} T={T} {kind} {dtype}", flush=True)
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype], (dims, r, T, kind, dtype))


def test_radius_above_the_general_limit_is_rejected():
    import paper_2105_06676_amd as sfft
    g = to_dev(np.ones((40, 40)), "f64")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic(g, np.ones((19, 19)) / 361, 3)  # r = 9
    assert e.value.code == -2
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic(to_dev(np.ones((41, 40)), "f64"), np.ones((7, 7)) / 49, 3)  # r = 3, 41 not 7-smooth
    assert e.value.code == -2


def _mixed_list():
    """(input, coeffs, T, dtype) for problems of every kind a batch may hold."""
    out = []
    specs = [((64, 48), 1, 30, "f64"), ((101, 64), 1, 25, "f64"), ((97,), 2, 40, "f32"), ((60, 50), 3, 12, "f64"),
             ((1000,), 4, 9, "f32"), ((30, 42), 2, 50, "f32"), ((13, 11, 12), 1, 6, "f64"), ((20, 18, 16), 3, 4, "f32")]
    for k, (dims, r, T, dt) in enumerate(specs):
        c = wl.box_random_coeffs(400 + k, len(dims), r)
        a = wl.uniform(400 + k, "grid", int(np.prod(dims))).reshape(dims)
        out.append((a, c, T, dt))
    return out


def test_batch_holds_non_smooth_and_wide_radius_problems():
    import torch
    import paper_2105_06676_amd as sfft
    probs = _mixed_list()
    grids = [to_dev(a, dt) for a, c, T, dt in probs]
    sfft.batch([(g, c, T) for g, (a, c, T, dt) in zip(grids, probs)])
    torch.cuda.synchronize()
    for g, (a, c, T, dt) in zip(grids, probs):
        ref = oracle.periodic(rounded_input(a, dt), c, T)
        assert_close(g.cpu().numpy().astype(np.float64), ref, TOL[dt], (a.shape, T, dt))


def test_server_holds_non_smooth_and_wide_radius_problems():
    import torch
    import paper_2105_06676_amd as sfft
    probs = _mixed_list()
    srv = sfft.Server(0, 1 << 30, 16)
    grids = [to_dev(a, dt) for a, c, T, dt in probs]
    torch.cuda.synchronize()
    tickets = [srv.submit(g, c, T) for g, (a, c, T, dt) in zip(grids, probs)]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(probs) and st["peak_bytes"] <= st["budget_bytes"]
    for g, (a, c, T, dt) in zip(grids, probs):
        ref = oracle.periodic(rounded_input(a, dt), c, T)
        assert_close(g.cpu().numpy().astype(np.float64), ref, TOL[dt], (a.shape, T, dt))
