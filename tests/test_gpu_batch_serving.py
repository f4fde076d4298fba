"""Batched launches, graph replay and the continuous-batching server.

* a batch of uneven problems (1-D/2-D/3-D, FP32/FP64, different T, periodic and
  aperiodic) gives every problem exactly the result of solving it alone, and
  matches the oracle;
* a captured graph replayed several times, with eager work between replays,
  reproduces the eager batch every time;
* the server returns each request's result bit-identical to the request solved
  alone, also when a tiny HBM budget forces queueing, and rejects invalid or
  oversize requests at submit.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rel_l2, rounded_input, to_dev

pytestmark = pytest.mark.gpu


def _mix(seed=7, n=14):
    rng = np.random.default_rng(seed)
    shapes = [(4096,), (96,), (1000,), (64, 48), (30, 42), (128, 128), (24, 20, 18), (16, 32, 8),
              (8192,), (7, 9), (256, 100), (50, 60), (12, 12, 12), (3000,)]
    probs = []
    for i in range(n):
        dims = shapes[i % len(shapes)]
        r = 1 + (i % 2)
        if len(dims) == 3 and r == 2 and max(dims) > 20:
            r = 1
        c = wl.box_random_coeffs(seed * 100 + i, len(dims), r)
        T = int(rng.integers(1, 3000))
        dtype = "f32" if i % 3 == 0 else "f64"
        a = wl.uniform(seed * 100 + i, "grid", int(np.prod(dims))).reshape(dims)
        probs.append((a, c, T, dtype))
    return probs


def test_batch_equals_alone_and_oracle():
    import torch
    import paper_2105_06676_amd as sfft
    probs = _mix()
    alone = []
    for a, c, T, dt in probs:
        g = to_dev(a, dt)
        sfft.periodic(g, c, T)
        alone.append(g)
    grids = [to_dev(a, dt) for a, c, T, dt in probs]
    sfft.batch([(g, c, T) for g, (a, c, T, dt) in zip(grids, probs)])
    torch.cuda.synchronize()
    for g, al, (a, c, T, dt) in zip(grids, alone, probs):
        assert torch.equal(g, al)
        if a.size <= 70000:
            ref = oracle.periodic(rounded_input(a, dt), c, T)
            assert_close(g.cpu().numpy().astype(np.float64), ref, TOL[dt])


def test_batch_with_aperiodic_members():
    import torch
    import paper_2105_06676_amd as sfft
    c = wl.box_random_coeffs(3, 2, 1)
    ap = wl.uniform(3, "grid", 42 * 38).reshape(42, 38)
    pe = wl.uniform(4, "grid", 40 * 36).reshape(40, 36)
    ga, gp = to_dev(ap, "f64"), to_dev(pe, "f64")
    sfft.batch([(ga, c, 21, True), (gp, c, 33)])
    torch.cuda.synchronize()
    assert_close(ga.cpu().numpy(), oracle.aperiodic(ap, c, 21), 1e-12)
    assert_close(gp.cpu().numpy(), oracle.periodic(pe, c, 33), 1e-12)


def test_batch_rejects_invalid_member_without_running():
    import torch
    import paper_2105_06676_amd as sfft
    c = wl.box_random_coeffs(3, 2, 1)
    good = to_dev(np.ones((16, 16)), "f64")
    bad = to_dev(np.ones((11, 16)), "f64")
    wide = np.ones((7, 7)) / 49  # radius 3 needs 7-smooth extents; 11 is not
    with pytest.raises(sfft.SfftError) as e:
        sfft.batch([(good, c, 5), (bad, wide, 5)])
    assert "problem 1" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(good, torch.ones_like(good))


def test_graph_replays_match_eager():
    import torch
    import paper_2105_06676_amd as sfft
    probs = _mix(seed=9, n=8)
    a0 = [to_dev(a, dt) for a, c, T, dt in probs]
    eager = [x.clone() for x in a0]
    sfft.batch([(g, c, T) for g, (a, c, T, dt) in zip(eager, probs)])
    grids = [x.clone() for x in a0]
    graph = sfft.Graph([(g, c, T) for g, (a, c, T, dt) in zip(grids, probs)])
    for rep in range(3):
        for g, x in zip(grids, a0):
            g.copy_(x)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        # unrelated eager work between replays
        sfft.periodic(to_dev(np.ones((32, 32)), "f32"), wl.jacobi5_coeffs(), 3)
        for g, e in zip(grids, eager):
            assert torch.equal(g, e), rep
    graph.close()


def _serve(probs, budget=0, slots=0):
    import torch
    import paper_2105_06676_amd as sfft
    srv = sfft.Server(0, budget, slots)
    grids = [to_dev(a, dt) for a, c, T, dt in probs]
    torch.cuda.synchronize()
    tickets = [srv.submit(g, c, T) for g, (a, c, T, dt) in zip(grids, probs)]
    for t in tickets:
        srv.wait(t)
    stats = srv.stats()
    times = [srv.times(t) for t in tickets]
    srv.close()
    return grids, stats, times


def test_server_results_equal_alone():
    import torch
    import paper_2105_06676_amd as sfft
    probs = _mix(seed=11, n=24)
    grids, stats, times = _serve(probs)
    assert stats["completed"] == len(probs)
    for g, (a, c, T, dt) in zip(grids, probs):
        al = to_dev(a, dt)
        sfft.periodic(al, c, T)
        torch.cuda.synchronize()
        assert torch.equal(g, al)
    assert all(d >= s >= 0 for s, d in times)


def test_server_tiny_budget_forces_queueing():
    import torch
    import paper_2105_06676_amd as sfft
    probs = _mix(seed=12, n=10)
    # a budget that holds about one of the larger requests at a time
    grids, stats, _ = _serve(probs, budget=4 << 20, slots=2)
    assert stats["completed"] == len(probs)
    assert stats["batches"] >= len(probs) // 2
    assert stats["peak_bytes"] <= 4 << 20
    for g, (a, c, T, dt) in zip(grids, probs):
        al = to_dev(a, dt)
        sfft.periodic(al, c, T)
        torch.cuda.synchronize()
        assert torch.equal(g, al)


def test_server_rejects_bad_requests():
    import paper_2105_06676_amd as sfft
    srv = sfft.Server(0, 1 << 20, 4)
    c = wl.jacobi5_coeffs()
    with pytest.raises(sfft.SfftError):
        srv.submit(to_dev(np.ones((13, 16)), "f32"), np.ones((7, 7)) / 49, 5)  # radius 3 on a non-7-smooth extent
    with pytest.raises(sfft.SfftError):
        srv.submit(to_dev(np.ones((16, 16)), "f32"), c, -1)  # negative T
    with pytest.raises(sfft.SfftError) as e:
        srv.submit(to_dev(np.ones((1024, 1024)), "f64"), c, 5)  # workspace above the budget
    assert e.value.code == -3
    srv.close()


# ------------------------------------------------------------ serving mix --

def _ncoef(req):
    return (2 * req.radius + 1) ** req.ndim


def test_server_staggered_mix_against_oracle():
    """Requests of the serving mix's distribution (d = 1/2/3, r = 1/2, T log-uniform
    up to 1e5, FP32 and FP64; cells capped at 2^20 for the test) arrive staggered
    while earlier ones run.  Every served result is checked against the FP64 loop
    oracle where its cost fits the test's budget, the rest bit for bit against the
    same problem solved alone."""
    import time

    import torch
    import paper_2105_06676_amd as sfft
    reqs = wl.serving_mix(48, seed=31, log2_cells=(10.0, 20.0), max_T=1e5)
    assert {r.ndim for r in reqs} == {1, 2, 3} and {r.radius for r in reqs} == {1, 2}
    assert {r.dtype for r in reqs} == {"f32", "f64"} and max(r.T for r in reqs) >= 10000
    srv = sfft.Server(0, 2 << 30, 16)
    grids = [to_dev(r.grid(), r.dtype) for r in reqs]
    torch.cuda.synchronize()
    span = 0.05  # seconds over which the arrivals are spread
    scale = span / max(reqs[-1].arrival_s, 1e-9)
    t0 = time.perf_counter()
    tickets = []
    for r, g in zip(reqs, grids):
        while time.perf_counter() - t0 < r.arrival_s * scale:
            pass
        tickets.append(srv.submit(g, r.coeffs, r.T))
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["batches"] >= 2
    # oracle for the cheapest results, within a budget of coefficient-updates
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].cells * reqs[i].T * _ncoef(reqs[i]))
    budget, checked = 2.0e9, set()
    for i in order:
        cost = reqs[i].cells * reqs[i].T * _ncoef(reqs[i])
        if cost > budget:
            break
        budget -= cost
        r = reqs[i]
        print(f"oracle check: request {i} dims={r.dims} r={r.radius} T={r.T} {r.dtype}", flush=True)
        ref = oracle.periodic(rounded_input(r.grid(), r.dtype), r.coeffs, r.T)
        assert_close(grids[i].cpu().numpy().astype(np.float64), ref, TOL[r.dtype], (r.dims, r.T, r.dtype))
        checked.add(i)
    assert len(checked) >= 12
    assert {reqs[i].ndim for i in checked} == {1, 2, 3}
    for i, (r, g) in enumerate(zip(reqs, grids)):
        if i in checked:
            continue
        al = to_dev(r.grid(), r.dtype)
        sfft.periodic(al, r.coeffs, r.T)
        torch.cuda.synchronize()
        assert torch.equal(g, al), (i, r.dims, r.T, r.dtype)


def test_server_batches_overlap_on_the_device():
    """A request arriving while an earlier batch runs is launched on another
    stream at once: the two batches' device spans overlap."""
    import time

    import torch
    import paper_2105_06676_amd as sfft
    c = wl.jacobi5_coeffs()
    srv = sfft.Server(0, 4 << 30, 8)
    a = wl.uniform(41, "grid", 4096 * 4096).reshape(4096, 4096)
    grids = [to_dev(a, "f64") for _ in range(4)]
    torch.cuda.synchronize()
    tickets = []
    for g in grids:
        tickets.append(srv.submit(g, c, 1000))
        time.sleep(50e-6)
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    dev = st["device"]
    assert dev["batches_timed"] == st["batches"] >= 2
    assert dev["max_concurrent_batches"] >= 2, dev
    assert dev["sum_batch_ms"] > dev["busy_ms"], dev
    ref = to_dev(a, "f64")
    sfft.periodic(ref, c, 1000)
    torch.cuda.synchronize()
    for g in grids:
        assert torch.equal(g, ref)


def test_server_aperiodic_requests_in_their_budget_and_against_oracle():
    """Aperiodic requests run inside their own block of the HBM budget, sized at
    submit by the solver's bookkeeping: a budget smaller than that block rejects
    the request, and served results match the aperiodic loop oracle."""
    import torch
    import paper_2105_06676_amd as sfft
    c2 = wl.box_random_coeffs(51, 2, 1)
    big = to_dev(np.zeros((514, 514)), "f64")
    small_srv = sfft.Server(0, 1 << 20, 4)
    with pytest.raises(sfft.SfftError) as e:
        small_srv.submit(big, c2, 300, True)  # needs several 2 MB level buffers
    assert e.value.code == -3
    small_srv.close()
    cases = [((60, 50), c2, 40, "f64"), ((60, 50), c2, 7, "f32"), ((300,), wl.box_random_coeffs(52, 1, 2), 90, "f64"),
             ((20, 18, 16), wl.box_random_coeffs(53, 3, 1), 9, "f64"), ((130, 100), c2, 100, "f32")]
    srv = sfft.Server(0, 1 << 30, 8)
    items = []
    for k, (dims, c, T, dt) in enumerate(cases):
        r = (c.shape[0] - 1) // 2
        a = wl.uniform(60 + k, "grid", int(np.prod([n + 2 * r for n in dims]))).reshape([n + 2 * r for n in dims])
        g = to_dev(a, dt)
        items.append((a, c, T, dt, g, srv.submit(g, c, T, True)))
    # periodic requests in the same stream of arrivals
    p = wl.uniform(70, "grid", 64 * 48).reshape(64, 48)
    gp = to_dev(p, "f64")
    tp = srv.submit(gp, c2, 33)
    for it in items:
        srv.wait(it[5])
    srv.wait(tp)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(cases) + 1
    assert st["peak_bytes"] <= st["budget_bytes"]
    torch.cuda.synchronize()
    for a, c, T, dt, g, _ in items:
        ref = oracle.aperiodic(rounded_input(a, dt), c, T)
        assert_close(g.cpu().numpy().astype(np.float64), ref, TOL[dt], (a.shape, T, dt))
    assert_close(gp.cpu().numpy(), oracle.periodic(p, c2, 33), TOL["f64"])
