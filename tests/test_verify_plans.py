"""Host-side verification of every pass schedule the solver builds (no GPU):
each pass's address range, from its descriptor's loop bounds and strides, lies
inside the buffer it addresses; row counts and tile coverage match the transform
extents.  Covered: the aperiodic solves of the GPU suite's shapes (every
recursion depth, slab layouts of both faces, biased stencils, both boundary
conditions, the 1-D FP64 slab shapes), the full-size aperiodic workload, and
periodic schedules of every kernel family (power-of-two, mixed-radix, generic,
split axes, 1-D, 3-D)."""
import contextlib

import numpy as np
import pytest

import workloads as wl


@contextlib.contextmanager
def cutoff(value):
    import paper_2105_06676_amd as sfft
    sfft.set_option("aperiodic_cutoff", value)
    try:
        yield
    finally:
        sfft.set_option("aperiodic_cutoff", 0)


def _ok(rep, what):
    assert rep["failures"] == 0, (what, rep["errors"][:5])
    assert rep["checked"] > 0, what


APERIODIC = []
for dims in [(10,), (37,), (64,), (300,), (1000,), (4097,), (8, 8), (13, 29), (40, 40), (64, 50), (100, 7),
             (33, 1), (200, 180), (6, 7, 8), (12, 12, 12), (20, 16, 10), (50, 60, 40)]:
    for r in (1, 2):
        for T in (1, 5, 17, 40, 300):
            for cut in (0, 1, 3, 16):
                if (sum(dims) + 3 * r + T + cut) % 3 or (cut == 16 and len(dims) > 1):
                    continue  # (a 16-step base case needs a 1-D band to fit one LDS tile)
                APERIODIC.append((dims, r, T, cut))


@pytest.mark.parametrize("kind", ["fixed", "reflect"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_verify_aperiodic_suite_shapes(kind, dtype):
    import paper_2105_06676_amd as sfft
    n = 0
    for dims, r, T, cut in APERIODIC:
        if kind == "reflect" and min(dims) < r:
            continue
        c = wl.box_random_coeffs(5, len(dims), r)
        with cutoff(cut):
            rep = sfft.verify(dims, c, T, dtype, kind)
        _ok(rep, (dims, r, T, cut))
        n += rep["checked"]
    assert n > 1000


def test_verify_aperiodic_biased_stencils():
    import paper_2105_06676_amd as sfft
    for dims, offs, r, T, cut in [((300,), [(-1,), (0,)], 1, 150, 8), ((257,), [(-2,), (-1,), (0,)], 2, 90, 4),
                                  ((120, 100), [(-1, 0), (0, -1), (0, 0)], 1, 60, 0),
                                  ((90, 110), [(1, 0), (0, 1), (0, 0), (1, 1)], 1, 45, 3),
                                  ((20, 18, 16), [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0)], 1, 24, 0)]:
        c = np.zeros((2 * r + 1,) * len(dims))
        for o in offs:
            c[tuple(oi + r for oi in o)] = 1.0 / len(offs)
        for dt in ("f32", "f64"):
            with cutoff(cut):
                _ok(sfft.verify(dims, c, T, dt, "fixed"), (dims, offs))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_verify_aperiodic_full_size_workload(dtype):
    import paper_2105_06676_amd as sfft
    w = wl.config("box2d_aperiodic_4096")
    rep = sfft.verify(w.dims, w.coeffs, w.T, dtype, "fixed")
    _ok(rep, w.dims)
    assert rep["checked"] > 500


@pytest.mark.parametrize("dims", [(8192, 8192), (8000, 8000), (6300, 6720), (4000, 4000), (512, 512, 512),
                                  (400, 400, 400), (800, 800, 800), (65536,), (16384,), (1 << 20,), (2000, 1000),
                                  (250, 160), (96, 768), (75, 50), (20, 40, 100), (640,), (1536, 40), (3, 5),
                                  (1,), (2, 2, 2),
                                  # 7- and 9-point families, gather stages, odd real rows, long 1-D
                                  # axes with complex middle rows, single strided passes up to 1024
                                  (49, 98), (343, 16), (54, 486), (35, 84), (210, 60), (105, 70, 20),
                                  (64, 125), (12, 105), (10, 12, 35), (125,), (945,), (100000,), (18522,),
                                  (1536, 4096), (1280, 64), (640, 200, 256), (1470, 2800)])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_verify_periodic_schedules(dims, dtype):
    import paper_2105_06676_amd as sfft
    c = wl.box_random_coeffs(3, len(dims), 1)
    _ok(sfft.verify(dims, c, 100, dtype), dims)
    c3 = wl.box_random_coeffs(3, len(dims), 3)
    try:
        rep = sfft.verify(dims, c3, 100, dtype)
    except sfft.SfftError as e:
        # the unfused schedule of wide stencils needs a 1-D axis within one row
        assert len(dims) == 1 and dims[0] > 8192 and "EUNSUPPORTED" in str(e), (dims, e)
        return
    _ok(rep, (dims, "radius 3"))
