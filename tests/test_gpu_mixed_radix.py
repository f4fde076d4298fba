"""The register mixed-radix kernels (7-smooth transform lengths held 5, 7, 9, 10,
12, 14, 15, 20, 21 or 25 points per thread) against the FP64 loop oracle: every family,
rows (real-to-complex, complex-to-real, the whole 1-D solve) and strided axes
(forward, inverse, fused middle pass, split twiddles), every mode visible (T = 1
with an asymmetric stencil) and long damped runs; batched launches that mix these
kernels with the other families; the pass schedule uses them where expected."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_periodic, rounded_input, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [
    (2000, 1000),     # rows 500 = 4 * 125; columns 2000 = 16 x 125
    (250, 160),       # rows 80 = 16 * 5 (FP64: 10 points); columns 250 = 2 * 125
    (96, 768),        # rows 384 = 2^7 * 3 (12 points); columns 96 = 2^5 * 3
    (75, 50),         # columns 75 = 3 * 25 (generic), rows 25 = 5^2
    (20, 40, 100),    # 3-D: rows 50, columns 40 and 20
    (640,),           # 1-D whole solve, L = 320 = 2^6 * 5
    (1536,),          # 1-D whole solve, L = 768 = 2^8 * 3
    (8000, 64),       # the paper's 8000: columns 8000 = 64 x 125
    # lengths mixing 3, 5 and 7 (12-, 14-, 15- and 21-point threads, middle stages
    # whose radix does not divide the points per thread)
    (630, 420),       # columns 630 = 2 3^2 5 7, rows 210
    (1470, 90),       # columns 1470 = 2 3 5 7^2, rows 45 = 3^2 5
    (210, 3360),      # rows 1680 = 2^4 3 5 7 (the 6720 rows of the 6300 x 6720 torus halved twice)
    (63, 105, 42),    # 3-D: 63 = 3^2 7, 105 = 3 5 7, rows 21
    (6300, 16),       # columns 6300 = 2^2 3^2 5^2 7 split in levels
    # 7- and 9-point threads (7^b, 3^b, 2 3^b) and the gather form (a last radix
    # that divides no Q: the outputs are read back from LDS in natural order)
    (49, 98),         # columns 49 = 7^2, rows 49
    (343, 16),        # columns 343 = 7^3
    (27, 162),        # columns 27 = 3^3, rows 81 = 3^4
    (54, 486),        # columns 54 = 2 3^3 (radix 2 guarded), rows 243 = 3^5
    (35, 84),         # columns 35 = 5 7 (gather), rows 42 = 2 3 7 (gather)
    (210, 60),        # columns 210 = 2 3 5 7 (gather), rows 30 = 2 3 5 (gather)
    (105, 70, 20),    # 3-D: 105 = 3 5 7 and 70 = 2 5 7 (gather)
    (175, 126),       # columns 175 = 5^2 7 (gather), rows 63 = 3^2 7
    (189, 20),        # columns 189 = 3^3 7
    (1050, 16),       # columns 1050 = 2 3 5^2 7 split in levels
    # odd real rows: one n-point complex transform per row, the half spectrum
    # stored, the mirrors rebuilt as conjugates on the way back
    (64, 125),        # rows 125 = 5^3
    (30, 49),         # rows 49 = 7^2
    (20, 27),         # rows 27 = 3^3
    (12, 105),        # rows 105 = 3 5 7 (gather)
    (10, 12, 35),     # 3-D, rows 35 = 5 7 (gather)
    (125,),           # 1-D whole solve, odd
    (343,),           # 1-D whole solve, 7^3
    (945,),           # 1-D whole solve, 3^3 5 7
    # 10-point rows with a guarded radix-4 middle stage (the rows' own kernel variant)
    (16, 8000),       # rows 4000 = 10 10 4 10
    (6, 800),         # rows 400 = 10 4 10
    (8000,),          # 1-D whole solve, L = 4000
    # long 1-D axes: strided levels, then a complex row middle pass on these kernels
    (100000,),        # 25 x 4000
    (62500,),         # 20 x 3125
    (18522,),         # 6 x 3087 = 3^2 7^3
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", SHAPES)
def test_mixed_radix_full_spectrum(shape, dtype):
    c = wl.box_random_coeffs(900 + len(shape), len(shape), 1)
    a0 = wl.uniform(900 + shape[0], "grid", int(np.prod(shape))).reshape(shape)
    print(f"mixed radix T=1: {shape} {dtype}", flush=True)
    ref = oracle.periodic(rounded_input(a0, dtype), c, 1)
    assert_close(gpu_periodic(a0, c, 1, dtype), ref, TOL[dtype], (shape, dtype))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(2000, 1000), (96, 768), (20, 40, 100), (640,), (630, 420), (210, 3360),
                                   (49, 98), (35, 84), (210, 60), (54, 486), (64, 125), (945,)])
def test_mixed_radix_long_damped(shape, dtype):
    rng = np.random.default_rng(31)
    c = np.abs(rng.uniform(size=(3,) * len(shape)))
    c = 0.97 * c / c.sum()
    a0 = wl.uniform(31, "grid", int(np.prod(shape))).reshape(shape)
    T = 120
    ref = oracle.periodic(rounded_input(a0, dtype), c, T)
    assert_close(gpu_periodic(a0, c, T, dtype), ref, TOL[dtype], (shape, dtype))


def test_mixed_radix_kernels_are_planned():
    import paper_2105_06676_amd as sfft
    d = sfft.plan_describe((2000, 1000), "f32")
    mixed = [p for p in d["passes"] if p.get("mixed_q")]
    assert len(mixed) >= 3, d["passes"]
    d = sfft.plan_describe((2000, 1000), "f64")
    assert any(p.get("mixed_q") == 10 for p in d["passes"]), d["passes"]


def test_batch_with_mixed_radix_members_equals_alone():
    import torch
    import paper_2105_06676_amd as sfft
    probs = []
    for k, (shape, dt) in enumerate([((2000, 1000), "f32"), ((250, 160), "f64"), ((96, 768), "f32"),
                                     ((250, 160), "f32"), ((1000, 640), "f32"), ((640,), "f64")]):
        c = wl.box_random_coeffs(950 + k, len(shape), 1 + (k % 2))
        a = wl.uniform(950 + k, "grid", int(np.prod(shape))).reshape(shape)
        probs.append((a, c, 37 + k, dt))
    alone = []
    for a, c, T, dt in probs:
        g = to_dev(a, dt)
        sfft.periodic(g, c, T)
        alone.append(g)
    grids = [to_dev(a, dt) for a, c, T, dt in probs]
    sfft.batch([(g, c, T) for g, (a, c, T, dt) in zip(grids, probs)])
    torch.cuda.synchronize()
    for g, al in zip(grids, alone):
        assert torch.equal(g, al)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batch_groups_mixed_members_by_last_radix(dt):
    """Members with the same points per thread but different last-stage radices
    (e.g. 96- and 48-point axes of the 12-point family) run in separate launches
    and each equals its solve alone."""
    import torch
    import paper_2105_06676_amd as sfft
    shapes = [(192, 96), (96, 192), (96, 48), (48, 96), (384,), (192,), (1536, 40)]
    probs = []
    for k, shape in enumerate(shapes):
        c = wl.box_random_coeffs(970 + k, len(shape), 1)
        a = wl.uniform(970 + k, "grid", int(np.prod(shape))).reshape(shape)
        probs.append((a, c, 11 + k))
    alone = []
    for a, c, T in probs:
        g = to_dev(a, dt)
        sfft.periodic(g, c, T)
        alone.append(g)
    grids = [to_dev(a, dt) for a, c, T in probs]
    sfft.batch([(g, c, T) for g, (a, c, T) in zip(grids, probs)])
    torch.cuda.synchronize()
    for g, al, (a, c, T) in zip(grids, alone, probs):
        assert torch.equal(g, al), a.shape
    # and against the oracle
    for g, (a, c, T) in zip(grids, probs):
        ref = oracle.periodic(rounded_input(a, dt), c, T)
        assert_close(g.cpu().numpy().astype(np.float64), ref, TOL[dt], a.shape)
