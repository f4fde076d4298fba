"""The seeded input generator: SplitMix64 values, distributions and workload recipes."""
import numpy as np

import workloads as w


def test_splitmix64_known_values():
    # state 0: outputs mix(1*gamma), mix(2*gamma), mix(3*gamma) of the published generator
    z = w._mix(np.arange(1, 4, dtype=np.uint64) * w.GAMMA)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_range_and_offsets():
    u = w.uniform(3, "grid", 10000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.02
    assert np.array_equal(w.uniform(3, "grid", 5, start=100), u[100:105])
    assert not np.array_equal(w.uniform(3, "coef", 5), u[:5])


def test_gaussian_moments():
    g = w.gaussian(4, "grid", 20000)
    assert abs(g.mean()) < 0.03 and abs(g.std() - 1.0) < 0.03


def test_coefficients_sum_exactly_one():
    for c in (w.star7_random_coeffs(3), w.box_random_coeffs(4, 2, 1), w.box_random_coeffs(7, 3, 2)):
        assert c.sum() == 1.0 and (c >= 0).all()
    c3 = w.config("star3d_512").coeffs
    assert c3[1, 1, 1] >= 0.4 and np.count_nonzero(c3) == 7


def test_crop_matches_full_grid():
    for name, side in (("jacobi2d_8192", 8), ("star3d_512", 2)):
        cfg = w.config(name)
        small = w.Workload(cfg.name, cfg.ndim, (side * 3,) * cfg.ndim, cfg.radius, cfg.T,
                           cfg.coeffs, cfg.seed, cfg.init)
        # crop of a grid whose rows have the full-size stride
        crop = w.crop_grid(cfg, side)
        full_rows = cfg.dims[-1]
        for lead in np.ndindex(*(side,) * (cfg.ndim - 1)):
            off = 0
            stride = 1
            strides = []
            for n in reversed(cfg.dims):
                strides.append(stride)
                stride *= n
            strides = list(reversed(strides))
            off = sum(l * s for l, s in zip(lead, strides[:-1]))
            if cfg.init == "uniform":
                row = w.uniform(cfg.seed, "grid", side, start=off)
            else:
                row = w.gaussian(cfg.seed, "grid", off + side)[off:]
            assert np.array_equal(crop[lead], row)
        assert small.dims[-1] != full_rows


def test_serving_mix_shapes():
    reqs = w.serving_mix(200)
    assert all(1 <= r.ndim <= 3 for r in reqs)
    assert all(2 ** 9 <= r.cells <= 2 ** 25 for r in reqs)
    assert all(1 <= r.T <= 100000 and r.radius in (1, 2) for r in reqs)
    assert all(w._is_7smooth(n) for r in reqs for n in r.dims)
    assert sorted(r.arrival_s for r in reqs) == [r.arrival_s for r in reqs]
