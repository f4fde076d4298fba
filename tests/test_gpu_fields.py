"""Vector-valued fields on the GPU against the oracle's coupled periodic loop.

m fields evolve together (field i at t+1 = sum_j stencil (i, j) applied to field j
at t); the library transforms all fields as one batch, raises every mode's m x m
symbol matrix to the power T in FP64, and transforms back.  Tolerances are the
scalar path's: relative L2 against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rel_l2, rounded_input, to_dev

pytestmark = pytest.mark.gpu


def _system(seed, m, d, r, sym=False):
    """Coupling blocks c_ij = R_ij * S_ij: R a seeded orthogonal m x m matrix and
    S_ij positive stencils of sum 1, so the zero mode's matrix is R itself (it
    rotates without decay) while every block keeps its own stencil.  sym: every
    S_ij point-symmetric (real symbol matrices)."""
    rng = np.random.default_rng(seed)
    R, _ = np.linalg.qr(rng.standard_normal((m, m)))
    c = np.zeros((m, m) + (2 * r + 1,) * d)
    for i in range(m):
        for j in range(m):
            S = wl.box_random_coeffs(seed * 16 + 4 * i + j, d, r)
            if sym:
                S = 0.5 * (S + np.flip(S))
            c[i, j] = R[i, j] * S
    return c


def _gpu(a, c, T, dtype):
    import torch
    import paper_2105_06676_amd as sfft
    g = to_dev(a, dtype)
    sfft.periodic_fields(g, c, T)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


CASES = [
    ((96,), 2, 1, 37), ((1000,), 3, 2, 500), ((105,), 2, 1, 20), ((16384,), 2, 1, 300),
    ((64, 48), 2, 1, 100), ((30, 42), 3, 1, 77), ((96, 80), 4, 1, 400), ((50, 60), 1, 2, 64),
    ((256, 100), 2, 2, 150), ((16, 12, 10), 2, 1, 45), ((8, 8, 8), 3, 1, 12), ((24, 20, 18), 4, 1, 200),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("dims,m,r,T", CASES)
def test_fields_match_oracle(dims, m, r, T, sym, dtype):
    d = len(dims)
    c = _system(7 + m + r + d, m, d, r, sym)
    a = wl.uniform(7 + len(dims) + m, "grid", m * int(np.prod(dims))).reshape((m,) + dims)
    got = _gpu(a, c, T, dtype)
    want = oracle.periodic_fields(rounded_input(a, dtype), c, T)
    assert_close(got, want, TOL[dtype])


def test_one_field_is_the_scalar_stencil():
    c = wl.box_random_coeffs(11, 2, 1)
    a = wl.uniform(11, "grid", 72 * 60).reshape(1, 72, 60)
    got = _gpu(a, c[None, None], 250, "f64")
    assert_close(got[0], oracle.periodic(a[0], c, 250), 1e-12)


def test_block_diagonal_fields_are_independent():
    import torch
    import paper_2105_06676_amd as sfft
    cs = [wl.box_random_coeffs(20 + i, 2, 1) for i in range(3)]
    c = np.zeros((3, 3, 3, 3))
    for i in range(3):
        c[i, i] = cs[i]
    a = wl.uniform(12, "grid", 3 * 64 * 64).reshape(3, 64, 64)
    got = _gpu(a, c, 640, "f64")
    for i in range(3):
        g = to_dev(a[i], "f64")
        sfft.periodic(g, cs[i], 640)
        torch.cuda.synchronize()
        assert_close(got[i], g.cpu().numpy(), 1e-12)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_leapfrog_wave_cosine_mode_full_size(dtype):
    # 2-D leapfrog a_{t+1} = 2 a_t - a_{t-1} + k Lap a_t on 2048^2: a cosine mode with
    # a_{-1} = cos(phi) a_0 evolves as cos(t phi) a_0, cos(phi) = 1 - 2k (sin^2(q0/2) + sin^2(q1/2))
    n, k, T = 2048, 0.2, 1500
    k0, k1 = 3, 5
    q0, q1 = 2 * np.pi * k0 / n, 2 * np.pi * k1 / n
    phi = np.arccos(1 - 2 * k * (np.sin(q0 / 2) ** 2 + np.sin(q1 / 2) ** 2))
    x = np.arange(n)
    mode = np.cos(q0 * x)[:, None] * np.cos(q1 * x)[None, :]
    c = np.zeros((2, 2, 3, 3))
    c[0, 0] = [[0, k, 0], [k, 2 - 4 * k, k], [0, k, 0]]
    c[0, 1, 1, 1] = -1.0
    c[1, 0, 1, 1] = 1.0
    a = np.stack([mode, np.cos(phi) * mode])
    got = _gpu(a, c, T, dtype)
    # The 2 x 2 step matrix of this mode has the eigenvalues exp(+-i phi), phi = 0.008:
    # nearly a double eigenvalue, so its T-th power has entries of order 1/sin(phi)
    # that cancel in the result; FP64 rounding then leaves about
    # T * eps / sin(phi) * log2(T) ~ 2e-10 (the reference's own arccos near 1 adds
    # ~1e-11).  FP32 passes keep their 1e-5 budget.
    tol = 1e-5 if dtype == "f32" else 2e-9
    assert_close(got[0], np.cos(T * phi) * mode, tol)
    assert_close(got[1], np.cos((T - 1) * phi) * mode, tol)


def test_affine_update_through_a_constant_field():
    S = wl.box_random_coeffs(13, 2, 1)
    S *= 0.9 / S.sum()
    c = np.zeros((2, 2, 3, 3))
    c[0, 0] = S
    c[0, 1, 1, 1] = 1.0
    c[1, 1, 1, 1] = 1.0
    a0 = wl.uniform(13, "grid", 80 * 70).reshape(80, 70)
    a = np.stack([a0, np.full_like(a0, 0.375)])
    got = _gpu(a, c, 123, "f64")
    assert_close(got, oracle.periodic_fields(a, c, 123), 1e-12)
    assert np.allclose(got[1], 0.375, rtol=0, atol=1e-13)


def test_T_zero_is_a_no_op():
    import torch
    import paper_2105_06676_amd as sfft
    g = to_dev(wl.uniform(14, "grid", 2 * 32 * 32).reshape(2, 32, 32), "f32")
    before = g.clone()
    sfft.periodic_fields(g, _system(14, 2, 2, 1), 0)
    torch.cuda.synchronize()
    assert torch.equal(g, before)


def test_fields_rejects_bad_arguments_without_touching_the_grid():
    import torch
    import paper_2105_06676_amd as sfft
    g = to_dev(np.ones((5, 16, 16)), "f64")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_fields(g, np.zeros((5, 5, 3, 3)), 3)
    assert e.value.code == -2
    g2 = to_dev(np.ones((2, 13, 16)), "f64")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_fields(g2, np.zeros((2, 2, 7, 7)), 3)  # radius 3
    assert e.value.code == -2
    g3 = to_dev(np.ones((2, 32768)), "f32")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_fields(g3, np.zeros((2, 2, 3)), 3)
    assert e.value.code == -2
    c = np.zeros((2, 2, 3, 3))
    c[1, 0, 0, 0] = np.nan
    g4 = to_dev(np.ones((2, 16, 16)), "f64")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_fields(g4, c, 3)
    assert e.value.code == -1
    torch.cuda.synchronize()
    for t in (g, g2, g3, g4):
        assert torch.equal(t, torch.ones_like(t))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_wave_workload_full_size_invariants(dtype):
    """The 4096^2 leapfrog workload: starting at rest, the zero mode's 2 x 2 matrix
    [[2, -1], [1, 0]] keeps the mean of both fields; the stencil is symmetric under
    swapping the axes, so a symmetric input stays symmetric; the scheme is stable."""
    import torch
    import paper_2105_06676_amd as sfft
    w = wl.config("wave2d_leapfrog_4096")
    a = w.grid()
    a = 0.5 * (a + a.transpose(0, 2, 1))
    g = to_dev(a, dtype)
    sfft.periodic_fields(g, w.coeffs, w.T)
    torch.cuda.synchronize()
    out = g.double()
    tol = 1e-5 if dtype == "f32" else 1e-12
    m0 = float(np.mean(a[0]))
    assert abs(float(out[0].mean()) - m0) <= tol * abs(m0)
    assert abs(float(out[1].mean()) - m0) <= tol * abs(m0)
    assert float((out[0] - out[0].T).norm() / out[0].norm()) <= tol
    assert bool(torch.isfinite(out).all()) and float(out.abs().max()) < 10.0
