"""Implicit stencils on the GPU (Q a_{t+1} = S a_t) against the oracle's
pseudo-inverse solve, plus full-size properties.  Tolerances as for the scalar
path (relative L2 against the FP64 oracle)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rel_l2, rounded_input, to_dev

pytestmark = pytest.mark.gpu


def _ident(d, r=1):
    c = np.zeros((2 * r + 1,) * d)
    c[(r,) * d] = 1.0
    return c


def _lap(d, k, r=1):
    c = np.zeros((2 * r + 1,) * d)
    for a in range(d):
        for s in (-1, 1):
            idx = [r] * d
            idx[a] += s
            c[tuple(idx)] = k
    c[(r,) * d] = -2 * d * k
    return c


def _gpu(a, q, s, T, dtype):
    import torch
    import paper_2105_06676_amd as sfft
    g = to_dev(a, dtype)
    sfft.periodic_implicit(g, q, s, T)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


def _random_q(seed, d, r):
    """Diagonally dominant, not symmetric: 2 I minus a random stencil of sum 1."""
    return 2.0 * _ident(d, r) - wl.box_random_coeffs(seed, d, r)


CASES = [
    ("backward_euler_1d", (96,), lambda: (_ident(1) - _lap(1, 0.8), _ident(1)), 50),
    ("crank_nicolson_2d", (48, 40), lambda: (_ident(2) - _lap(2, 0.6), _ident(2) + _lap(2, 0.6)), 30),
    ("random_2d", (30, 42), lambda: (_random_q(5, 2, 1), wl.box_random_coeffs(6, 2, 1)), 25),
    ("random_2d_r2", (36, 20), lambda: (_random_q(7, 2, 2), wl.box_random_coeffs(8, 2, 2)), 12),
    ("backward_euler_3d", (12, 10, 8), lambda: (_ident(3) - _lap(3, 0.5), _ident(3)), 20),
    ("random_1d_r2", (120,), lambda: (_random_q(9, 1, 2), wl.box_random_coeffs(10, 1, 2)), 40),
    ("power_of_two_2d", (64, 64), lambda: (_ident(2) - _lap(2, 1.5), _ident(2)), 200),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,dims,make,T", CASES, ids=[c[0] for c in CASES])
def test_implicit_matches_oracle(name, dims, make, T, dtype):
    q, s = make()
    a = wl.uniform(30 + len(dims), "grid", int(np.prod(dims))).reshape(dims)
    got = _gpu(a, q, s, T, dtype)
    want = oracle.implicit_periodic(rounded_input(a, dtype), q, s, T)
    assert_close(got, want, TOL[dtype])


@pytest.mark.parametrize("dims", [(64,), (16, 12)])
def test_singular_q_uses_the_pseudo_inverse(dims):
    # Q = Laplacian annihilates the constant mode: that mode is dropped, the rest inverted
    d = len(dims)
    q, s = _lap(d, 1.0), _ident(d)
    a = wl.uniform(31, "grid", int(np.prod(dims))).reshape(dims)
    T = 3
    got = _gpu(a, q, s, T, "f64")
    want = oracle.implicit_periodic(a, q, s, T)
    # Q^+ amplifies the lowest nonzero mode by 1 / lambda_min (about 100 here) per
    # step; the symbol of that mode carries an absolute error of a few eps * sum|q|,
    # so both sides agree to about T * eps * sum|q| / lambda_min relative.
    lam_min = 4 * min(np.sin(np.pi / n) ** 2 for n in dims)
    tol = 10 * T * np.finfo(float).eps * np.abs(q).sum() / lam_min
    assert_close(got, want, tol)
    assert abs(got.mean()) <= 1e-12 * np.abs(got).max()


def test_identity_q_is_the_explicit_stencil():
    import torch
    import paper_2105_06676_amd as sfft
    s = wl.box_random_coeffs(12, 2, 1)
    a = wl.uniform(32, "grid", 56 * 48).reshape(56, 48)
    got = _gpu(a, _ident(2), s, 333, "f64")
    g = to_dev(a, "f64")
    sfft.periodic(g, s, 333)
    torch.cuda.synchronize()
    assert_close(got, g.cpu().numpy(), 1e-12)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_backward_euler_full_size_properties(dtype):
    """4096^2 backward-Euler heat (kappa = 2, T = 1000): the sum is conserved
    (lambda_R(0) = 1), an axis-symmetric input stays symmetric, values stay within
    the initial range (the update is a positive averaging)."""
    import torch
    import paper_2105_06676_amd as sfft
    n = 4096
    a = wl.uniform(33, "grid", n * n).reshape(n, n)
    a = 0.5 * (a + a.T)
    g = to_dev(a, dtype)
    sfft.periodic_implicit(g, _ident(2) - _lap(2, 2.0), _ident(2), 1000)
    torch.cuda.synchronize()
    out = g.double()
    tol = 1e-5 if dtype == "f32" else 1e-12
    assert abs(float(out.sum()) - float(a.sum())) <= tol * float(a.sum())
    assert float((out - out.T).norm() / out.norm()) <= tol
    assert float(out.min()) >= a.min() - tol and float(out.max()) <= a.max() + tol


def test_implicit_rejects_bad_arguments():
    import torch
    import paper_2105_06676_amd as sfft
    g = to_dev(np.ones((13, 16)), "f64")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_implicit(g, _ident(2, 3), _ident(2, 3), 3)  # radius 3
    assert e.value.code == -2
    with pytest.raises(ValueError):
        sfft.periodic_implicit(to_dev(np.ones((16, 16)), "f64"), _ident(2, 2), _ident(2, 1), 3)
    q = _ident(2)
    q[0, 0] = np.inf
    g2 = to_dev(np.ones((16, 16)), "f64")
    with pytest.raises(sfft.SfftError) as e:
        sfft.periodic_implicit(g2, q, _ident(2), 3)
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert torch.equal(g, torch.ones_like(g)) and torch.equal(g2, torch.ones_like(g2))
