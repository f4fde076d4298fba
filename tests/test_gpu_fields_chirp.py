"""Coupled fields and implicit stencils on extents with a prime factor above 7
(chirp-z transforms on those axes, the symbol-matrix power over the full
spectrum), against the FP64 oracle: the coupled periodic loop and the
pseudo-inverse implicit solve."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, rounded_input, to_dev

pytestmark = pytest.mark.gpu


def _system(seed, m, d, r, sym=False):
    """Blocks c_ij = R_ij * S_ij (R orthogonal, S_ij positive stencils of sum 1):
    the zero mode rotates without decay, every block keeps its own stencil."""
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


FIELD_CASES = [
    ((211,), 2, 1, 40), ((97,), 3, 2, 25), ((1009,), 2, 1, 300),
    ((37, 64), 2, 1, 60), ((48, 41), 3, 1, 33), ((53, 59), 2, 2, 20), ((11, 13), 4, 1, 17),
    ((13, 8, 11), 2, 1, 15), ((7, 17, 10), 3, 1, 9),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("dims,m,r,T", FIELD_CASES)
def test_fields_on_prime_extents_match_oracle(dims, m, r, T, sym, dtype):
    import torch
    import paper_2105_06676_amd as sfft
    d = len(dims)
    c = _system(40 + m + r + d, m, d, r, sym)
    a = wl.uniform(41 + sum(dims) + m, "grid", m * int(np.prod(dims))).reshape((m,) + dims)
    g = to_dev(a, dtype)
    sfft.periodic_fields(g, c, T)
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64)
    want = oracle.periodic_fields(rounded_input(a, dtype), c, T)
    assert_close(got, want, TOL[dtype], (dims, m, r, T, sym))


def _ident(d, r=1):
    c = np.zeros((2 * r + 1,) * d)
    c[(r,) * d] = 1.0
    return c


def _lap(d, k, r=1):
    c = np.zeros((2 * r + 1,) * d)
    for ax in range(d):
        for s in (-1, 1):
            idx = [r] * d
            idx[ax] += s
            c[tuple(idx)] = k
    c[(r,) * d] = -2 * d * k
    return c


IMPLICIT_CASES = [
    ("backward_euler_1d_prime", (101,), lambda: (_ident(1) - _lap(1, 0.8), _ident(1)), 50),
    ("crank_nicolson_2d_prime", (47, 40), lambda: (_ident(2) - _lap(2, 0.6), _ident(2) + _lap(2, 0.6)), 30),
    ("random_2d_prime", (31, 43), lambda: (2.0 * _ident(2) - wl.box_random_coeffs(5, 2, 1),
                                           wl.box_random_coeffs(6, 2, 1)), 25),
    ("backward_euler_3d_prime", (11, 10, 13), lambda: (_ident(3) - _lap(3, 0.5), _ident(3)), 20),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,dims,make,T", IMPLICIT_CASES, ids=[c[0] for c in IMPLICIT_CASES])
def test_implicit_on_prime_extents_matches_oracle(name, dims, make, T, dtype):
    import torch
    import paper_2105_06676_amd as sfft
    q, s = make()
    a = wl.uniform(50 + len(dims), "grid", int(np.prod(dims))).reshape(dims)
    g = to_dev(a, dtype)
    sfft.periodic_implicit(g, q, s, T)
    torch.cuda.synchronize()
    want = oracle.implicit_periodic(rounded_input(a, dtype), q, s, T)
    assert_close(g.cpu().numpy().astype(np.float64), want, TOL[dtype], name)


def test_singular_q_on_a_prime_torus_uses_the_pseudo_inverse():
    import torch
    import paper_2105_06676_amd as sfft
    dims = (29, 12)
    q, s = _lap(2, 1.0), _ident(2)
    a = wl.uniform(57, "grid", int(np.prod(dims))).reshape(dims)
    T = 3
    g = to_dev(a, "f64")
    sfft.periodic_implicit(g, q, s, T)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    want = oracle.implicit_periodic(a, q, s, T)
    lam_min = 4 * min(np.sin(np.pi / n) ** 2 for n in dims)
    tol = 10 * T * np.finfo(float).eps * np.abs(q).sum() / lam_min
    assert_close(got, want, tol)
    assert abs(got.mean()) <= 1e-12 * np.abs(got).max()


def test_fields_on_prime_extents_with_one_field_equal_the_scalar_solve():
    """m = 1 through the fields pipeline and the scalar chirp-z solve agree to rounding."""
    import torch
    import paper_2105_06676_amd as sfft
    dims = (61, 36)
    c = wl.box_random_coeffs(58, 2, 1)
    a = wl.uniform(58, "grid", int(np.prod(dims))).reshape(dims)
    g1 = to_dev(a[None], "f64")
    sfft.periodic_fields(g1, c[None, None], 77)
    g2 = to_dev(a, "f64")
    sfft.periodic(g2, c, 77)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g1[0].cpu().numpy(), g2.cpu().numpy(), rtol=0, atol=1e-13)
