"""Pins of the vector-valued-field oracle (``oracle.periodic_fields``) against
facts fixed independently of it: the scalar oracle on block-diagonal systems,
closed forms (Fibonacci, rotations, an affine update, a second-order-in-time
recurrence), and an exact rational matrix power on tiny grids.

The system is the vector-valued extension of the periodic problem (Sec. 3 and
the appendix on vector-valued fields): field i at t+1 is the sum over j of the
circulant stencil (i, j) applied to field j at t.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _blocks(m, d, r):
    return np.zeros((m, m) + (2 * r + 1,) * d)


def test_block_diagonal_is_independent_scalar_solves():
    rng = np.random.default_rng(1)
    dims, r, T = (9, 7), 1, 13
    c = _blocks(3, 2, r)
    for i in range(3):
        c[i, i] = rng.random((3, 3)) / 9.0
    a = rng.random((3,) + dims)
    got = oracle.periodic_fields(a, c, T)
    for i in range(3):
        assert np.array_equal(got[i], oracle.periodic(a[i], c[i, i], T))


def test_fibonacci_pointwise_pair():
    # a0' = a0 + a1, a1' = a0 (r = 0): a0_T = F(T+1) a0 + F(T) a1, exact in FP64 for T <= 70
    c = _blocks(2, 1, 0)
    c[0, 0, 0] = c[0, 1, 0] = c[1, 0, 0] = 1.0
    a = np.array([[3.0, -2.0, 5.0], [1.0, 4.0, 0.0]])
    fib = [0, 1]
    for _ in range(80):
        fib.append(fib[-1] + fib[-2])
    for T in (0, 1, 2, 10, 70):
        got = oracle.periodic_fields(a, c, T)
        want0 = fib[T + 1] * a[0] + fib[T] * a[1]
        want1 = fib[T] * a[0] + fib[T - 1 if T else 1] * a[1] if T else a[1]
        assert np.array_equal(got[0], want0), T
        assert np.array_equal(got[1], want1), T


def test_pointwise_rotation():
    th = 0.3
    c = _blocks(2, 2, 0)
    c[0, 0, 0, 0], c[0, 1, 0, 0] = np.cos(th), -np.sin(th)
    c[1, 0, 0, 0], c[1, 1, 0, 0] = np.sin(th), np.cos(th)
    rng = np.random.default_rng(2)
    a = rng.random((2, 4, 3))
    T = 57
    got = oracle.periodic_fields(a, c, T)
    ct, st = np.cos(T * th), np.sin(T * th)
    assert np.allclose(got[0], ct * a[0] - st * a[1], rtol=0, atol=1e-12)
    assert np.allclose(got[1], st * a[0] + ct * a[1], rtol=0, atol=1e-12)


def test_affine_update_through_a_constant_field():
    # a' = S a + b with b held in a second field (S^(0,1) = I, S^(1,1) = I, S^(1,0) = 0):
    # a_T = S^T a_0 + b * (1 - s^T) / (1 - s) where s is the coefficient sum of S.
    rng = np.random.default_rng(3)
    dims, r, T = (8, 6), 1, 21
    S = rng.random((3, 3))
    S *= 0.75 / S.sum()
    s = S.sum()
    b = 0.625
    c = _blocks(2, 2, r)
    c[0, 0] = S
    c[0, 1, 1, 1] = 1.0
    c[1, 1, 1, 1] = 1.0
    a0 = rng.random(dims)
    got = oracle.periodic_fields(np.stack([a0, np.full(dims, b)]), c, T)
    want = oracle.periodic(a0, S, T) + b * (1 - s ** T) / (1 - s)
    assert np.allclose(got[0], want, rtol=0, atol=1e-13)
    assert np.array_equal(got[1], np.full(dims, b))


def test_second_order_in_time_wave_recurrence():
    # leapfrog a_{t+1} = 2 a_t - a_{t-1} + k (a_t[x+1] - 2 a_t[x] + a_t[x-1]) as fields (a_t, a_{t-1});
    # a cosine mode with a_{-1} = cos(phi) a_0 evolves as cos(t phi) a_0, cos phi = 1 - 2k sin^2(q/2)
    n, kq, k = 32, 3, 0.4
    q = 2 * np.pi * kq / n
    x = np.arange(n)
    phi = np.arccos(1 - 2 * k * np.sin(q / 2) ** 2)
    c = _blocks(2, 1, 1)
    c[0, 0] = [k, 2 - 2 * k, k]
    c[0, 1, 1] = -1.0
    c[1, 0, 1] = 1.0
    a = np.stack([np.cos(q * x), np.cos(phi) * np.cos(q * x)])
    for T in (1, 7, 100):
        got = oracle.periodic_fields(a, c, T)
        assert np.allclose(got[0], np.cos(T * phi) * np.cos(q * x), rtol=0, atol=1e-12), T
        assert np.allclose(got[1], np.cos((T - 1) * phi) * np.cos(q * x), rtol=0, atol=1e-12), T


@pytest.mark.parametrize("dims,m,r,T", [((5,), 2, 1, 6), ((4, 3), 3, 1, 4), ((3, 2, 2), 2, 1, 3), ((6,), 3, 2, 5)])
def test_exact_rational_matrix_power(dims, m, r, T):
    # build the (m N) x (m N) update matrix from its definition and apply it T times
    # in exact rationals; small integer coefficients and data keep FP64 exact
    rng = np.random.default_rng(4 + m + r)
    d = len(dims)
    c = rng.integers(-2, 3, size=(m, m) + (2 * r + 1,) * d).astype(np.float64)
    a = rng.integers(-3, 4, size=(m,) + dims).astype(np.float64)
    N = int(np.prod(dims))
    cells = list(np.ndindex(*dims))
    index = {cell: k for k, cell in enumerate(cells)}
    M = [[Fraction(0)] * (m * N) for _ in range(m * N)]
    for i in range(m):
        for j in range(m):
            for cell in cells:
                for off in np.ndindex(*(2 * r + 1,) * d):
                    o = [t - r for t in off]
                    nb = tuple((x + oo) % n for x, oo, n in zip(cell, o, dims))
                    M[i * N + index[cell]][j * N + index[nb]] += Fraction(int(c[(i, j) + off]))
    v = [Fraction(int(x)) for x in a.reshape(-1)]
    for _ in range(T):
        v = [sum(M[p][q] * v[q] for q in range(m * N) if M[p][q]) for p in range(m * N)]
    want = np.array([float(x) for x in v]).reshape(a.shape)
    assert np.array_equal(oracle.periodic_fields(a, c, T), want)
