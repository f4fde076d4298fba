"""Pins of the implicit-stencil oracle (``oracle.implicit_periodic``): the update
``Q a_{t+1} = S a_t`` of the appendix on implicit stencils, solved with the
pseudo-inverse of the circulant Q.  Checked against the explicit loop oracle
(Q = I), the defining residual (applying Q and S with the explicit loop), closed
forms for single Fourier modes (backward Euler, Crank-Nicolson), the projection
property of a singular Q, and conservation."""
import numpy as np

import oracle


def _lap1(k):
    return np.array([k, -2 * k, k])


def _lap2(k):
    c = np.zeros((3, 3))
    c[0, 1] = c[2, 1] = c[1, 0] = c[1, 2] = k
    c[1, 1] = -4 * k
    return c


def _ident(d):
    c = np.zeros((3,) * d)
    c[(1,) * d] = 1.0
    return c


def test_identity_q_is_the_explicit_stencil():
    rng = np.random.default_rng(1)
    s = rng.random((3, 3))
    s /= s.sum()
    a = rng.random((12, 10))
    assert np.allclose(oracle.implicit_periodic(a, _ident(2), s, 9), oracle.periodic(a, s, 9), rtol=0, atol=1e-14)


def test_each_step_satisfies_the_implicit_equation():
    rng = np.random.default_rng(2)
    q = _ident(2) - _lap2(0.3)
    q[0, 0] = 0.05  # not symmetric: a general invertible Q
    s = rng.random((3, 3))
    s /= s.sum()
    a0 = rng.random((16, 14))
    a1 = oracle.implicit_periodic(a0, q, s, 1)
    assert np.allclose(oracle.periodic(a1, q, 1), oracle.periodic(a0, s, 1), rtol=0, atol=1e-13)


def test_backward_euler_cosine_mode():
    n, kq, kappa, T = 40, 3, 0.7, 25
    th = 2 * np.pi * kq / n
    x = np.arange(n)
    a = np.cos(th * x)
    got = oracle.implicit_periodic(a, _ident(1) - _lap1(kappa), _ident(1), T)
    factor = 1.0 / (1.0 + 4 * kappa * np.sin(th / 2) ** 2)
    assert np.allclose(got, factor ** T * a, rtol=0, atol=1e-13)


def test_crank_nicolson_2d_mode():
    n0, n1, k0, k1, kappa, T = 16, 12, 2, 5, 0.9, 17
    t0, t1 = 2 * np.pi * k0 / n0, 2 * np.pi * k1 / n1
    mode = np.cos(t0 * np.arange(n0))[:, None] * np.sin(t1 * np.arange(n1))[None, :]
    lam_lap = -4 * (np.sin(t0 / 2) ** 2 + np.sin(t1 / 2) ** 2)
    q = _ident(2) - _lap2(kappa / 2)
    s = _ident(2) + _lap2(kappa / 2)
    got = oracle.implicit_periodic(mode, q, s, T)
    factor = (1 + kappa / 2 * lam_lap) / (1 - kappa / 2 * lam_lap)
    assert np.allclose(got, factor ** T * mode, rtol=0, atol=1e-13)


def test_singular_q_projects_out_its_null_space():
    # Q = 1-D Laplacian annihilates constants: Q^+ returns the zero-mean part's
    # preimage, so the result has zero mean and Q a_1 = a_0 - mean(a_0)
    rng = np.random.default_rng(3)
    a0 = rng.random(24)
    a1 = oracle.implicit_periodic(a0, _lap1(1.0), _ident(1), 1)
    assert abs(a1.mean()) < 1e-13
    assert np.allclose(oracle.periodic(a1, _lap1(1.0), 1), a0 - a0.mean(), rtol=0, atol=1e-12)


def test_backward_euler_conserves_the_sum():
    rng = np.random.default_rng(4)
    a = rng.random((3, 5, 7))
    q = _ident(3)
    q[1, 1, 1] += 0.6
    for off in ((0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)):
        q[off] -= 0.1
    got = oracle.implicit_periodic(a, q, _ident(3), 11)
    assert abs(got.sum() - a.sum()) < 1e-12
