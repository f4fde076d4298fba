"""Pins of the oracle's reflecting (zero-flux, Neumann) boundary, Sec. 4.

The oracle refills the frame before every step with the mirror image of the
interior about the cell faces.  These tests check it against what the
mathematics fixes, none of them by retyping the oracle's mirror rule:

* closed form: the half-sample cosines cos(pi k (i + 1/2) / n) are eigenvectors
  of every stencil that is symmetric along each axis under this boundary (the
  DCT-II basis), with eigenvalue sum_o c[o] prod_a cos(pi k_a o_a / n_a);
* a library routine: for such stencils T steps equal scipy's orthonormal DCT-II,
  multiplication by the eigenvalues to the power T, and the inverse DCT-II;
* another library route for any stencil: numpy's ``pad(mode="symmetric")``
  followed by scipy's ``correlate(mode="valid")``, exact on integers;
* invariants: a constant field scales by sum(c)^T for any stencil, and the
  interior sum is conserved by symmetric stencils whose coefficients sum to 1.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.signal

import oracle


def _framed(interior, r, fill=0.0):
    """Interior array placed inside an r-wide frame of `fill`."""
    return np.pad(np.asarray(interior, dtype=np.float64), r, mode="constant", constant_values=fill)


def _inner(a, r):
    return a[tuple(slice(r, s - r) for s in a.shape)]


def _sym_stencil(rng, d, r):
    """Coefficients symmetric along every axis: c[o] = c[o'] whenever |o| = |o'|."""
    shape = (2 * r + 1,) * d
    base = rng.uniform(0.1, 1.0, size=(r + 1,) * d)
    c = np.zeros(shape)
    for idx in np.ndindex(*shape):
        c[idx] = base[tuple(abs(i - r) for i in idx)]
    return c


def _eigen(c, dims, ks):
    r = (c.shape[0] - 1) // 2
    lam = 0.0
    for idx in np.ndindex(*c.shape):
        o = [i - r for i in idx]
        lam += c[idx] * np.prod([np.cos(np.pi * k * oa / n) for k, oa, n in zip(ks, o, dims)])
    return lam


@pytest.mark.parametrize("dims,r,ks", [((12,), 1, (3,)), ((15,), 2, (7,)), ((9, 10), 1, (2, 5)),
                                        ((7, 6), 2, (4, 1)), ((5, 6, 4), 1, (1, 2, 3))])
def test_reflect_half_sample_cosine_is_eigenvector(dims, r, ks):
    rng = np.random.default_rng(11)
    c = _sym_stencil(rng, len(dims), r)
    c /= c.sum()
    mode = np.ones(dims)
    for ax, (k, n) in enumerate(zip(ks, dims)):
        shape = [1] * len(dims)
        shape[ax] = n
        mode = mode * np.cos(np.pi * k * (np.arange(n) + 0.5) / n).reshape(shape)
    T = 9
    out = _inner(oracle.aperiodic(_framed(mode, r, fill=123.0), c, T, bc="reflect"), r)
    lam = _eigen(c, dims, ks)
    np.testing.assert_allclose(out, lam ** T * mode, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims,r", [((40,), 1), ((33,), 3), ((11, 13), 2), ((6, 7, 8), 1)])
def test_reflect_equals_dct_ii_evolution(dims, r):
    rng = np.random.default_rng(5)
    c = _sym_stencil(rng, len(dims), r)
    c /= c.sum() * 1.02
    a0 = rng.standard_normal(dims)
    T = 13
    out = _inner(oracle.aperiodic(_framed(a0, r), c, T, bc="reflect"), r)
    grids = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    lam = np.zeros(dims)
    for idx in np.ndindex(*c.shape):
        o = [i - r for i in idx]
        term = np.ones(dims)
        for g, oa, n in zip(grids, o, dims):
            term = term * np.cos(np.pi * g * oa / n)
        lam += c[idx] * term
    ref = scipy.fft.idctn(lam ** T * scipy.fft.dctn(a0, type=2, norm="ortho"), type=2, norm="ortho")
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dims,r", [((9,), 1), ((8,), 2), ((5, 6), 1), ((4, 5), 2), ((3, 4, 5), 1)])
def test_reflect_exact_integers_against_symmetric_pad(dims, r):
    """Any stencil (asymmetric here): each step is numpy's symmetric pad of the
    interior followed by scipy's valid-mode correlation; integers keep both exact."""
    rng = np.random.default_rng(sum(dims) + r)
    c = rng.integers(-2, 3, size=(2 * r + 1,) * len(dims)).astype(np.float64)
    a0 = rng.integers(-3, 4, size=dims).astype(np.float64)
    T = 4
    out = _inner(oracle.aperiodic(_framed(a0, r, fill=-77.0), c, T, bc="reflect"), r)
    x = a0.copy()
    for _ in range(T):
        x = scipy.signal.correlate(np.pad(x, r, mode="symmetric"), c, mode="valid", method="direct")
    assert np.abs(x).max() < 2 ** 52
    np.testing.assert_array_equal(out, x)


@pytest.mark.parametrize("dims,r", [((17,), 2), ((6, 9), 1), ((4, 5, 3), 2)])
def test_reflect_constant_field_scales_by_coefficient_sum(dims, r):
    rng = np.random.default_rng(2)
    c = rng.uniform(-0.3, 0.6, size=(2 * r + 1,) * len(dims))
    T = 6
    out = _inner(oracle.aperiodic(_framed(np.full(dims, 2.5), r, fill=9.0), c, T, bc="reflect"), r)
    np.testing.assert_allclose(out, 2.5 * c.sum() ** T, rtol=1e-13, atol=0)


def test_reflect_conserves_sum_for_symmetric_stencil():
    rng = np.random.default_rng(8)
    c = _sym_stencil(rng, 2, 2)
    c /= c.sum()
    a0 = rng.uniform(0, 1, size=(14, 9))
    out = _inner(oracle.aperiodic(_framed(a0, 2), c, 50, bc="reflect"), 2)
    assert abs(out.sum() - a0.sum()) < 1e-12 * a0.size


def test_reflect_returned_frame_mirrors_interior_and_fixed_is_unchanged():
    rng = np.random.default_rng(4)
    c = rng.uniform(0, 0.2, size=(3, 3))
    a = _framed(rng.standard_normal((5, 4)), 1, fill=3.0)
    out = oracle.aperiodic(a, c, 3, bc="reflect")
    np.testing.assert_array_equal(out, np.pad(_inner(out, 1), 1, mode="symmetric"))
    fixed = oracle.aperiodic(a, c, 3)
    np.testing.assert_array_equal(fixed[0], a[0])
    np.testing.assert_array_equal(fixed[:, -1], a[:, -1])


def test_reflect_rejects_interior_narrower_than_radius_and_unknown_bc():
    c = np.ones((5,)) / 5
    with pytest.raises(ValueError):
        oracle.aperiodic(np.zeros(1 + 4), c, 1, bc="reflect")
    with pytest.raises(ValueError):
        oracle.aperiodic(np.zeros(9), c, 1, bc="periodic")
    # T = 0 returns the interior unchanged
    a = np.arange(9.0)
    np.testing.assert_array_equal(_inner(oracle.aperiodic(a, c, 0, bc="reflect"), 2), a[2:-2])
