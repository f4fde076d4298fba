"""Pins for the oracle: each test checks it against something other than itself.

Each pin is chosen so a plausible mistake (a wrong sign, a transposed offset, a
dropped term, an off-by-one in the frame) fails at least one of them:

* the paper's printed 4x4 stencil matrix (appendix "Stencil Matrix Example");
* exact matrix powers in Python integers (brute force on tiny grids);
* the affine augmented-matrix form of a fixed frame (appendix on vector-valued
  fields, affine example) in exact integers;
* closed forms: single Fourier modes, the binomial kernel of (1/4, 1/2, 1/4)^T,
  pure shifts, pointwise scaling, conservation;
* structural facts of Sec. 4: cells farther than sigma*T from the frame do not see
  it and match the periodic solve.
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle
import workloads
from conftest import golden_path


def _printed_matrix():
    rows = []
    with open(golden_path("stencil_matrix_4x4.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return rows


# ---------------------------------------------------------------------------

def test_printed_matrix_columns():
    """S e_j from the loop equals column j of the printed matrix (orientation pin)."""
    M = _printed_matrix()
    c = np.array([-2.0, 1.0, 3.0])
    for j in range(4):
        e = np.zeros(4)
        e[j] = 1.0
        col = oracle.periodic(e, c, 1)
        assert col.tolist() == [float(M[i][j]) for i in range(4)]


def _int_matmul(A, B):
    n, m, p = len(A), len(B), len(B[0])
    return [[sum(A[i][k] * B[k][j] for k in range(m)) for j in range(p)] for i in range(n)]


def test_printed_matrix_powers():
    """S^T x for T = 2, 3, 5 equals the integer matrix power of the printed matrix."""
    M = _printed_matrix()
    c = np.array([-2.0, 1.0, 3.0])
    x = [1, 2, 3, 4]
    for T in (2, 3, 5):
        P = [[int(i == j) for j in range(4)] for i in range(4)]
        for _ in range(T):
            P = _int_matmul(M, P)
        expect = [sum(P[i][j] * x[j] for j in range(4)) for i in range(4)]
        got = oracle.periodic(np.array(x, dtype=float), c, T)
        assert got.tolist() == [float(v) for v in expect]


def test_symbol_is_eigenvalues_of_printed_matrix():
    """Lambda = F s (appendix, eigenvalue-FFT relation) gives M v_k = Lambda_k v_k for
    the modes v_k[m] = exp(+2 pi i k m / 4) of the printed matrix, and the values
    are the eigenvalues a library eigen-solver finds for it."""
    M = np.array(_printed_matrix(), dtype=float)
    lam = oracle.symbol(np.array([-2.0, 1.0, 3.0]), [4])
    m = np.arange(4)
    for k in range(4):
        v = np.exp(2j * np.pi * k * m / 4)
        np.testing.assert_allclose(M @ v, lam[k] * v, atol=1e-12)
    ev = np.linalg.eigvals(M)
    for lk in lam:
        assert np.min(np.abs(ev - lk)) < 1e-9
    # a zero eigenvalue: everything in mode 2 is annihilated after one step
    assert abs(lam[2]) < 1e-15


# ---------------------------------------------------------------------------

def _dense_periodic(c_int, dims):
    """Dense integer matrix of one periodic step (weights scaled by the common denominator)."""
    d = len(dims)
    r = (len(c_int) - 1) // 2 if d == 1 else (np.asarray(c_int).shape[0] - 1) // 2
    N = int(np.prod(dims))
    A = [[0] * N for _ in range(N)]
    carr = np.asarray(c_int, dtype=object)
    for i in range(N):
        ii = np.unravel_index(i, dims)
        for idx in np.ndindex(*carr.shape):
            o = [k - r for k in idx]
            jj = tuple((a + b) % n for a, b, n in zip(ii, o, dims))
            j = int(np.ravel_multi_index(jj, dims))
            A[i][j] += int(carr[idx])
    return A


def _matvec(A, x):
    return [sum(a * b for a, b in zip(row, x)) for row in A]


@pytest.mark.parametrize("dims,T", [((7,), 9), ((5, 6), 6), ((3, 4, 2), 5), ((2,), 12), ((1, 5), 8)])
def test_exact_matrix_power_periodic(dims, T):
    """Dyadic weights and integer data keep every loop value exact in FP64, so the
    loop must equal the exact integer matrix power bit for bit (brute force)."""
    d = len(dims)
    rng = np.random.default_rng(7 + T)
    den = 8
    shape = (3,) * d
    c_int = rng.integers(-3, 4, size=shape)
    c_int.flat[0] = 2  # keep at least one asymmetric entry
    c = c_int.astype(float) / den
    x = rng.integers(-8, 9, size=dims)
    A = _dense_periodic(c_int, dims)
    v = [int(t) for t in x.ravel()]
    for _ in range(T):
        v = _matvec(A, v)
    expect = np.array([float(Fraction(t, den ** T)) for t in v]).reshape(dims)
    got = oracle.periodic(x.astype(float), c, T)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("dims,r,T", [((9,), 3, 6), ((13,), 4, 5), ((5,), 4, 4), ((8, 9), 3, 3), ((4, 3, 5), 3, 2),
                                     ((11,), 8, 3)])
def test_exact_matrix_power_periodic_wide_radius(dims, r, T):
    """The loop for radii above 2 (extents shorter than 2r + 1 alias offsets
    modulo the extent) against the exact integer matrix power."""
    d = len(dims)
    rng = np.random.default_rng(40 + r + T)
    den = 16
    c_int = rng.integers(-4, 5, size=(2 * r + 1,) * d)
    c_int.flat[0] = 3
    c = c_int.astype(float) / den
    x = rng.integers(-8, 9, size=dims)
    A = _dense_periodic(c_int, dims)
    v = [int(t) for t in x.ravel()]
    for _ in range(T):
        v = _matvec(A, v)
    expect = np.array([float(Fraction(t, den ** T)) for t in v]).reshape(dims)
    got = oracle.periodic(x.astype(float), c, T)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("dims,T", [((6,), 7), ((4, 5), 5), ((3, 3, 2), 4), ((2, 2), 9)])
def test_exact_affine_power_aperiodic(dims, T):
    """Fixed frame as an affine map: state (interior, 1) evolves by [[S_int, b], [0, 1]]
    (the affine-stencil construction of the appendix on vector-valued fields);
    its exact integer power must equal the aperiodic loop."""
    d = len(dims)
    r = 1
    rng = np.random.default_rng(11 + T)
    den = 8
    c_int = rng.integers(-3, 4, size=(3,) * d)
    c = c_int.astype(float) / den
    store = tuple(n + 2 * r for n in dims)
    full = rng.integers(-8, 9, size=store)
    interior_idx = [ii for ii in np.ndindex(*store) if all(r <= a < r + n for a, n in zip(ii, dims))]
    pos = {ii: k for k, ii in enumerate(interior_idx)}
    N = len(interior_idx)
    # scaled step: den * x_{t+1} = S_int x_t + b  (all integers)
    A = [[0] * (N + 1) for _ in range(N + 1)]
    for ii in interior_idx:
        i = pos[ii]
        for idx in np.ndindex(*c_int.shape):
            o = [k - r for k in idx]
            jj = tuple(a + b for a, b in zip(ii, o))
            w = int(c_int[idx])
            if jj in pos:
                A[i][pos[jj]] += w
            else:
                A[i][N] += w * int(full[jj])
    # homogeneous coordinate carries the scale: 1 -> den
    A[N][N] = den
    v = [int(full[ii]) for ii in interior_idx] + [1]
    for _ in range(T):
        v = _matvec(A, v)
    expect = full.astype(float)
    for ii in interior_idx:
        expect[ii] = float(Fraction(v[pos[ii]], den ** T))
    got = oracle.aperiodic(full.astype(float), c, T)
    assert np.array_equal(got, expect)


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,T", [(64, 3, 100), (50, 7, 37), (128, 1, 1000)])
def test_single_cosine_mode_heat(n, k, T):
    """cos mode k under (1/4, 1/2, 1/4) scales by (1/2 + 1/2 cos(2 pi k / n))^T."""
    m = np.arange(n)
    a0 = np.cos(2 * np.pi * k * m / n)
    lam = 0.5 + 0.5 * np.cos(2 * np.pi * k / n)
    got = oracle.periodic(a0, workloads.heat1d_coeffs(), T)
    np.testing.assert_allclose(got, lam ** T * a0, rtol=0, atol=4 * T * 2.2e-16)


def test_single_mode_asymmetric_2d():
    """An asymmetric 2-D stencil moves a mode by the phase of lambda:
    a_T = Re(lambda^T exp(2 pi i (k.m / n))), lambda = sum_o c_o exp(+2 pi i o.k / n)."""
    n0, n1, k0, k1, T = 12, 10, 2, 3, 9
    rng = np.random.default_rng(3)
    c = rng.random((3, 3))
    c /= c.sum()
    m0, m1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    phase = 2 * np.pi * (k0 * m0 / n0 + k1 * m1 / n1)
    lam = sum(c[o0 + 1, o1 + 1] * np.exp(2j * np.pi * (o0 * k0 / n0 + o1 * k1 / n1))
              for o0 in (-1, 0, 1) for o1 in (-1, 0, 1))
    got = oracle.periodic(np.cos(phase), c, T)
    np.testing.assert_allclose(got, np.real(lam ** T * np.exp(1j * phase)), atol=1e-13)


# ---------------------------------------------------------------------------

def test_conservation():
    c = workloads.box_random_coeffs(9, 2, 2)
    assert c.sum() == 1.0
    a0 = workloads.uniform(9, "grid", 30 * 20).reshape(30, 20)
    got = oracle.periodic(a0, c, 50)
    assert abs(got.sum() - a0.sum()) <= 1e-12 * abs(a0.sum())


@pytest.mark.slow
def test_binomial_closed_form_full_heat1d():
    """(1/4, 1/2, 1/4)^{*T} is Binomial(2T, 1/2): a_T[n] = sum_m C(2T, m) 4^-T a_0[(n + m - T) mod N],
    weights computed as exact integers over 4^T and rounded once (textbook identity)."""
    w = workloads.config("heat1d_65536")
    a0 = w.grid()
    T = w.T
    N = a0.shape[0]
    weights = [float(Fraction(comb(2 * T, m), 4 ** T)) for m in range(2 * T + 1)]
    expect = np.zeros(N)
    for m, wt in enumerate(weights):
        if wt == 0.0:
            continue
        expect += wt * np.roll(a0, -(m - T))
    got = oracle.periodic(a0, w.coeffs, T)
    err = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    assert err < 1e-13


@pytest.mark.parametrize("dims,shift_axis", [((17,), 0), ((6, 9), 1), ((4, 5, 6), 0)])
def test_pure_shift(dims, shift_axis):
    """c[+1 along one axis] = 1 gives a_T[n] = a_0[(n + T e) mod N] exactly."""
    d = len(dims)
    c = np.zeros((3,) * d)
    idx = [1] * d
    idx[shift_axis] = 2
    c[tuple(idx)] = 1.0
    a0 = workloads.uniform(5, "grid", int(np.prod(dims))).reshape(dims)
    T = 23
    got = oracle.periodic(a0, c, T)
    assert np.array_equal(got, np.roll(a0, -T, axis=shift_axis))


def test_translation_invariance():
    c = workloads.box_random_coeffs(12, 2, 1)
    a0 = workloads.uniform(12, "grid", 15 * 11).reshape(15, 11)
    T = 13
    base = oracle.periodic(a0, c, T)
    shifted = oracle.periodic(np.roll(a0, (4, -3), axis=(0, 1)), c, T)
    assert np.array_equal(shifted, np.roll(base, (4, -3), axis=(0, 1)))


def test_identity_and_one_step_and_pointwise():
    a0 = workloads.uniform(13, "grid", 40).reshape(5, 8)
    c = workloads.box_random_coeffs(13, 2, 1)
    assert np.array_equal(oracle.periodic(a0, c, 0), a0)
    one = oracle.periodic(a0, c, 1)
    hand = np.zeros_like(a0)
    for o0 in (-1, 0, 1):
        for o1 in (-1, 0, 1):
            hand += c[o0 + 1, o1 + 1] * np.roll(a0, (-o0, -o1), axis=(0, 1))
    np.testing.assert_allclose(one, hand, rtol=0, atol=1e-15)
    c0 = np.array([[0.75]])
    np.testing.assert_allclose(oracle.periodic(a0, c0, 7), 0.75 ** 7 * a0, rtol=1e-15)


def test_tiny_extent_aliasing():
    """Extents smaller than 2r+1 alias offsets modulo n, exactly as '% N' does."""
    c = np.array([0.1, 0.2, 0.3, 0.25, 0.15])  # r = 2
    a0 = np.array([1.0, -2.0])
    # n = 2: offsets -2, 0, +2 hit cell i, offsets -1, +1 hit the other cell
    same = c[0] + c[2] + c[4]
    other = c[1] + c[3]
    expect = np.array([same * 1.0 + other * -2.0, same * -2.0 + other * 1.0])
    np.testing.assert_allclose(oracle.periodic(a0, c, 1), expect, rtol=1e-15)


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,r,T", [((40,), 1, 9), ((30, 26), 1, 6), ((24, 20), 2, 3), ((14, 12, 16), 1, 3)])
def test_aperiodic_interior_matches_periodic(dims, r, T):
    """Cells farther than r*T from the frame never see it (Sec. 4, region of influence),
    so they equal the periodic solve of the interior grid bit for bit."""
    d = len(dims)
    c = workloads.box_random_coeffs(21, d, r)
    store = tuple(n + 2 * r for n in dims)
    a = workloads.uniform(21, "grid", int(np.prod(store))).reshape(store)
    ap = oracle.aperiodic(a, c, T)
    inner = tuple(slice(r, r + n) for n in dims)
    per = oracle.periodic(a[inner], c, T)
    mask = oracle.dist(dims) > r * T
    assert mask.any()
    assert np.array_equal(ap[inner][mask], per[mask])


def test_frame_unchanged_and_roi():
    """The frame is read-only; perturbing it changes only cells with dist <= r*T."""
    dims, r, T = (33, 29), 1, 7
    c = workloads.box_random_coeffs(22, 2, r)
    store = tuple(n + 2 * r for n in dims)
    a = workloads.uniform(22, "grid", int(np.prod(store))).reshape(store)
    b = a.copy()
    b[0, :] += 1.0
    b[:, -1] -= 0.5
    ra, rb = oracle.aperiodic(a, c, T), oracle.aperiodic(b, c, T)
    assert np.array_equal(ra[0, :], a[0, :]) and np.array_equal(ra[:, -1], a[:, -1])
    inner = tuple(slice(r, r + n) for n in dims)
    far = oracle.dist(dims) > r * T
    near = oracle.dist(dims) == 1
    assert np.array_equal(ra[inner][far], rb[inner][far])
    assert not np.array_equal(ra[inner][near], rb[inner][near])


def test_dist_brute_force():
    dims = (5, 7, 4)
    dd = oracle.dist(dims)
    for ii in np.ndindex(*dims):
        expect = 1 + min(min(i, n - 1 - i) for i, n in zip(ii, dims))
        assert dd[ii] == expect


# ---------------------------------------------------------------- symbol / power

def test_symbol_closed_forms():
    n = 48
    k = np.arange(n)
    np.testing.assert_allclose(oracle.symbol(workloads.heat1d_coeffs(), [n]),
                               0.5 + 0.5 * np.cos(2 * np.pi * k / n), atol=1e-15)
    n0, n1 = 12, 20
    k0, k1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    expect = 0.2 * (1 + 2 * np.cos(2 * np.pi * k0 / n0) + 2 * np.cos(2 * np.pi * k1 / n1))
    np.testing.assert_allclose(oracle.symbol(workloads.jacobi5_coeffs(), [n0, n1]), expect, atol=1e-15)


def test_symbol_power_exact_gaussian_integers():
    """(a + b i)^T for dyadic a, b is exact in 60 digits at these sizes: compare
    against exact Gaussian-integer powers."""
    vals = [(3, -1, 2), (1, 1, 1), (-5, 2, 3), (0, 0, 0)]
    for a, b, sh in vals:
        z = complex(a / 2 ** sh, b / 2 ** sh)
        for T in (0, 1, 2, 7, 13):
            re, im = 1, 0
            for _ in range(T):
                re, im = re * a - im * b, re * b + im * a
            ex = complex(float(Fraction(re, 2 ** (sh * T))), float(Fraction(im, 2 ** (sh * T))))
            got = oracle.symbol_power(np.array([z]), T)[0]
            assert got == ex


def test_symbol_power_unit_modulus_phase():
    phi = 0.731
    z = np.exp(1j * phi)
    T = 4096
    got = oracle.symbol_power(np.array([z]), T)[0]
    # |z| differs from 1 by at most an ulp; the phase must be T * arg(z)
    assert abs(np.angle(got) - np.angle(np.exp(1j * T * np.angle(z)))) < 1e-12
