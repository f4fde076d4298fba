"""Oracle for the FFT stencil solver: plain, slow, obviously correct CPU code.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_2105_06676_amd``) never imports it and shares no code with it.

Contents
--------
``periodic(a, coeffs, T)``
    T sweeps of the periodic nested loop in FP64 (C, ``loops.c``): the plain
    definition ``a_T = S^T a_0`` of the paper's periodic problem (Sec. 3, the
    periodic looping algorithm; d-D form in the appendix on d-D grids).
``aperiodic(a, coeffs, T, bc="fixed")``
    The aperiodic nested loop with a fixed r-wide frame (Sec. 2 aperiodic looping
    algorithm; Sec. 4 for what StencilFFT-A must reproduce).  ``bc="reflect"``:
    the zero-flux (Neumann) boundary Sec. 4 names among the base case's options,
    the frame refilled before every step with the mirror image of the interior.
``periodic_fields(a, coeffs, T)``
    T sweeps of the periodic loop for m coupled scalar fields (the vector-valued
    extension of Sec. 3 and its appendix): field i at t+1 is the sum over j of
    stencil (i, j) applied to field j at t.
``implicit_periodic(a, q, s, T)``
    Implicit stencils (appendix on implicit stencils): each step solves
    ``Q a_{t+1} = S a_t`` with the Moore-Penrose pseudo-inverse of the circulant
    matrix Q, ``a_{t+1} = Q^+ S a_t`` (the minimum-norm least-squares solution;
    for circulant Q this is the paper's inverse-or-zero rule per eigenvalue).  The
    matrices are built from their definition; ``S a`` is one sweep of the loop, the
    solve is a sparse LU when Q is nonsingular and a dense pseudo-inverse (SVD)
    otherwise.
``symbol(coeffs, dims)``
    Step 1(i) of the periodic algorithm written literally: build the first column
    ``s`` of the circulant matrix and take its N-point DFT (appendix, eigenvalue-FFT
    relation).  numpy's FFT serves as the DFT primitive.
``symbol_power(lam, T)``
    Step 2: ``lam**T`` by binary repeated squaring (Sec. 3, repeated squaring),
    carried out in 60-digit decimal arithmetic so that the FP64 GPU value can be
    judged against a reference far more accurate than itself.
``dist(shape_interior)``
    Distance of every interior cell to the fixed frame, 1 + min over faces
    (Sec. 4's region-of-influence notation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from decimal import Decimal, getcontext
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "loops.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``loops.c`` into ``liboracle.so`` (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_periodic", "oracle_aperiodic"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int]
        lib.oracle_periodic_fields.restype = ctypes.c_int
        lib.oracle_periodic_fields.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_int64, ctypes.c_int]
        lib.oracle_aperiodic_bc.restype = ctypes.c_int
        lib.oracle_aperiodic_bc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                            ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def _check_coeffs(coeffs: np.ndarray, ndim: int) -> int:
    c = np.asarray(coeffs)
    if c.ndim != ndim or len(set(c.shape)) != 1 or c.shape[0] % 2 != 1:
        raise ValueError(f"coefficients must be (2r+1,)*{ndim}, got {c.shape}")
    return (c.shape[0] - 1) // 2


def periodic(a: np.ndarray, coeffs: np.ndarray, T: int, nthreads: int = 0) -> np.ndarray:
    """``a_T`` after T periodic sweeps; input is widened to float64 (exact for float32)."""
    x = np.ascontiguousarray(a, dtype=np.float64).copy()
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    r = _check_coeffs(c, x.ndim)
    dims = (ctypes.c_int64 * x.ndim)(*x.shape)
    rc = _load().oracle_periodic(x.ctypes.data, x.ndim, dims, c.ctypes.data, r, int(T), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_periodic failed ({rc})")
    return x


def periodic_fields(a: np.ndarray, coeffs: np.ndarray, T: int, nthreads: int = 0) -> np.ndarray:
    """m coupled fields: ``a`` has shape (m, *dims), ``coeffs`` (m, m, *(2r+1,)*d);
    block ``coeffs[i, j]`` is the stencil from field j at t to field i at t+1."""
    x = np.ascontiguousarray(a, dtype=np.float64).copy()
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    m, d = x.shape[0], x.ndim - 1
    if c.ndim != d + 2 or c.shape[0] != m or c.shape[1] != m:
        raise ValueError(f"coefficients must be ({m}, {m}) + (2r+1,)*{d}, got {c.shape}")
    r = _check_coeffs(c[0, 0], d)
    dims = (ctypes.c_int64 * d)(*x.shape[1:])
    rc = _load().oracle_periodic_fields(x.ctypes.data, m, d, dims, c.ctypes.data, r, int(T), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_periodic_fields failed ({rc})")
    return x


def stencil_matrix(coeffs: np.ndarray, dims: Sequence[int]):
    """The N x N periodic stencil matrix (scipy CSR): row i holds c[o] at column
    (i + o) mod n (the periodic loop's neighbour convention), duplicates summed."""
    import scipy.sparse as sp
    c = np.asarray(coeffs, dtype=np.float64)
    d = len(dims)
    r = (c.shape[0] - 1) // 2
    N = int(np.prod(dims))
    cells = np.arange(N)
    coords = np.unravel_index(cells, tuple(dims))
    rows, cols, vals = [], [], []
    for off in np.ndindex(*c.shape):
        w = c[off]
        if w == 0.0:
            continue
        nb = tuple((coords[a] + (off[a] - r)) % dims[a] for a in range(d))
        rows.append(cells)
        cols.append(np.ravel_multi_index(nb, tuple(dims)))
        vals.append(np.full(N, w))
    if not rows:
        return sp.csr_matrix((N, N))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def implicit_periodic(a: np.ndarray, q: np.ndarray, s: np.ndarray, T: int, rcond: float = 1e-13) -> np.ndarray:
    """``a_T`` of ``Q a_{t+1} = S a_t`` on a periodic grid: ``a_{t+1} = Q^+ (S a_t)``.
    ``rcond``: singular values below rcond * (largest) count as zero when Q is singular."""
    import scipy.sparse.linalg as spla
    x = np.ascontiguousarray(a, dtype=np.float64).copy()
    qq = np.ascontiguousarray(q, dtype=np.float64)
    ss = np.ascontiguousarray(s, dtype=np.float64)
    _check_coeffs(qq, x.ndim)
    _check_coeffs(ss, x.ndim)
    dims = x.shape
    Q = stencil_matrix(qq, dims).tocsc()
    solve = None
    try:
        lu = spla.splu(Q)
        # a usable factorisation: no (near-)zero pivot
        piv = np.abs(lu.U.diagonal())
        if piv.min() > rcond * max(piv.max(), 1e-300):
            solve = lu.solve
    except RuntimeError:
        solve = None
    if solve is None:
        Qp = np.linalg.pinv(Q.toarray(), rcond=rcond)
        solve = lambda b: Qp @ b  # noqa: E731
    for _ in range(int(T)):
        x = solve(periodic(x, ss, 1).reshape(-1)).reshape(dims)
    return x


BCS = {"fixed": 0, "reflect": 1}


def aperiodic(a: np.ndarray, coeffs: np.ndarray, T: int, nthreads: int = 0, bc: str = "fixed") -> np.ndarray:
    """``a`` has extents n_i + 2r; the interior evolves T steps.

    ``bc="fixed"``: the r-wide frame holds fixed boundary values.  ``bc="reflect"``:
    before every step the frame is the mirror image of the interior about the
    cell faces (zero-flux boundary); the frame's input values are ignored and the
    returned frame is the mirror image of the final interior."""
    if bc not in BCS:
        raise ValueError(f"bc must be one of {sorted(BCS)}")
    x = np.ascontiguousarray(a, dtype=np.float64).copy()
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    r = _check_coeffs(c, x.ndim)
    interior = [s - 2 * r for s in x.shape]
    if min(interior) < 1:
        raise ValueError("interior extents must be >= 1")
    if bc == "reflect" and min(interior) < r:
        raise ValueError("a reflecting boundary needs interior extents >= r")
    dims = (ctypes.c_int64 * x.ndim)(*interior)
    rc = _load().oracle_aperiodic_bc(x.ctypes.data, x.ndim, dims, c.ctypes.data, r, int(T), BCS[bc],
                                     int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_aperiodic_bc failed ({rc})")
    return x


def first_column(coeffs: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """First column ``s[m] = S[m, 0]`` of the circulant stencil matrix.

    Row 0 of ``S`` updates cell 0 from neighbour ``(0 + o) mod n`` with weight
    ``c[o]``, so ``S[0, o mod n] += c[o]``; circulance ``S[i, j] = s[i - j]`` (Sec. 3)
    then gives ``s[(-o) mod n] += c[o]`` (offsets alias modulo n for tiny grids)."""
    c = np.asarray(coeffs, dtype=np.float64)
    d = c.ndim
    r = (c.shape[0] - 1) // 2
    s = np.zeros(tuple(dims), dtype=np.float64)
    for idx in np.ndindex(*c.shape):
        o = [k - r for k in idx]
        pos = tuple((-oi) % n for oi, n in zip(o, dims))
        s[pos] += c[idx]
    return s


def symbol(coeffs: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """``Lambda = F s``: unnormalised forward DFT (exponent -2 pi i) of the first column."""
    return np.fft.fftn(first_column(coeffs, dims))


def symbol_power(lam: np.ndarray, T: int, digits: int = 60) -> np.ndarray:
    """``lam**T`` elementwise by binary repeated squaring in ``digits``-digit decimals.

    The FP64 inputs are taken as exact; only the powering is done here.  Slow: meant
    for a few thousand elements."""
    getcontext().prec = digits
    flat = np.asarray(lam, dtype=np.complex128).ravel()
    out = np.empty_like(flat)
    for i, z in enumerate(flat):
        vr, vi = Decimal(1), Decimal(0)
        sr, si = Decimal(float(z.real)), Decimal(float(z.imag))
        R = int(T)
        while R > 0:
            if R & 1:
                vr, vi = vr * sr - vi * si, vr * si + vi * sr
            R >>= 1
            if R:
                sr, si = sr * sr - si * si, 2 * sr * si
        out[i] = complex(float(vr), float(vi))
    return out.reshape(np.shape(lam))


def dist(interior: Sequence[int]) -> np.ndarray:
    """``1 + min over faces`` of the index distance of each interior cell to the frame."""
    d = None
    for ax, n in enumerate(interior):
        i = np.arange(n)
        di = np.minimum(i + 1, n - i)
        shape = [1] * len(interior)
        shape[ax] = n
        di = di.reshape(shape)
        d = di if d is None else np.minimum(d, di)
    return np.broadcast_to(d, tuple(interior)).copy()
