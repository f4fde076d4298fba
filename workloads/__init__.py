"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws numbers and builds stencil-coefficient arrays and grids of
the shapes used by the periodic / aperiodic stencil workloads.  It holds none of
the stencil method's arithmetic (no symbol, no FFT, no time stepping), so both the
oracle and the HIP path can consume what it produces without sharing any code.

Random numbers come from a counter-based SplitMix64 generator written from its
published definition (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): value ``i`` of a stream is ``mix(key + (i + 1) * GAMMA)``
with ``GAMMA = 0x9E3779B97F4A7C15`` and the two-multiply finaliser ``mix``.  The
stream key is derived from ``(seed, purpose)`` so grids and coefficients of one
workload are independent streams.

Coefficient layout (the same everywhere in this repository): a ``(2r+1,)*d`` float64
array indexed by neighbour offset ``o + r`` per axis, row-major over ``o_0..o_{d-1}``;
entry ``c[o]`` multiplies ``a[(i + o) mod n]`` when updating cell ``i`` (the periodic
loop's neighbour convention ``S[i, (i + j) % N]``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (uint64 in, uint64 out, wrapping arithmetic)."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _fnv1a64(text: str) -> int:
    h = 0xCBF29CE484222325
    for b in text.encode():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def stream_key(seed: int, purpose: str) -> np.uint64:
    with np.errstate(over="ignore"):
        k = _mix(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
        return np.uint64(int(k) ^ _fnv1a64(purpose))


def raw_u64(seed: int, purpose: str, count: int, start: int = 0) -> np.ndarray:
    """Values ``start .. start+count-1`` of the (seed, purpose) stream as uint64."""
    key = stream_key(seed, purpose)
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + idx * GAMMA)


def uniform(seed: int, purpose: str, count: int, start: int = 0) -> np.ndarray:
    """Uniform [0, 1) doubles: top 53 bits of each 64-bit value times 2**-53."""
    z = raw_u64(seed, purpose, count, start)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian(seed: int, purpose: str, count: int) -> np.ndarray:
    """Standard normal doubles by Box-Muller on pairs (1 - u1, u2) of the uniform stream."""
    m = (count + 1) // 2
    u = uniform(seed, purpose, 2 * m)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * m, dtype=np.float64)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:count]


def snap_coefficients(c: np.ndarray, centre_index: Tuple[int, ...], bits: int = 40) -> np.ndarray:
    """Round every coefficient but the centre to a multiple of 2**-bits and let the
    centre absorb the residue, so the coefficients sum to exactly 1 in float64."""
    scale = float(2 ** bits)
    ints = np.rint(c * scale).astype(np.int64)
    ints[centre_index] = 0
    ints[centre_index] = (1 << bits) - int(ints.sum())
    return ints.astype(np.float64) / scale


def box_shape(ndim: int, r: int) -> Tuple[int, ...]:
    return (2 * r + 1,) * ndim


def centre(ndim: int, r: int) -> Tuple[int, ...]:
    return (r,) * ndim


# ---------------------------------------------------------------------------
# Named workloads (stand-ins for the paper's heat1d / jacobi2d / heat3d runs,
# whose benchmark coefficients are not available).
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ndim: int
    dims: Tuple[int, ...]          # interior extents (evolved cells)
    radius: int
    T: int
    coeffs: np.ndarray             # (2r+1,)*ndim float64
    seed: int
    init: str                      # "uniform" | "gaussian"
    aperiodic: bool = False
    dtypes: Tuple[str, ...] = ("f64",)
    notes: str = ""
    fields: int = 1                # coupled fields (coeffs then (m, m) + (2r+1,)*ndim)
    implicit_q: Optional[np.ndarray] = None  # implicit update Q a_{t+1} = S a_t (coeffs = S)
    bc: str = "fixed"              # aperiodic boundary: "fixed" frame or "reflect" (zero flux)

    @property
    def storage_dims(self) -> Tuple[int, ...]:
        if self.aperiodic:
            return tuple(n + 2 * self.radius for n in self.dims)
        return self.dims

    def grid(self, dims: Optional[Tuple[int, ...]] = None) -> np.ndarray:
        """The seeded initial array (float64, row-major, storage extents)."""
        dims = tuple(dims) if dims is not None else self.storage_dims
        n = int(np.prod(dims))
        if self.init == "uniform":
            v = uniform(self.seed, "grid", n)
        elif self.init == "gaussian":
            v = gaussian(self.seed, "grid", n)
        else:
            raise ValueError(self.init)
        v = v.reshape(dims)
        if self.fields > 1:
            # every field starts from the same seeded array (a wave field at rest:
            # the previous step equals the current one)
            v = np.stack([v] * self.fields)
        return v


def heat1d_coeffs() -> np.ndarray:
    return np.array([0.25, 0.5, 0.25], dtype=np.float64)


def jacobi5_coeffs() -> np.ndarray:
    c = np.zeros((3, 3), dtype=np.float64)
    c[1, 1] = 0.2
    c[0, 1] = c[2, 1] = c[1, 0] = c[1, 2] = 0.2
    return c


def identity_coeffs(ndim: int) -> np.ndarray:
    c = np.zeros((3,) * ndim, dtype=np.float64)
    c[(1,) * ndim] = 1.0
    return c


def backward_euler2d_q(kappa: float) -> np.ndarray:
    """Q = I - kappa * (5-point Laplacian): the implicit side of a backward-Euler heat step."""
    c = np.zeros((3, 3), dtype=np.float64)
    c[1, 1] = 1.0 + 4.0 * kappa
    c[0, 1] = c[2, 1] = c[1, 0] = c[1, 2] = -kappa
    return c


def leapfrog2d_coeffs(kappa: float) -> np.ndarray:
    """Second-order-in-time 2-D wave update a_{t+1} = 2 a_t - a_{t-1} + kappa * (5-point
    Laplacian of a_t), as two fields (a_t, a_{t-1}): blocks (0,0) = 2 I + kappa Lap,
    (0,1) = -I, (1,0) = I, (1,1) = 0.  Stable for kappa <= 1/2."""
    c = np.zeros((2, 2, 3, 3), dtype=np.float64)
    c[0, 0, 1, 1] = 2.0 - 4.0 * kappa
    c[0, 0, 0, 1] = c[0, 0, 2, 1] = c[0, 0, 1, 0] = c[0, 0, 1, 2] = kappa
    c[0, 1, 1, 1] = -1.0
    c[1, 0, 1, 1] = 1.0
    return c


def star7_random_coeffs(seed: int) -> np.ndarray:
    """7-point star with random weights: centre 0.4 + 0.2*u0, the six neighbours share
    1 - centre in proportion to u1..u6 (order -x, +x, -y, +y, -z, +z with x = axis 0),
    then snapped so the sum is exactly 1."""
    u = uniform(seed, "coef", 7)
    ctr = 0.4 + 0.2 * u[0]
    w = (1.0 - ctr) * u[1:] / u[1:].sum()
    c = np.zeros((3, 3, 3), dtype=np.float64)
    c[1, 1, 1] = ctr
    c[0, 1, 1], c[2, 1, 1] = w[0], w[1]
    c[1, 0, 1], c[1, 2, 1] = w[2], w[3]
    c[1, 1, 0], c[1, 1, 2] = w[4], w[5]
    return snap_coefficients(c, (1, 1, 1))


def box_random_coeffs(seed: int, ndim: int, r: int, purpose: str = "coef") -> np.ndarray:
    """Full (2r+1)^d box of U[0,1) weights normalised to sum 1, snapped to 2**-40."""
    shape = box_shape(ndim, r)
    u = uniform(seed, purpose, int(np.prod(shape))).reshape(shape)
    return snap_coefficients(u / u.sum(), centre(ndim, r))


def config(name: str) -> Workload:
    """The five named workloads at full size."""
    if name == "heat1d_65536":
        return Workload("heat1d_65536", 1, (65536,), 1, 1024, heat1d_coeffs(), 1, "uniform",
                        dtypes=("f64",), notes="1-D periodic 3-point heat")
    if name == "jacobi2d_8192":
        return Workload("jacobi2d_8192", 2, (8192, 8192), 1, 4096, jacobi5_coeffs(), 2, "uniform",
                        dtypes=("f32", "f64"), notes="2-D periodic 5-point Jacobi")
    if name == "star3d_512":
        return Workload("star3d_512", 3, (512, 512, 512), 1, 1000, star7_random_coeffs(3), 3,
                        "gaussian", dtypes=("f32",), notes="3-D periodic random 7-point star")
    if name == "box2d_aperiodic_4096":
        return Workload("box2d_aperiodic_4096", 2, (4096, 4096), 1, 512, box_random_coeffs(4, 2, 1), 4,
                        "uniform", aperiodic=True, dtypes=("f64", "f32"),
                        notes="2-D aperiodic 9-point box, fixed frame")
    if name == "box2d_reflect_4096":
        return Workload("box2d_reflect_4096", 2, (4096, 4096), 1, 512, box_random_coeffs(4, 2, 1), 4,
                        "uniform", aperiodic=True, dtypes=("f64", "f32"), bc="reflect",
                        notes="2-D aperiodic 9-point box, reflecting (zero-flux) frame")
    if name == "upwind2d_aperiodic_4096":
        c = np.zeros((3, 3), dtype=np.float64)
        c[1, 1], c[0, 1], c[1, 0] = 0.5, 0.25, 0.25
        return Workload("upwind2d_aperiodic_4096", 2, (4096, 4096), 1, 512, c, 9, "uniform", aperiodic=True,
                        dtypes=("f64", "f32"), notes="2-D aperiodic upwind 3-point stencil, fixed frame")
    if name == "jacobi2d_6300x6720_smooth":
        return Workload("jacobi2d_6300x6720_smooth", 2, (6300, 6720), 1, 4096, jacobi5_coeffs(), 8, "uniform",
                        dtypes=("f32", "f64"),
                        notes="2-D periodic 5-point Jacobi on a 7-smooth, non-power-of-two torus "
                              "(6300 = 2^2 3^2 5^2 7, 6720 = 2^6 3 5 7; mixed-radix transforms)")
    if name == "jacobi2d_8000_smooth":
        return Workload("jacobi2d_8000_smooth", 2, (8000, 8000), 1, 100000, jacobi5_coeffs(), 10, "uniform",
                        dtypes=("f32", "f64"),
                        notes="2-D periodic 5-point Jacobi at the paper's 2-D size and step count "
                              "(8000 = 2^6 5^3: mixed-radix transforms)")
    if name == "heat3d_800_smooth":
        c = np.zeros((3, 3, 3), dtype=np.float64)
        c[1, 1, 1] = 0.4
        c[0, 1, 1] = c[2, 1, 1] = c[1, 0, 1] = c[1, 2, 1] = c[1, 1, 0] = c[1, 1, 2] = 0.1
        return Workload("heat3d_800_smooth", 3, (800, 800, 800), 1, 10000, c, 11, "uniform",
                        dtypes=("f32",),
                        notes="3-D periodic 7-point heat at the paper's 3-D size and step count "
                              "(800 = 2^5 5^2: mixed-radix transforms)")
    if name == "jacobi2d_8191_prime":
        return Workload("jacobi2d_8191_prime", 2, (8191, 8191), 1, 4096, jacobi5_coeffs(), 8, "uniform",
                        dtypes=("f32", "f64"),
                        notes="2-D periodic 5-point Jacobi on a prime torus (chirp-z transforms)")
    if name == "heat2d_backward_euler_4096":
        return Workload("heat2d_backward_euler_4096", 2, (4096, 4096), 1, 1000, identity_coeffs(2), 7, "uniform",
                        dtypes=("f32", "f64"), implicit_q=backward_euler2d_q(2.0),
                        notes="2-D backward-Euler heat step (I - kappa Lap) a_{t+1} = a_t, kappa = 2")
    if name == "wave2d_leapfrog_4096":
        return Workload("wave2d_leapfrog_4096", 2, (4096, 4096), 1, 2048, leapfrog2d_coeffs(0.25), 6, "uniform",
                        dtypes=("f32", "f64"), fields=2,
                        notes="2-D leapfrog wave equation as two coupled periodic fields")
    raise KeyError(name)


def crop_grid(w: Workload, side: int) -> np.ndarray:
    """Leading ``side^d`` corner of the seeded full-size grid of ``w``, generated
    without materialising the full grid (rows are drawn from their stream offsets)."""
    dims = w.storage_dims
    out = np.empty((side,) * w.ndim, dtype=np.float64)
    if w.init != "uniform" and w.init != "gaussian":
        raise ValueError(w.init)
    strides = [int(np.prod(dims[i + 1:])) for i in range(w.ndim)]
    idx = np.indices((side,) * (w.ndim - 1)).reshape(w.ndim - 1, -1).T if w.ndim > 1 else [()]
    for lead in idx:
        off = sum(int(l) * s for l, s in zip(lead, strides[:-1]))
        if w.init == "uniform":
            row = uniform(w.seed, "grid", side, start=off)
        else:
            # Box-Muller consumes uniforms in pairs; draw the enclosing even range.
            s0 = off - (off % 2)
            m = side + (off % 2)
            m += m % 2
            u = uniform(w.seed, "grid", m, start=s0)
            u1, u2 = 1.0 - u[0::2], u[1::2]
            rad = np.sqrt(-2.0 * np.log(u1))
            g = np.empty(m, dtype=np.float64)
            g[0::2] = rad * np.cos(2.0 * np.pi * u2)
            g[1::2] = rad * np.sin(2.0 * np.pi * u2)
            row = g[off % 2: off % 2 + side]
        out[tuple(lead)] = row
    return out


# ---------------------------------------------------------------------------
# Serving mix: a Poisson stream of periodic requests.
# ---------------------------------------------------------------------------

def _is_7smooth(n: int) -> bool:
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


_SMOOTH = None


def _smooth_numbers(limit: int = 1 << 26):
    global _SMOOTH
    if _SMOOTH is None:
        out = []
        p2 = 1
        while p2 <= limit:
            p3 = p2
            while p3 <= limit:
                p5 = p3
                while p5 <= limit:
                    p7 = p5
                    while p7 <= limit:
                        out.append(p7)
                        p7 *= 7
                    p5 *= 5
                p3 *= 3
            p2 *= 2
        _SMOOTH = np.array(sorted(out), dtype=np.float64)
    return _SMOOTH


def nearest_7smooth(x: float) -> int:
    """The 7-smooth integer closest to x in log distance."""
    sm = _smooth_numbers()
    j = int(np.searchsorted(sm, x))
    cands = [sm[k] for k in (j - 1, j) if 0 <= k < len(sm)]
    return int(min(cands, key=lambda v: abs(math.log(v) - math.log(x))))


@dataclass
class Request:
    rid: int
    arrival_s: float
    ndim: int
    dims: Tuple[int, ...]
    radius: int
    T: int
    dtype: str
    coeffs: np.ndarray = field(repr=False)
    seed: int = 0

    @property
    def cells(self) -> int:
        return int(np.prod(self.dims))

    def grid(self) -> np.ndarray:
        return uniform(self.seed, f"req{self.rid}", self.cells).reshape(self.dims)


def serving_mix(count: int = 10000, seed: int = 5, rate_per_s: float = 1000.0,
                log2_cells=(10.0, 24.0), max_T: float = 1e5, smooth: bool = True) -> list:
    """Requests of the serving mix: d ~ U{1,2,3}; log2(N) ~ U[10, 24]; extents
    N^(1/d) * 2^delta_i with sum(delta) = 0, delta ~ U[-1/2, 1/2], each rounded to the
    nearest 7-smooth integer (smooth=True) or to the nearest integer; r ~ U{1,2};
    full box weights normalised and snapped; T = round(10^u), u ~ U[0, log10(max_T)];
    dtype f32/f64 with probability 1/2; Poisson arrivals at ``rate_per_s``."""
    per = 16
    u = uniform(seed, "mix", per * count).reshape(count, per)
    reqs = []
    t = 0.0
    for i in range(count):
        row = u[i]
        t += -math.log(1.0 - row[0]) / rate_per_s
        d = 1 + min(2, int(row[1] * 3))
        lg = log2_cells[0] + (log2_cells[1] - log2_cells[0]) * row[2]
        delta = row[3:3 + d] - 0.5
        delta = delta - delta.mean() if d > 1 else np.zeros(1)
        base = 2.0 ** (lg / d)
        dims = tuple(nearest_7smooth(base * 2.0 ** float(dl)) if smooth else max(1, int(round(base * 2.0 ** float(dl))))
                     for dl in delta)
        r = 1 + int(row[6] * 2)
        T = max(1, int(round(10.0 ** (row[7] * math.log10(max_T)))))
        dtype = "f32" if row[8] < 0.5 else "f64"
        coeffs = box_random_coeffs(seed * 1000003 + i, d, r, purpose="reqcoef")
        reqs.append(Request(i, t, d, dims, r, T, dtype, coeffs, seed=seed))
    return reqs
