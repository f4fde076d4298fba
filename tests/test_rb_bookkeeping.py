"""The reading of RecursiveBoundary (Sec. 4) used by the HIP aperiodic solver,
checked on the CPU: executing the same band bookkeeping with the oracle's loops
in place of the GPU's slab solves and base case must reproduce the aperiodic
loop bit for bit.

The executor below is test harness code, not a CPU path of the product: it
restates the plan in entry times (a face of axis k enters a cell at distance dist
after ceil(dist / reach_k) steps; ell = min over the faces the stencil reads
toward; interior kept at ell > T; RB(T) = base case for T <= cutoff, else
step 1 = slabs of band (0, 2T] over T1 = floor(T/2) steps kept on (T1, T + T2]
plus RB(T1); step 2 = slabs of band (0, T + T2] over T2 steps kept on (T2, T]
plus RB(T2); a slab of axis k is reach_k cells deep per step of entry time; each
cell taken from the slab of the face that enters it first, slabs zero-padded to
7-smooth extents) so that the reading itself is pinned.
"""
import numpy as np
import pytest

import oracle
import workloads as wl


def _pad7(n):
    def smooth(m):
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        return m == 1
    while not smooth(n):
        n += 1
    return n


def _rb_execute(a, c, r, T, cutoff):
    d = a.ndim
    n = [s - 2 * r for s in a.shape]
    inner = tuple(slice(r, r + x) for x in n)
    # reach per axis and the faces the stencil reads toward
    nz = [tuple(i - r for i in idx) for idx in np.ndindex(*c.shape) if c[idx] != 0]
    reach = [max([abs(o[k]) for o in nz] + [0]) for k in range(d)]
    act = [[any(o[k] < 0 for o in nz), any(o[k] > 0 for o in nz)] for k in range(d)]
    big = 1 << 40

    def ent(g):
        """(first face, entry time): ceil(distance / reach) per face, min over the
        active faces in face order (axis 0 low, axis 0 high, axis 1 low, ...)."""
        best, face = big, -1
        for k in range(d):
            for side in (0, 1):
                if not act[k][side]:
                    continue
                dist = g[k] + 1 if side == 0 else n[k] - g[k]
                e = -(-dist // reach[k])
                if e < best:
                    best, face = e, 2 * k + side
        return face, best

    depth = [(-(-n[k] // 2) if act[k][0] and act[k][1] else n[k]) for k in range(d)]
    maxell = min([-(-depth[k] // reach[k]) for k in range(d) if act[k][0] or act[k][1]] + [big])

    def slabs(src, dst, w, steps, lo, hi):
        if lo >= maxell or hi <= lo:
            return
        for ax in range(d):
            if not (act[ax][0] or act[ax][1]) or reach[ax] * lo >= depth[ax]:
                continue
            ta = min(reach[ax] * w, n[ax])
            ext = [ta if k == ax else n[k] for k in range(d)]
            if ta >= n[ax]:
                sides = [-1]
            else:
                sides = [s_ for s_ in (0, 1) if act[ax][s_]]
            for side in sides:
                org = [0] * d
                if side == 1:
                    org[ax] = n[ax] - ta
                box = src[tuple(slice(r + o, r + o + e) for o, e in zip(org, ext))]
                big_box = np.zeros([_pad7(e) for e in ext])
                big_box[tuple(slice(0, e) for e in ext)] = box
                res = oracle.periodic(big_box, c, steps)
                for idx in np.ndindex(*ext):
                    g = [o + i for o, i in zip(org, idx)]
                    f, e = ent(g)
                    if lo < e <= hi and f // 2 == ax and (side < 0 or (f & 1) == side):
                        dst[tuple(r + x for x in g)] = res[idx]

    def base(src, dst, tau):
        fr = a.copy()
        fr[inner] = src[inner]
        res = oracle.aperiodic(fr, c, tau)
        for idx in np.ndindex(*n):
            if ent(idx)[1] <= tau:
                g = tuple(r + i for i in idx)
                dst[g] = res[g]

    def rb(src, dst, T):
        if T <= cutoff:
            base(src, dst, T)
            return
        T1 = T // 2
        T2 = T - T1
        mid = np.full_like(a, np.nan)
        slabs(src, mid, 2 * T, T1, T1, T + T2)
        rb(src, mid, T1)
        slabs(mid, dst, T + T2, T2, T2, T)
        rb(mid, dst, T2)

    out = a.copy()
    per = oracle.periodic(a[inner], c, T)
    band = a.copy()
    rb(a, band, T)
    for idx in np.ndindex(*n):
        g = tuple(r + i for i in idx)
        out[g] = per[idx] if ent(idx)[1] > T else band[g]
    return out


def _offsets_stencil(offs, r, d, seed):
    c = np.zeros((2 * r + 1,) * d)
    w = wl.uniform(seed, "coef", len(offs)) + 0.1
    for o, x in zip(offs, w / w.sum()):
        c[tuple(oi + r for oi in o)] = x
    return c


@pytest.mark.parametrize("dims,offs,r,T,cutoff", [
    ((31,), [(-2,), (-1,), (0,)], 2, 9, 1),                                       # upwind, reach 2
    ((26, 22), [(-2, 0), (2, 0), (0, -1), (0, 1), (0, 0)], 2, 7, 1),             # reach 2 / 1
    ((20, 24), [(-2, 0), (-1, -1), (0, 0), (1, 1), (0, 1)], 2, 6, 1),            # biased, reach 2 / 1
    ((12, 14, 10), [(0, -2, 0), (0, 2, 0), (-1, 0, 0), (0, 0, 1), (0, 0, 0)], 2, 5, 1),
])
def test_per_axis_entry_times_reproduce_loop(dims, offs, r, T, cutoff):
    """Stencils whose reach differs between axes: bands, slabs and base-case strips
    scale per axis (ceil(distance / reach)), and the result is still the loop's."""
    d = len(dims)
    c = _offsets_stencil(offs, r, d, 60 + T)
    store = tuple(x + 2 * r for x in dims)
    a = wl.uniform(61 + T, "grid", int(np.prod(store))).reshape(store)
    ref = oracle.aperiodic(a, c, T)
    got = _rb_execute(a, c, r, T, cutoff)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dims,r,T,cutoff", [((10,), 1, 2, 1), ((23,), 2, 9, 1), ((13, 29), 1, 17, 3),
                                             ((9, 8, 10), 1, 5, 1), ((24, 20), 2, 7, 1), ((30, 18), 1, 11, 2)])
def test_recursive_boundary_reading_reproduces_loop(dims, r, T, cutoff):
    d = len(dims)
    c = wl.box_random_coeffs(31 + T, d, r)
    store = tuple(x + 2 * r for x in dims)
    a = wl.uniform(31 + T, "grid", int(np.prod(store))).reshape(store)
    ref = oracle.aperiodic(a, c, T)
    got = _rb_execute(a, c, r, T, cutoff)
    assert np.array_equal(got, ref)
