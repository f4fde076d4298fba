"""The reading of RecursiveBoundary (Sec. 4) used by the HIP aperiodic solver,
checked on the CPU: executing the same band bookkeeping with the oracle's loops
in place of the GPU's slab solves and base case must reproduce the aperiodic
loop bit for bit.

The executor below is test harness code, not a CPU path of the product: it
restates the plan (interior kept at dist > rT; RB(T) = base case for T <= cutoff,
else step 1 = slabs of band (0, 2rT] over T1 = floor(T/2) steps kept on
(rT1, rT + rT2] plus RB(T1); step 2 = slabs of band (0, rT + rT2] over T2 steps
kept on (rT2, rT] plus RB(T2); each cell taken from the slab of its nearest
face, slabs zero-padded to 7-smooth extents) so that the reading itself is pinned.
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
    maxdist = min((x + 1) // 2 for x in n)

    def faces(g):
        fd = []
        for k in range(d):
            fd += [g[k] + 1, n[k] - g[k]]
        dd = min(fd)
        return fd.index(dd), dd

    def slabs(src, dst, w, steps, lo, hi):
        if lo >= maxdist or hi <= lo:
            return
        for ax in range(d):
            ta = min(w, n[ax])
            ext = [ta if k == ax else n[k] for k in range(d)]
            sides = [0, 1] if ta < n[ax] else [-1]
            for side in sides:
                org = [0] * d
                if side == 1:
                    org[ax] = n[ax] - ta
                box = src[tuple(slice(r + o, r + o + e) for o, e in zip(org, ext))]
                big = np.zeros([_pad7(e) for e in ext])
                big[tuple(slice(0, e) for e in ext)] = box
                res = oracle.periodic(big, c, steps)
                for idx in np.ndindex(*ext):
                    g = [o + i for o, i in zip(org, idx)]
                    f, dd = faces(g)
                    if lo < dd <= hi and f // 2 == ax and (side < 0 or (f & 1) == side):
                        dst[tuple(r + x for x in g)] = res[idx]

    def base(src, dst, tau):
        fr = a.copy()
        fr[inner] = src[inner]
        res = oracle.aperiodic(fr, c, tau)
        for idx in np.ndindex(*n):
            if faces(idx)[1] <= r * tau:
                g = tuple(r + i for i in idx)
                dst[g] = res[g]

    def rb(src, dst, T):
        if T <= cutoff:
            base(src, dst, T)
            return
        T1 = T // 2
        T2 = T - T1
        mid = np.full_like(a, np.nan)
        slabs(src, mid, 2 * r * T, T1, r * T1, r * T + r * T2)
        rb(src, mid, T1)
        slabs(mid, dst, r * T + r * T2, T2, r * T2, r * T)
        rb(mid, dst, T2)

    out = a.copy()
    per = oracle.periodic(a[inner], c, T)
    band = a.copy()
    rb(a, band, T)
    for idx in np.ndindex(*n):
        g = tuple(r + i for i in idx)
        out[g] = per[idx] if faces(idx)[1] > r * T else band[g]
    return out


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
