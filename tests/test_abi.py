"""CPU-side checks of the C ABI: the library loads, exports every declared symbol,
rejects invalid arguments before touching the GPU, and plans without a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "stencil_fft.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:int|void|const char\*)\s+\**\s*(\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_2105_06676_amd as s
    names = _declared_functions()
    assert "stencil_fft_periodic" in names and "stencil_fft_aperiodic" in names
    assert len(names) >= 15
    for n in names:
        assert hasattr(s.lib, n), n


def test_measurement_probes_load_and_reject_bad_shapes():
    """The probe library (measurements only, not the solver) exports both probes;
    the strip probe refuses shapes it cannot run before any device work."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2105_06676_amd", "libsfft_probe.so"))
    assert hasattr(lib, "sfft_probe_dft16") and hasattr(lib, "sfft_probe_strip")
    f = lib.sfft_probe_strip
    f.restype = ctypes.c_float
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, ctypes.c_void_p]
    assert f(3, 0, None, None, 16, 8, 1, None) < 0      # W must be 1 or 2
    assert f(1, 0, None, None, 8, 16, 1, None) < 0      # columns beyond the pitch
    assert f(2, 1, None, None, 16, 8, 0, None) < 0      # no repetitions


def test_invalid_arguments_are_rejected_without_a_gpu():
    import paper_2105_06676_amd as s
    lib = s.lib
    f = lib.stencil_fft_periodic
    dims = (ctypes.c_int64 * 2)(8, 8)
    c = np.ones((3, 3)) / 9
    cp = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(0x1000)
    # null grid
    assert f(None, 0, 2, dims, cp, 1, 5, None) == -1
    # bad ndim, dtype, radius, T
    assert f(fake, 0, 4, dims, cp, 1, 5, None) == -1
    assert f(fake, 7, 2, dims, cp, 1, 5, None) == -1
    assert f(fake, 0, 2, dims, cp, -1, 5, None) == -1
    assert f(fake, 0, 2, dims, cp, 1, -5, None) == -1
    # non-finite coefficient
    bad = c.copy()
    bad[1, 1] = np.nan
    assert f(fake, 0, 2, dims, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1, 5, None) == -1
    assert "not finite" in s._binding._last_error().decode()
    # zero extent
    z = (ctypes.c_int64 * 2)(0, 8)
    assert f(fake, 0, 2, z, cp, 1, 5, None) == -1
    # extents beyond the supported range (any extent up to 2^30 is accepted; those
    # with a prime factor above 7 take the chirp-z path)
    p = (ctypes.c_int64 * 2)((1 << 31) + 1, 8)
    assert f(fake, 0, 2, p, cp, 1, 5, None) == -2
    assert "2^30" in s._binding._last_error().decode()
    # the fields entry point takes at most 4 fields (checked before any device work)
    ff = s._binding._periodic_fields
    p = (ctypes.c_int64 * 2)(11, 8)
    assert ff(fake, 0, 5, 2, p, cp, 1, 5, None) == -2
    assert "4 fields" in s._binding._last_error().decode()
    # boundary conditions of the aperiodic entry point
    fb = lib.stencil_fft_aperiodic_bc
    fb.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                   ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    assert fb(fake, 0, 2, dims, cp, 1, 5, 7, None) == -1
    assert "boundary" in s._binding._last_error().decode()
    c5 = np.ones((5, 5)) / 25
    small = (ctypes.c_int64 * 2)(8, 1)
    assert fb(fake, 0, 2, small, c5.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, 5, 1, None) == -1
    assert "reflecting" in s._binding._last_error().decode()


def test_unknown_option_rejected():
    import paper_2105_06676_amd as s
    with pytest.raises(s.SfftError):
        s.set_option("no_such_option", 1)
    with pytest.raises(s.SfftError):
        s.set_option("col_max", 100)


@pytest.mark.parametrize("dims,dtype", [((65536,), "f64"), ((8192, 8192), "f32"), ((8192, 8192), "f64"),
                                        ((512, 512, 512), "f32"), ((1000,), "f64"), ((1, 64), "f32"),
                                        ((7, 9, 5), "f64"), ((1 << 24,), "f32")])
def test_plan_schedule_shape(dims, dtype):
    """The schedule has 2*(number of passes per axis) - 1 passes with one fused middle
    pass, and its model bytes add up per pass."""
    import paper_2105_06676_amd as s
    p = s.plan_describe(dims, dtype)
    modes = [q["mode"] for q in p["passes"]]
    assert modes.count("mid") == 1
    mid = modes.index("mid")
    assert all(m == "fwd" for m in modes[:mid]) and all(m == "inv" for m in modes[mid + 1:])
    assert len(modes[:mid]) == len(modes[mid + 1:])
    assert p["model_bytes"] == sum(q["model_bytes"] for q in p["passes"])
    # every sub-transform length factors the extent
    for a, lev in enumerate(p["levels"]):
        assert int(np.prod(lev)) == dims[a]
    for q in p["passes"]:
        assert int(np.prod(q["radices"] or [1])) == q["L"]
        assert q["lds_bytes"] <= 160 * 1024


@pytest.mark.parametrize("n", [32768, 65536, 1 << 17, 1 << 20])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_long_power_of_two_axes_stay_on_register_kernels(n, dtype):
    """A 1-D power-of-two extent too long for one row pass is split so that every
    level (the strided cofactor included) runs on the register kernels: the strided
    levels are at least 16 points long."""
    import paper_2105_06676_amd as s
    p = s.plan_describe((n,), dtype)
    assert all(q["fast"] == 1 for q in p["passes"]), [(q["name"], q["L"], q["fast"]) for q in p["passes"]]
    assert all(q["L"] >= 16 for q in p["passes"])
