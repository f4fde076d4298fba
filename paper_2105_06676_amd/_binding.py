"""ctypes binding of libstencilfft.so: argument marshalling only."""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libstencilfft.so")

if not os.path.exists(library_path):
    raise ImportError(
        f"{library_path} is missing: build it with `python -m paper_2105_06676_amd.build` "
        "(the solver has no CPU fallback)")

# torch is imported first so that its HIP runtime is the one in the process: the
# library then binds to that same runtime (by soname) instead of loading a second
# copy, which would not share devices, streams or allocations with torch.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(library_path)

SFFT_F32, SFFT_F64 = 0, 1
ERRORS = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "ENOMEM", -4: "EHIP", -5: "EBUSY", -6: "ENOTFOUND"}

_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class _Problem(ctypes.Structure):
    _fields_ = [("grid", _vp), ("dtype", ctypes.c_int), ("ndim", ctypes.c_int),
                ("dims", ctypes.c_int64 * 3), ("coeffs", _dp), ("radius", ctypes.c_int),
                ("T", ctypes.c_int64), ("aperiodic", ctypes.c_int)]


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_periodic = _sig("stencil_fft_periodic", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, _vp])
_periodic_noalloc = _sig("stencil_fft_periodic_noalloc", ctypes.c_int,
                         [_vp, ctypes.c_int, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, _vp])
_periodic_fields = _sig("stencil_fft_periodic_fields", ctypes.c_int,
                       [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, _vp])
_periodic_implicit = _sig("stencil_fft_periodic_implicit", ctypes.c_int,
                         [_vp, ctypes.c_int, ctypes.c_int, _i64p, _dp, _dp, ctypes.c_int, ctypes.c_int64, _vp])
_aperiodic = _sig("stencil_fft_aperiodic", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, _vp])
_aperiodic_bc = _sig("stencil_fft_aperiodic_bc", ctypes.c_int,
                     [_vp, ctypes.c_int, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp])
SFFT_BC_FIXED, SFFT_BC_REFLECT = 0, 1
_BCS = {"fixed": SFFT_BC_FIXED, "reflect": SFFT_BC_REFLECT}
_last_error = _sig("stencil_fft_last_error", ctypes.c_char_p, [])
_symbol_power = _sig("stencil_fft_symbol_power", ctypes.c_int, [_vp, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, _vp])
_batch = _sig("stencil_fft_batch", ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int, _vp])
_set_option = _sig("stencil_fft_set_option", ctypes.c_int, [ctypes.c_char_p, ctypes.c_int64])
_profile = _sig("stencil_fft_profile", ctypes.c_int, [ctypes.c_int])
_profile_read = _sig("stencil_fft_profile_read", ctypes.c_int, [ctypes.c_char_p, ctypes.c_int64])
_plan_describe = _sig("stencil_fft_plan_describe", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_char_p, ctypes.c_int64])
_version = _sig("stencil_fft_version", ctypes.c_char_p, [])
_verify = _sig("stencil_fft_verify", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64,
                                                   ctypes.c_int, ctypes.c_char_p, ctypes.c_int64])
_tune = _sig("stencil_fft_tune", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_int64])
_tune_save = _sig("stencil_fft_tune_save", ctypes.c_int, [ctypes.c_char_p])
_tune_load = _sig("stencil_fft_tune_load", ctypes.c_int, [ctypes.c_char_p])
_tune_clear = _sig("stencil_fft_tune_clear", ctypes.c_int, [])
_srv_create = _sig("sfft_server_create", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_uint64, ctypes.c_int])
_srv_submit = _sig("sfft_server_submit", ctypes.c_int, [_vp, ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_uint64)])
_srv_poll = _sig("sfft_server_poll", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)])
_srv_wait = _sig("sfft_server_wait", ctypes.c_int, [_vp, ctypes.c_uint64])
_srv_stats = _sig("sfft_server_stats", ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int64])
_srv_destroy = _sig("sfft_server_destroy", None, [_vp])
_srv_times = _sig("sfft_server_ticket_times", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)])
_graph_create = _sig("stencil_fft_graph_create", ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(_vp)])
_graph_launch = _sig("stencil_fft_graph_launch", ctypes.c_int, [_vp, _vp])
_graph_destroy = _sig("stencil_fft_graph_destroy", None, [_vp])


class SfftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise SfftError(rc, _last_error().decode())
    return rc


def version() -> str:
    return _version().decode()


def tune(dims, dtype: str = "f32", reps: int = 5, device: int = 0) -> dict:
    """Autotune the strided-axis factorisations of a periodic shape (see
    stencil_fft_tune); returns the tuner's report."""
    import torch
    d = (ctypes.c_int64 * len(dims))(*dims)
    buf = ctypes.create_string_buffer(1 << 20)
    with torch.cuda.device(device):
        _check(_tune(len(dims), d, SFFT_F64 if dtype == "f64" else SFFT_F32, int(reps), buf, len(buf)))
    return json.loads(buf.value.decode())


def tune_save(path: str):
    _check(_tune_save(path.encode()))


def tune_load(path: str):
    _check(_tune_load(path.encode()))


def tune_clear():
    _check(_tune_clear())


def _coeffs(coeffs, ndim: int):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    if c.ndim != ndim or len(set(c.shape)) != 1 or c.shape[0] % 2 != 1:
        raise ValueError(f"coefficients must have shape (2r+1,)*{ndim}, got {c.shape}")
    return c, (c.shape[0] - 1) // 2


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return SFFT_F32
    if t.dtype == torch.float64:
        return SFFT_F64
    raise TypeError(f"grid dtype must be float32 or float64, got {t.dtype}")


def _stream(t, stream):
    import torch
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return torch.cuda.current_stream(t.device).cuda_stream


def _check_grid(t):
    if not t.is_cuda:
        raise ValueError("grid must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("grid must be contiguous")


def periodic(grid, coeffs, T: int, stream=None):
    """Evolve ``grid`` (CUDA tensor, float32/float64, 1-3 dims) T steps in place
    under the periodic stencil ``coeffs`` ((2r+1,)*ndim array, c[o] multiplies a[i+o])."""
    import torch
    _check_grid(grid)
    c, r = _coeffs(coeffs, grid.dim())
    dims = (ctypes.c_int64 * grid.dim())(*grid.shape)
    with torch.cuda.device(grid.device):
        _check(_periodic(grid.data_ptr(), _dtype_code(grid), grid.dim(), dims,
                         c.ctypes.data_as(_dp), r, int(T), _stream(grid, stream)))
    return grid


def periodic_noalloc(grid, coeffs, T: int, stream=None):
    """``periodic`` through the entry point that allocates no device memory
    (7-smooth extents; tables and workspace in the library's fixed device array)."""
    import torch
    _check_grid(grid)
    c, r = _coeffs(coeffs, grid.dim())
    dims = (ctypes.c_int64 * grid.dim())(*grid.shape)
    with torch.cuda.device(grid.device):
        _check(_periodic_noalloc(grid.data_ptr(), _dtype_code(grid), grid.dim(), dims,
                                 c.ctypes.data_as(_dp), r, int(T), _stream(grid, stream)))
    return grid


def periodic_fields(grid, coeffs, T: int, stream=None):
    """Evolve m coupled fields T steps in place: ``grid`` has shape (m, *dims),
    ``coeffs`` shape (m, m, *(2r+1,)*ndim); block (i, j) weights field j's
    neighbours in field i's update."""
    import torch
    _check_grid(grid)
    m, d = grid.shape[0], grid.dim() - 1
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    if c.ndim != d + 2 or c.shape[:2] != (m, m):
        raise ValueError(f"coefficients must have shape ({m}, {m}) + (2r+1,)*{d}, got {c.shape}")
    _, r = _coeffs(c[0, 0], d)
    dims = (ctypes.c_int64 * d)(*grid.shape[1:])
    with torch.cuda.device(grid.device):
        _check(_periodic_fields(grid.data_ptr(), _dtype_code(grid), m, d, dims, c.ctypes.data_as(_dp), r, int(T),
                                _stream(grid, stream)))
    return grid


def periodic_implicit(grid, q_coeffs, s_coeffs, T: int, stream=None):
    """Evolve ``grid`` T steps in place under the implicit update Q a_{t+1} = S a_t
    (both stencils (2r+1,)*ndim arrays of the same radius)."""
    import torch
    _check_grid(grid)
    q, r = _coeffs(q_coeffs, grid.dim())
    s_, r2 = _coeffs(s_coeffs, grid.dim())
    if r != r2:
        raise ValueError("Q and S must have the same radius (pad the smaller with zeros)")
    dims = (ctypes.c_int64 * grid.dim())(*grid.shape)
    with torch.cuda.device(grid.device):
        _check(_periodic_implicit(grid.data_ptr(), _dtype_code(grid), grid.dim(), dims, q.ctypes.data_as(_dp),
                                  s_.ctypes.data_as(_dp), r, int(T), _stream(grid, stream)))
    return grid


def aperiodic(grid, coeffs, T: int, stream=None, bc: str = "fixed"):
    """Evolve the interior of ``grid`` T steps in place (grid extents are interior
    extents + 2r).  ``bc="fixed"``: the outer r-wide frame holds fixed boundary
    values; ``bc="reflect"``: zero-flux boundary, the frame is not read (before
    every step it stands for the mirror image of the interior)."""
    import torch
    _check_grid(grid)
    if bc not in _BCS:
        raise ValueError(f"bc must be one of {sorted(_BCS)}")
    c, r = _coeffs(coeffs, grid.dim())
    interior = [s - 2 * r for s in grid.shape]
    dims = (ctypes.c_int64 * grid.dim())(*interior)
    with torch.cuda.device(grid.device):
        if bc == "fixed":
            _check(_aperiodic(grid.data_ptr(), _dtype_code(grid), grid.dim(), dims,
                              c.ctypes.data_as(_dp), r, int(T), _stream(grid, stream)))
        else:
            _check(_aperiodic_bc(grid.data_ptr(), _dtype_code(grid), grid.dim(), dims,
                                 c.ctypes.data_as(_dp), r, int(T), _BCS[bc], _stream(grid, stream)))
    return grid


def verify(dims: Sequence[int], coeffs, T: int, dtype: str = "f32", kind="periodic") -> dict:
    """Host-side check of the pass schedules of a solve against its buffers (no
    device).  kind: "periodic", "fixed" or "reflect" (aperiodic frames; dims are
    interior extents).  Returns {"checked", "failures", "errors"}."""
    kinds = {"periodic": 0, "fixed": 1, "reflect": 2}
    c, r = _coeffs(coeffs, len(dims))
    d = (ctypes.c_int64 * len(dims))(*dims)
    buf = ctypes.create_string_buffer(1 << 16)
    rc = _verify(SFFT_F64 if dtype == "f64" else SFFT_F32, len(dims), d, c.ctypes.data_as(_dp), r, int(T),
                 kinds[kind], buf, len(buf))
    _check(rc)
    return json.loads(buf.value.decode())


def symbol_power(out, dims: Sequence[int], coeffs, T: int, stream=None):
    """Write lambda(k)^T (complex128, natural order, shape ``dims``) into ``out``."""
    import torch
    _check_grid(out)
    if out.dtype != torch.complex128 or tuple(out.shape) != tuple(dims):
        raise ValueError("out must be a complex128 tensor of shape dims")
    c, r = _coeffs(coeffs, len(dims))
    d = (ctypes.c_int64 * len(dims))(*dims)
    with torch.cuda.device(out.device):
        _check(_symbol_power(out.data_ptr(), len(dims), d, c.ctypes.data_as(_dp), r, int(T), _stream(out, stream)))
    return out


def _kind(aperiodic_) -> int:
    """sfft_problem.aperiodic from False/True or a boundary name."""
    if isinstance(aperiodic_, str):
        if aperiodic_ not in _BCS:
            raise ValueError(f"boundary must be one of {sorted(_BCS)}")
        return 1 + _BCS[aperiodic_]
    return 1 if aperiodic_ else 0


def _problem(grid, coeffs, T, aperiodic_, keep):
    _check_grid(grid)
    c, r = _coeffs(coeffs, grid.dim())
    keep.append(c)
    p = _Problem()
    p.grid = grid.data_ptr()
    p.dtype = _dtype_code(grid)
    p.ndim = grid.dim()
    ext = [s - 2 * r for s in grid.shape] if aperiodic_ else list(grid.shape)
    for a in range(3):
        p.dims[a] = ext[a] if a < grid.dim() else 1
    p.coeffs = c.ctypes.data_as(_dp)
    p.radius = r
    p.T = int(T)
    p.aperiodic = _kind(aperiodic_)
    return p


def batch(problems, stream=None):
    """Solve a list of ``(grid, coeffs, T)`` or ``(grid, coeffs, T, aperiodic)`` in
    batched launches on one stream (``aperiodic``: False, True = fixed frame,
    or a boundary name, "fixed" or "reflect")."""
    import torch
    keep = []
    arr = (_Problem * len(problems))()
    dev = None
    for i, pr in enumerate(problems):
        grid, coeffs, T = pr[0], pr[1], pr[2]
        ap = pr[3] if len(pr) > 3 else False
        arr[i] = _problem(grid, coeffs, T, ap, keep)
        dev = grid.device
    if not problems:
        return
    with torch.cuda.device(dev):
        _check(_batch(arr, len(problems), _stream(problems[0][0], stream)))


class Graph:
    """A batch of periodic problems captured into a hipGraph; each launch() advances
    every bound grid by its T steps again."""

    def __init__(self, problems):
        import torch
        self._keep = []
        arr = (_Problem * len(problems))()
        for i, pr in enumerate(problems):
            arr[i] = _problem(pr[0], pr[1], pr[2], False, self._keep)
        self._grids = [pr[0] for pr in problems]
        self._h = _vp()
        with torch.cuda.device(problems[0][0].device):
            _check(_graph_create(arr, len(problems), ctypes.byref(self._h)))

    def launch(self, stream=None):
        _check(_graph_launch(self._h, _stream(self._grids[0], stream)))

    def close(self):
        if self._h:
            _graph_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching stencil server (one per device)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_slots: int = 0):
        self._h = _vp()
        _check(_srv_create(ctypes.byref(self._h), int(device), int(hbm_budget_bytes), int(max_slots)))
        self._keep = {}

    def submit(self, grid, coeffs, T: int, aperiodic_=False) -> int:
        keep = []
        p = _problem(grid, coeffs, T, aperiodic_, keep)
        t = ctypes.c_uint64()
        _check(_srv_submit(self._h, ctypes.byref(p), ctypes.byref(t)))
        self._keep[t.value] = (grid, keep)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        _check(_srv_poll(self._h, ticket, ctypes.byref(done)))
        if done.value:
            self._keep.pop(ticket, None)
        return bool(done.value)

    def wait(self, ticket: int):
        _check(_srv_wait(self._h, ticket))
        self._keep.pop(ticket, None)

    def times(self, ticket: int):
        """(submit, done) in seconds since the server started; done is -1 while pending."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(_srv_times(self._h, ticket, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def stats(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(_srv_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            _srv_destroy(self._h)
            self._h = _vp()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_option(name: str, value: int):
    _check(_set_option(name.encode(), int(value)))


def profile_start():
    _check(_profile(1))


def profile_stop():
    _check(_profile(0))


def profile_read() -> dict:
    buf = ctypes.create_string_buffer(1 << 20)
    _check(_profile_read(buf, len(buf)))
    return json.loads(buf.value.decode())


def plan_describe(dims: Sequence[int], dtype: str = "f32") -> dict:
    d = (ctypes.c_int64 * len(dims))(*dims)
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_plan_describe(len(dims), d, SFFT_F64 if dtype == "f64" else SFFT_F32, buf, len(buf)))
    return json.loads(buf.value.decode())
