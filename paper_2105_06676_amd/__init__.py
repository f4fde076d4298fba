"""FFT stencil solver for AMD MI355X (gfx950).

Python binding over ``libstencilfft.so`` (C ABI in ``include/stencil_fft.h``).
It only marshals arguments: device memory comes from torch tensors, streams from
``torch.cuda.current_stream()``, and every step of a solve runs in the HIP kernels
of the library.  Importing this package fails loudly when the library has not
been built (``python -m paper_2105_06676_amd.build``); there is no CPU fallback.
"""
from ._binding import (  # noqa: F401
    Graph,
    SfftError,
    Server,
    aperiodic,
    batch,
    lib,
    library_path,
    periodic,
    periodic_fields,
    periodic_noalloc,
    periodic_implicit,
    plan_describe,
    profile_read,
    profile_start,
    profile_stop,
    set_option,
    symbol_power,
    tune,
    tune_clear,
    tune_load,
    tune_save,
    verify,
    version,
)
