"""Two-stage NMF for streaming data on MI355X (gfx950).

The compute path is the HIP library built from ``csrc/`` (C ABI in
``include/nmf.h``); ``_lib`` is its ctypes binding and ``synth`` draws seeded
synthetic inputs.
"""
from ._lib import (NMF, Batch, NMFError, Options, Report, default_options, load, workspace_bytes,  # noqa: F401
                   EXPORTS, NMF_OK, NMF_CONVERGED, NMF_EINVAL, NMF_ENOMEM, NMF_EDEVICE, NMF_ENOTCONV,
                   NMF_ESINGULAR, NMF_ESTATE, NMF_ECAPACITY)
