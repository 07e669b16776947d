"""MI355X (gfx950) library for the reionization-redshift hot path of AMBER.

Trac et al., "AMBER: A Semi-numerical Abundance Matching Box for the Epoch of
Reionization", arXiv:2109.10375.  The compute lives in ``libamber.so`` (HIP
kernels behind the C-ABI in ``include/amber.h``); this package only marshals
torch tensors, streams and structs into those calls.  There is no CPU path: if
the library is missing, every call raises.
"""
from ._lib import (  # noqa: F401
    AmberError,
    Batch,
    BatchItem,
    History,
    Plan,
    STATUS_BAD_W,
    STATUS_NAN_J,
    STATUS_RANGE,
    fft_schedules,
    lib,
    library_path,
)
from .tune import tune_plan  # noqa: F401

__all__ = ["AmberError", "Batch", "BatchItem", "History", "Plan", "fft_schedules", "lib", "library_path", "tune_plan",
           "STATUS_NAN_J", "STATUS_BAD_W", "STATUS_RANGE"]
