"""MI355X-native truncated-EM sparse coding (BSC, TSC, MCA).

The truncated E-step, the FP64 M-step and the serving loop run in the HIP
library libprosper.so (C ABI in include/prosper.h); this package is its thin
Python binding plus the EM driver objects of the paper's user interface.
"""
from ._lib import MODELS, PRECISIONS, ProsperError, load, state_count, state_table  # noqa: F401

__all__ = ["MODELS", "PRECISIONS", "ProsperError", "load", "state_count", "state_table"]
