"""MI355X-native truncated-EM sparse coding (BSC, TSC, MCA, MMCA).

The truncated E-step, the FP64 M-step and the serving loop run in the HIP
library libprosper.so (C ABI in include/prosper.h).  This package holds its
thin Python binding (`api`: E-step, M-step, contexts and accumulators on
torch device tensors; `serve`: the request server), the model, annealing
and EM driver objects of the paper's user interface (`em`: BSC_ET, TSC_ET,
MCA_ET, MMCA_ET, LinearAnnealing, EM), and the build of the library
(`build`).
"""
from ._lib import MODELS, PRECISIONS, ProsperError, load, state_count, state_table  # noqa: F401

__all__ = ["MODELS", "PRECISIONS", "ProsperError", "load", "state_count", "state_table"]
