"""FP64 CPU oracle for the truncated E-step and M-step (test infrastructure).

Only tests/, ``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg
may import this package.  The GPU library never calls it and shares no code
with it.
"""
from .prosper_oracle import *  # noqa: F401,F403
from .prosper_oracle import __all__  # noqa: F401
