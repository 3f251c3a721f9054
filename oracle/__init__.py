"""CPU FP64 oracle for the split pressure-gradient projection (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  See ``ppe_oracle`` for the definitions it follows.
"""
from .ppe_oracle import *  # noqa: F401,F403
from .ppe_oracle import __all__  # noqa: F401
