"""Plain FP64 CPU oracle of the WCSPH step (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP product path never does.
"""
from .oracle import *  # noqa: F401,F403
