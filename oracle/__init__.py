"""FP64 CPU oracle for the Barnes-Hut force path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark use it to check and time the GPU library.  The
GPU library never imports, links or calls anything in this package.
"""
from .bh import *  # noqa: F401,F403
