"""Barnes-Hut gravity on one MI355X (gfx950): HIP kernels behind a C ABI.

The compute path lives in the shared library built from ``csrc/``; the
``bh`` module binds it with ctypes.  Importing this package loads nothing;
``from paper_1907_02289_amd import bh`` loads the library.
"""
