"""MI355X-native certification of k-sparse GLM branch-and-bound nodes (arXiv 2502.09502).

The compute path is libcertglm.so (hand-written HIP kernels for gfx950 behind a C ABI,
``include/certglm.h``); ``_lib`` is its ctypes binding and ``synth`` the seeded input generator.
"""
from . import synth  # noqa: F401
