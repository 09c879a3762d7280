"""Helpers shared by the GPU tests."""
import functools

import numpy as np

from paper_2502_09502_amd import _lib


@functools.lru_cache(maxsize=1)
def ctx():
    return _lib.Context(0)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)
