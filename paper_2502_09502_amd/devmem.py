"""Device buffers for callers of the C ABI that hand over device memory (no torch needed).

The HIP runtime used here is the one libcertglm.so itself links (libamdhip64.so.7, loaded with
the library), so the pointers are valid in the library's device context. Plumbing only: a
buffer is hipMalloc'ed memory with host <-> device copies; no computation happens here.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib

_hip = None
_H2D, _D2H = 1, 2


def _rt():
    global _hip
    if _hip is None:
        _lib.load()  # the library first: its runtime is the one this handle resolves to
        hip = C.CDLL("libamdhip64.so.7")
        hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        hip.hipFree.argtypes = [C.c_void_p]
        hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        hip.hipSetDevice.argtypes = [C.c_int]
        hip.hipDeviceSynchronize.argtypes = []
        _hip = hip
    return _hip


# the ABI's element types (cgl_dtype) by numpy dtype; BF16 travels as uint16 bit patterns
CGL_DTYPE = {np.dtype(np.float64): _lib.F64, np.dtype(np.float32): _lib.F32,
             np.dtype(np.uint16): _lib.BF16}


class DeviceArray:
    """A C-contiguous array in device memory: shape, numpy dtype, data_ptr()."""

    def __init__(self, shape, dtype, device: int = 0):
        self.shape = tuple(int(s) for s in np.atleast_1d(shape)) if not isinstance(shape, tuple) \
            else tuple(int(s) for s in shape)
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        self.device = device
        hip = _rt()
        if hip.hipSetDevice(device) != 0:
            raise RuntimeError("hipSetDevice failed")
        self._ptr = C.c_void_p()
        if hip.hipMalloc(C.byref(self._ptr), C.c_size_t(max(self.nbytes, 8))) != 0:
            raise MemoryError("hipMalloc failed")

    @classmethod
    def from_numpy(cls, a: np.ndarray, device: int = 0) -> "DeviceArray":
        a = np.ascontiguousarray(a)
        d = cls(a.shape, a.dtype, device)
        d.upload(a)
        return d

    def data_ptr(self) -> int:
        return int(self._ptr.value or 0)

    def upload(self, a: np.ndarray) -> None:
        a = np.ascontiguousarray(a, dtype=self.dtype)
        if a.nbytes != self.nbytes:
            raise ValueError("size mismatch")
        if _rt().hipMemcpy(self._ptr, a.ctypes.data_as(C.c_void_p), a.nbytes, _H2D) != 0:
            raise RuntimeError("hipMemcpy to the device failed")

    def numpy(self) -> np.ndarray:
        out = np.empty(self.shape, self.dtype)
        if _rt().hipMemcpy(out.ctypes.data_as(C.c_void_p), self._ptr, self.nbytes, _D2H) != 0:
            raise RuntimeError("hipMemcpy to the host failed")
        return out

    def free(self) -> None:
        if self._ptr.value:
            _rt().hipFree(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Stream:
    """A HIP stream (default priority, non-blocking) for a context the caller synchronises."""

    def __init__(self, device: int = 0):
        hip = _rt()
        hip.hipStreamCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        hip.hipStreamSynchronize.argtypes = [C.c_void_p]
        hip.hipStreamDestroy.argtypes = [C.c_void_p]
        if hip.hipSetDevice(device) != 0:
            raise RuntimeError("hipSetDevice failed")
        self.h = C.c_void_p()
        if hip.hipStreamCreateWithFlags(C.byref(self.h), 1) != 0:  # hipStreamNonBlocking
            raise RuntimeError("hipStreamCreateWithFlags failed")

    def synchronize(self) -> None:
        if _rt().hipStreamSynchronize(self.h) != 0:
            raise RuntimeError("hipStreamSynchronize failed")

    def close(self) -> None:
        if self.h.value:
            _rt().hipStreamDestroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
