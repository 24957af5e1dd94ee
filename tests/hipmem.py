"""Device buffers for tests through the HIP runtime's C interface (ctypes).

Test plumbing only: it lets the GPU tests hand device pointers to the
library's entry points (device arcs, device seeds, device signature
destinations) without a tensor library.
"""
import ctypes
import sys

import numpy as np

_hip = None
H2D, D2H = 1, 2


def hip():
    global _hip
    if _hip is None:
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        h.hipFree.argtypes = [ctypes.c_void_p]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipDeviceSynchronize.argtypes = []
        _hip = h
    return _hip


class DeviceArray:
    """A device copy of a numpy array; duck-types the tensor attributes the binding reads."""
    is_cuda = True

    def __init__(self, host=None, dtype=None, count=None):
        if host is not None:
            host = np.ascontiguousarray(host)
            dtype, count = host.dtype, host.size
        self.dtype = np.dtype(dtype)
        self.count = int(count)
        self.nbytes = max(1, self.count * self.dtype.itemsize)
        self.ptr = ctypes.c_void_p()
        rc = hip().hipMalloc(ctypes.byref(self.ptr), self.nbytes)
        assert rc == 0, f"hipMalloc failed: {rc}"
        if host is not None and self.count:
            rc = hip().hipMemcpy(self.ptr, host.ctypes.data_as(ctypes.c_void_p), self.nbytes, H2D)
            assert rc == 0, f"hipMemcpy failed: {rc}"

    def data_ptr(self) -> int:
        return int(self.ptr.value)

    def numel(self) -> int:
        return self.count

    def to_host(self) -> np.ndarray:
        out = np.empty(self.count, dtype=self.dtype)
        if self.count:
            assert hip().hipDeviceSynchronize() == 0
            rc = hip().hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), self.ptr, self.nbytes, D2H)
            assert rc == 0, f"hipMemcpy failed: {rc}"
        return out

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():   # bound at definition: the module's globals may be gone at exit
            return
        try:
            self.free()
        except Exception:
            pass
