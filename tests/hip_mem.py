"""Device memory and streams of the HIP runtime libaf4.so is linked against,
through ctypes, as a caller of the C ABI holds them (torch bundles a HIP
runtime of its own, whose streams the library cannot wait on)."""
import ctypes

import numpy as np

from paper_2510_11527_amd import af

_hip = None
H2D, D2H = 1, 2


def hip():
    """The HIP runtime libaf4.so uses (loaded with it)."""
    global _hip
    if _hip is None:
        af.lib()
        H = ctypes.CDLL("libamdhip64.so.7")
        vp = ctypes.c_void_p
        H.hipMalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t]
        H.hipFree.argtypes = [vp]
        H.hipMemcpy.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int]
        H.hipStreamCreate.argtypes = [ctypes.POINTER(vp)]
        H.hipStreamDestroy.argtypes = [vp]
        H.hipHostMalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, ctypes.c_uint]
        H.hipHostFree.argtypes = [vp]
        H.hipMemcpyAsync.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
        H.hipStreamSynchronize.argtypes = [vp]
        for f in ("hipMalloc", "hipFree", "hipMemcpy", "hipStreamCreate", "hipStreamDestroy", "hipDeviceSynchronize",
                  "hipHostMalloc", "hipHostFree", "hipMemcpyAsync", "hipStreamSynchronize"):
            getattr(H, f).restype = ctypes.c_int
        _hip = H
    return _hip


class DeviceBlock:
    """The DoFs as one device block with kind stride ncell + pad; the padding
    holds NaN, which no kernel may read."""

    def __init__(self, U, precision, pad):
        ncell = np.asarray(U[0]).size
        self.dtype = np.float32 if precision == 32 else np.float64
        host = np.full((len(U), ncell + pad), np.nan, dtype=self.dtype)
        for z, u in enumerate(U):
            host[z, :ncell] = np.asarray(u).reshape(-1)
        self.shape = host.shape
        self.ncell = ncell
        self.kstride = ncell + pad
        self.ptr = ctypes.c_void_p()
        assert hip().hipMalloc(ctypes.byref(self.ptr), host.nbytes) == 0
        assert hip().hipMemcpy(self.ptr, host.ctypes.data, host.nbytes, H2D) == 0
        assert hip().hipDeviceSynchronize() == 0

    def kinds(self):
        """Device addresses of the kinds."""
        isz = np.dtype(self.dtype).itemsize
        return [self.ptr.value + z * self.kstride * isz for z in range(self.shape[0])]

    def read(self):
        host = np.empty(self.shape, dtype=self.dtype)
        assert hip().hipMemcpy(host.ctypes.data, self.ptr, host.nbytes, D2H) == 0
        return [host[z, :self.ncell].copy() for z in range(self.shape[0])], host[:, self.ncell:].copy()

    def free(self):
        assert hip().hipFree(self.ptr) == 0


class PinnedBuffer:
    """Page-locked host memory (hipHostMalloc) seen as a numpy array."""

    def __init__(self, nbytes):
        self.ptr = ctypes.c_void_p()
        assert hip().hipHostMalloc(ctypes.byref(self.ptr), nbytes, 0) == 0
        self.nbytes = nbytes

    def array(self, dtype, count):
        buf = (ctypes.c_char * self.nbytes).from_address(self.ptr.value)
        return np.frombuffer(buf, dtype=dtype, count=count)

    def free(self):
        assert hip().hipHostFree(self.ptr) == 0
