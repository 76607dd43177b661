"""The tuned multi-core fp32 CPU implementation of EDGE (the comparison
point on the host's cores; not the oracle, which stays plain fp64)."""
import ctypes
import os

import numpy as np

from .build import LIB

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built (python -m paper_2503_10855_amd.cpu.build)")
        _lib = ctypes.CDLL(LIB)
        _lib.hx_cpu_edge_detect_many.restype = ctypes.c_int
    return _lib


def edge_detect_many(imgs, ksize=5, sigma=1.0, theta=0.1, nthreads=1):
    """Masks (uint8) and M of each float32 image, on nthreads host threads."""
    n = len(imgs)
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in imgs]
    masks = [np.empty(a.shape, np.uint8) for a in arrs]
    P = ctypes.POINTER(ctypes.c_float)
    U = ctypes.POINTER(ctypes.c_uint8)
    I64 = ctypes.c_int64 * n
    src = (P * n)(*[a.ctypes.data_as(P) for a in arrs])
    dst = (U * n)(*[m.ctypes.data_as(U) for m in masks])
    Ms = np.zeros(n, np.float64)
    rc = lib().hx_cpu_edge_detect_many(
        n, src, I64(*[a.shape[0] for a in arrs]), I64(*[a.shape[1] for a in arrs]),
        I64(*[a.shape[1] for a in arrs]), dst, I64(*[a.shape[1] for a in arrs]),
        ctypes.c_int(ksize), ctypes.c_double(sigma), ctypes.c_double(theta),
        ctypes.c_int(nthreads), Ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("hx_cpu_edge_detect_many rejected its arguments")
    return masks, Ms
