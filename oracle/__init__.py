"""ctypes loader for the EDGE oracle (oracle/libhx_oracle.so).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only tests/, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It imports
nothing from paper_2503_10855_amd; the product path never imports it.

The stage definitions (O1..O8) and the reading of the paper they rest on are
in oracle/hxo.h; SRAD's (S1..S3) in oracle/hxo_srad.h.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64


def lib():
    """Load (building first if absent) the oracle shared library.  The
    environment variable HXO_ORACLE_LIB names another build to load instead
    (the mutation tests load deliberately broken copies this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("HXO_ORACLE_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        L.hxo_gauss_weights.argtypes = [ctypes.c_int32, ctypes.c_double, _f64p]
        L.hxo_blur.argtypes = [_f32p, _i64, _i64, _i64, ctypes.c_int32,
                               ctypes.c_double, _f64p]
        L.hxo_laplacian.argtypes = [_f64p, _i64, _i64, _f64p]
        L.hxo_zero_crossing.argtypes = [_f64p, _i64, _i64, _u8p]
        L.hxo_sobel.argtypes = [_f64p, _i64, _i64, _f64p]
        L.hxo_max.argtypes = [_f64p, _i64]
        L.hxo_max.restype = ctypes.c_double
        L.hxo_threshold.argtypes = [_u8p, _f64p, _i64, _i64, ctypes.c_double,
                                    _u8p, _i64]
        L.hxo_edge_detect.argtypes = [_f32p, _i64, _i64, _i64, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_double, _u8p,
                                      _i64, _f64p, _f64p, _f64p, _u8p, _f64p]
        L.hxo_edge_detect_many.argtypes = [
            ctypes.c_int32, ctypes.POINTER(_f32p), ctypes.POINTER(_i64),
            ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int32,
            ctypes.c_double, ctypes.c_double, ctypes.POINTER(_u8p),
            ctypes.POINTER(_i64), _f64p, ctypes.c_int32]
        L.hxo_srad_stats.argtypes = [_f64p, _i64, _i64, _f64p, _f64p, _f64p]
        L.hxo_srad_coeff.argtypes = [_f64p, _i64, _i64, ctypes.c_double, _f64p]
        L.hxo_srad_update.argtypes = [_f64p, _f64p, _i64, _i64, ctypes.c_double, _f64p]
        L.hxo_srad.argtypes = [_f32p, _i64, _i64, _i64, ctypes.c_int32, ctypes.c_double,
                               _f64p, _f64p]
        for name in ("hxo_gauss_weights", "hxo_blur", "hxo_laplacian",
                     "hxo_zero_crossing", "hxo_sobel", "hxo_threshold",
                     "hxo_edge_detect", "hxo_edge_detect_many", "hxo_srad_stats",
                     "hxo_srad_coeff", "hxo_srad_update", "hxo_srad"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments")


def _img2d(img):
    img = np.asarray(img)
    if img.dtype != np.float32 or img.ndim != 2:
        raise TypeError("oracle input must be a 2-D float32 array")
    if img.strides[1] != 4 or img.strides[0] % 4:
        img = np.ascontiguousarray(img)
    return img, img.strides[0] // 4


def gauss_weights(ksize, sigma):
    """O1: normalised sampled Gaussian of length ksize."""
    g = np.zeros(max(ksize, 1), np.float64)
    _check(lib().hxo_gauss_weights(ksize, sigma, _p(g, _f64p)), "weights")
    return g


def blur(img, ksize=5, sigma=1.0):
    """O2+O3: direct 2-D clamped Gaussian sum, fp64."""
    img, pitch = _img2d(img)
    H, W = img.shape
    B = np.empty((H, W), np.float64)
    _check(lib().hxo_blur(_p(img, _f32p), H, W, pitch, ksize, sigma,
                          _p(B, _f64p)), "blur")
    return B


def laplacian(B):
    """O4 on a dense fp64 image."""
    B = np.ascontiguousarray(B, np.float64)
    L = np.empty_like(B)
    _check(lib().hxo_laplacian(_p(B, _f64p), *B.shape, _p(L, _f64p)),
           "laplacian")
    return L


def zero_crossing(L):
    """O5 on a dense fp64 image; returns uint8 in {0,1}."""
    L = np.ascontiguousarray(L, np.float64)
    Z = np.empty(L.shape, np.uint8)
    _check(lib().hxo_zero_crossing(_p(L, _f64p), *L.shape, _p(Z, _u8p)),
           "zero_crossing")
    return Z


def sobel(B):
    """O6: Sobel magnitude G of a dense fp64 image."""
    B = np.ascontiguousarray(B, np.float64)
    G = np.empty_like(B)
    _check(lib().hxo_sobel(_p(B, _f64p), *B.shape, _p(G, _f64p)), "sobel")
    return G


def max_reduce(G):
    """O7: sequential max."""
    G = np.ascontiguousarray(G, np.float64).ravel()
    return float(lib().hxo_max(_p(G, _f64p), G.size))


def threshold(Z, G, tau):
    """O8: mask = Z == 1 and G > tau."""
    Z = np.ascontiguousarray(Z, np.uint8)
    G = np.ascontiguousarray(G, np.float64)
    H, W = G.shape
    m = np.empty((H, W), np.uint8)
    _check(lib().hxo_threshold(_p(Z, _u8p), _p(G, _f64p), H, W, tau,
                               _p(m, _u8p), W), "threshold")
    return m


def edge_detect(img, ksize=5, sigma=1.0, theta=0.1, stages=False):
    """O1..O8 for one image.

    Returns a dict with 'mask' (uint8 HxW), 'M' (float), and, when stages is
    true, the fp64 stage images 'B', 'L', 'G' and the uint8 'Z'.
    """
    img, pitch = _img2d(img)
    H, W = img.shape
    mask = np.empty((H, W), np.uint8)
    M = ctypes.c_double(0.0)
    out = {}
    if stages:
        B = np.empty((H, W), np.float64)
        L = np.empty((H, W), np.float64)
        Z = np.empty((H, W), np.uint8)
        G = np.empty((H, W), np.float64)
        ptrs = (_p(B, _f64p), _p(L, _f64p), _p(Z, _u8p), _p(G, _f64p))
        out.update(B=B, L=L, Z=Z, G=G)
    else:
        ptrs = (None, None, None, None)
    _check(lib().hxo_edge_detect(_p(img, _f32p), H, W, pitch, ksize, sigma,
                                 theta, _p(mask, _u8p), W, ctypes.byref(M),
                                 *ptrs), "edge_detect")
    out.update(mask=mask, M=M.value)
    return out


def edge_detect_many(imgs, ksize=5, sigma=1.0, theta=0.1, nthreads=1):
    """O1..O8 for a list of images, one image per worker thread.

    Returns (masks, Ms).  Identical to calling edge_detect on each image.
    """
    n = len(imgs)
    arrs = [_img2d(a) for a in imgs]
    masks = [np.empty(a.shape, np.uint8) for a, _ in arrs]
    Ms = np.zeros(n, np.float64)
    I = (_f32p * n)(*[_p(a, _f32p) for a, _ in arrs])
    Hs = (_i64 * n)(*[a.shape[0] for a, _ in arrs])
    Ws = (_i64 * n)(*[a.shape[1] for a, _ in arrs])
    Ps = (_i64 * n)(*[p for _, p in arrs])
    Mk = (_u8p * n)(*[_p(m, _u8p) for m in masks])
    MP = (_i64 * n)(*[m.shape[1] for m in masks])
    _check(lib().hxo_edge_detect_many(n, I, Hs, Ws, Ps, ksize, sigma, theta,
                                      Mk, MP, _p(Ms, _f64p), nthreads),
           "edge_detect_many")
    return masks, Ms


# ---------------------------------------------------------------- SRAD --
def _dense64(J):
    J = np.ascontiguousarray(J, dtype=np.float64)
    if J.ndim != 2:
        raise TypeError("SRAD oracle input must be 2-D")
    return J


def srad_stats(J):
    """S1 on a 2-D array: (q0^2, mean, var), in fp64."""
    J = _dense64(J)
    q, m, v = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().hxo_srad_stats(_p(J, _f64p), J.shape[0], J.shape[1], ctypes.byref(q),
                                ctypes.byref(m), ctypes.byref(v)), "srad_stats")
    return q.value, m.value, v.value


def srad_coeff(J, q0sqr):
    """S2: the diffusion coefficient c of every pixel."""
    J = _dense64(J)
    c = np.empty_like(J)
    _check(lib().hxo_srad_coeff(_p(J, _f64p), J.shape[0], J.shape[1], q0sqr, _p(c, _f64p)),
           "srad_coeff")
    return c


def srad_update(J, c, lam):
    """S3: J + lambda/4 * D."""
    J, c = _dense64(J), _dense64(c)
    out = np.empty_like(J)
    _check(lib().hxo_srad_update(_p(J, _f64p), _p(c, _f64p), J.shape[0], J.shape[1], lam,
                                 _p(out, _f64p)), "srad_update")
    return out


def srad(img, niter, lam):
    """niter SRAD iterations of an fp32 image: (J after them, q0^2 of each)."""
    a, pitch = _img2d(img)
    out = np.empty(a.shape, np.float64)
    q = np.zeros(max(niter, 1), np.float64)
    _check(lib().hxo_srad(_p(a, _f32p), a.shape[0], a.shape[1], pitch, niter, lam,
                          _p(out, _f64p), _p(q, _f64p)), "srad")
    return out, q[:niter]
