"""ctypes binding of libhx.so (include/hx.h).

Argument marshalling only: every step of the pipeline runs in the HIP
kernels behind the C ABI.  torch supplies device memory and streams.
Importing this module loads libhx.so and raises ImportError if it has not
been built (``python -m paper_2503_10855_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhx.so")

HX_OK, HX_E_INVALID, HX_E_NOMEM, HX_E_HIP, HX_E_UNSUPPORTED, HX_E_BUSY, \
    HX_E_PENDING, HX_E_NOT_FOUND = range(8)
PASS_AUTO, PASS_STORE, PASS_RECOMPUTE, PASS_SPECULATE = 0, 1, 2, 3
FORM_IMAGE, FORM_STAGES, FORM_BATCH, FORM_BATCH_STORE, FORM_SRAD = 1, 2, 4, 8, 16
FORM_ALL = 31
REDUCE_TREE, REDUCE_TWO_LEVEL, REDUCE_SEQUENTIAL = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [("ksize", ctypes.c_int32), ("sigma", ctypes.c_float),
                ("thresh_frac", ctypes.c_float), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("fusion_depth", ctypes.c_int32),
                ("pass_mode", ctypes.c_int32), ("max_pixels", ctypes.c_int64),
                ("max_images", ctypes.c_int64), ("forms", ctypes.c_int32),
                ("batch_contexts", ctypes.c_int32)]


class Image(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("height", ctypes.c_int64),
                ("width", ctypes.c_int64), ("src_pitch", ctypes.c_int64),
                ("mask", ctypes.c_void_p), ("mask_pitch", ctypes.c_int64)]


class Schedule(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("fusion_depth", ctypes.c_int32), ("pass_mode", ctypes.c_int32),
                ("reduce_mode", ctypes.c_int32)]

    def astuple(self):
        return (self.tile_w, self.tile_h, self.fusion_depth, self.pass_mode,
                self.reduce_mode)


class ServeParams(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32)]


_P = ctypes.c_void_p
_i32, _i64, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64

# name -> (restype, argtypes)
_SIGS = {
    "hx_pipeline_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int,
                                          ctypes.POINTER(_P)]),
    "hx_pipeline_destroy": (None, [_P]),
    "hx_edge_detect_static": (ctypes.c_int, [_P, ctypes.POINTER(Image), _P, _P]),
    "hx_autotune_batch": (ctypes.c_int, [_P, ctypes.POINTER(Image), _i32, ctypes.c_char_p,
                                         ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "hx_pipeline_memory": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(_u64)]),
    "hx_pipeline_sync": (ctypes.c_int, [_P]),
    "hx_pipeline_set_schedule": (ctypes.c_int, [_P, ctypes.POINTER(Schedule)]),
    "hx_pipeline_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "hx_pipeline_last_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "hx_pipeline_get_schedule": (ctypes.c_int, [_P, _i64, _i64,
                                                ctypes.POINTER(Schedule)]),
    "hx_edge_detect": (ctypes.c_int, [_P, ctypes.POINTER(Image), _P, _P]),
    "hx_edge_detect_batched": (ctypes.c_int, [_P, ctypes.POINTER(Image), _i32,
                                              _P, _P]),
    "hx_edge_detect_stages": (ctypes.c_int, [_P, ctypes.POINTER(Image), _P, _P,
                                             _P, _P, _P, _P]),
    "hx_autotune": (ctypes.c_int, [_P, _i64, _i64, ctypes.c_char_p]),
    "hx_autotune_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "hx_serve_create": (ctypes.c_int, [_P, ctypes.POINTER(ServeParams), _P,
                                       ctypes.c_size_t, ctypes.POINTER(_P)]),
    "hx_serve_submit": (ctypes.c_int, [_P, _P, _i64, _i64, _i64, ctypes.c_double,
                                       ctypes.POINTER(_u64)]),
    "hx_serve_poll": (ctypes.c_int, [_P, _u64, _P, _i64,
                                     ctypes.POINTER(ctypes.c_double)]),
    "hx_serve_poll_timed": (ctypes.c_int, [_P, _u64, _P, _i64,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
    "hx_serve_now": (ctypes.c_double, [_P]),
    "hx_serve_reserve": (ctypes.c_int, [_P, _i64, _i64, ctypes.POINTER(_P),
                                        ctypes.POINTER(_u64)]),
    "hx_serve_commit": (ctypes.c_int, [_P, _u64, ctypes.c_double]),
    "hx_serve_cancel": (ctypes.c_int, [_P, _u64]),
    "hx_serve_view": (ctypes.c_int, [_P, _u64, ctypes.POINTER(_P),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "hx_serve_release": (ctypes.c_int, [_P, _u64]),
    "hx_srad": (ctypes.c_int, [_P, _P, _i64, _i64, _i64, _i32, ctypes.c_float, _i32, _P,
                               _P]),
    "hx_schedule_compile": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(Schedule)]),
    "hx_schedule_to_text": (ctypes.c_int, [ctypes.POINTER(Schedule), ctypes.c_char_p,
                                           ctypes.c_size_t]),
    "hx_serve_stats": (ctypes.c_int, [_P, ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                      ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "hx_serve_destroy": (ctypes.c_int, [_P]),
    "hx_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "hx_last_error": (ctypes.c_char_p, []),
}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2503_10855_amd/build.py")
_lib = ctypes.CDLL(LIB_PATH)
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class HxError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.hx_last_error().decode(errors="replace")
        name = _lib.hx_status_str(status).decode()
        super().__init__(f"{where}: {name}: {msg}")


def _check(st, where):
    if st != HX_OK:
        raise HxError(st, where)


def raw():
    """The loaded ctypes library (for ABI-level tests)."""
    return _lib


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def image_desc(src: torch.Tensor, mask: torch.Tensor) -> Image:
    if src.dtype != torch.float32 or src.dim() != 2 or src.stride(1) != 1:
        raise TypeError("src must be a 2-D float32 tensor with unit column stride")
    if mask.dtype != torch.uint8 or mask.dim() != 2 or mask.stride(1) != 1:
        raise TypeError("mask must be a 2-D uint8 tensor with unit column stride")
    if tuple(mask.shape) != tuple(src.shape):
        raise ValueError("mask and src shapes differ")
    if not (src.is_cuda and mask.is_cuda):
        raise ValueError("src and mask must be device tensors")
    H, W = src.shape
    return Image(src.data_ptr(), H, W, src.stride(0), mask.data_ptr(), mask.stride(0))


def compile_schedule(text):
    """Schedule text -> (tile_w, tile_h, fusion_depth, pass_mode,
    reduce_mode); HxError if it does not parse, apply or lower."""
    s = Schedule()
    _check(_lib.hx_schedule_compile(text.encode(), ctypes.byref(s)), "hx_schedule_compile")
    return s.astuple()


def schedule_text(sched):
    """The canonical schedule text of a (tile_w, tile_h, depth, pass, reduce)."""
    s = Schedule(*sched)
    buf = ctypes.create_string_buffer(1024)
    _check(_lib.hx_schedule_to_text(ctypes.byref(s), buf, len(buf)), "hx_schedule_to_text")
    return buf.value.decode()


class Pipeline:
    """An hx_pipeline: constants, dynamic-constant sizes and scratch."""

    def __init__(self, ksize=5, sigma=1.0, theta=0.1, max_pixels=1 << 25,
                 max_images=1024, device=0, tile_w=0, tile_h=0, fusion_depth=0,
                 pass_mode=0, forms=0, batch_contexts=0):
        self.params = Params(ksize, sigma, theta, tile_w, tile_h, fusion_depth,
                             pass_mode, max_pixels, max_images, forms, batch_contexts)
        self.device = device
        h = _P()
        _check(_lib.hx_pipeline_create(ctypes.byref(self.params), device,
                                       ctypes.byref(h)), "hx_pipeline_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.hx_pipeline_destroy(self._h)
            self._h = None

    def memory(self):
        """(device bytes, pinned host bytes, allocation calls) the pipeline
        holds; allocation calls stay constant after creation."""
        d, h, n = ctypes.c_size_t(), ctypes.c_size_t(), _u64()
        _check(_lib.hx_pipeline_memory(self._h, ctypes.byref(d), ctypes.byref(h),
                                       ctypes.byref(n)), "hx_pipeline_memory")
        return d.value, h.value, n.value

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, tile_w=None, tile_h=None, fusion_depth=None,
                     pass_mode=PASS_STORE, reduce_mode=REDUCE_TREE):
        """Force a schedule; with no arguments restore automatic choice."""
        if tile_w is None:
            _check(_lib.hx_pipeline_set_schedule(self._h, None), "set_schedule")
            return
        s = Schedule(tile_w, tile_h, fusion_depth, pass_mode, reduce_mode)
        _check(_lib.hx_pipeline_set_schedule(self._h, ctypes.byref(s)),
               "set_schedule")

    def set_schedule_text(self, text):
        """Force the schedule a schedule program compiles to."""
        self.set_schedule(*compile_schedule(text))

    def schedule(self, H, W):
        s = Schedule()
        _check(_lib.hx_pipeline_get_schedule(self._h, H, W, ctypes.byref(s)),
               "get_schedule")
        return s.astuple()

    def sync(self):
        _check(_lib.hx_pipeline_sync(self._h), "hx_pipeline_sync")

    def set_timing(self, enable=True):
        _check(_lib.hx_pipeline_set_timing(self._h, 1 if enable else 0), "set_timing")

    def last_timing(self):
        """(reset, pass 1, pass 2, pass 0) durations in ms of the last
        batched call made in timing mode (waits for it); pass 0 runs under
        SPECULATE only and is 0 otherwise."""
        ms = (ctypes.c_float * 4)()
        _check(_lib.hx_pipeline_last_timing(self._h, ms), "last_timing")
        return tuple(ms)

    def edge_detect(self, src, mask=None, dmax=None, stream=None):
        if mask is None:
            mask = torch.empty(src.shape, dtype=torch.uint8, device=src.device)
        d = image_desc(src, mask)
        _check(_lib.hx_edge_detect(self._h, ctypes.byref(d),
                                   dmax.data_ptr() if dmax is not None else None,
                                   _stream(stream)), "hx_edge_detect")
        return mask

    def edge_detect_static(self, src, mask=None, dmax=None, stream=None):
        """hx_edge_detect_static: the per-image fused form with its scratch
        in the library's fixed device array (no allocation; calls that
        overlap on one GPU race)."""
        if mask is None:
            mask = torch.empty(src.shape, dtype=torch.uint8, device=src.device)
        d = image_desc(src, mask)
        _check(_lib.hx_edge_detect_static(self._h, ctypes.byref(d),
                                          dmax.data_ptr() if dmax is not None else None,
                                          _stream(stream)), "hx_edge_detect_static")
        return mask

    def edge_detect_batched(self, srcs, masks=None, dmax=None, stream=None):
        if masks is None:
            masks = [torch.empty(s.shape, dtype=torch.uint8, device=s.device)
                     for s in srcs]
        n = len(srcs)
        arr = (Image * n)(*[image_desc(s, m) for s, m in zip(srcs, masks)])
        _check(_lib.hx_edge_detect_batched(
            self._h, arr, n, dmax.data_ptr() if dmax is not None else None,
            _stream(stream)), "hx_edge_detect_batched")
        return masks

    def prepare_batch(self, srcs, masks=None, dmax=None):
        """Marshal the descriptors of a batch once; the returned object's
        run() makes the batched call without rebuilding them."""
        return PreparedBatch(self, srcs, masks, dmax)

    def edge_detect_stages(self, src, stream=None, stages=("B", "L", "Z", "G")):
        """The stage hook: a dict of device tensors B, L, Z, G (those named in
        `stages`), M and mask.  Depth 1 by default; under a forced depth-2
        (depth-3) schedule L (B) is kept on chip and cannot be asked for."""
        H, W = src.shape
        dev = src.device
        out = dict(M=torch.empty(1, dtype=torch.float32, device=dev),
                   mask=torch.empty((H, W), dtype=torch.uint8, device=dev))
        for k in stages:
            out[k] = torch.empty((H, W), dtype=torch.uint8 if k == "Z" else torch.float32,
                                 device=dev)
        d = image_desc(src, out["mask"])
        ptr = lambda k: out[k].data_ptr() if k in out else None  # noqa: E731
        _check(_lib.hx_edge_detect_stages(
            self._h, ctypes.byref(d), ptr("B"), ptr("L"), ptr("Z"), ptr("G"),
            out["M"].data_ptr(), _stream(stream)), "hx_edge_detect_stages")
        return out

    def srad(self, J, niter, lam=0.5, fused=True, q_log=None, stream=None):
        """niter SRAD iterations on the fp32 device tensor J (H, W), in
        place; q_log (float64 device tensor of niter, optional) receives
        q0^2 of each iteration."""
        assert J.dtype == torch.float32 and J.dim() == 2 and J.stride(1) == 1
        _check(_lib.hx_srad(self._h, J.data_ptr(), J.shape[0], J.shape[1], J.stride(0),
                            niter, lam, 1 if fused else 0,
                            q_log.data_ptr() if q_log is not None else None,
                            _stream(stream)), "hx_srad")
        return J

    def autotune(self, H, W, cache_path=None):
        _check(_lib.hx_autotune(self._h, H, W,
                                cache_path.encode() if cache_path else None),
               "hx_autotune")
        return self.schedule(H, W)

    def autotune_batch(self, srcs, masks=None, cache_path=None):
        """Time the batched call on this batch under every candidate tile
        height and pass structure; keep the fastest for batches of its class.
        Returns (tile_h, pass_mode)."""
        if masks is None:
            masks = [torch.empty(s.shape, dtype=torch.uint8, device=s.device) for s in srcs]
        n = len(srcs)
        arr = (Image * n)(*[image_desc(s, m) for s, m in zip(srcs, masks)])
        th, pm = _i32(), _i32()
        _check(_lib.hx_autotune_batch(self._h, arr, n,
                                      cache_path.encode() if cache_path else None,
                                      ctypes.byref(th), ctypes.byref(pm)), "hx_autotune_batch")
        return th.value, pm.value

    def autotune_load(self, cache_path):
        _check(_lib.hx_autotune_load(self._h, cache_path.encode()),
               "hx_autotune_load")


class PreparedBatch:
    """A batch whose C descriptors are built once (see Pipeline.prepare_batch).
    The tensors are kept alive by this object."""

    def __init__(self, pipeline, srcs, masks=None, dmax=None):
        if masks is None:
            masks = [torch.empty(s.shape, dtype=torch.uint8, device=s.device)
                     for s in srcs]
        self.pipeline, self.srcs, self.masks, self.dmax = pipeline, srcs, masks, dmax
        self.n = len(srcs)
        self.arr = (Image * self.n)(*[image_desc(s, m) for s, m in zip(srcs, masks)])
        self.dmax_ptr = dmax.data_ptr() if dmax is not None else None

    def run(self, stream=None):
        _check(_lib.hx_edge_detect_batched(self.pipeline.handle, self.arr, self.n,
                                           self.dmax_ptr, _stream(stream)),
               "hx_edge_detect_batched")
        return self.masks


class Server:
    """An hx_server: continuous-batching request loop over a device arena."""

    def __init__(self, pipeline: Pipeline, hbm_budget, streams=4, max_batch=64,
                 arena: torch.Tensor = None):
        if arena is None:
            # The pipeline's own scratch counts against the budget; the arena
            # holds the rest (hx_serve_create refuses a budget below it).
            rest = max(hbm_budget - pipeline.memory()[0], 1 << 12)
            arena = torch.empty(rest, dtype=torch.uint8, device=f"cuda:{pipeline.device}")
        self.arena = arena
        self.pipeline = pipeline
        self.sp = ServeParams(hbm_budget, streams, max_batch)
        h = _P()
        _check(_lib.hx_serve_create(pipeline.handle, ctypes.byref(self.sp),
                                    arena.data_ptr(), arena.numel(),
                                    ctypes.byref(h)), "hx_serve_create")
        self._h = h

    def now(self):
        return _lib.hx_serve_now(self._h)

    def submit(self, img, arrival=None):
        """img: host float32 numpy array (H, W); a row-strided view (a crop)
        is passed with its pitch, without a copy.  Returns a ticket; raises
        HxError (status HX_E_PENDING) if the pinned pool is full until
        finished requests are polled."""
        t = self.try_submit(img, arrival)
        if t is None:
            raise HxError(HX_E_PENDING, "hx_serve_submit")
        return t

    def try_submit(self, img, arrival=None):
        """submit(), but None while the pinned pool is full."""
        import numpy as np
        a = img
        if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.ndim == 2
                and a.strides[1] == 4 and a.strides[0] % 4 == 0
                and a.strides[0] >= 4 * a.shape[1]):
            a = np.ascontiguousarray(a, dtype=np.float32)
        t = _u64()
        st = _lib.hx_serve_submit(self._h, a.ctypes.data, a.shape[0], a.shape[1],
                                  a.strides[0] // 4,
                                  self.now() if arrival is None else arrival,
                                  ctypes.byref(t))
        if st == HX_E_PENDING:
            return None
        _check(st, "hx_serve_submit")
        return t.value

    def poll(self, ticket, shape, out=None):
        """Returns (mask, latency_s) when done, or None while pending.  `out`
        (uint8, C-contiguous, of `shape`) receives the mask if given."""
        r = self.poll_timed(ticket, shape, out)
        return None if r is None else r[:2]

    def poll_timed(self, ticket, shape, out=None):
        """Returns (mask, latency_s, service_s) when done, or None while
        pending; service_s runs from the batch's launch to the mask on the host."""
        import numpy as np
        m = np.empty(shape, dtype=np.uint8) if out is None else out
        if m.shape != tuple(shape) or m.dtype != np.uint8 or not m.flags.c_contiguous:
            raise ValueError("out must be a C-contiguous uint8 array of the request's shape")
        lat = ctypes.c_double()
        svc = ctypes.c_double()
        st = _lib.hx_serve_poll_timed(self._h, ticket, m.ctypes.data, shape[1],
                                      ctypes.byref(lat), ctypes.byref(svc))
        if st == HX_E_PENDING:
            return None
        _check(st, "hx_serve_poll_timed")
        return m, lat.value, svc.value

    def reserve(self, shape):
        """Zero-copy submission: (ticket, slot), slot a float32 numpy array
        of `shape` over the server's pinned pool, to be filled by the
        caller and then queued with commit(ticket); None while the pool is
        full."""
        import numpy as np
        h, w = shape
        ptr, t = _P(), _u64()
        st = _lib.hx_serve_reserve(self._h, h, w, ctypes.byref(ptr), ctypes.byref(t))
        if st == HX_E_PENDING:
            return None
        _check(st, "hx_serve_reserve")
        buf = (ctypes.c_float * (h * w)).from_address(ptr.value)
        return t.value, np.ctypeslib.as_array(buf).reshape(h, w)

    def commit(self, ticket, arrival=None):
        """Queue a reserved slot (the slot must not be written afterwards)."""
        _check(_lib.hx_serve_commit(self._h, ticket,
                                    self.now() if arrival is None else arrival),
               "hx_serve_commit")

    def cancel(self, ticket):
        _check(_lib.hx_serve_cancel(self._h, ticket), "hx_serve_cancel")

    def view(self, ticket, shape):
        """Zero-copy collection: (mask, latency_s, service_s) with mask a
        read-only uint8 numpy view of the pinned pool, valid until
        release(ticket); None while pending."""
        import numpy as np
        h, w = shape
        ptr = _P()
        lat, svc = ctypes.c_double(), ctypes.c_double()
        st = _lib.hx_serve_view(self._h, ticket, ctypes.byref(ptr), ctypes.byref(lat),
                                ctypes.byref(svc))
        if st == HX_E_PENDING:
            return None
        _check(st, "hx_serve_view")
        buf = (ctypes.c_uint8 * (h * w)).from_address(ptr.value)
        m = np.ctypeslib.as_array(buf).reshape(h, w)
        m.flags.writeable = False
        return m, lat.value, svc.value

    def release(self, ticket):
        _check(_lib.hx_serve_release(self._h, ticket), "hx_serve_release")

    def stats(self):
        v = [_u64() for _ in range(4)]
        _check(_lib.hx_serve_stats(self._h, *[ctypes.byref(x) for x in v]),
               "hx_serve_stats")
        return dict(completed=v[0].value, batches=v[1].value, pixels=v[2].value,
                    peak_bytes=v[3].value)

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.hx_serve_destroy(self._h), "hx_serve_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
