"""ctypes binding of ``libirfilter.so`` (declared in ``include/irfilter.h``).

Argument marshalling only: every step of the filter runs in the library's HIP
kernels.  Functions take torch CUDA tensors (torch provides device memory and
streams) and pass their data pointers, row pitches and the current stream to the
C entry points of the same name.  A 2-D tensor is one frame ``[H, W]`` whose row
pitch is ``stride(0) * element_size()``; a 3-D tensor ``[N, H, W]`` is a stack.
Pixel types: ``torch.uint8`` and ``torch.uint16`` (``torch.int16`` is accepted
as raw 16-bit storage and filtered as unsigned).

If the shared library has not been built, every call raises
``LibraryNotBuilt``: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libirfilter.so")

IRF_U8 = 1
IRF_U16 = 2

STATUS = {
    0: "IRF_OK", -1: "IRF_ERR_NULL", -2: "IRF_ERR_DIMS", -3: "IRF_ERR_PITCH", -4: "IRF_ERR_DTYPE",
    -5: "IRF_ERR_WINDOW", -6: "IRF_ERR_PASSES", -7: "IRF_ERR_ALIAS", -8: "IRF_ERR_HIP",
    -9: "IRF_ERR_NOMEM", -10: "IRF_ERR_CAPACITY", -11: "IRF_ERR_TUNING",
}

# name -> (restype, argtypes); mirrors include/irfilter.h
_vp, _sz, _i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
SIGNATURES = {
    "ir_filter_detect": (_i32, [_vp, _sz, _vp, _sz, _i32, _i32, _i32, _i32, _vp, _vp]),
    "ir_filter_detect_directional": (_i32, [_vp, _sz, _vp, _sz, _i32, _i32, _i32, _vp, _vp]),
    "ir_filter_median": (_i32, [_vp, _sz, _vp, _sz, _vp, _sz, _i32, _i32, _i32, _i32, _vp]),
    "ir_filter_run": (_i32, [_vp, _sz, _vp, _sz, _i32, _i32, _i32, _i32, _i32, _vp, _sz, _vp, _vp]),
    "ir_filter_run_noalloc": (_i32, [_vp, _sz, _vp, _sz, _i32, _i32, _i32, _i32, _i32, _vp, _vp]),
    "ir_filter_run_frames": (_i32, [_vp, _sz, _sz, _vp, _sz, _sz, _i32, _i32, _i32, _i32, _i32, _i32,
                                    _vp, _sz, _sz, _vp, _vp]),
    "ir_filter_plan_create": (_i32, [ctypes.POINTER(ctypes.c_void_p), _i32, _i32, ctypes.c_uint]),
    "ir_filter_run_batch": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "ir_filter_plan_destroy": (None, [_vp]),
    "ir_filter_frame_tiles": (_i32, [_i32, _i32]),
    "ir_filter_status_string": (ctypes.c_char_p, [_i32]),
    "ir_filter_version": (_i32, []),
    "ir_filter_get_tuning": (_i32, [_i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "ir_filter_set_tuning": (_i32, [_i32, _i32, _i32, _i32]),
    "ir_filter_get_fusion": (_i32, [_i32, _i32, ctypes.POINTER(_i32)]),
    "ir_filter_set_fusion": (_i32, [_i32, _i32, _i32]),
    "ir_filter_resolve_fusion": (_i32, [_i32, _i32, _i32, _i32, ctypes.POINTER(_i32)]),
    "ir_filter_set_batch_threads": (_i32, [_i32]),
    "ir_filter_get_batch_threads": (_i32, []),
    "ir_filter_plan_frame_tiles": (_i32, [_vp, _i32, _i32]),
    "ir_filter_server_create": (_i32, [ctypes.POINTER(ctypes.c_void_p), _sz, _i32, _i32, _i32, ctypes.c_uint]),
    "ir_filter_server_register_stream": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32]),
    "ir_filter_server_submit": (_i32, [_vp, _vp, _i32]),
    "ir_filter_server_poll": (_i32, [_vp]),
    "ir_filter_server_run": (_i32, [_vp]),
    "ir_filter_server_completed": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double), _i32]),
    "ir_filter_server_now": (ctypes.c_double, [_vp]),
    "ir_filter_server_steps": (_i32, [_vp]),
    "ir_filter_server_arena_used": (_sz, [_vp]),
    "ir_filter_server_resident_bytes": (_sz, [_vp]),
    "ir_filter_server_destroy": (None, [_vp]),
}

IRF_SELECT_NETWORK = 1
IRF_SELECT_BISECT = 2
IRF_SELECT_GROUP = 3
IRF_SELECT_HIST = 4
SELECT_NAMES = {IRF_SELECT_NETWORK: "network", IRF_SELECT_BISECT: "bisect", IRF_SELECT_GROUP: "group",
                IRF_SELECT_HIST: "hist"}
MAX_WINDOW = 63        # single-frame and stack entry points
MAX_BATCH_WINDOW = 31  # batch plans and the server


IRF_PLAN_GRAPH = 1


class IrfFrame(ctypes.Structure):
    """Mirror of ``irf_frame``."""
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("src_pitch", ctypes.c_size_t),
                ("dst_pitch", ctypes.c_size_t), ("width", ctypes.c_int), ("height", ctypes.c_int),
                ("dtype", ctypes.c_int), ("window", ctypes.c_int)]


class IrfRequest(ctypes.Structure):
    """Mirror of ``irf_request``."""
    _fields_ = [("id", ctypes.c_uint64), ("host_src", ctypes.c_void_p), ("host_dst", ctypes.c_void_p),
                ("src_pitch", ctypes.c_size_t), ("dst_pitch", ctypes.c_size_t), ("width", ctypes.c_int),
                ("height", ctypes.c_int), ("dtype", ctypes.c_int), ("window", ctypes.c_int),
                ("stream_id", ctypes.c_int), ("arrival", ctypes.c_double)]


class LibraryNotBuilt(ImportError):
    pass


class IrfError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({status_string(status)})")


_lib = None


def load(path: Optional[str] = None):
    """Load the library (once) and declare its signatures."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise LibraryNotBuilt(f"{p} is missing: run paper_1201_3972_amd.build.build() first")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().ir_filter_status_string(status).decode()
    except LibraryNotBuilt:
        return STATUS.get(status, "unknown")


def _check(fn: str, status: int) -> None:
    if status != 0:
        raise IrfError(fn, status)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.uint8:
        return IRF_U8
    if t.dtype in (torch.uint16, torch.int16):
        return IRF_U16
    raise TypeError(f"unsupported pixel type {t.dtype}; use uint8 or uint16")


def _frame(t, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D [H, W]")
    if t.stride(1) != 1:
        raise ValueError(f"{name} rows must be contiguous")
    return t.data_ptr(), t.stride(0) * t.element_size()


def _stack(t, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 3:
        raise ValueError(f"{name} must be 3-D [N, H, W]")
    if t.stride(2) != 1:
        raise ValueError(f"{name} rows must be contiguous")
    es = t.element_size()
    return t.data_ptr(), t.stride(1) * es, t.stride(0) * es


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _same(a, b, what: str):
    if a.shape != b.shape or _dtype_code(a) != _dtype_code(b):
        raise ValueError(f"{what} must match the source shape and pixel type")


def _counts(t, need: int, name: str = "flagged_count"):
    """Pointer of a device count array of at least ``need`` 64-bit entries
    (None passes through): the kernels write it with 64-bit atomics, so a host
    tensor, a narrower type or too few entries is refused here."""
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise ValueError(f"{name} must hold 64-bit integers (torch.int64 or torch.uint64)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < need:
        raise ValueError(f"{name} needs at least {need} entries, has {t.numel()}")
    return t.data_ptr()


def _mask(mask, src):
    import torch
    if mask.dtype != torch.uint8:
        raise ValueError("mask must be uint8")
    if tuple(mask.shape) != tuple(src.shape):
        raise ValueError("mask must have the source shape")


def ir_filter_detect(src, mask, window: int, flagged_count=None, stream=None) -> None:
    """Noise mask (uint8, 1 = noisy) of ``src``; optional uint64 count tensor (1 element)."""
    sp, spitch = _frame(src, "src")
    mp, mpitch = _frame(mask, "mask")
    H, W = src.shape
    _mask(mask, src)
    cp = _counts(flagged_count, 1)
    _check("ir_filter_detect", load().ir_filter_detect(sp, spitch, mp, mpitch, W, H, _dtype_code(src),
                                                       window, cp, _stream(stream)))


def ir_filter_detect_directional(src, mask, flagged_count=None, stream=None) -> None:
    """Mask of the opt-in directional detector (not the paper's detector; see
    include/irfilter.h): 1 where the pixel lies outside its two neighbours'
    range on all four lines of its 3x3 window."""
    sp, spitch = _frame(src, "src")
    mp, mpitch = _frame(mask, "mask")
    H, W = src.shape
    _mask(mask, src)
    cp = _counts(flagged_count, 1)
    _check("ir_filter_detect_directional",
           load().ir_filter_detect_directional(sp, spitch, mp, mpitch, W, H, _dtype_code(src), cp,
                                               _stream(stream)))


def ir_filter_median(src, dst, window: int, mask=None, stream=None) -> None:
    """Window median where ``mask`` != 0 (every pixel when ``mask`` is None)."""
    _same(src, dst, "dst")
    if mask is not None:
        _mask(mask, src)
    sp, spitch = _frame(src, "src")
    dp, dpitch = _frame(dst, "dst")
    mp, mpitch = (None, 0) if mask is None else _frame(mask, "mask")
    H, W = src.shape
    _check("ir_filter_median", load().ir_filter_median(sp, spitch, mp, mpitch, dp, dpitch, W, H,
                                                       _dtype_code(src), window, _stream(stream)))


def ir_filter_run(src, dst, window: int, passes: int = 1, scratch=None, flagged_count=None,
                  stream=None) -> None:
    """FNR ``passes`` times; ``flagged_count`` (uint64/int64, ``passes`` elements) is optional."""
    _same(src, dst, "dst")
    if scratch is not None:
        _same(src, scratch, "scratch")
    sp, spitch = _frame(src, "src")
    dp, dpitch = _frame(dst, "dst")
    xp, xpitch = (None, 0) if scratch is None else _frame(scratch, "scratch")
    H, W = src.shape
    cp = _counts(flagged_count, passes)
    _check("ir_filter_run", load().ir_filter_run(sp, spitch, dp, dpitch, W, H, _dtype_code(src), window,
                                                 passes, xp, xpitch, cp, _stream(stream)))


def ir_filter_run_noalloc(src, dst, window: int, passes: int = 1, flagged_count=None, stream=None) -> None:
    """``ir_filter_run`` whose intermediate passes use the library's own
    per-GPU device array (no scratch argument, nothing allocated per call);
    calls that overlap on one GPU share that array and race."""
    _same(src, dst, "dst")
    sp, spitch = _frame(src, "src")
    dp, dpitch = _frame(dst, "dst")
    H, W = src.shape
    cp = _counts(flagged_count, passes)
    _check("ir_filter_run_noalloc", load().ir_filter_run_noalloc(sp, spitch, dp, dpitch, W, H, _dtype_code(src),
                                                                 window, passes, cp, _stream(stream)))


def ir_filter_run_frames(src, dst, window: int, passes: int = 1, scratch=None, flagged_count=None,
                         stream=None) -> None:
    """FNR over a stack ``[N, H, W]``: one launch per pass, or per pair of passes
    where the library fuses two passes into one launch (see ``set_fusion``);
    results and per-pass counts are the same either way."""
    _same(src, dst, "dst")
    if scratch is not None:
        _same(src, scratch, "scratch")
    sp, spitch, sstride = _stack(src, "src")
    dp, dpitch, dstride = _stack(dst, "dst")
    xp, xpitch, xstride = (None, 0, 0) if scratch is None else _stack(scratch, "scratch")
    N, H, W = src.shape
    cp = _counts(flagged_count, passes)
    _check("ir_filter_run_frames",
           load().ir_filter_run_frames(sp, spitch, sstride, dp, dpitch, dstride, W, H, N, _dtype_code(src),
                                       window, passes, xp, xpitch, xstride, cp, _stream(stream)))


def version() -> int:
    return load().ir_filter_version()


def _dtype_arg(dtype) -> int:
    if dtype in (IRF_U8, IRF_U16):
        return dtype
    if dtype in ("u8", "uint8"):
        return IRF_U8
    if dtype in ("u16", "uint16"):
        return IRF_U16
    raise ValueError(f"pixel type {dtype!r}: use 'u8', 'u16', IRF_U8 or IRF_U16")


def get_tuning(dtype, window: int):
    """(threads, select) used by the single-size entry points for this pixel type and window."""
    t, sel = ctypes.c_int(), ctypes.c_int()
    _check("ir_filter_get_tuning", load().ir_filter_get_tuning(_dtype_arg(dtype), window, ctypes.byref(t),
                                                               ctypes.byref(sel)))
    return t.value, sel.value


def set_tuning(dtype, window: int, threads: int, select: int) -> None:
    """Set (threads, select) for a pixel type and window; (0, 0) restores the default."""
    _check("ir_filter_set_tuning", load().ir_filter_set_tuning(_dtype_arg(dtype), window, threads, select))


FUSION_AUTO = -1


def get_fusion(dtype, window: int) -> int:
    """Fusion setting of (dtype, window): the fused kernel's workgroup size,
    0 for separate launches, or FUSION_AUTO (the library's automatic choice)."""
    t = ctypes.c_int()
    _check("ir_filter_get_fusion", load().ir_filter_get_fusion(_dtype_arg(dtype), window, ctypes.byref(t)))
    return t.value


def resolve_fusion(dtype, window: int, width: int, height: int) -> int:
    """What a run of two or more passes over width x height frames uses: the
    fused workgroup size, or 0 for separate passes."""
    t = ctypes.c_int()
    _check("ir_filter_resolve_fusion", load().ir_filter_resolve_fusion(_dtype_arg(dtype), window, width, height,
                                                                       ctypes.byref(t)))
    return t.value


def set_fusion(dtype, window: int, threads: int) -> None:
    """Fuse pairs of passes with workgroups of `threads` (256 or 512), run
    passes separately (0), or leave it to the library (FUSION_AUTO, the default,
    which runs separate passes)."""
    _check("ir_filter_set_fusion", load().ir_filter_set_fusion(_dtype_arg(dtype), window, threads))


def set_batch_threads(threads: int) -> None:
    """Workgroup size of batch plans created from now on (128, 256, or 0 for the default)."""
    _check("ir_filter_set_batch_threads", load().ir_filter_set_batch_threads(threads))


def get_batch_threads() -> int:
    return load().ir_filter_get_batch_threads()


def frame_tiles(width: int, height: int) -> int:
    return load().ir_filter_frame_tiles(width, height)


class Plan:
    """Owner of an ``irf_plan``: batches of uneven frames in one persistent launch.

    ``run(items)`` takes ``(src, dst, window)`` triples of 2-D CUDA tensors (each
    frame may have its own size, pixel type and window)."""

    def __init__(self, max_frames: int, max_tiles: int, graph: bool = False):
        self._lib = load()
        self._ptr = ctypes.c_void_p()
        _check("ir_filter_plan_create",
               self._lib.ir_filter_plan_create(ctypes.byref(self._ptr), max_frames, max_tiles,
                                               IRF_PLAN_GRAPH if graph else 0))
        self.max_frames, self.max_tiles, self.graph = max_frames, max_tiles, graph

    @staticmethod
    def frames(items) -> "ctypes.Array":
        arr = (IrfFrame * len(items))()
        for i, (src, dst, window) in enumerate(items):
            _same(src, dst, "dst")
            sp, spitch = _frame(src, "src")
            dp, dpitch = _frame(dst, "dst")
            H, W = src.shape
            arr[i] = IrfFrame(sp, dp, spitch, dpitch, W, H, _dtype_code(src), window)
        return arr

    def run(self, items, flagged_counts=None, stream=None) -> None:
        self.run_frames(self.frames(items), len(items), flagged_counts, stream)

    def run_frames(self, arr, n: int, flagged_counts=None, stream=None) -> None:
        """Run prepared ``IrfFrame`` descriptors (see :meth:`frames`)."""
        if self._ptr is None:
            raise RuntimeError("plan is closed")
        cp = _counts(flagged_counts, n, "flagged_counts")
        _check("ir_filter_run_batch", self._lib.ir_filter_run_batch(self._ptr, arr, n, cp, _stream(stream)))

    def close(self) -> None:
        if self._ptr is not None and self._ptr.value:
            self._lib.ir_filter_plan_destroy(self._ptr)
        self._ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
