"""CPU oracle of the FNR filter -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never loads it.  It wraps ``fnr_oracle.c``
(plain C, built with gcc) through ctypes and takes/returns numpy arrays.

Every function follows the paper's definition (Section 3.3 detector with
Eq. 3a/3b and Step 2, Section 3.4 median replacement by introsort, Section 4
whole-image passes); the C file states the readings taken where the paper is
silent.
"""

from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fnr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class SortStats(ctypes.Structure):
    _fields_ = [("scans", ctypes.c_uint64), ("sorts", ctypes.c_uint64), ("partitions", ctypes.c_uint64),
                ("heapsorts", ctypes.c_uint64), ("insertions", ctypes.c_uint64)]


_lib = None


def _configure(lib):
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    lib.oracle_introsort.argtypes = [vp, i32, vp]
    lib.oracle_introsort.restype = None
    lib.oracle_introsort_depth.argtypes = [vp, i32, i32, vp]
    lib.oracle_introsort_depth.restype = None
    lib.oracle_window.argtypes = [vp, sz, i32, i32, i32, i32, i32, i32, vp]
    lib.oracle_window.restype = i32
    lib.oracle_detect.argtypes = [vp, sz, vp, sz, i32, i32, i32, i32, vp]
    lib.oracle_detect.restype = i32
    lib.oracle_median.argtypes = [vp, sz, vp, sz, vp, sz, i32, i32, i32, i32, vp, vp]
    lib.oracle_median.restype = i32
    lib.oracle_fnr.argtypes = [vp, sz, vp, sz, i32, i32, i32, i32, i32, vp, vp]
    lib.oracle_fnr.restype = i32
    lib.oracle_detect_directional.argtypes = [vp, sz, vp, sz, i32, i32, i32, vp]
    lib.oracle_detect_directional.restype = i32
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Run the wrappers against another build of the oracle source (the
    mutation tests use this to check that the pins catch planted mistakes)."""
    global _lib
    saved = _load()
    _lib = _configure(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def compile_source(source: str, out_path: str) -> str:
    """Build ``source`` (C text) as a shared library at ``out_path``."""
    c_path = out_path + ".c"
    with open(c_path, "w") as fh:
        fh.write(source)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", out_path, c_path])
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _frame(a: np.ndarray) -> Tuple[np.ndarray, int]:
    if a.ndim != 2 or a.dtype not in (np.uint8, np.uint16):
        raise TypeError("frame must be a 2-D uint8 or uint16 array")
    a = np.ascontiguousarray(a)
    return a, a.itemsize


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def introsort(values, depth_limit: Optional[int] = None) -> Tuple[np.ndarray, SortStats]:
    """Sort a copy of ``values`` (uint32) with the oracle's introsort."""
    a = np.array(values, dtype=np.uint32, copy=True)
    st = SortStats()
    lib = _load()
    if depth_limit is None:
        lib.oracle_introsort(_ptr(a), a.size, ctypes.byref(st))
    else:
        lib.oracle_introsort_depth(_ptr(a), a.size, depth_limit, ctypes.byref(st))
    return a, st


def window(frame: np.ndarray, x: int, y: int, k: int) -> np.ndarray:
    """S_xy of pixel (x, y) in the paper's listing order (k*k values)."""
    f, b = _frame(frame)
    H, W = f.shape
    S = np.zeros(k * k, dtype=np.uint32)
    rc = _load().oracle_window(_ptr(f), f.strides[0], W, H, b, k, x, y, _ptr(S))
    if rc:
        raise ValueError(f"oracle_window rejected its arguments ({rc})")
    return S


def detect(frame: np.ndarray, k: int) -> Tuple[np.ndarray, int]:
    """Noise mask (1 = noisy) and noisy-pixel count of one detection pass."""
    f, b = _frame(frame)
    H, W = f.shape
    mask = np.zeros((H, W), dtype=np.uint8)
    cnt = ctypes.c_uint64(0)
    rc = _load().oracle_detect(_ptr(f), f.strides[0], _ptr(mask), mask.strides[0], W, H, b, k,
                               ctypes.byref(cnt))
    if rc:
        raise ValueError(f"oracle_detect rejected its arguments ({rc})")
    return mask, int(cnt.value)


def detect_directional(frame: np.ndarray) -> Tuple[np.ndarray, int]:
    """Opt-in directional detector, a reading of Fig. 1's caption (not the
    paper's detector): a pixel is noisy when, on each of the four lines through
    it in its 3x3 window (row, column, both diagonals), its grey level lies
    outside the range of its two neighbours.  Returns (mask, count)."""
    f, b = _frame(frame)
    H, W = f.shape
    mask = np.zeros((H, W), dtype=np.uint8)
    cnt = ctypes.c_uint64(0)
    rc = _load().oracle_detect_directional(_ptr(f), f.strides[0], _ptr(mask), mask.strides[0], W, H, b,
                                           ctypes.byref(cnt))
    if rc:
        raise ValueError(f"oracle_detect_directional rejected its arguments ({rc})")
    return mask, int(cnt.value)


def median(frame: np.ndarray, k: int, mask: Optional[np.ndarray] = None,
           stats: Optional[SortStats] = None) -> Tuple[np.ndarray, int]:
    """Window median where ``mask`` != 0 (everywhere if None); returns (out, sorts)."""
    f, b = _frame(frame)
    H, W = f.shape
    out = np.zeros_like(f)
    m = None
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.shape != f.shape:
            raise ValueError("mask shape must match the frame")
    sorts = ctypes.c_uint64(0)
    rc = _load().oracle_median(_ptr(f), f.strides[0], _ptr(m), 0 if m is None else m.strides[0],
                               _ptr(out), out.strides[0], W, H, b, k, ctypes.byref(sorts),
                               None if stats is None else ctypes.byref(stats))
    if rc:
        raise ValueError(f"oracle_median rejected its arguments ({rc})")
    return out, int(sorts.value)


def fnr(frame: np.ndarray, k: int, passes: int = 1,
        stats: Optional[SortStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """FNR applied ``passes`` times; returns (output, per-pass noisy counts)."""
    f, b = _frame(frame)
    H, W = f.shape
    out = np.zeros_like(f)
    counts = np.zeros(max(passes, 1), dtype=np.uint64)
    rc = _load().oracle_fnr(_ptr(f), f.strides[0], _ptr(out), out.strides[0], W, H, b, k, passes,
                            _ptr(counts), None if stats is None else ctypes.byref(stats))
    if rc:
        raise ValueError(f"oracle_fnr rejected its arguments ({rc})")
    return out, counts


def fnr_at(frame: np.ndarray, k: int, points) -> np.ndarray:
    """One FNR pass evaluated at the (x, y) pixels in ``points`` only, each from
    its own window: the centre value unless it equals the minimum or maximum of
    S_xy (Section 3.3, Eq. 3a/3b), else element (k*k - 1)/2 of S_xy sorted by the
    oracle's introsort (Section 3.4).  For sampled checks of frames too large
    for :func:`fnr`."""
    f, _ = _frame(frame)
    out = np.zeros(len(points), dtype=np.uint32)
    for i, (x, y) in enumerate(points):
        S = window(f, int(x), int(y), k)
        c = int(f[y, x])
        if c == int(S.min()) or c == int(S.max()):
            out[i] = introsort(S)[0][(k * k - 1) // 2]
        else:
            out[i] = c
    return out
