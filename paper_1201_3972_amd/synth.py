"""Seeded synthetic infrared frames.

The paper evaluates on one real 364x244 8-bit infrared street scene with 20 % and
30 % impulse noise (Section 4.2, Fig. 2-4).  That image is not available, so every
input here is synthetic, built to have the same structure: a smooth thermal field
(a surface whose temperature varies monotonically, Section 3), thin bright lines,
small text strokes, optional Gaussian read noise, and impulse noise applied last.

This module only draws inputs.  It holds none of the filter's arithmetic (no window
extrema, no medians), so both the CPU oracle and the GPU path can take their inputs
from it without sharing any of the method's code.

Recipe (all in float64, then ``np.rint`` and clip):

* field: ``a*x/W + b*y/H`` with ``a, b ~ U(0.2, 0.6)`` plus 8 Gaussian blobs (centre
  uniform in the frame, sigma ``~ U(0.03, 0.12) * min(W, H)``, amplitude
  ``~ U(-0.6, 0.9)``), normalised to [0, 1] and mapped to the dtype's field range;
* four 1-px lines (two horizontal, one vertical, one diagonal) at field + ``line``;
* twelve random 3x5 stroke glyphs (each cell on with p = 0.6) at field +- ``glyph``;
* optional read noise ``N(0, sigma^2)``;
* impulses: every pixel independently with probability ``density``;
  salt-and-pepper sets 0 or MAX (1/2 each), random-valued sets ``U{0..MAX}``,
  mixed picks one of the two per pixel with probability 1/2.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BASE_SEED = 12013972

# (field low, field high, line step, glyph step, impulse MAX) per pixel type.
_RANGES = {
    "u8": (40.0, 200.0, 60.0, 80.0, 255),
    "u16": (1000.0, 15000.0, 4000.0, 80.0 * 64.0, 16383),
}
_NP_DTYPE = {"u8": np.uint8, "u16": np.uint16}
NOISE_KINDS = ("none", "sp", "rv", "mixed")


@dataclasses.dataclass(frozen=True)
class FrameSpec:
    width: int
    height: int
    dtype: str = "u8"  # "u8" or "u16" (u16 frames carry 14-bit data)
    noise: str = "sp"  # one of NOISE_KINDS
    density: float = 0.2
    read_sigma: float = 0.0
    seed: int = BASE_SEED
    structures: bool = True

    def __post_init__(self):
        if self.dtype not in _NP_DTYPE:
            raise ValueError(f"dtype must be u8 or u16, got {self.dtype!r}")
        if self.noise not in NOISE_KINDS:
            raise ValueError(f"noise must be one of {NOISE_KINDS}, got {self.noise!r}")
        if self.width < 1 or self.height < 1:
            raise ValueError("frame must be at least 1x1")


def impulse_max(dtype: str) -> int:
    return _RANGES[dtype][4]


def config_seed(config_index: int, frame_index: Optional[int] = None) -> int:
    """Seed of config ``i`` (``BASE + i``) or of frame ``j`` in it (``BASE + 1000 i + j``)."""
    if frame_index is None:
        return BASE_SEED + config_index
    return BASE_SEED + 1000 * config_index + frame_index


def _field(rng: np.random.Generator, W: int, H: int) -> np.ndarray:
    xs = np.arange(W, dtype=np.float64)
    ys = np.arange(H, dtype=np.float64)
    a, b = rng.uniform(0.2, 0.6, size=2)
    f = a * xs[None, :] / W + b * ys[:, None] / H
    for _ in range(8):
        cx = rng.uniform(0, W)
        cy = rng.uniform(0, H)
        s = rng.uniform(0.03, 0.12) * min(W, H)
        amp = rng.uniform(-0.6, 0.9)
        gx = np.exp(-((xs - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((ys - cy) ** 2) / (2.0 * s * s))
        f = f + amp * gy[:, None] * gx[None, :]
    lo, hi = f.min(), f.max()
    if hi > lo:
        f = (f - lo) / (hi - lo)
    else:
        f = np.zeros_like(f)
    return f


def _structures(rng: np.random.Generator, f: np.ndarray, line: float, glyph: float) -> np.ndarray:
    H, W = f.shape
    f = f.copy()
    for _ in range(2):  # horizontal lines
        f[rng.integers(0, H), :] += line
    f[:, rng.integers(0, W)] += line  # vertical line
    x0 = int(rng.integers(0, W))  # diagonal line
    n = min(H, W)
    idx = np.arange(n)
    f[idx, (x0 + idx) % W] += line
    for _ in range(12):  # 3 wide x 5 tall stroke glyphs
        cells = rng.random((5, 3)) < 0.6
        sign = 1.0 if rng.random() < 0.5 else -1.0
        gy = int(rng.integers(0, max(1, H - 4)))
        gx = int(rng.integers(0, max(1, W - 2)))
        sub = f[gy:gy + 5, gx:gx + 3]
        sub += sign * glyph * cells[: sub.shape[0], : sub.shape[1]]
    return f


def clean_frame(spec: FrameSpec) -> np.ndarray:
    """The noise-free part of :func:`make_frame` (field, structures, read noise)."""
    return _make(spec, impulses=False)


def make_frame(spec: FrameSpec) -> np.ndarray:
    """One ``H x W`` frame of ``spec.dtype`` drawn from ``spec.seed``."""
    return _make(spec, impulses=True)


def _make(spec: FrameSpec, impulses: bool) -> np.ndarray:
    lo, hi, line, glyph, vmax = _RANGES[spec.dtype]
    rng = np.random.default_rng(spec.seed)
    f = lo + (hi - lo) * _field(rng, spec.width, spec.height)
    if spec.structures:
        f = _structures(rng, f, line, glyph)
    if spec.read_sigma > 0:
        f = f + rng.normal(0.0, spec.read_sigma, size=f.shape)
    img = np.clip(np.rint(f), 0, vmax).astype(_NP_DTYPE[spec.dtype])
    if not impulses or spec.noise == "none" or spec.density <= 0:
        return img
    hit = rng.random(img.shape) < spec.density
    salt = rng.random(img.shape) < 0.5
    rv = rng.integers(0, vmax + 1, size=img.shape).astype(img.dtype)
    if spec.noise == "sp":
        use_sp = np.ones(img.shape, dtype=bool)
    elif spec.noise == "rv":
        use_sp = np.zeros(img.shape, dtype=bool)
    else:
        use_sp = rng.random(img.shape) < 0.5
    sp = np.where(salt, vmax, 0).astype(img.dtype)
    noisy = np.where(use_sp, sp, rv)
    return np.where(hit, noisy, img).astype(img.dtype)


def random_frame(rng: np.random.Generator, width: int, height: int, dtype: str, alphabet: Optional[int] = None) -> np.ndarray:
    """Unstructured frame: uniform values, or values in ``0..alphabet-1`` to force ties."""
    vmax = 255 if dtype == "u8" else 65535
    hi = vmax + 1 if alphabet is None else alphabet
    return rng.integers(0, hi, size=(height, width)).astype(_NP_DTYPE[dtype])


# ----------------------------------------------------------------------------
# Workload recipes (sizes and noise mixes of the evaluation workloads)
# ----------------------------------------------------------------------------

def c1_frame() -> np.ndarray:
    """320x240 u8, field 40-200 with lines and glyphs, 20 % salt-and-pepper (3x3 window)."""
    return make_frame(FrameSpec(320, 240, "u8", "sp", 0.20, 0.0, config_seed(0)))


C2_DENSITIES = (0.10, 0.30, 0.60)
C2_WINDOWS = (5, 7)


def c2_spec(density: float, frame_index: int = 0) -> FrameSpec:
    """640x512 u16 14-bit field, read noise sigma 20, random-valued impulses."""
    return FrameSpec(640, 512, "u16", "rv", density, 20.0, config_seed(1, frame_index))


def c2_frames(n_per_density: int = 1) -> List[np.ndarray]:
    out = []
    j = 0
    for d in C2_DENSITIES:
        for _ in range(n_per_density):
            out.append(make_frame(c2_spec(d, j)))
            j += 1
    return out


C3_WINDOWS = (3, 5, 7, 9, 11, 15)


def c3_spec(frame_index: int = 0) -> FrameSpec:
    """1920x1080 u16 14-bit, read noise sigma 20, 40 % mixed impulses."""
    return FrameSpec(1920, 1080, "u16", "mixed", 0.40, 20.0, config_seed(2, frame_index))


@dataclasses.dataclass(frozen=True)
class BatchItem:
    spec: FrameSpec
    window: int


def c4_items(n: int = 256, seed: Optional[int] = None) -> List[BatchItem]:
    """Uneven batch: W ~ U{160..1280}, H ~ U{120..1024}, dtype u8/u16 (1/2 each),
    window in {3,5,7,9}, density ~ U(0.05, 0.60), mixed impulses."""
    rng = np.random.default_rng(config_seed(3) if seed is None else seed)
    items = []
    for j in range(n):
        W = int(rng.integers(160, 1281))
        H = int(rng.integers(120, 1025))
        dt = "u8" if rng.random() < 0.5 else "u16"
        k = int(rng.choice([3, 5, 7, 9]))
        d = float(rng.uniform(0.05, 0.60))
        items.append(BatchItem(FrameSpec(W, H, dt, "mixed", d, 0.0 if dt == "u8" else 20.0,
                                         config_seed(3, j)), k))
    return items
