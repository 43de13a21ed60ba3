"""Quality metric of the paper's evaluation (host side, not the filter itself).

PSNR, Section 4.2 Eq. (5): 10 log10(MAX^2 / MSE), MSE the mean squared
difference between the original (noise-free) and the processed frame, MAX the
largest grey level (255 for 8-bit frames)."""

from __future__ import annotations

import numpy as np


def psnr(reference: np.ndarray, processed: np.ndarray, max_value: float = None) -> float:
    """PSNR in dB of ``processed`` against ``reference`` (inf when identical)."""
    if reference.shape != processed.shape:
        raise ValueError("frames must have the same shape")
    if max_value is None:
        max_value = 255.0 if reference.dtype == np.uint8 else 16383.0
    mse = float(np.mean((reference.astype(np.float64) - processed.astype(np.float64)) ** 2))
    if mse == 0.0:
        return float("inf")
    return 10.0 * np.log10(max_value * max_value / mse)
