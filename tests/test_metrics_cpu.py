"""PSNR (Eq. 5) against closed forms."""

import math

import numpy as np
import pytest

from paper_1201_3972_amd import metrics


def test_identical_frames_are_infinite():
    a = np.arange(100, dtype=np.uint8).reshape(10, 10)
    assert metrics.psnr(a, a) == math.inf


def test_constant_offset_closed_form():
    a = np.full((8, 8), 100, np.uint8)
    b = a + 5  # MSE = 25
    assert metrics.psnr(a, b) == pytest.approx(10 * math.log10(255 ** 2 / 25))


def test_single_pixel_error_and_max_value():
    a = np.zeros((10, 10), np.uint16)
    b = a.copy()
    b[3, 4] = 100  # MSE = 100^2 / 100 = 100
    assert metrics.psnr(a, b, max_value=16383) == pytest.approx(10 * math.log10(16383 ** 2 / 100))
    assert metrics.psnr(a, b) == pytest.approx(10 * math.log10(16383 ** 2 / 100))  # 14-bit default


def test_symmetric_and_shape_checked():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 256, (16, 16), dtype=np.uint8)
    b = rng.integers(0, 256, (16, 16), dtype=np.uint8)
    assert metrics.psnr(a, b) == pytest.approx(metrics.psnr(b, a))
    with pytest.raises(ValueError):
        metrics.psnr(a, b[:8])
