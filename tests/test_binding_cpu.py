"""Python-binding argument checks that run before any library call.

Each case is refused by the binding (ValueError) before it reaches the C ABI,
so these run without a GPU: the tensors are CPU tensors and the checks that
fail come first.  A device tensor is needed only where the check under test
follows the device check; those cases use a stand-in object."""

import pytest
import torch

from paper_1201_3972_amd import irfilter


class FakeCuda:
    """Stands in for a CUDA tensor in the checks on count arrays."""

    def __init__(self, dtype=torch.int64, n=1, contiguous=True):
        self.is_cuda = True
        self.dtype = dtype
        self._n = n
        self._c = contiguous

    def is_contiguous(self):
        return self._c

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


def test_counts_must_be_device_64bit_contiguous_and_long_enough():
    assert irfilter._counts(None, 3) is None
    with pytest.raises(ValueError, match="CUDA"):
        irfilter._counts(torch.zeros(4, dtype=torch.int64), 1)
    with pytest.raises(ValueError, match="64-bit"):
        irfilter._counts(FakeCuda(torch.int32, 4), 1)
    with pytest.raises(ValueError, match="contiguous"):
        irfilter._counts(FakeCuda(n=4, contiguous=False), 1)
    with pytest.raises(ValueError, match="at least 2"):
        irfilter._counts(FakeCuda(n=1), 2)
    assert irfilter._counts(FakeCuda(n=2), 2) == 0x1000
    assert irfilter._counts(FakeCuda(torch.uint64, 5), 5) == 0x1000


def test_mask_must_be_uint8_of_the_source_shape():
    src = torch.zeros((8, 9), dtype=torch.uint16)
    with pytest.raises(ValueError, match="uint8"):
        irfilter._mask(torch.zeros((8, 9), dtype=torch.int16), src)
    with pytest.raises(ValueError, match="shape"):
        irfilter._mask(torch.zeros((8, 8), dtype=torch.uint8), src)
    irfilter._mask(torch.zeros((8, 9), dtype=torch.uint8), src)


def test_scratch_must_match_the_source():
    src = torch.zeros((8, 9), dtype=torch.uint8)
    with pytest.raises(ValueError, match="scratch"):
        irfilter.ir_filter_run(src, torch.zeros_like(src), 3, passes=2, scratch=torch.zeros((7, 9), dtype=torch.uint8))
    with pytest.raises(ValueError, match="scratch"):
        irfilter.ir_filter_run_frames(src[None], torch.zeros_like(src[None]), 3, passes=2,
                                      scratch=torch.zeros((1, 8, 9), dtype=torch.uint16))


def test_median_checks_the_mask_first():
    src = torch.zeros((8, 9), dtype=torch.uint8)
    with pytest.raises(ValueError, match="mask"):
        irfilter.ir_filter_median(src, torch.zeros_like(src), 3, mask=torch.zeros((9, 9), dtype=torch.uint8))
