"""The two detection paths of the stack kernel.

A tile whose staged values all lie below 0x4000 (every 8-bit frame, 14-bit
data) takes the horizontal min / max through the three-input half-precision
instructions; any other tile takes the packed integer path.  Both must give
the oracle's flags, medians and counts: frames just below and at the switch
value, frames of small values (subnormal bit patterns, zero, ties), and frames
whose tiles take different paths side by side, at every window of the stack
kernel's detector, with both workgroup sizes, in the whole-filter and the
mask-writing modes."""

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter
from tests.gpu_helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WINDOWS = [3, 5, 7, 9, 11, 13, 15, 17, 21, 31]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


@pytest.fixture
def threads():
    touched = []

    def set_(k, t):
        sel = irfilter.IRF_SELECT_NETWORK if k <= 15 else irfilter.IRF_SELECT_GROUP
        irfilter.set_tuning("u16", k, t, sel)
        touched.append(k)

    yield set_
    for k in touched:
        irfilter.set_tuning("u16", k, 0, 0)


def frames(seed):
    rng = np.random.default_rng(seed)
    H, W = 150, 300  # three tile columns (the last ragged), several tile rows
    out = {}
    # just below the switch value, ties at the top
    out["below"] = rng.integers(0x3F00, 0x4000, size=(H, W)).astype(np.uint16)
    # just at and above it
    out["at"] = rng.integers(0x3FF0, 0x4010, size=(H, W)).astype(np.uint16)
    # small values: zero and half-precision subnormal bit patterns, few levels
    out["small"] = rng.choice(np.array([0, 1, 2, 3, 0x3FF, 0x400, 0x401], dtype=np.uint16), size=(H, W))
    # a 14-bit frame with one block of 16-bit values: neighbouring tiles take
    # different paths, and windows straddle them
    f = rng.integers(0, 0x4000, size=(H, W)).astype(np.uint16)
    f[40:90, 100:230] = rng.integers(0x4000, 0x10000, size=(50, 130)).astype(np.uint16)
    out["mixed"] = f
    # single large values scattered through a 14-bit frame with impulses
    g = rng.integers(2000, 3000, size=(H, W)).astype(np.uint16)
    g[rng.random((H, W)) < 0.2] = 0
    g[rng.random((H, W)) < 0.001] = 0xFFFF
    out["sparse_large"] = g
    return out


@pytest.mark.parametrize("t", [128, 256])
@pytest.mark.parametrize("k", WINDOWS)
def test_fnr_both_paths(dev, threads, k, t):
    threads(k, t)
    for name, f in frames(900 + k).items():
        say(f"case f16 detect fnr {name} k={k} t={t}")
        src = to_dev(torch, f, dev)
        dst = torch.empty_like(src)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
        torch.cuda.synchronize()
        want, wc = oracle.fnr(f, k)
        got = to_host(torch, dst)
        assert np.array_equal(got, want), (name, int((got != want).sum()))
        assert int(cnt.item()) == int(wc[0]), name


@pytest.mark.parametrize("k", [3, 5, 7, 9, 15, 25])
def test_detect_mask_both_paths(dev, k):
    for name, f in frames(950 + k).items():
        say(f"case f16 detect mask {name} k={k}")
        src = to_dev(torch, f, dev)
        mask = torch.full(f.shape, 9, dtype=torch.uint8, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        irfilter.ir_filter_detect(src, mask, k, flagged_count=cnt)
        torch.cuda.synchronize()
        wmask, wcount = oracle.detect(f, k)
        assert np.array_equal(mask.cpu().numpy(), wmask.astype(np.uint8)), name
        assert int(cnt.item()) == int(wcount), name


def test_u8_frames_and_stack(dev):
    # 8-bit frames always qualify; a stack mixing a 14-bit and a 16-bit frame
    rng = np.random.default_rng(5)
    f8 = rng.integers(0, 256, size=(97, 260)).astype(np.uint8)
    for k in (3, 5, 7, 11):
        say(f"case f16 detect u8 k={k}")
        src = to_dev(torch, f8, dev)
        dst = torch.empty_like(src)
        irfilter.ir_filter_run(src, dst, k)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(torch, dst), oracle.fnr(f8, k)[0]), k
    a = rng.integers(0, 0x4000, size=(120, 256)).astype(np.uint16)
    b = rng.integers(0, 0x10000, size=(120, 256)).astype(np.uint16)
    st = np.stack([a, b, a])
    say("case f16 detect stack 14/16/14-bit")
    src = to_dev(torch, st, dev)
    dst = torch.empty_like(src)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run_frames(src, dst, 7, flagged_count=cnt)
    torch.cuda.synchronize()
    out = to_host(torch, dst)
    tot = 0
    for i in range(3):
        want, wc = oracle.fnr(st[i], 7)
        assert np.array_equal(out[i], want), i
        tot += int(wc[0])
    assert int(cnt.item()) == tot
