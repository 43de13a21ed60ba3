"""GPU parity at the size limits of the C ABI.

Frames up to IRF_MAX_DIM (32768) on a side, stacks larger than 4 GiB (64-bit
frame offsets) and row pitches just under 2^24 bytes (32-bit offsets inside a
frame close to their limit).  Frames too large for the whole-frame oracle are
checked at sampled pixels: each sample's window is cut out with its
neighbourhood and evaluated by the oracle on the crop, which clamps exactly as
the full frame does because the crop ends where the frame ends.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


def to_dev(a, dev):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).to(dev).view(torch.uint16)
    return torch.from_numpy(a).to(dev)


def to_host(t):
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def sampled_points(W, H, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(int(x), int(y)) for x, y in zip(rng.integers(0, W, n), rng.integers(0, H, n))]
    return pts + [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1), (W // 2, 0), (0, H // 2)]


def oracle_at(frame, k, pts):
    """FNR output at each point from the oracle run on a crop around its window."""
    H, W = frame.shape
    r = k // 2
    out = []
    for x, y in pts:
        x0, y0 = max(0, x - r), max(0, y - r)
        crop = np.ascontiguousarray(frame[y0:min(H, y + r + 1), x0:min(W, x + r + 1)])
        out.append(int(oracle.fnr_at(crop, k, [(x - x0, y - y0)])[0]))
    return np.array(out)


def gpu_at(t, pts):
    idx_y = torch.tensor([y for _, y in pts], device=t.device)
    idx_x = torch.tensor([x for x, _ in pts], device=t.device)
    v = t.view(torch.int16)[idx_y, idx_x] if t.dtype == torch.uint16 else t[idx_y, idx_x]
    v = v.cpu().numpy()
    return (v.view(np.uint16) if t.dtype == torch.uint16 else v).astype(np.int64)


@pytest.mark.parametrize("W,H,dt,k", [(32768, 40, "u16", 5), (40, 32768, "u8", 7), (32768, 9, "u8", 31),
                                      (5, 32768, "u16", 17)])
def test_widest_and_tallest_frames(dev, W, H, dt, k):
    f = synth.make_frame(synth.FrameSpec(W, H, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0, W + H + k))
    say(f"case limits {dt} {W}x{H} k={k}")
    want, wc = oracle.fnr(f, k)
    src = to_dev(f, dev)
    dst = torch.empty_like(src)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(dst), want)
    assert int(cnt.item()) == int(wc[0])


def test_largest_frame(dev):
    """32768 x 32768 u16 (2 GiB), 3x3 and 7x7: sampled pixels against the oracle,
    and the count against the detector's own mask."""
    N = 32768
    say("case limits 32768x32768 u16: generating")
    rng = np.random.default_rng(32768)
    f = rng.integers(0, 16384, size=(N, N), dtype=np.uint16)
    f[rng.integers(0, N, 4_000_000), rng.integers(0, N, 4_000_000)] = 16383  # salt
    src = to_dev(f, dev)
    dst = torch.empty_like(src)
    mask = torch.empty((N, N), dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    dcnt = torch.zeros(1, dtype=torch.int64, device=dev)
    pts = sampled_points(N, N, 1500, 5)
    for k in (3, 7):
        say(f"case limits 32768x32768 u16 k={k}")
        irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
        irfilter.ir_filter_detect(src, mask, k, flagged_count=dcnt)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gpu_at(dst, pts), oracle_at(f, k, pts))
        assert int(cnt.item()) == int(dcnt.item()) == int(mask.sum(dtype=torch.int64).item())
    del src, dst, mask
    torch.cuda.empty_cache()


def test_stack_beyond_4gib(dev):
    """Three 32768 x 24576 u16 frames (4.5 GiB): frame offsets need 64 bits."""
    n, W, H, k = 3, 32768, 24576, 5
    say("case limits stack of 3 x 32768x24576 u16: generating")
    rng = np.random.default_rng(77)
    src = torch.empty((n, H, W), dtype=torch.uint16, device=dev)
    frames = []
    for i in range(n):
        f = rng.integers(1000, 3000, size=(H, W), dtype=np.uint16)
        f[rng.integers(0, H, 1_000_000), rng.integers(0, W, 1_000_000)] = 0  # pepper
        src[i].copy_(to_dev(f, dev))
        frames.append(f)
    dst = torch.empty_like(src)
    say("case limits stack of 3: run")
    irfilter.ir_filter_run_frames(src, dst, k)
    torch.cuda.synchronize()
    pts = sampled_points(W, H, 1000, 6)
    for i in range(n):
        np.testing.assert_array_equal(gpu_at(dst[i], pts), oracle_at(frames[i], k, pts))
    del src, dst
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_pitch_just_below_2_24(dev, dt):
    """Rows 2^24 - 64 bytes apart over 250 rows: in-frame byte offsets reach
    4.18e9, just under the 32-bit limit the host enforces."""
    W, H, k = 1000, 250, 5
    b = 2 if dt == "u16" else 1
    pitch = (1 << 24) - 64
    f = synth.make_frame(synth.FrameSpec(W, H, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0, 2024))
    want, wc = oracle.fnr(f, k)
    tdt = torch.uint16 if dt == "u16" else torch.uint8
    say(f"case limits pitch 2^24-64 {dt}")
    big = torch.zeros((H, pitch // b), dtype=torch.int16 if dt == "u16" else torch.uint8, device=dev)
    big[:, :W].copy_(to_dev(f, dev).view(torch.int16) if dt == "u16" else to_dev(f, dev))
    src = big.view(tdt)[:, :W]
    dbig = torch.zeros_like(big)
    dst = dbig.view(tdt)[:, :W]
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(dst.contiguous()), want)
    assert int(cnt.item()) == int(wc[0])
    assert not dbig[:, W:W + 64].any() and not dbig[:, -64:].any()
    del big, dbig
    torch.cuda.empty_cache()
