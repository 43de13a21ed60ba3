"""GPU parity of the windows above 15x15 (17x17 .. 31x31).

Detection is the same separable min/max on a wider LDS halo; the median of a
flagged pixel is found by a group of 8 or 16 lanes (grey-level bisection with
group sums).  Every output pixel, mask byte and count must equal the oracle's
(the paper's detector and introsort median, Sections 3.3-3.4).
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LARGE = [17, 19, 21, 23, 25, 27, 29, 31]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


@pytest.fixture
def threads():
    """Set the workgroup size (and selection) of (dtype, window) for one test;
    restores the defaults after."""
    touched = []

    def set_(dt, k, t, sel=irfilter.IRF_SELECT_GROUP):
        irfilter.set_tuning(dt, k, t, sel)
        touched.append((dt, k))

    yield set_
    for dt, k in touched:
        irfilter.set_tuning(dt, k, 0, 0)


def to_dev(a, dev):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).to(dev).view(torch.uint16)
    return torch.from_numpy(a).to(dev)


def to_host(t):
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ; first at (x={x}, y={y}): "
                             f"gpu {got[y, x]} oracle {want[y, x]}")


def check_fnr(frame, k, dev, passes=1, tag=""):
    say(f"case large fnr {tag} {frame.dtype} {frame.shape[1]}x{frame.shape[0]} k={k} passes={passes}")
    want, wcounts = oracle.fnr(frame, k, passes)
    src = to_dev(frame, dev)
    dst = torch.empty_like(src)
    scr = torch.empty_like(src) if passes > 1 else None
    cnt = torch.zeros(passes, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run(src, dst, k, passes=passes, scratch=scr, flagged_count=cnt)
    torch.cuda.synchronize()
    assert_same(to_host(dst), want, f"fnr k={k}")
    np.testing.assert_array_equal(cnt.cpu().numpy().astype(np.uint64), wcounts)


SELECTS = [irfilter.IRF_SELECT_GROUP, irfilter.IRF_SELECT_HIST]


@pytest.mark.parametrize("sel", SELECTS)
@pytest.mark.parametrize("t", [128, 256])
@pytest.mark.parametrize("k", LARGE)
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_fnr_every_window(dev, threads, dt, k, t, sel):
    # 2 tiles across (the second ragged) and several tile rows, mixed impulses
    threads(dt, k, t, sel)
    f = synth.make_frame(synth.FrameSpec(203, 149, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0, 1700 + k))
    check_fnr(f, k, dev, tag=f"t{t} {irfilter.SELECT_NAMES[sel]}")


@pytest.mark.parametrize("k", [17, 23, 31])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_detect_median_and_plain_median(dev, dt, k):
    f = synth.make_frame(synth.FrameSpec(150, 97, dt, "rv" if dt == "u16" else "sp", 0.25,
                                         20.0 if dt == "u16" else 0.0, 1800 + k))
    src = to_dev(f, dev)
    say(f"case large detect {dt} k={k}")
    mask = torch.full(f.shape, 7, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_detect(src, mask, k, flagged_count=cnt)
    torch.cuda.synchronize()
    wmask, wcount = oracle.detect(f, k)
    assert_same(mask.cpu().numpy(), wmask.astype(np.uint8), f"mask k={k}")
    assert int(cnt.item()) == int(wcount)
    say(f"case large masked median {dt} k={k}")
    dst = torch.empty_like(src)
    irfilter.ir_filter_median(src, dst, k, mask=mask)
    torch.cuda.synchronize()
    assert_same(to_host(dst), oracle.median(f, k, wmask)[0], f"masked median k={k}")
    say(f"case large plain median {dt} k={k}")
    irfilter.ir_filter_median(src, dst, k)
    torch.cuda.synchronize()
    assert_same(to_host(dst), oracle.median(f, k)[0], f"median filter k={k}")


@pytest.mark.parametrize("W,H,k", [(1, 1, 31), (2, 3, 17), (5, 40, 31), (40, 5, 25), (31, 31, 31),
                                   (128, 1, 19), (129, 64, 27), (257, 65, 21), (300, 33, 29)])
def test_shapes(dev, W, H, k):
    for dt in ("u8", "u16"):
        f = synth.make_frame(synth.FrameSpec(W, H, dt, "mixed", 0.35, 0.0 if dt == "u8" else 20.0, W * 7 + H))
        check_fnr(f, k, dev)


@pytest.mark.parametrize("sel", SELECTS)
@pytest.mark.parametrize("k", [17, 31])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_ties_and_extremes(dev, threads, dt, k, sel):
    threads(dt, k, 256, sel)
    rng = np.random.default_rng(k + (dt == "u16"))
    check_fnr(synth.random_frame(rng, 140, 90, dt, alphabet=3), k, dev, tag="ties")
    vmax = 255 if dt == "u8" else 65535
    npdt = np.uint8 if dt == "u8" else np.uint16
    check_fnr(np.where(rng.random((90, 140)) < 0.5, 0, vmax).astype(npdt), k, dev, tag="s&p")
    say(f"case large constant {dt} k={k}")
    for val in (0, vmax):
        f = np.full((40, 70), val, dtype=npdt)
        src = to_dev(f, dev)
        dst = torch.empty_like(src)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
        torch.cuda.synchronize()
        assert_same(to_host(dst), f, "constant frame")
        assert int(cnt.item()) == f.size


@pytest.mark.parametrize("sel", SELECTS)
def test_full_16bit_range(dev, threads, sel):
    rng = np.random.default_rng(31)
    f = rng.integers(0, 65536, size=(80, 150)).astype(np.uint16)
    for k in (17, 21, 31):
        threads("u16", k, 256, sel)
        check_fnr(f, k, dev, tag=f"16-bit {irfilter.SELECT_NAMES[sel]}")


@pytest.mark.parametrize("k", [17, 25, 31])
def test_hist_masked_and_plain_median(dev, threads, k):
    # the radix select serves every mode that selects: masked and plain medians
    for dt in ("u8", "u16"):
        threads(dt, k, 128, irfilter.IRF_SELECT_HIST)
        f = synth.make_frame(synth.FrameSpec(141, 75, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0, 1850 + k))
        src = to_dev(f, dev)
        mask = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
        irfilter.ir_filter_detect(src, mask, k)
        dst = torch.empty_like(src)
        say(f"case hist masked median {dt} k={k}")
        irfilter.ir_filter_median(src, dst, k, mask=mask)
        torch.cuda.synchronize()
        wmask, _ = oracle.detect(f, k)
        assert_same(to_host(dst), oracle.median(f, k, wmask)[0], f"hist masked median k={k}")
        say(f"case hist plain median {dt} k={k}")
        irfilter.ir_filter_median(src, dst, k)
        torch.cuda.synchronize()
        assert_same(to_host(dst), oracle.median(f, k)[0], f"hist median filter k={k}")


def test_two_passes_and_stack(dev):
    f = synth.make_frame(synth.FrameSpec(170, 120, "u16", "mixed", 0.4, 20.0, 1901))
    check_fnr(f, 19, dev, passes=2)
    N, W, H, k = 4, 133, 71, 25
    frames = [synth.make_frame(synth.FrameSpec(W, H, "u8", "sp", 0.1 + 0.1 * i, 0.0, 1910 + i)) for i in range(N)]
    say("case large stack")
    src = to_dev(np.stack(frames), dev)
    dst = torch.empty_like(src)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run_frames(src, dst, k, flagged_count=cnt)
    torch.cuda.synchronize()
    out = to_host(dst)
    tot = 0
    for i, fr in enumerate(frames):
        want, wc = oracle.fnr(fr, k)
        assert_same(out[i], want, f"stack frame {i}")
        tot += int(wc[0])
    assert int(cnt.item()) == tot


def test_batch_takes_large_windows_beside_small_ones(dev):
    # batch plans run windows above 15x15 in kernels of their own, in the same
    # batch as small windows; each frame equals its single launch, and 33 is refused
    rng = np.random.default_rng(1717)
    frames = [rng.integers(0, 1 << 14, size=(70 + 13 * i, 90 + 29 * i)).astype(np.uint16) for i in range(4)]
    wins = [7, 17, 31, 9]
    srcs = [to_dev(f, dev) for f in frames]
    dsts = [torch.empty_like(s) for s in srcs]
    refs = [torch.empty_like(s) for s in srcs]
    say("case large windows in a batch")
    tiles = sum(irfilter.frame_tiles(f.shape[1], f.shape[0]) for f in frames)
    with irfilter.Plan(4, tiles) as plan:
        plan.run([(s, d, k) for s, d, k in zip(srcs, dsts, wins)])
        for s, r, k in zip(srcs, refs, wins):
            irfilter.ir_filter_run(s, r, k)
        torch.cuda.synchronize()
        for d, r, k in zip(dsts, refs, wins):
            assert torch.equal(d.view(torch.int16), r.view(torch.int16)), k
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(srcs[0], dsts[0], 7), (srcs[1], dsts[1], 33)])
        assert e.value.status == -5
