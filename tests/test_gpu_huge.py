"""GPU parity of the windows above 31x31 (33x33 .. 63x63).

Tiles stage a 32-pixel halo on each side; the median of a flagged pixel is
found by a group of 16 or 32 lanes (grey-level bisection, the 32-lane groups
summing their counts across two DPP rows).  Every output pixel, mask byte and
count must equal the oracle's (the paper's detector and introsort median,
Sections 3.3-3.4)."""

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, synth
from tests.gpu_helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HUGE = [33, 35, 39, 41, 47, 55, 63]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ; first at (x={x}, y={y}): "
                             f"gpu {got[y, x]} oracle {want[y, x]}")


def check_fnr(frame, k, dev, passes=1, tag=""):
    say(f"case huge fnr {tag} {frame.dtype} {frame.shape[1]}x{frame.shape[0]} k={k} passes={passes}")
    want, wcounts = oracle.fnr(frame, k, passes)
    src = to_dev(torch, frame, dev)
    dst = torch.empty_like(src)
    scr = torch.empty_like(src) if passes > 1 else None
    cnt = torch.zeros(passes, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run(src, dst, k, passes=passes, scratch=scr, flagged_count=cnt)
    torch.cuda.synchronize()
    assert_same(to_host(torch, dst), want, f"fnr k={k}")
    np.testing.assert_array_equal(cnt.cpu().numpy().astype(np.uint64), wcounts)


def test_defaults_and_tuning():
    for k in HUGE:
        assert irfilter.get_tuning("u16", k) == (128, irfilter.IRF_SELECT_GROUP)
        with pytest.raises(irfilter.IrfError):
            irfilter.set_tuning("u16", k, 256, irfilter.IRF_SELECT_GROUP)


@pytest.mark.parametrize("k", HUGE)
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_fnr_every_window(dev, dt, k):
    # 2 tiles across (the second ragged) and several tile rows, mixed impulses
    f = synth.make_frame(synth.FrameSpec(190, 101, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0, 3300 + k))
    check_fnr(f, k, dev)


@pytest.mark.parametrize("k", [33, 45, 63])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_detect_median_and_plain_median(dev, dt, k):
    f = synth.make_frame(synth.FrameSpec(150, 77, dt, "rv" if dt == "u16" else "sp", 0.25,
                                         20.0 if dt == "u16" else 0.0, 3400 + k))
    src = to_dev(torch, f, dev)
    say(f"case huge detect {dt} k={k}")
    mask = torch.full(f.shape, 7, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_detect(src, mask, k, flagged_count=cnt)
    torch.cuda.synchronize()
    wmask, wcount = oracle.detect(f, k)
    assert_same(mask.cpu().numpy(), wmask.astype(np.uint8), f"mask k={k}")
    assert int(cnt.item()) == int(wcount)
    say(f"case huge masked median {dt} k={k}")
    dst = torch.empty_like(src)
    irfilter.ir_filter_median(src, dst, k, mask=mask)
    torch.cuda.synchronize()
    assert_same(to_host(torch, dst), oracle.median(f, k, wmask)[0], f"masked median k={k}")
    say(f"case huge plain median {dt} k={k}")
    irfilter.ir_filter_median(src, dst, k)
    torch.cuda.synchronize()
    assert_same(to_host(torch, dst), oracle.median(f, k)[0], f"median filter k={k}")


@pytest.mark.parametrize("W,H,k", [(1, 1, 63), (2, 3, 33), (5, 70, 63), (70, 5, 41), (63, 63, 63),
                                   (128, 1, 35), (129, 40, 47), (257, 33, 39), (300, 33, 55)])
def test_shapes(dev, W, H, k):
    for dt in ("u8", "u16"):
        f = synth.make_frame(synth.FrameSpec(W, H, dt, "mixed", 0.35, 0.0 if dt == "u8" else 20.0, W * 11 + H))
        check_fnr(f, k, dev)


@pytest.mark.parametrize("k", [33, 63])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_ties_extremes_and_full_range(dev, dt, k):
    rng = np.random.default_rng(k + (dt == "u16"))
    check_fnr(synth.random_frame(rng, 140, 70, dt, alphabet=3), k, dev, tag="ties")
    vmax = 255 if dt == "u8" else 65535
    npdt = np.uint8 if dt == "u8" else np.uint16
    check_fnr(np.where(rng.random((70, 140)) < 0.5, 0, vmax).astype(npdt), k, dev, tag="s&p")
    check_fnr(rng.integers(0, vmax + 1, size=(60, 150)).astype(npdt), k, dev, tag="full range")
    say(f"case huge constant {dt} k={k}")
    f = np.full((40, 70), vmax, dtype=npdt)
    src = to_dev(torch, f, dev)
    dst = torch.empty_like(src)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
    torch.cuda.synchronize()
    assert_same(to_host(torch, dst), f, "constant frame")
    assert int(cnt.item()) == f.size


def test_two_passes_stack_and_batch_limit(dev):
    f = synth.make_frame(synth.FrameSpec(130, 90, "u16", "mixed", 0.4, 20.0, 3501))
    check_fnr(f, 37, dev, passes=2)
    N, W, H, k = 3, 133, 61, 51
    frames = [synth.make_frame(synth.FrameSpec(W, H, "u8", "sp", 0.1 + 0.1 * i, 0.0, 3510 + i)) for i in range(N)]
    say("case huge stack")
    src = to_dev(torch, np.stack(frames), dev)
    dst = torch.empty_like(src)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_run_frames(src, dst, k, flagged_count=cnt)
    torch.cuda.synchronize()
    out = to_host(torch, dst)
    tot = 0
    for i, fr in enumerate(frames):
        want, wc = oracle.fnr(fr, k)
        assert_same(out[i], want, f"stack frame {i}")
        tot += int(wc[0])
    assert int(cnt.item()) == tot
    # batch plans stop at 31x31
    with irfilter.Plan(2, 64) as plan:
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(src[0], dst[0], 33)])
        assert e.value.status == -5
