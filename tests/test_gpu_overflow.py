"""Tiles whose flagged pixels overflow the 5x5 and 7x7 stack kernels' list (more
than 3/8 of the tile; the 7x7 standard median filter keeps a slot per pixel):
they select in rounds and store every median straight to the frame after
storing the tile unfiltered.  Frames with flag rates from about
a third to all pixels, ragged sizes and both workgroup sizes, against the
oracle (whole frames, every pixel and the count)."""

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, synth
from tests.gpu_helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


@pytest.fixture
def tuning():
    touched = []

    def set_(dt, k, t, sel):
        irfilter.set_tuning(dt, k, t, sel)
        touched.append((dt, k))

    yield set_
    for dt, k in touched:
        irfilter.set_tuning(dt, k, 0, 0)


def frames(dt, seed):
    rng = np.random.default_rng(seed)
    vmax = 255 if dt == "u8" else 65535
    npdt = np.uint8 if dt == "u8" else np.uint16
    yield "alphabet 2", rng.integers(0, 2, size=(150, 301)).astype(npdt)          # ties everywhere
    yield "alphabet 3", rng.integers(0, 3, size=(131, 260)).astype(npdt)
    yield "constant", np.full((97, 200), 7, dtype=npdt)                            # every pixel flagged
    yield "s&p 70%", np.where(rng.random((140, 333)) < 0.7,
                               np.where(rng.random((140, 333)) < 0.5, 0, vmax), 100).astype(npdt)
    yield "mixed 60%", synth.make_frame(synth.FrameSpec(290, 171, dt, "mixed", 0.6, 0.0 if dt == "u8" else 20.0,
                                                         seed))


@pytest.mark.parametrize("sel", [irfilter.IRF_SELECT_NETWORK, irfilter.IRF_SELECT_BISECT])
@pytest.mark.parametrize("t", [128, 256])
@pytest.mark.parametrize("k", [5, 7, 9, 13])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_dense_flags_match_oracle(dev, tuning, dt, k, t, sel):
    tuning(dt, k, t, sel)
    for name, f in frames(dt, 4000 + k):
        say(f"case overflow {name} {dt} k={k} t={t} sel={sel}")
        src = to_dev(torch, f, dev)
        dst = torch.empty_like(src)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        irfilter.ir_filter_run(src, dst, k, flagged_count=cnt)
        torch.cuda.synchronize()
        want, wc = oracle.fnr(f, k)
        got = to_host(torch, dst)
        assert np.array_equal(got, want), (name, int((got != want).sum()))
        assert int(cnt.item()) == int(wc[0]), name


@pytest.mark.parametrize("k", [5, 7, 17])
def test_dense_flags_plain_median_and_stack(dev, k):
    # the standard median filter flags every pixel; a stack with padded rows
    f = np.random.default_rng(k).integers(0, 1 << 14, size=(3, 133, 270)).astype(np.uint16)
    src = torch.zeros((3, 133, 272), dtype=torch.int16, device=dev).view(torch.uint16)[:, :, :270]
    src.copy_(to_dev(torch, f, dev))
    dst = torch.full((3, 133, 272), 0x5a5a, dtype=torch.int16, device=dev).view(torch.uint16)
    say(f"case overflow plain median k={k}")
    for i in range(3):
        irfilter.ir_filter_median(src[i], dst[i, :, :270], k)
    torch.cuda.synchronize()
    out = to_host(torch, dst)
    for i in range(3):
        assert np.array_equal(out[i, :, :270], oracle.median(f[i], k)[0]), i
    assert (out[:, :, 270:] == 0x5a5a).all()  # row padding untouched


@pytest.mark.parametrize("k", [5, 7])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_dense_caller_mask(dev, dt, k):
    # the masked median with a caller mask that marks about 70 % of the pixels
    rng = np.random.default_rng(77 + (dt == "u16") + 2 * k)
    hi = 256 if dt == "u8" else 1 << 14
    f = rng.integers(0, hi, size=(150, 261)).astype(np.uint8 if dt == "u8" else np.uint16)
    mask = (rng.random(f.shape) < 0.7).astype(np.uint8)
    src = to_dev(torch, f, dev)
    m = torch.from_numpy(mask).to(dev)
    dst = torch.empty_like(src)
    say(f"case overflow caller mask {dt} k={k}")
    irfilter.ir_filter_median(src, dst, k, mask=m)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(torch, dst), oracle.median(f, k, mask)[0])


@pytest.mark.parametrize("k", [5, 7])
def test_overflow_stack_and_sparse_neighbours(dev, k):
    # a stack whose frames alternate between sparse flags (the list holds them)
    # and dense ones (rounds), with 128 and 256 threads: both paths side by side
    rng = np.random.default_rng(500 + k)
    sparse = synth.make_frame(synth.FrameSpec(640, 128, "u16", "rv", 0.3, 20.0, 600 + k))
    dense = np.where(rng.random((128, 640)) < 0.6, np.where(rng.random((128, 640)) < 0.5, 0, 65535),
                     sparse).astype(np.uint16)
    st = np.stack([sparse, dense, sparse, dense])
    for t in (128, 256):
        irfilter.set_tuning("u16", k, t, irfilter.IRF_SELECT_NETWORK)
        try:
            say(f"case overflow stack k={k} t={t}")
            src = to_dev(torch, st, dev)
            dst = torch.empty_like(src)
            cnt = torch.zeros(1, dtype=torch.int64, device=dev)
            irfilter.ir_filter_run_frames(src, dst, k, flagged_count=cnt)
            torch.cuda.synchronize()
        finally:
            irfilter.set_tuning("u16", k, 0, 0)
        out = to_host(torch, dst)
        tot = 0
        for i in range(len(st)):
            want, wc = oracle.fnr(st[i], k)
            assert np.array_equal(out[i], want), (i, t)
            tot += int(wc[0])
        assert int(cnt.item()) == tot
