"""GPU parity of the opt-in directional detector (``ir_filter_detect_directional``).

Not the paper's detector: a reading of Fig. 1's caption, pinned in
``tests/test_oracle_directional.py``.  The mask and count must equal the
oracle's bit for bit, and composing the mask with ``ir_filter_median`` must
equal the oracle's masked median.
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


def check(frame, dev, tag=""):
    say(f"case directional {tag} {frame.dtype} {frame.shape[1]}x{frame.shape[0]}")
    want, wc = oracle.detect_directional(frame)
    src = to_dev(frame, dev)
    mask = torch.full(frame.shape, 9, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    irfilter.ir_filter_detect_directional(src, mask, flagged_count=cnt)
    torch.cuda.synchronize()
    got = mask.cpu().numpy()
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError(f"{len(bad)} mask bytes differ; first at (x={x}, y={y}): gpu {got[y, x]} "
                             f"oracle {want[y, x]}")
    assert int(cnt.item()) == wc
    return mask


def _shapes():
    rng = np.random.default_rng(44)
    dims = [1, 2, 3, 4, 5, 7, 8, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200, 257]
    return [(int(rng.choice(dims)), int(rng.choice(dims)), "u8" if i % 2 else "u16", ["sp", "rv", "mixed"][i % 3],
             3000 + i) for i in range(30)]


@pytest.mark.parametrize("W,H,dt,noise,seed", _shapes())
def test_shapes(dev, W, H, dt, noise, seed):
    f = synth.make_frame(synth.FrameSpec(W, H, dt, noise, 0.3, 0.0 if dt == "u8" else 20.0, seed))
    check(f, dev)


@pytest.mark.parametrize("threads", [128, 256])
@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_workgroup_sizes_and_ties(dev, dt, threads):
    irfilter.set_tuning(dt, 3, threads, irfilter.IRF_SELECT_NETWORK)
    try:
        rng = np.random.default_rng(threads)
        check(synth.random_frame(rng, 300, 170, dt, alphabet=3), dev, tag=f"t{threads} ties")
        check(synth.random_frame(rng, 300, 170, dt), dev, tag=f"t{threads} uniform")
        check(synth.make_frame(synth.c2_spec(0.3, 0)) if dt == "u16" else synth.c1_frame(), dev,
              tag=f"t{threads} workload")
    finally:
        irfilter.set_tuning(dt, 3, 0, 0)


def test_lines_kept_and_impulses_found(dev):
    f = np.full((64, 200), 50, dtype=np.uint8)
    f[10, 5:190] = 220            # one-pixel row
    f[15:60, 100] = 10            # one-pixel column
    idx = np.arange(20, 60)
    f[idx, idx + 20] = 230        # diagonal
    f[40, 150] = 255              # impulses
    f[30, 170] = 0
    m = check(f, dev, tag="lines").cpu().numpy()
    assert m[40, 150] == 1 and m[30, 170] == 1
    assert not m[10, 6:189].any()


@pytest.mark.parametrize("dt", ["u8", "u16"])
def test_unaligned_layout(dev, dt):
    W, H, off = 203, 150, 3
    f = synth.make_frame(synth.FrameSpec(W, H, dt, "mixed", 0.3, 20.0 if dt == "u16" else 0.0, 61))
    want, wc = oracle.detect_directional(f)
    big = np.zeros((H, W + 37), dtype=f.dtype)
    big[:, off:off + W] = f
    src = to_dev(big, dev)[:, off:off + W]
    mbig = torch.full((H, W + 29), 5, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    say(f"case directional unaligned {dt}")
    irfilter.ir_filter_detect_directional(src, mbig[:, 1:1 + W], flagged_count=cnt)
    torch.cuda.synchronize()
    out = mbig.cpu().numpy()
    np.testing.assert_array_equal(out[:, 1:1 + W], want)
    assert (out[:, 0] == 5).all() and (out[:, 1 + W:] == 5).all()
    assert int(cnt.item()) == wc


@pytest.mark.parametrize("k", [3, 5, 9])
def test_composed_with_the_masked_median(dev, k):
    f = synth.make_frame(synth.FrameSpec(364, 244, "u8", "sp", 0.2, 0.0, 62 + k))
    mask = check(f, dev, tag=f"compose k={k}")
    src = to_dev(f, dev)
    dst = torch.empty_like(src)
    irfilter.ir_filter_median(src, dst, k, mask=mask)
    torch.cuda.synchronize()
    want, _ = oracle.median(f, k, oracle.detect_directional(f)[0])
    np.testing.assert_array_equal(to_host(dst), want)
