"""GPU parity of every tuning choice: each (workgroup size, selection
algorithm) kernel must give the oracle's result bit for bit, for every window
and pixel type, in every mode, and batches must too under either batch
workgroup size.  Also a short autotuner run."""

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import autotune, irfilter, synth
from tests.gpu_helpers import same, say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WINDOWS = (3, 5, 7, 9, 11, 13, 15)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    for dt in ("u8", "u16"):
        for k in WINDOWS:
            irfilter.set_tuning(dt, k, 0, 0)
    irfilter.set_batch_threads(0)


_FRAMES = {}


def frames(dt):
    """Two frames per pixel type: 150x70 with mixed impulses at 30 % (ragged
    tiles of both heights) and 33x9 at 60 %."""
    if dt not in _FRAMES:
        sig = 0.0 if dt == "u8" else 20.0
        _FRAMES[dt] = [synth.make_frame(synth.FrameSpec(150, 70, dt, "mixed", 0.3, sig, 901 + (dt == "u16"))),
                       synth.make_frame(synth.FrameSpec(33, 9, dt, "mixed", 0.6, sig, 903 + (dt == "u16")))]
    return _FRAMES[dt]


_WANT = {}


def want(dt, k, i, what):
    key = (dt, k, i, what)
    if key not in _WANT:
        f = frames(dt)[i]
        if what == "fnr":
            _WANT[key] = oracle.fnr(f, k)[0]
        elif what == "median":
            _WANT[key] = oracle.median(f, k)[0]
        else:
            _WANT[key] = oracle.detect(f, k)[0].astype(np.uint8)
    return _WANT[key]


@pytest.mark.parametrize("dt", ["u8", "u16"])
@pytest.mark.parametrize("k", WINDOWS)
def test_every_choice_matches_oracle(dev, dt, k):
    for threads, sel in autotune.candidates(k):
        say(f"tuning {dt} {k}x{k} threads={threads} select={sel}")
        irfilter.set_tuning(dt, k, threads, sel)
        for i, f in enumerate(frames(dt)):
            src = to_dev(torch, f, dev)
            dst = torch.empty_like(src)
            irfilter.ir_filter_run(src, dst, k)
            med = torch.empty_like(src)
            irfilter.ir_filter_median(src, med, k)
            mask = torch.empty(f.shape, dtype=torch.uint8, device=dev)
            irfilter.ir_filter_detect(src, mask, k)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(torch, dst), want(dt, k, i, "fnr")), (threads, sel, i)
            assert np.array_equal(to_host(torch, med), want(dt, k, i, "median")), (threads, sel, i)
            assert np.array_equal(mask.cpu().numpy(), want(dt, k, i, "detect")), (threads, sel, i)
        # a stack (one launch over several frames)
        f = frames(dt)[0]
        src = to_dev(torch, np.stack([f, f[::-1].copy(), f]), dev)
        dst = torch.empty_like(src)
        irfilter.ir_filter_run_frames(src, dst, k)
        torch.cuda.synchronize()
        got = to_host(torch, dst)
        assert np.array_equal(got[0], want(dt, k, 0, "fnr"))
        assert np.array_equal(got[2], want(dt, k, 0, "fnr"))
        assert np.array_equal(got[1], oracle.fnr(f[::-1].copy(), k)[0])


def test_masked_median_every_choice(dev):
    f = frames("u16")[0]
    rng = np.random.default_rng(5)
    m = (rng.random(f.shape) < 0.3).astype(np.uint8)
    exp = np.where(m != 0, oracle.median(f, 9)[0], f)
    src = to_dev(torch, f, dev)
    mask = torch.from_numpy(m).to(dev)
    for threads, sel in autotune.candidates(9):
        irfilter.set_tuning("u16", 9, threads, sel)
        dst = torch.empty_like(src)
        irfilter.ir_filter_median(src, dst, 9, mask=mask)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(torch, dst), exp), (threads, sel)


@pytest.mark.parametrize("threads", [128, 256])
def test_batch_under_either_workgroup_size(dev, threads):
    irfilter.set_batch_threads(threads)
    rng = np.random.default_rng(77)
    specs = []
    for j in range(24):
        dt = "u8" if j % 2 else "u16"
        W, H = int(rng.integers(1, 300)), int(rng.integers(1, 200))
        specs.append((synth.FrameSpec(W, H, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0, 7000 + j),
                      WINDOWS[j % len(WINDOWS)]))
    fr = [synth.make_frame(s) for s, _ in specs]
    srcs = [to_dev(torch, f, dev) for f in fr]
    dsts = [torch.empty_like(x) for x in srcs]
    tiles = sum(irfilter.frame_tiles(f.shape[1], f.shape[0]) for f in fr)
    with irfilter.Plan(len(fr), tiles) as plan:
        say(f"batch threads={threads} tiles={tiles}")
        plan.run([(a, b, k) for a, b, (_, k) in zip(srcs, dsts, specs)])
        torch.cuda.synchronize()
    for f, d, (_, k) in zip(fr, dsts, specs):
        assert np.array_equal(to_host(torch, d), oracle.fnr(f, k)[0])


def test_autotuner_short_run(dev):
    say("autotune short run")
    pool = [synth.make_frame(synth.FrameSpec(256, 96, "u16", "rv", 0.3, 20.0, 31))]
    out = autotune.tune_single(torch, "u16", windows=(5, 13), frames=4, rounds=1, reps=1, pool=pool)
    for k in ("5", "13"):
        ent = out[k]
        assert (ent["threads"], autotune.SELECT_BY_NAME[ent["select"]]) in autotune.candidates(int(k))
        assert irfilter.get_tuning("u16", int(k)) == (ent["threads"], autotune.SELECT_BY_NAME[ent["select"]])
        assert len(ent["ms"]) == len(autotune.candidates(int(k)))
    fu = autotune.tune_fusion(torch, "u16", windows=(3, 9, 11), frames=4, rounds=1, reps=1, pool=pool)
    assert set(fu) == {"3", "9"}  # no fused kernel above 9x9
    for k, ent in fu.items():
        assert ent["threads"] in autotune.FUSION_CHOICES + (irfilter.FUSION_AUTO,)
        assert irfilter.get_fusion("u16", int(k)) == ent["threads"]
        if ent["threads"] == irfilter.FUSION_AUTO:
            assert ent["auto"] == irfilter.resolve_fusion("u16", int(k), 256, 96)
        irfilter.set_fusion("u16", int(k), -1)
    b = autotune.tune_batch(torch, n=12, rounds=1, reps=1)
    assert b["threads"] in (128, 256) and irfilter.get_batch_threads() == b["threads"]
