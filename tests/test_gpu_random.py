"""Seeded random GPU parity cases across the whole surface of the C ABI.

Each case draws a frame shape, pixel type, window (3..63), noise, entry point
(the whole filter with 1-3 passes, detection, the masked or plain median, the
directional detector), kernel choices (workgroup size, selection algorithm,
fusion of passes) and a layout (aligned or offset rows), and checks the result
and counts against the oracle bit for bit.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_CASES = 160
WINDOWS = [3, 5, 7, 9, 11, 13, 15, 17, 21, 25, 31, 33, 45, 63]
WEIGHTS = [.15, .15, .13, .11, .08, .06, .06, .06, .05, .04, .04, .03, .02, .02]


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
    t = t.contiguous()
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def draw(case):
    rng = np.random.default_rng(90_000 + case)
    k = int(rng.choice(WINDOWS, p=WEIGHTS))
    dt = "u8" if rng.random() < 0.5 else "u16"
    W, H = int(rng.integers(1, 600)), int(rng.integers(1, 300))
    if k >= 17:
        W, H = min(W, 260), min(H, 160)
    if k >= 33:
        W, H = min(W, 200), min(H, 120)
    op = str(rng.choice(["run", "run", "run", "detect", "masked", "median", "directional"]))
    passes = int(rng.choice([1, 2, 3], p=[.6, .3, .1])) if op == "run" else 1
    noise = str(rng.choice(["sp", "rv", "mixed", "none"]))
    density = float(rng.uniform(0.05, 0.6))
    seed = int(rng.integers(1 << 30))
    ties = rng.random() < 0.1
    sels = ([irfilter.IRF_SELECT_NETWORK, irfilter.IRF_SELECT_BISECT] if k <= 15 else
            [irfilter.IRF_SELECT_GROUP, irfilter.IRF_SELECT_HIST] if k <= 31 else [irfilter.IRF_SELECT_GROUP])
    threads, sel = int(rng.choice([128, 256] if k <= 31 else [128])), int(rng.choice(sels))
    fusion = int(rng.choice([-1, 0, 256, 512])) if k <= 9 else int(rng.choice([-1, 0]))
    off = int(rng.choice([0, 0, 1, 3]))
    return dict(k=k, dt=dt, W=W, H=H, op=op, passes=passes, noise=noise, density=density, seed=seed, ties=ties,
                threads=threads, sel=sel, fusion=fusion, off=off, rng=rng)


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_case(dev, case):
    c = draw(case)
    k, dt, W, H, off = c["k"], c["dt"], c["W"], c["H"], c["off"]
    if c["ties"]:
        f = synth.random_frame(c["rng"], W, H, dt, alphabet=int(c["rng"].integers(2, 5)))
    else:
        f = synth.make_frame(synth.FrameSpec(W, H, dt, c["noise"], c["density"], 0.0 if dt == "u8" else 20.0,
                                             c["seed"]))
    say(f"case random {case}: {dt} {W}x{H} k={k} op={c['op']} passes={c['passes']} threads={c['threads']} "
        f"select={c['sel']} fusion={c['fusion']} off={off}")
    irfilter.set_tuning(dt, k, c["threads"], c["sel"])
    irfilter.set_fusion(dt, k, c["fusion"])
    try:
        big = np.zeros((H, W + 8), dtype=f.dtype)
        big[:, off:off + W] = f
        src = to_dev(big, dev)[:, off:off + W]
        out_big = torch.zeros((H, W + 8), dtype=src.dtype if c["op"] not in ("detect", "directional")
                              else torch.uint8, device=dev)
        out = out_big[:, off:off + W]
        cnt = torch.zeros(max(c["passes"], 1), dtype=torch.int64, device=dev)
        if c["op"] == "run":
            scr = torch.empty((H, W), dtype=src.dtype, device=dev)
            irfilter.ir_filter_run(src, out, k, passes=c["passes"], scratch=scr, flagged_count=cnt)
            want, wc = oracle.fnr(f, k, c["passes"])
        elif c["op"] == "detect":
            irfilter.ir_filter_detect(src, out, k, flagged_count=cnt)
            want, n = oracle.detect(f, k)
            wc = np.array([n], dtype=np.uint64)
        elif c["op"] == "directional":
            irfilter.ir_filter_detect_directional(src, out, flagged_count=cnt)
            want, n = oracle.detect_directional(f)
            wc = np.array([n], dtype=np.uint64)
        else:
            mask = None
            if c["op"] == "masked":
                m = (c["rng"].random((H, W)) < c["density"]).astype(np.uint8)
                mask = to_dev(m, dev)
            irfilter.ir_filter_median(src, out, k, mask=mask)
            want = oracle.median(f, k, None if mask is None else m)[0]
            wc = None
        torch.cuda.synchronize()
        got = to_host(out)
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            y, x = bad[0]
            raise AssertionError(f"{len(bad)} values differ; first at (x={x}, y={y}): gpu {got[y, x]} "
                                 f"oracle {want[y, x]}")
        if wc is not None:
            np.testing.assert_array_equal(cnt.cpu().numpy().astype(np.uint64), wc)
        padding = to_host(out_big)
        assert not padding[:, :off].any() and not padding[:, off + W:].any()
    finally:
        irfilter.set_tuning(dt, k, 0, 0)
        irfilter.set_fusion(dt, k, -1)
