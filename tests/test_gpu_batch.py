"""GPU parity of the batched form: one persistent launch over uneven frames.

Every frame of a batch must equal the oracle's FNR result for that frame alone
(tolerance zero), and the per-frame noisy counts must match.  Graph replays are
checked one by one, with other device work and synchronisations between them.
"""

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, synth
from tests.gpu_helpers import full, same, say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


ALL_WINDOWS = tuple(range(3, 32, 2))


def make_batch(seed, n, max_w=420, max_h=300, windows=ALL_WINDOWS):
    rng = np.random.default_rng(seed)
    specs = []
    for j in range(n):
        W = int(rng.integers(1, max_w + 1)) if j % 5 else int(rng.integers(1, 20))
        H = int(rng.integers(1, max_h + 1)) if j % 7 else int(rng.integers(1, 20))
        dt = "u8" if rng.random() < 0.5 else "u16"
        k = int(rng.choice(windows))
        d = float(rng.uniform(0.05, 0.6))
        specs.append((synth.FrameSpec(W, H, dt, "mixed", d, 0.0 if dt == "u8" else 20.0, seed * 1000 + j), k))
    return specs


def run_and_check(dev, plan, specs, tag):
    frames = [synth.make_frame(s) for s, _ in specs]
    srcs = [to_dev(torch, f, dev) for f in frames]
    dsts = [torch.empty_like(s) for s in srcs]
    cnt = torch.zeros(len(specs), dtype=torch.int64, device=dev)
    say(f"case batch {tag}: {len(specs)} frames")
    plan.run([(s, d, k) for s, d, (_, k) in zip(srcs, dsts, specs)], flagged_counts=cnt)
    torch.cuda.synchronize()
    counts = cnt.cpu().numpy()
    for i, (f, (spec, k)) in enumerate(zip(frames, specs)):
        want, wc = oracle.fnr(f, k)
        got = to_host(torch, dsts[i])
        assert np.array_equal(got, want), (tag, i, spec, k, int((got != want).sum()))
        assert counts[i] == wc[0], (tag, i)
    return srcs, dsts


@pytest.mark.parametrize("graph", [False, True])
def test_uneven_batch_matches_oracle(dev, graph):
    specs = make_batch(11, 40)
    tiles = sum(irfilter.frame_tiles(s.width, s.height) for s, _ in specs)
    with irfilter.Plan(64, tiles + 10, graph=graph) as plan:
        run_and_check(dev, plan, specs, f"graph={graph}")


def test_graph_replays_with_changing_batches(dev):
    with irfilter.Plan(32, 4000, graph=True) as plan:
        for rep in range(5):
            # each batch uses another set of window classes (3..9, 11..15, single
            # windows above 15x15), so most replays first capture a new graph
            wins = [(3, 5, 7, 9), (3, 5, 7, 9, 13), (9, 17), (5, 25, 31), (3, 5, 7, 9)][rep]
            specs = make_batch(100 + rep, 12 + 3 * rep, windows=wins)
            run_and_check(dev, plan, specs, f"replay {rep}")
            # unrelated eager work between replays
            x = torch.randn(1 << 20, device=dev)
            torch.cuda.synchronize()
            assert torch.isfinite(x.sum())


def test_consecutive_batches_without_sync(dev):
    # several batches queued back to back on one stream reuse the plan's two
    # table sets alternately; every result must still be right
    rng_specs = [make_batch(200 + i, 10, windows=(5, 7)) for i in range(5)]
    with irfilter.Plan(16, 2000) as plan:
        pending = []
        for i, specs in enumerate(rng_specs):
            frames = [synth.make_frame(s) for s, _ in specs]
            srcs = [to_dev(torch, f, dev) for f in frames]
            dsts = [torch.empty_like(s) for s in srcs]
            plan.run([(s, d, k) for s, d, (_, k) in zip(srcs, dsts, specs)])
            pending.append((frames, specs, dsts))
        torch.cuda.synchronize()
        for frames, specs, dsts in pending:
            for f, (_, k), d in zip(frames, specs, dsts):
                assert np.array_equal(to_host(torch, d), oracle.fnr(f, k)[0])


def test_batch_equals_per_frame_launches_at_workload_size(dev):
    """The uneven-batch workload (256 frames, 160x120 .. 1280x1024, u8/u16,
    windows 3/5/7/9, 5-60 % mixed impulses): batch output equals the plain
    per-frame launch for every frame; every 16th frame also equals the oracle."""
    items = synth.c4_items(256)
    frames = [synth.make_frame(it.spec) for it in items]
    srcs = [to_dev(torch, f, dev) for f in frames]
    dsts = [torch.empty_like(s) for s in srcs]
    refs = [torch.empty_like(s) for s in srcs]
    tiles = sum(irfilter.frame_tiles(f.shape[1], f.shape[0]) for f in frames)
    cnt = torch.zeros(len(items), dtype=torch.int64, device=dev)
    say(f"case c4 batch: {len(items)} frames, {tiles} tiles")
    with irfilter.Plan(256, tiles, graph=True) as plan:
        plan.run([(s, d, it.window) for s, d, it in zip(srcs, dsts, items)], flagged_counts=cnt)
    c1 = torch.zeros(1, dtype=torch.int64, device=dev)
    per = []
    for s, r, it in zip(srcs, refs, items):
        irfilter.ir_filter_run(s, r, it.window, flagged_count=c1)
        per.append(c1.clone())
    torch.cuda.synchronize()
    counts = cnt.cpu().numpy()
    for i in range(len(items)):
        assert same(torch, dsts[i], refs[i]), i
        assert counts[i] == int(per[i].item()), i
    for i in range(0, len(items), 16):
        want, wc = oracle.fnr(frames[i], items[i].window)
        assert np.array_equal(to_host(torch, dsts[i]), want), i
        assert counts[i] == wc[0]


def test_batch_validation(dev):
    a = full(torch, (64, 64), 5, torch.uint8, dev)
    b = torch.empty_like(a)
    with irfilter.Plan(2, 8) as plan:
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(a, b, 3), (b, a, 3)])  # one frame's dst is another's src
        assert e.value.status == -7
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(a, b, 3)] * 3)  # more frames than the plan holds
        assert e.value.status == -10
        big = torch.empty((64 * 9, 128), dtype=torch.uint8, device=dev)
        big2 = torch.empty_like(big)
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(big, big2, 3)])  # 9 tiles > 8
        assert e.value.status == -10
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(a, b, 4)])
        assert e.value.status == -5
        with pytest.raises(irfilter.IrfError) as e:
            plan.run([(a, b, 33)])
        assert e.value.status == -5
        plan.run([(a, b, 3)])
        torch.cuda.synchronize()
        assert same(torch, b, a)


@pytest.mark.parametrize("graph", [False, True])
def test_every_window_class_in_one_batch(dev, graph):
    # one frame per window 3..31 and pixel type, tiny and ragged sizes included
    specs = []
    for j, k in enumerate(ALL_WINDOWS):
        for dt in ("u8", "u16"):
            W, H = (37 + 29 * j) % 300 + 1, (11 + 17 * j) % 200 + 1
            specs.append((synth.FrameSpec(W, H, dt, "mixed", 0.3, 0.0 if dt == "u8" else 20.0,
                                          7000 + 2 * j + (dt == "u16")), k))
    tiles = sum(irfilter.frame_tiles(s.width, s.height) for s, _ in specs)
    with irfilter.Plan(len(specs), tiles, graph=graph) as plan:
        run_and_check(dev, plan, specs, f"all classes graph={graph}")
