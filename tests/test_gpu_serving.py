"""GPU tests of the continuous-batching server: every served result equals the
result of the same frame filtered alone, and admission respects the memory
budget."""

import numpy as np
import pytest

import oracle
from paper_1201_3972_amd import irfilter, serving, synth
from tests.gpu_helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    irfilter.load()
    return torch.device("cuda:0")


def alone(dev, host_src, window):
    src = host_src.to(dev)
    dst = torch.empty_like(src)
    irfilter.ir_filter_run(src, dst, window)
    torch.cuda.synchronize()
    return to_host(torch, dst)


def test_results_in_the_mix_equal_results_alone(dev):
    streams, reqs = serving.video_workload(torch, seed=5, duration=0.6, n_streams=8, frames_per_stream=2)
    say(f"case serving mix: {len(reqs)} requests")
    srv = serving.Server(memory_budget=160 << 20, max_inflight=3)
    for s in streams:
        srv.register_stream(s.stream_id, s.width, s.height, s.dtype)
    for r in reqs:
        srv.submit(r)
    srv.run_until_idle()
    srv.close()
    assert len(srv.completed) == len(reqs)
    assert srv.steps < len(reqs)  # requests were batched together
    cache = {}
    for r in reqs:
        key = (r.host_src.data_ptr(), r.window)
        if key not in cache:
            cache[key] = alone(dev, r.host_src, r.window)
        assert np.array_equal(to_host(torch, r.host_dst), cache[key]), r.rid
        assert r.latency is not None and r.latency >= 0
    # the video frames also against the oracle (one per distinct frame and window)
    seen = set()
    for r in reqs:
        key = (r.host_src.data_ptr(), r.window)
        if r.stream_id is not None and key not in seen:
            seen.add(key)
            want, _ = oracle.fnr(to_host(torch, r.host_src), r.window)
            assert np.array_equal(to_host(torch, r.host_dst), want)


def test_memory_budget_serialises_large_frames(dev):
    _, reqs = serving.video_workload(torch, seed=9, duration=0.3, n_streams=2, large_fraction=0.5,
                                     frames_per_stream=1)
    large = [r for r in reqs if r.stream_id is None]
    assert len(large) >= 2
    nb = serving.frame_bytes(3840, 2160, "u16")
    # room for one large frame (input + output) and nothing else: one-off
    # frames go through the arena one at a time
    srv = serving.Server(memory_budget=2 * serving._round(nb), max_inflight=3)
    for r in reqs:
        srv.submit(r)
    srv.run_until_idle()
    srv.close()
    assert len(srv.completed) == len(reqs)
    assert srv.arena_used == 0
    ref = {}
    for r in large:
        key = (r.host_src.data_ptr(), r.window)
        if key not in ref:
            ref[key] = alone(dev, r.host_src, r.window)
        assert np.array_equal(to_host(torch, r.host_dst), ref[key])


def test_request_larger_than_budget_is_reported(dev):
    _, reqs = serving.video_workload(torch, seed=3, duration=0.2, n_streams=1, large_fraction=0.5,
                                     frames_per_stream=1)
    srv = serving.Server(memory_budget=1 << 20, max_inflight=2)
    for r in reqs:
        srv.submit(r)
    with pytest.raises(RuntimeError):
        srv.run_until_idle()
    srv.close()


def test_windows_above_31_are_rejected_at_submission(dev):
    # the server runs batch plans, which take windows up to IRF_MAX_BATCH_WINDOW (31)
    src = torch.zeros((64, 64), dtype=torch.uint8).pin_memory()
    srv = serving.Server(memory_budget=1 << 24, max_inflight=2)
    try:
        srv.submit(serving.Request(1, 0.0, src, 33))
        with pytest.raises(irfilter.IrfError) as e:
            srv.run_until_idle()
        assert e.value.status == -5
    finally:
        srv.close()


def test_large_windows_are_served_like_alone(dev):
    # one-off frames with windows above 15x15 beside small-window ones: each
    # result equals the same frame filtered alone, and the oracle
    specs = [(synth.FrameSpec(300, 200, "u16", "mixed", 0.3, 20.0, 9100), 21),
             (synth.FrameSpec(257, 129, "u8", "sp", 0.2, 0.0, 9101), 31),
             (synth.FrameSpec(640, 512, "u16", "rv", 0.3, 20.0, 9102), 5),
             (synth.FrameSpec(190, 77, "u8", "mixed", 0.4, 0.0, 9103), 17)]
    srv = serving.Server(memory_budget=1 << 26, max_inflight=2)
    reqs = []
    try:
        for i, (spec, k) in enumerate(specs):
            f = synth.make_frame(spec)
            t = torch.from_numpy(f.view(np.int16)).view(torch.uint16) if f.dtype == np.uint16 else torch.from_numpy(f)
            reqs.append((f, k, serving.Request(i, 0.0005 * i, t.pin_memory(), k)))
            srv.submit(reqs[-1][2])
        say("case serving: large windows beside small ones")
        srv.run_until_idle()
    finally:
        srv.close()
    for f, k, r in reqs:
        got = r.host_dst.view(torch.int16).numpy().view(np.uint16) if f.dtype == np.uint16 else r.host_dst.numpy()
        src = to_dev(torch, f, dev)
        alone = torch.empty_like(src)
        irfilter.ir_filter_run(src, alone, k)
        torch.cuda.synchronize()
        assert np.array_equal(got, to_host(torch, alone)), (f.shape, k)
        assert np.array_equal(got, oracle.fnr(f, k)[0]), (f.shape, k)
