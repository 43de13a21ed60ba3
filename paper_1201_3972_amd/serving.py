"""Continuous-batching request loop for video-frame FNR filtering on one GPU.

Requests (one frame each, any size / pixel type / window) arrive over time.  The
engine keeps up to ``max_inflight`` batches on the device at once:

* admission -- an arrived request is admitted into the next batch when device
  memory for its input and output is available: frames of a registered video
  stream use that stream's resident slot (allocated once, kept for the stream's
  lifetime, reused frame after frame); other frames take space from a bounded
  device arena and give it back when their result has reached the host.  A
  request that does not fit waits; nothing is dropped.
* one step -- the admitted requests are copied host -> device on the copy
  stream, filtered by ONE batched launch (``irfilter.Plan``, a persistent
  kernel over all their tiles) on the compute stream, and copied back on the
  copy stream; events order the three.  Steps are issued while earlier ones are
  still running, so copies of one batch overlap the kernel of another.
* completion -- a batch is complete when its device -> host copy has finished;
  each request's latency is completion minus arrival (host clock).

Only the host-side bookkeeping lives here; all filtering runs in the HIP
kernels behind the C ABI.  Streams are created at the default priority.
"""

from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import irfilter

_ALIGN = 4096


def frame_bytes(width: int, height: int, dtype: str) -> int:
    return width * height * (1 if dtype == "u8" else 2)


def _round(n: int) -> int:
    return (n + _ALIGN - 1) // _ALIGN * _ALIGN


class DeviceArena:
    """First-fit allocator over one preallocated device buffer (the memory
    budget for transient frames).  Offsets are aligned to 4 KiB; freed blocks
    coalesce with their neighbours."""

    def __init__(self, torch, nbytes: int, device):
        self.torch = torch
        self.capacity = _round(nbytes)
        self.buf = torch.empty(self.capacity, dtype=torch.uint8, device=device)
        self.free: List[Tuple[int, int]] = [(0, self.capacity)]  # (offset, size), sorted
        self.used = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        need = _round(nbytes)
        for i, (off, size) in enumerate(self.free):
            if size >= need:
                if size == need:
                    del self.free[i]
                else:
                    self.free[i] = (off + need, size - need)
                self.used += need
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        need = _round(nbytes)
        self.used -= need
        blocks = self.free
        i = 0
        while i < len(blocks) and blocks[i][0] < off:
            i += 1
        blocks.insert(i, (off, need))
        # merge with the next, then with the previous
        if i + 1 < len(blocks) and blocks[i][0] + blocks[i][1] == blocks[i + 1][0]:
            blocks[i] = (blocks[i][0], blocks[i][1] + blocks[i + 1][1])
            del blocks[i + 1]
        if i > 0 and blocks[i - 1][0] + blocks[i - 1][1] == blocks[i][0]:
            blocks[i - 1] = (blocks[i - 1][0], blocks[i - 1][1] + blocks[i][1])
            del blocks[i]

    def view(self, off: int, width: int, height: int, dtype: str):
        t = self.torch
        n = frame_bytes(width, height, dtype)
        v = self.buf[off:off + n]
        return (v.view(t.uint8) if dtype == "u8" else v.view(t.uint16)).view(height, width)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds, on the engine's clock
    host_src: object        # pinned torch tensor [H, W]
    window: int
    stream_id: Optional[int] = None  # registered video stream, or None for a one-off frame
    host_dst: object = None  # pinned torch tensor [H, W], filled by the engine
    done: Optional[float] = None

    @property
    def shape(self):
        return tuple(self.host_src.shape)

    @property
    def dtype(self) -> str:
        return "u8" if self.host_src.element_size() == 1 else "u16"

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class _Slot:
    """Resident device buffers of one registered video stream."""

    def __init__(self, torch, width, height, dtype, device):
        td = torch.uint8 if dtype == "u8" else torch.uint16
        self.src = torch.empty((height, width), dtype=td, device=device)
        self.dst = torch.empty_like(self.src)
        self.busy = False


class _Batch:
    def __init__(self, reqs, ev_done, arena_blocks, slots):
        self.reqs = reqs
        self.ev_done = ev_done
        self.arena_blocks = arena_blocks  # [(offset, nbytes)]
        self.slots = slots


class Server:
    """Continuous-batching FNR server on one GPU (see the module docstring)."""

    def __init__(self, memory_budget: int, max_batch_frames: int = 512, max_batch_tiles: int = 1 << 16,
                 max_inflight: int = 3, graph: bool = True, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena = DeviceArena(torch, memory_budget, self.device)
        self.plans = [irfilter.Plan(max_batch_frames, max_batch_tiles, graph=graph)
                      for _ in range(max_inflight)]
        self.max_batch_frames = max_batch_frames
        self.max_batch_tiles = max_batch_tiles
        self.max_inflight = max_inflight
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.compute_stream = torch.cuda.Stream(device=self.device)
        self.slots: Dict[int, _Slot] = {}
        self.future: collections.deque = collections.deque()  # not yet arrived, by arrival
        self.pending: collections.deque = collections.deque()  # arrived, not admitted
        self.inflight: collections.deque = collections.deque()
        self.completed: List[Request] = []
        self.steps = 0
        self.batch_sizes: List[int] = []
        self._plan_i = 0
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def register_stream(self, stream_id: int, width: int, height: int, dtype: str, depth: int = 2) -> None:
        """Give a video stream ``depth`` resident device slots for its whole
        lifetime; a frame takes any free slot of its stream, so up to ``depth``
        consecutive frames of one stream can be in flight together."""
        self.slots[stream_id] = [_Slot(self.torch, width, height, dtype, self.device) for _ in range(depth)]

    def submit(self, req: Request) -> None:
        """Queue a request; it becomes eligible once the engine clock passes
        ``req.arrival`` (submit in arrival order)."""
        if req.host_dst is None:
            req.host_dst = self.torch.empty_like(req.host_src, pin_memory=True)
        if self.future and req.arrival < self.future[-1].arrival:
            raise ValueError("submit requests in arrival order")
        self.future.append(req)

    def _arrive(self) -> None:
        now = self.now()
        while self.future and self.future[0].arrival <= now:
            self.pending.append(self.future.popleft())

    # -- engine ---------------------------------------------------------------
    def _admit(self):
        """Arrived requests that fit now, in arrival order (a request that does
        not fit does not block later ones that do)."""
        admitted, blocks, slots = [], [], []
        tiles = 0
        keep = collections.deque()
        while self.pending:
            r = self.pending.popleft()
            if len(admitted) >= self.max_batch_frames:
                keep.append(r)
                continue
            H, W = r.shape
            nt = irfilter.frame_tiles(W, H)
            if tiles + nt > self.max_batch_tiles:
                keep.append(r)
                continue
            if r.stream_id is not None and r.stream_id in self.slots:
                s = next((x for x in self.slots[r.stream_id] if not x.busy), None)
                if s is None or (r.shape != tuple(s.src.shape)):
                    keep.append(r)  # the stream's earlier frames still own its slots
                    continue
                s.busy = True
                slots.append(s)
                admitted.append((r, s.src, s.dst))
            else:
                nb = frame_bytes(W, H, r.dtype)
                a = self.arena.alloc(nb)
                b = self.arena.alloc(nb) if a is not None else None
                if b is None:
                    if a is not None:
                        self.arena.release(a, nb)
                    keep.append(r)
                    continue
                blocks += [(a, nb), (b, nb)]
                admitted.append((r, self.arena.view(a, W, H, r.dtype), self.arena.view(b, W, H, r.dtype)))
            tiles += nt
        self.pending = keep
        return admitted, blocks, slots

    def _issue(self, admitted, blocks, slots) -> None:
        torch = self.torch
        cs, ks = self.copy_stream, self.compute_stream
        with torch.cuda.stream(cs):
            for r, dsrc, _ in admitted:
                dsrc.copy_(r.host_src, non_blocking=True)
        ev_in = torch.cuda.Event()
        ev_in.record(cs)
        ks.wait_event(ev_in)
        plan = self.plans[self._plan_i]
        self._plan_i = (self._plan_i + 1) % len(self.plans)
        plan.run([(dsrc, ddst, r.window) for r, dsrc, ddst in admitted], stream=ks)
        ev_k = torch.cuda.Event()
        ev_k.record(ks)
        cs.wait_event(ev_k)
        with torch.cuda.stream(cs):
            for r, _, ddst in admitted:
                r.host_dst.copy_(ddst, non_blocking=True)
        ev_done = torch.cuda.Event()
        ev_done.record(cs)
        self.inflight.append(_Batch([r for r, _, _ in admitted], ev_done, blocks, slots))
        self.steps += 1
        self.batch_sizes.append(len(admitted))

    def _retire(self, block: bool = False) -> int:
        n = 0
        while self.inflight:
            b = self.inflight[0]
            if block:
                b.ev_done.synchronize()
            elif not b.ev_done.query():
                break
            t = self.now()
            for r in b.reqs:
                r.done = t
            self.completed.extend(b.reqs)
            for off, nb in b.arena_blocks:
                self.arena.release(off, nb)
            for slot in b.slots:
                slot.busy = False
            self.inflight.popleft()
            n += 1
            block = False
        return n

    def poll(self) -> bool:
        """One engine iteration: retire finished batches, then issue a new one
        if there is room and arrived work fits.  Returns True on progress."""
        progressed = self._retire() > 0
        self._arrive()
        if len(self.inflight) < self.max_inflight and self.pending:
            admitted, blocks, slots = self._admit()
            if admitted:
                self._issue(admitted, blocks, slots)
                progressed = True
        return progressed

    def run_until_idle(self, idle_sleep: float = 50e-6) -> None:
        """Serve until every submitted request has completed."""
        while self.future or self.pending or self.inflight:
            if self.poll():
                continue
            if len(self.inflight) >= self.max_inflight:
                self._retire(block=True)  # wait for the oldest batch
            elif self.inflight:
                time.sleep(idle_sleep)  # completions or arrivals will come
            elif self.pending:
                raise RuntimeError("an arrived request does not fit the device-memory budget")
            else:
                wait = self.future[0].arrival - self.now()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))

    def close(self) -> None:
        self._retire(block=True)
        for p in self.plans:
            p.close()


# ----------------------------------------------------------------------------
# workload: video streams with Poisson arrivals plus occasional large frames
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class StreamSpec:
    stream_id: int
    width: int
    height: int
    dtype: str
    window: int
    fps: float


def poisson_arrivals(rng: np.random.Generator, rate: float, duration: float) -> np.ndarray:
    """Arrival times of a Poisson process of ``rate`` per second on [0, duration)."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.asarray(out)
        out.append(t)


def video_workload(torch, seed: int, duration: float, n_streams: int = 32, fps: float = 30.0,
                   large_fraction: float = 0.05, windows: Sequence[int] = (3, 5, 7, 9),
                   frames_per_stream: int = 4, rate_scale: float = 1.0):
    """The serving workload: ``n_streams`` 640x512 u16 streams at ``fps`` with
    exponential inter-arrival times, plus 3840x2160 u16 frames making up
    ``large_fraction`` of all requests; each stream keeps one window, each large
    frame draws one.  Frame content comes from a small pool of distinct
    synthetic frames per stream (pinned host memory)."""
    from . import synth

    rng = np.random.default_rng(seed)
    streams = [StreamSpec(i, 640, 512, "u16", int(rng.choice(windows)), fps) for i in range(n_streams)]
    pools = {}
    for s in streams:
        pools[s.stream_id] = [
            torch.from_numpy(synth.make_frame(synth.FrameSpec(
                640, 512, "u16", "rv", float(rng.uniform(0.05, 0.4)), 20.0,
                seed * 100000 + s.stream_id * 100 + j)).view(np.int16)).view(torch.uint16).pin_memory()
            for j in range(frames_per_stream)]
    large_pool = [torch.from_numpy(synth.make_frame(synth.FrameSpec(
        3840, 2160, "u16", "mixed", 0.3, 20.0, seed * 100000 + 99000 + j)).view(np.int16)).view(torch.uint16).pin_memory()
        for j in range(2)]
    reqs = []
    rid = 0
    for s in streams:
        for j, t in enumerate(poisson_arrivals(rng, s.fps * rate_scale, duration)):
            reqs.append(Request(rid, float(t), pools[s.stream_id][j % frames_per_stream], s.window, s.stream_id))
            rid += 1
    n_video = len(reqs)
    large_rate = n_video / duration * large_fraction / (1.0 - large_fraction)
    for j, t in enumerate(poisson_arrivals(rng, large_rate, duration)):
        reqs.append(Request(rid, float(t), large_pool[j % len(large_pool)], int(rng.choice(windows)), None))
        rid += 1
    reqs.sort(key=lambda r: r.arrival)
    return streams, reqs


def summarize(reqs: Sequence[Request], wall: float) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None]) * 1e3
    px = sum(r.shape[0] * r.shape[1] for r in reqs if r.done is not None)
    return {"requests": len(reqs), "completed": int(len(lat)),
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
            "max_ms": round(float(lat.max()), 3) if len(lat) else None,
            "MP_per_s": round(px / wall / 1e6, 1), "wall_s": round(wall, 3)}
