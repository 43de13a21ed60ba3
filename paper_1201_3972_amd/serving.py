"""Continuous-batching request loop for video-frame FNR filtering on one GPU.

Requests (one frame each, any size / pixel type / window) arrive over time and
are served by the library's native engine (``ir_filter_server_*`` in
``include/irfilter.h``, ``csrc/server.hip``), which keeps up to
``max_inflight`` batches on the device at once:

* admission -- an arrived request is admitted into the next batch when device
  memory for its input and output is available: frames of a registered video
  stream use that stream's resident slots (allocated once, kept for the
  stream's lifetime, reused frame after frame); other frames take space from a
  bounded device arena and give it back when their result has reached the
  host.  A request that does not fit waits; nothing is dropped.
* one step -- the admitted requests are copied host -> device on a copy
  stream, filtered by ONE batched launch (a persistent kernel over all their
  tiles) on a compute stream, and copied back on the copy stream; events order
  the three.  Steps are issued while earlier ones are still running, so copies
  of one batch overlap the kernel of another.
* completion -- a batch is complete when its device -> host copy has finished;
  each request's latency is completion minus arrival on the engine's clock.

This module only marshals requests (pinned torch tensors) into the engine and
reads completions back; admission, copies, launches and timing are native.
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import irfilter

_ALIGN = 4096


def frame_bytes(width: int, height: int, dtype: str) -> int:
    return width * height * (1 if dtype == "u8" else 2)


def _round(n: int) -> int:
    return (n + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the engine starts serving
    host_src: object        # pinned torch tensor [H, W]
    window: int
    stream_id: Optional[int] = None  # video stream (one-off frame if None or not registered)
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


class Server:
    """Continuous-batching FNR server on one GPU (see the module docstring)."""

    def __init__(self, memory_budget: int, max_batch_frames: int = 512, max_batch_tiles: int = 1 << 16,
                 max_inflight: int = 3, graph: bool = True, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self._lib = irfilter.load()
        self._ptr = ctypes.c_void_p()
        irfilter._check("ir_filter_server_create", self._lib.ir_filter_server_create(
            ctypes.byref(self._ptr), memory_budget, max_batch_frames, max_batch_tiles, max_inflight,
            irfilter.IRF_PLAN_GRAPH if graph else 0))
        self.max_inflight = max_inflight
        self._queued: List[Request] = []
        self._by_id: Dict[int, Request] = {}
        self._offset: Optional[float] = None  # engine clock at which serving started
        self._last_arrival = float("-inf")
        self._streams = set()
        self.completed: List[Request] = []

    # -- set-up ----------------------------------------------------------------
    def register_stream(self, stream_id: int, width: int, height: int, dtype: str, depth: int = 2) -> None:
        """Give a video stream ``depth`` resident device slots for its whole
        lifetime; a frame takes any free slot of its stream, so up to ``depth``
        consecutive frames of one stream can be in flight together."""
        irfilter._check("ir_filter_server_register_stream", self._lib.ir_filter_server_register_stream(
            self._ptr, stream_id, width, height, irfilter._dtype_arg(dtype), depth))
        self._streams.add(stream_id)

    def submit(self, req: Request) -> None:
        """Queue a request (in arrival order); it is handed to the engine when
        serving starts, and admitted once the engine clock passes its arrival."""
        if req.host_dst is None:
            req.host_dst = self.torch.empty_like(req.host_src, pin_memory=True)
        if req.arrival < self._last_arrival:
            raise ValueError("submit requests in arrival order")
        self._last_arrival = req.arrival
        self._queued.append(req)

    # -- engine ----------------------------------------------------------------
    def now(self) -> float:
        return self._lib.ir_filter_server_now(self._ptr) - (self._offset or 0.0)

    @property
    def steps(self) -> int:
        return self._lib.ir_filter_server_steps(self._ptr)

    @property
    def arena_used(self) -> int:
        return self._lib.ir_filter_server_arena_used(self._ptr)

    @property
    def resident_bytes(self) -> int:
        """Device frame memory held: the arena plus every stream's resident slots."""
        return self._lib.ir_filter_server_resident_bytes(self._ptr)

    def _flush(self) -> None:
        if not self._queued:
            if self._offset is None:
                self._offset = self._lib.ir_filter_server_now(self._ptr)
            return
        arr = (irfilter.IrfRequest * len(self._queued))()
        for i, r in enumerate(self._queued):
            H, W = r.shape
            es = r.host_src.element_size()
            arr[i] = irfilter.IrfRequest(r.rid, r.host_src.data_ptr(), r.host_dst.data_ptr(),
                                         r.host_src.stride(0) * es, r.host_dst.stride(0) * es, W, H,
                                         irfilter.IRF_U8 if es == 1 else irfilter.IRF_U16, r.window,
                                         # frames of unregistered streams are one-off frames
                                         r.stream_id if r.stream_id in self._streams else -1,
                                         r.arrival)
            self._by_id[r.rid] = r
        # the engine clock is read once the array is built, so the time taken to
        # build it is not charged to the first requests' latency; arrivals move
        # onto the engine clock in one vectorised add
        if self._offset is None:
            self._offset = self._lib.ir_filter_server_now(self._ptr)
        arrivals = np.ndarray((len(arr),), dtype=np.float64, buffer=arr, offset=irfilter.IrfRequest.arrival.offset,
                              strides=(ctypes.sizeof(irfilter.IrfRequest),))
        arrivals += self._offset
        queued, self._queued = self._queued, []
        irfilter._check("ir_filter_server_submit", self._lib.ir_filter_server_submit(self._ptr, arr, len(queued)))

    def _collect(self) -> None:
        n = 256
        ids = (ctypes.c_uint64 * n)()
        lat = (ctypes.c_double * n)()
        while True:
            got = self._lib.ir_filter_server_completed(self._ptr, ids, lat, n)
            for i in range(got):
                r = self._by_id.pop(ids[i])
                r.done = r.arrival + lat[i]
                self.completed.append(r)
            if got < n:
                return

    def poll(self) -> bool:
        """One engine iteration; True on progress."""
        self._flush()
        st = self._lib.ir_filter_server_poll(self._ptr)
        if st < 0:
            raise irfilter.IrfError("ir_filter_server_poll", st)
        self._collect()
        return st > 0

    def run_until_idle(self) -> None:
        """Serve until every submitted request has completed."""
        self._flush()
        st = self._lib.ir_filter_server_run(self._ptr)
        self._collect()
        irfilter._check("ir_filter_server_run", st)

    def close(self) -> None:
        if self._ptr is not None and self._ptr.value:
            self._lib.ir_filter_server_destroy(self._ptr)
        self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
