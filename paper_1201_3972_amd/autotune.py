"""Autotuner: per pixel type and window, measure every (workgroup size,
selection algorithm) the library has a kernel for, and keep the fastest; for
two-pass runs, whether pairs of passes run fused (and with which workgroup
size) or as separate launches; for batches, the batch workgroup size.

All candidates compute the same order statistic, so a choice changes speed,
never results; the tuner still checks that every candidate's output equals the
untuned kernel's output bit for bit before timing it.  Times are HIP-event
times of whole launches over a stack resident in device memory, the candidates
of one window interleaved over several rounds (best round kept), so that clock
and cache state do not favour whichever runs first.

The table is kept as JSON under ``tuning/``, keyed by GPU architecture and ROCm
version (``tuning/<arch>_rocm<major.minor>.json``), and is applied to the
library with :func:`apply` (``load_cached`` does both).  Command line::

    python -m paper_1201_3972_amd.autotune [--quick] [--out PATH]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import irfilter

PKG = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(PKG, "tuning")
WINDOWS = (3, 5, 7, 9, 11, 13, 15)
LARGE_WINDOWS = (17, 19, 21, 23, 25, 27, 29, 31)  # group bisection or the radix select
# above 31x31 one kernel per window (group bisection, 128 threads): nothing to tune
LARGE_MAX_WINDOW = 31
SELECT_BY_NAME = {name: code for code, name in irfilter.SELECT_NAMES.items()}
NETWORK_MAX_WINDOW = 15
FUSED_MAX_WINDOW = 9
FUSION_CHOICES = (0, 256, 512)  # separate launches, fused with 256 or 512 threads
FUSION_MARGIN = 1.03  # a fixed fusion choice replaces the automatic one only if this much faster


def candidates(window: int) -> List[Tuple[int, int]]:
    """Every (threads, select) with a kernel for this window: networks and
    one-lane bisection up to 15x15, group bisection and the histogram radix
    select up to 31x31, group bisection on 128 threads above."""
    if window > LARGE_MAX_WINDOW:
        return [(128, irfilter.IRF_SELECT_GROUP)]
    if window <= NETWORK_MAX_WINDOW:
        sels = [irfilter.IRF_SELECT_NETWORK, irfilter.IRF_SELECT_BISECT]
    else:
        sels = [irfilter.IRF_SELECT_GROUP, irfilter.IRF_SELECT_HIST]
    return [(t, s) for t in (128, 256) for s in sels]


# ----------------------------------------------------------------------------
# cache
# ----------------------------------------------------------------------------

def cache_key(torch) -> Dict[str, str]:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    rocm = ".".join((torch.version.hip or "unknown").split(".")[:2])
    return {"arch": arch, "rocm": rocm}


def cache_path(key: Dict[str, str]) -> str:
    return os.path.join(TUNING_DIR, f"{key['arch']}_rocm{key['rocm']}.json")


def save(table: dict, path: str) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    os.replace(tmp, path)


def load_file(path: str) -> dict:
    with open(path) as fh:
        return json.load(fh)


def apply(table: dict) -> None:
    """Set the library's tuning from a table (entries it lacks keep their values)."""
    for dt, per_window in table.get("single", {}).items():
        for k, ent in per_window.items():
            irfilter.set_tuning(dt, int(k), int(ent["threads"]), SELECT_BY_NAME[ent["select"]])
    for dt, per_window in table.get("fusion", {}).items():
        for k, ent in per_window.items():
            irfilter.set_fusion(dt, int(k), int(ent["threads"]))
    if "batch" in table:
        irfilter.set_batch_threads(int(table["batch"]["threads"]))


def load_cached(torch, path: Optional[str] = None) -> Optional[dict]:
    """Apply the cached table for this GPU and ROCm version; None if there is none."""
    p = path or cache_path(cache_key(torch))
    if not os.path.exists(p):
        return None
    table = load_file(p)
    apply(table)
    return table


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def default_frames(dtype: str) -> List:
    """Distinct frames the single-size choices are timed on: 640x512 fields with
    random-valued impulses at 10/30/60 % and mixed impulses at 40 % (u16, read
    noise sigma 20), or salt-and-pepper at 20 % and mixed at 40 % (u8)."""
    from . import synth
    if dtype == "u16":
        specs = [synth.FrameSpec(640, 512, "u16", "rv", d, 20.0, synth.config_seed(5, j))
                 for j, d in enumerate((0.1, 0.3, 0.6))]
        specs.append(synth.FrameSpec(640, 512, "u16", "mixed", 0.4, 20.0, synth.config_seed(5, 3)))
    else:
        specs = [synth.FrameSpec(640, 512, "u8", "sp", 0.2, 0.0, synth.config_seed(5, 10)),
                 synth.FrameSpec(640, 512, "u8", "mixed", 0.4, 0.0, synth.config_seed(5, 11))]
    return [synth.make_frame(s) for s in specs]


def _stack(torch, frames, n: int):
    import numpy as np
    dev = torch.device("cuda:0")
    h, w = frames[0].shape
    if frames[0].dtype == np.uint16:
        out = torch.empty((n, h, w), dtype=torch.int16, device=dev)
        pool = [torch.from_numpy(np.ascontiguousarray(f).view(np.int16)).to(dev) for f in frames]
    else:
        out = torch.empty((n, h, w), dtype=torch.uint8, device=dev)
        pool = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames]
    for i in range(n):
        out[i].copy_(pool[i % len(pool)])
    return out.view(torch.uint16) if frames[0].dtype == np.uint16 else out


def _event_ms(torch, fn: Callable[[], None], reps: int) -> float:
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _same(torch, x, y) -> bool:
    if x.dtype == torch.uint16:
        return torch.equal(x.view(torch.int16), y.view(torch.int16))
    return torch.equal(x, y)


# ----------------------------------------------------------------------------
# tuning
# ----------------------------------------------------------------------------

def tune_single(torch, dtype: str, windows: Sequence[int] = WINDOWS, frames: int = 256, rounds: int = 3,
                reps: int = 5, pool=None, stack=None, log: Callable[[str], None] = lambda m: None) -> Dict[str, dict]:
    """Best (threads, select) per window for ``ir_filter_run_frames`` on a
    ``frames``-frame stack of ``pool`` (default: :func:`default_frames`), or on
    a device-resident ``stack`` given by the caller."""
    src = stack if stack is not None else _stack(torch, pool or default_frames(dtype), frames)
    dst = torch.empty_like(src)
    ref = torch.empty_like(src)
    out = {}
    for k in windows:
        before = irfilter.get_tuning(dtype, k)
        irfilter.set_tuning(dtype, k, 0, 0)
        irfilter.ir_filter_run_frames(src, ref, k)
        cands = candidates(k)
        for t, sel in cands:
            irfilter.set_tuning(dtype, k, t, sel)
            irfilter.ir_filter_run_frames(src, dst, k)
            torch.cuda.synchronize()
            if not _same(torch, dst, ref):
                irfilter.set_tuning(dtype, k, *before)
                raise RuntimeError(f"{dtype} {k}x{k}: threads={t} select={sel} differs from the untuned kernel")
        best = {c: float("inf") for c in cands}
        for _ in range(rounds):
            for t, sel in cands:
                irfilter.set_tuning(dtype, k, t, sel)
                ms = _event_ms(torch, lambda: irfilter.ir_filter_run_frames(src, dst, k), reps)
                best[(t, sel)] = min(best[(t, sel)], ms)
        (t, sel) = min(cands, key=lambda c: best[c])
        irfilter.set_tuning(dtype, k, t, sel)
        out[str(k)] = {"threads": t, "select": irfilter.SELECT_NAMES[sel],
                       "ms": {f"{tt}/{irfilter.SELECT_NAMES[ss]}": round(best[(tt, ss)], 4) for tt, ss in cands}}
        log(f"{dtype} {k}x{k}: {out[str(k)]['threads']} threads, {out[str(k)]['select']}  {out[str(k)]['ms']}")
    return out


def tune_fusion(torch, dtype: str, windows: Sequence[int] = (3, 5, 7, 9), frames: int = 256, rounds: int = 3,
                reps: int = 5, pool=None, log: Callable[[str], None] = lambda m: None) -> Dict[str, dict]:
    """Fused or separate passes, per window, for two-pass ``ir_filter_run_frames``
    on a ``frames``-frame stack of ``pool`` (default: :func:`default_frames`).
    The library's automatic choice (by tile coverage, per frame size) is kept
    unless a fixed choice beats it on this workload by FUSION_MARGIN."""
    src = _stack(torch, pool or default_frames(dtype), frames)
    dst = torch.empty_like(src)
    ref = torch.empty_like(src)
    scratch = torch.empty_like(src)
    out = {}
    for k in windows:
        if k > FUSED_MAX_WINDOW:
            continue
        before = irfilter.get_fusion(dtype, k)
        irfilter.set_fusion(dtype, k, 0)
        irfilter.ir_filter_run_frames(src, ref, k, passes=2, scratch=scratch)

        def run():
            irfilter.ir_filter_run_frames(src, dst, k, passes=2, scratch=scratch)

        for t in FUSION_CHOICES:
            irfilter.set_fusion(dtype, k, t)
            run()
            torch.cuda.synchronize()
            if not _same(torch, dst, ref):
                irfilter.set_fusion(dtype, k, before)
                raise RuntimeError(f"{dtype} {k}x{k}: two passes fused with {t} threads differ from separate passes")
        best = {t: float("inf") for t in FUSION_CHOICES}
        for _ in range(rounds):
            for t in FUSION_CHOICES:
                irfilter.set_fusion(dtype, k, t)
                best[t] = min(best[t], _event_ms(torch, run, reps))
        irfilter.set_fusion(dtype, k, irfilter.FUSION_AUTO)
        auto = irfilter.resolve_fusion(dtype, k, int(src.shape[2]), int(src.shape[1]))
        fastest = min(FUSION_CHOICES, key=lambda t: best[t])
        choice = irfilter.FUSION_AUTO if best[auto] <= best[fastest] * FUSION_MARGIN else fastest
        irfilter.set_fusion(dtype, k, choice)
        out[str(k)] = {"threads": choice, "auto": auto, "ms": {str(t): round(v, 4) for t, v in best.items()}}
        name = {irfilter.FUSION_AUTO: f"automatic ({auto})", 0: "separate"}.get(choice, f"fused, {choice} threads")
        log(f"{dtype} {k}x{k} two passes: {name}  {out[str(k)]['ms']}")
    return out


def tune_batch(torch, n: int = 256, rounds: int = 3, reps: int = 5,
               log: Callable[[str], None] = lambda m: None) -> dict:
    """Batch workgroup size on the uneven 256-frame batch (sizes 160x120 to
    1280x1024, u8 and u16, windows 3..9, mixed impulses at 5-60 %)."""
    import numpy as np
    from . import synth
    dev = torch.device("cuda:0")
    items = synth.c4_items(n)
    frames = [synth.make_frame(it.spec) for it in items]
    srcs = []
    for fr in frames:
        if fr.dtype == np.uint16:
            srcs.append(torch.from_numpy(fr.view(np.int16)).to(dev).view(torch.uint16))
        else:
            srcs.append(torch.from_numpy(fr).to(dev))
    dsts = [torch.empty_like(x) for x in srcs]
    refs = [torch.empty_like(x) for x in srcs]
    before = irfilter.get_batch_threads()
    plans = {}
    try:
        for t in (128, 256):
            irfilter.set_batch_threads(t)
            tiles = sum(irfilter.frame_tiles(fr.shape[1], fr.shape[0]) for fr in frames)
            plans[t] = irfilter.Plan(n, tiles)
        items3 = [(a, b, it.window) for a, b, it in zip(srcs, dsts, items)]
        arr = irfilter.Plan.frames(items3)
        arr_ref = irfilter.Plan.frames([(a, r, it.window) for a, r, it in zip(srcs, refs, items)])
        plans[128].run_frames(arr_ref, n)
        for t, p in plans.items():
            p.run_frames(arr, n)
            torch.cuda.synchronize()
            if not all(_same(torch, d, r) for d, r in zip(dsts, refs)):
                raise RuntimeError(f"batch with {t}-thread workgroups differs from the 128-thread batch")
        best = {t: float("inf") for t in plans}
        for _ in range(rounds):
            for t, p in plans.items():
                best[t] = min(best[t], _event_ms(torch, lambda: p.run_frames(arr, n), reps))
        choice = min(best, key=best.get)
    finally:
        for p in plans.values():
            p.close()
        irfilter.set_batch_threads(before if before != 128 else 0)
    irfilter.set_batch_threads(choice)
    out = {"threads": choice, "ms": {str(t): round(v, 4) for t, v in best.items()}}
    log(f"batch: {choice} threads  {out['ms']}")
    return out


def tune(torch, quick: bool = False, log: Callable[[str], None] = lambda m: None) -> dict:
    """Tune everything and apply the result; returns the table (not saved)."""
    t0 = time.time()
    frames = 64 if quick else 256
    rounds = 2 if quick else 3
    table = {"key": cache_key(torch), "workload": {
        "single": f"{frames} frames of 640x512 per pixel type (random-valued impulses at 10/30/60% and mixed "
                  f"at 40% for u16; salt-and-pepper 20% and mixed 40% for u8), run_frames, best of {rounds} "
                  "interleaved rounds",
        "large": f"windows 17..31: {frames // 32} frames of the same stacks, best of 2 rounds",
        "fusion": "the same stacks, two passes (windows up to 9x9)",
        "batch": "256 uneven frames (160x120..1280x1024, u8/u16, windows 3..9, mixed impulses 5-60%)"},
        "single": {}, "fusion": {}}
    for dt in ("u16", "u8"):
        table["single"][dt] = tune_single(torch, dt, frames=frames, rounds=rounds, log=log)
        table["single"][dt].update(tune_single(torch, dt, windows=LARGE_WINDOWS, frames=frames // 32,
                                               rounds=2, reps=2, log=log))
        table["fusion"][dt] = tune_fusion(torch, dt, frames=frames, rounds=rounds, log=log)
    table["batch"] = tune_batch(torch, rounds=rounds, log=log)
    table["seconds"] = round(time.time() - t0, 1)
    return table


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--quick", action="store_true", help="64-frame stacks and two rounds")
    ap.add_argument("--out", default=None, help="where to write the table (default: tuning/<arch>_rocm<ver>.json)")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 2
    table = tune(torch, quick=args.quick, log=lambda m: print(m, flush=True))
    path = args.out or cache_path(table["key"])
    save(table, path)
    print(f"wrote {path} ({table['seconds']} s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
