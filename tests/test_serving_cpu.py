"""Host-side serving logic that needs no GPU: the device-memory arena and the
arrival process (the arena is exercised on a CPU buffer)."""

import numpy as np
import torch

from paper_1201_3972_amd import serving


def test_arena_first_fit_and_coalescing():
    a = serving.DeviceArena(torch, 64 * 4096, "cpu")
    x = a.alloc(4096 * 10)
    y = a.alloc(100)            # rounds up to one page
    z = a.alloc(4096 * 20)
    assert (x, y, z) == (0, 40960, 45056)
    assert a.alloc(4096 * 40) is None  # only 33 pages left
    a.release(y, 100)
    assert a.alloc(4096) == 40960       # first fit reuses the hole
    a.release(40960, 4096)
    a.release(x, 4096 * 10)
    a.release(z, 4096 * 20)
    assert a.free == [(0, 64 * 4096)] and a.used == 0


def test_arena_random_alloc_release_never_overlaps():
    rng = np.random.default_rng(1)
    a = serving.DeviceArena(torch, 1 << 22, "cpu")
    live = {}
    for step in range(2000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            off = list(live)[int(rng.integers(len(live)))]
            a.release(off, live.pop(off))
        else:
            n = int(rng.integers(1, 1 << 17))
            off = a.alloc(n)
            if off is not None:
                live[off] = n
        spans = sorted((o, o + serving._round(n)) for o, n in live.items())
        assert all(spans[i][1] <= spans[i + 1][0] for i in range(len(spans) - 1))
        assert a.used == sum(serving._round(n) for n in live.values())
    for off, n in list(live.items()):
        a.release(off, n)
    assert a.free == [(0, a.capacity)]


def test_poisson_arrivals_rate():
    rng = np.random.default_rng(7)
    t = serving.poisson_arrivals(rng, 30.0, 200.0)
    assert np.all(np.diff(t) > 0) and t[-1] < 200.0
    assert abs(len(t) / 200.0 - 30.0) < 1.5
