"""Pins of the oracle's opt-in directional detector (a reading of Fig. 1's
caption; the figure is missing, so the paper fixes no values for it).

The rule read here: a pixel is noisy when, on each of the four lines through it
in its 3x3 window (row, column, both diagonals), its grey level lies outside
the range of its two neighbours; ties count as inside; window coordinates are
clamped to the frame.  Each pin below is a consequence of that rule chosen so
that a plausible slip fails it: pairing the wrong neighbours (dihedral
symmetry), a strict instead of an inclusive range (constant frames), "any line"
instead of "every line" (one-pixel lines), zero instead of replicated borders
(the border is never flagged).
"""

import numpy as np
import pytest

import oracle

DIHEDRAL = [
    lambda a: a, lambda a: np.rot90(a, 1), lambda a: np.rot90(a, 2), lambda a: np.rot90(a, 3),
    lambda a: a[:, ::-1], lambda a: a[::-1, :], lambda a: a.T, lambda a: np.rot90(a, 1)[:, ::-1],
]


def flags(f):
    m, c = oracle.detect_directional(np.ascontiguousarray(f))
    assert c == int(m.sum())
    return m


@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
def test_constant_frames_have_no_noise(dt):
    for val in (0, 7, np.iinfo(dt).max):
        assert not flags(np.full((9, 11), val, dtype=dt)).any()


def test_ramps_in_every_direction_have_no_noise():
    y, x = np.mgrid[0:20, 0:23]
    for g in (x, y, x + y, x - y + 40, 3 * x + 2 * y, (x * x) // 3, np.maximum(x, y)):
        assert not flags(g.astype(np.uint16)).any()


@pytest.mark.parametrize("val", [0, 255])
def test_interior_impulses_are_the_only_noise(val):
    y, x = np.mgrid[0:15, 0:17]
    for bg in (np.full((15, 17), 100), 60 + 4 * x + 3 * y):
        f = bg.astype(np.uint8)
        pts = [(3, 4), (8, 10), (12, 2), (5, 12)]
        for px, py in pts:
            f[py, px] = val
        want = np.zeros(f.shape, dtype=np.uint8)
        for px, py in pts:
            want[py, px] = 1
        np.testing.assert_array_equal(flags(f), want)


def test_one_pixel_lines_are_kept_while_the_extreme_detector_flags_them():
    for draw in ("row", "col", "diag", "anti"):
        f = np.full((16, 16), 50, dtype=np.uint8)
        idx = np.arange(2, 14)
        if draw == "row":
            f[7, idx] = 220
        elif draw == "col":
            f[idx, 7] = 220
        elif draw == "diag":
            f[idx, idx] = 220
        else:
            f[idx, 15 - idx] = 220
        line = f == 220
        assert not flags(f)[line].any()
        assert oracle.detect(f, 3)[0][line].all()  # the paper's detector removes such a line


def test_border_pixels_are_never_noise():
    rng = np.random.default_rng(4)
    for _ in range(20):
        f = rng.integers(0, 256, size=(int(rng.integers(1, 12)), int(rng.integers(1, 12)))).astype(np.uint8)
        m = flags(f)
        assert not m[0].any() and not m[-1].any() and not m[:, 0].any() and not m[:, -1].any()
    f = np.full((8, 8), 10, dtype=np.uint8)
    f[0, 0] = f[0, 5] = f[7, 7] = f[3, 0] = 250  # impulses on the border
    assert not flags(f).any()


def test_strict_extremes_are_noise_and_noise_differs_from_all_neighbours():
    rng = np.random.default_rng(9)
    for shape in ((20, 30), (7, 9)):
        f = rng.permutation(shape[0] * shape[1]).reshape(shape).astype(np.uint16)  # distinct values
        m = flags(f)
        p = np.pad(f, 1, mode="edge").astype(np.int64)
        H, W = shape
        nb = [p[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]
        c = f.astype(np.int64)
        strict = np.all([c > n for n in nb], axis=0) | np.all([c < n for n in nb], axis=0)
        inner = np.zeros(shape, dtype=bool)
        inner[1:-1, 1:-1] = True
        assert m[strict & inner].all()
    f = rng.integers(0, 3, size=(25, 25)).astype(np.uint8)  # many ties
    m = flags(f)
    p = np.pad(f, 1, mode="edge")
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                assert not (m.astype(bool) & (p[1 + dy:26 + dy, 1 + dx:26 + dx] == f)).any()


@pytest.mark.parametrize("seed", range(6))
def test_dihedral_symmetry(seed):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 4 if seed % 2 else 256, size=(13, 19)).astype(np.uint8)
    base = flags(f)
    for t in DIHEDRAL:
        np.testing.assert_array_equal(flags(t(f)), t(base))


def test_monotone_maps_and_complement_keep_the_flags():
    rng = np.random.default_rng(2)
    f = rng.integers(0, 200, size=(30, 31)).astype(np.uint16)
    base = flags(f)
    np.testing.assert_array_equal(flags((3 * f + 11).astype(np.uint16)), base)
    np.testing.assert_array_equal(flags((f.astype(np.int64) ** 2 // 7).astype(np.uint16)), base)
    np.testing.assert_array_equal(flags((65535 - f).astype(np.uint16)), base)
