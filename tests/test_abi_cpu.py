"""C-ABI checks that need no GPU: exported symbols and host-side validation.

Every call here is rejected by argument validation, which runs on the host
before any HIP call, so nothing reaches the device.  Pointers are plain host
addresses (never dereferenced).
"""

import ctypes
import os
import re
import subprocess

import pytest

from paper_1201_3972_amd import build as pkg_build
from paper_1201_3972_amd import irfilter

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irfilter.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(irfilter.LIB_PATH):
        pkg_build.build(force=False)
    return irfilter.load()


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ir_filter_\w+)\s*\(", text, re.M)))


def test_header_declares_the_three_paper_operations():
    names = header_functions()
    for n in ("ir_filter_detect", "ir_filter_median", "ir_filter_run"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", irfilter.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)$", out, re.M))
    for n in header_functions():
        assert n in exported, n
        assert hasattr(lib, n)


def test_binding_signatures_cover_the_header():
    assert set(header_functions()) == set(irfilter.SIGNATURES)


def test_version_and_status_strings(lib):
    assert lib.ir_filter_version() >> 16 == 1 and lib.ir_filter_version() & 0xffff >= 1
    for code, name in irfilter.STATUS.items():
        s = lib.ir_filter_status_string(code).decode()
        assert s and s != "unknown status", name
    assert lib.ir_filter_status_string(12345).decode() == "unknown status"


# fake, well separated host addresses (never touched: validation fails first)
SRC, DST, SCR, MASK, CNT = 1 << 32, 2 << 32, 3 << 32, 4 << 32, 5 << 32


def run(lib, src=SRC, sp=640, dst=DST, dp=640, W=320, H=240, dt=1, k=3, passes=1, scr=None, xp=0,
        cnt=None):
    return lib.ir_filter_run(src, sp, dst, dp, W, H, dt, k, passes, scr, xp, cnt, None)


@pytest.mark.parametrize("kw,want", [
    (dict(src=None), -1), (dict(dst=None), -1),
    (dict(W=0), -2), (dict(H=0), -2), (dict(W=-5), -2), (dict(W=32769), -2), (dict(H=40000), -2),
    (dict(dt=0), -4), (dict(dt=3), -4),
    (dict(k=1), -5), (dict(k=4), -5), (dict(k=32), -5), (dict(k=65), -5), (dict(k=0), -5), (dict(k=-3), -5),
    (dict(k=31, passes=0), -6),  # 31x31 is a valid window: validation reaches the pass count
    (dict(k=63, passes=0), -6),  # and so is 63x63
    (dict(passes=0), -6), (dict(passes=17), -6), (dict(passes=2), -6),
    (dict(sp=319), -3), (dict(dt=2, sp=639, dp=640), -3), (dict(dp=100), -3),
    (dict(dst=SRC + 1000), -7),
    (dict(dst=SRC + 640 * 239 + 319), -7),
    (dict(passes=2, scr=SRC + 5, xp=640), -7), (dict(passes=2, scr=DST, xp=640), -7),
    (dict(passes=2, scr=SCR, xp=10), -3),
    (dict(cnt=SRC + 8), -7),
    (dict(passes=2, scr=SCR, xp=640, cnt=SCR + 640 * 100), -7),  # counts inside scratch
    (dict(passes=2, scr=SCR, xp=640, cnt=SCR - 8), -7),  # second count is scratch's first byte
])
def test_run_validation(lib, kw, want):
    assert run(lib, **kw) == want


def test_pitch_and_span_limits(lib):
    # rows are addressed with 24-bit multiplies and 32-bit offsets inside a frame
    assert run(lib, sp=1 << 24) == -3
    assert run(lib, dp=1 << 24) == -3
    big = (1 << 24) - 16
    assert big * 299 + 320 >= 1 << 32
    assert run(lib, sp=big, H=300) == -3
    assert run(lib, dp=big, H=300) == -3
    f = lib.ir_filter_detect
    assert f(SRC, 640, MASK, 1 << 24, 320, 240, 1, 3, None, None) == -3


def test_last_byte_of_source_counts_for_aliasing(lib):
    end = SRC + 640 * 239 + 320  # one past the last byte read from src
    assert run(lib, dst=end - 1) == -7


def test_detect_validation(lib):
    f = lib.ir_filter_detect
    assert f(None, 640, MASK, 320, 320, 240, 1, 3, None, None) == -1
    assert f(SRC, 640, None, 320, 320, 240, 1, 3, None, None) == -1
    assert f(SRC, 640, MASK, 319, 320, 240, 1, 3, None, None) == -3
    assert f(SRC, 640, MASK, 320, 320, 240, 1, 2, None, None) == -5
    assert f(SRC, 640, SRC + 100, 320, 320, 240, 1, 3, None, None) == -7
    assert f(SRC, 640, MASK, 320, 320, 240, 1, 3, MASK + 64, None) == -7


def test_median_validation(lib):
    f = lib.ir_filter_median
    assert f(SRC, 640, None, 0, None, 640, 320, 240, 2, 3, None) == -1
    assert f(SRC, 640, MASK, 100, DST, 640, 320, 240, 2, 3, None) == -3
    assert f(SRC, 640, MASK, 320, DST, 640, 320, 240, 2, 65, None) == -5
    assert f(SRC, 640, None, 0, SRC, 640, 320, 240, 2, 3, None) == -7
    assert f(SRC, 640, DST, 320, DST, 640, 320, 240, 2, 3, None) == -7


def test_directional_detect_validation(lib):
    f = lib.ir_filter_detect_directional
    assert f(None, 640, MASK, 320, 320, 240, 2, None, None) == -1
    assert f(SRC, 640, None, 320, 320, 240, 2, None, None) == -1
    assert f(SRC, 640, MASK, 320, 0, 240, 2, None, None) == -2
    assert f(SRC, 640, MASK, 320, 320, 240, 5, None, None) == -4
    assert f(SRC, 639, MASK, 320, 320, 240, 2, None, None) == -3
    assert f(SRC, 640, MASK, 319, 320, 240, 2, None, None) == -3
    assert f(SRC, 640, SRC + 100, 320, 320, 240, 2, None, None) == -7
    assert f(SRC, 640, MASK, 320, 320, 240, 2, MASK + 8, None) == -7


def test_frames_validation(lib):
    f = lib.ir_filter_run_frames
    # stride smaller than one frame
    assert f(SRC, 640, 640 * 239, DST, 640, 640 * 240, 320, 240, 4, 2, 5, 1, None, 0, 0, None, None) == -3
    # stacks overlap in their last frame
    assert f(SRC, 640, 640 * 240, SRC + 640 * 240 * 3, 640, 640 * 240, 320, 240, 4, 2, 5, 1, None, 0, 0,
             None, None) == -7
    assert f(SRC, 640, 640 * 240, DST, 640, 640 * 240, 320, 240, 0, 2, 5, 1, None, 0, 0, None, None) == -2


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(irfilter.LibraryNotBuilt):
        irfilter.load(str(tmp_path / "nope.so"))


def test_plan_argument_checks_before_any_device_call(lib):
    import ctypes
    ptr = ctypes.c_void_p()
    assert lib.ir_filter_plan_create(None, 4, 4, 0) == -1
    assert lib.ir_filter_plan_create(ctypes.byref(ptr), 0, 4, 0) == -2
    assert lib.ir_filter_plan_create(ctypes.byref(ptr), 4, 0, 0) == -2
    assert ptr.value is None
    assert lib.ir_filter_run_batch(None, None, 1, None, None) == -1
    lib.ir_filter_plan_destroy(None)  # ignored


def test_frame_tile_count(lib):
    assert lib.ir_filter_frame_tiles(640, 512) == 5 * 16
    assert lib.ir_filter_frame_tiles(129, 65) == 2 * 3
    assert lib.ir_filter_frame_tiles(1, 1) == 1
    assert lib.ir_filter_frame_tiles(0, 5) == 0


def test_counts_just_outside_scratch_pass_validation(lib):
    # the two counts end right before scratch: validation passes the alias
    # check and fails on the next one (a pass count of 17)
    assert run(lib, passes=17, scr=SCR, xp=640, cnt=SCR - 16) == -6


def test_noalloc_rejects_frames_beyond_its_array_before_any_device_call(lib):
    f = lib.ir_filter_run_noalloc
    # 4096 x 4096 u16 fills the 32 MiB array exactly; one more row does not fit
    assert f(SRC, 8192, DST, 8192, 4096, 4097, 2, 3, 2, None, None) == -10
    assert f(SRC, 8192, DST, 8192, 32768, 32768, 2, 3, 3, None, None) == -10
    assert f(None, 8192, DST, 8192, 64, 64, 2, 3, 2, None, None) == -1
    assert f(SRC, 8192, DST, 8192, 64, 64, 2, 4, 2, None, None) == -5
    assert f(SRC, 8192, DST, 8192, 64, 64, 2, 3, 0, None, None) == -6
    assert f(SRC, 8192, DST, 8192, 64, 64, 2, 3, 17, None, None) == -6
