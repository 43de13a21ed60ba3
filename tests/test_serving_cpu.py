"""Host-side serving logic that needs no GPU: the arrival process and the
native engine's argument checks (which run before any HIP call)."""

import ctypes

import numpy as np
import pytest

from paper_1201_3972_amd import irfilter, serving


@pytest.fixture(scope="module")
def lib():
    try:
        return irfilter.load()
    except irfilter.LibraryNotBuilt:
        pytest.skip("library not built")


def test_poisson_arrivals_rate():
    rng = np.random.default_rng(7)
    t = serving.poisson_arrivals(rng, 30.0, 200.0)
    assert np.all(np.diff(t) > 0) and t[-1] < 200.0
    assert abs(len(t) / 200.0 - 30.0) < 1.5


def test_frame_bytes_and_rounding():
    assert serving.frame_bytes(640, 512, "u16") == 655360
    assert serving.frame_bytes(320, 240, "u8") == 76800
    assert serving._round(1) == 4096 and serving._round(4096) == 4096 and serving._round(4097) == 8192


def test_server_argument_checks(lib):
    ptr = ctypes.c_void_p()
    assert lib.ir_filter_server_create(None, 1 << 20, 8, 64, 2, 0) == -1
    assert lib.ir_filter_server_create(ctypes.byref(ptr), 1 << 20, 0, 64, 2, 0) == -2
    assert lib.ir_filter_server_create(ctypes.byref(ptr), 1 << 20, 8, 0, 2, 0) == -2
    assert lib.ir_filter_server_create(ctypes.byref(ptr), 1 << 20, 8, 64, 0, 0) == -2
    assert lib.ir_filter_server_create(ctypes.byref(ptr), 1 << 20, 8, 64, 9, 0) == -2
    assert ptr.value is None
    assert lib.ir_filter_server_register_stream(None, 0, 640, 512, 2, 2) == -1
    assert lib.ir_filter_server_submit(None, None, 0) == -1
    assert lib.ir_filter_server_poll(None) == -1
    assert lib.ir_filter_server_run(None) == -1
    assert lib.ir_filter_server_completed(None, None, None, 4) == 0
    assert lib.ir_filter_server_now(None) == 0.0
    assert lib.ir_filter_server_steps(None) == 0
    assert lib.ir_filter_server_arena_used(None) == 0
    lib.ir_filter_server_destroy(None)  # ignored


def test_request_struct_matches_the_header():
    # irf_request: u64, 2 pointers, 2 size_t, 5 ints, double (8-byte aligned)
    assert ctypes.sizeof(irfilter.IrfRequest) == 8 + 16 + 16 + 20 + 4 + 8
    assert irfilter.IrfRequest.arrival.offset == 64
