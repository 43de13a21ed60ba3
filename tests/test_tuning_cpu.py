"""Host side of the tuning table and the autotuner's cache (no device needed).

Tuning changes only which kernel runs, never the result: that is checked per
variant against the oracle in tests/test_gpu_tuning.py."""

import json

import pytest

from paper_1201_3972_amd import autotune, irfilter

pytestmark = pytest.mark.usefixtures("lib")


@pytest.fixture(scope="module")
def lib():
    try:
        return irfilter.load()
    except irfilter.LibraryNotBuilt:
        pytest.skip("library not built")


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    for dt in ("u8", "u16"):
        for k in range(3, 64, 2):
            irfilter.set_tuning(dt, k, 0, 0)
            irfilter.set_fusion(dt, k, -1)
    irfilter.set_batch_threads(0)


def test_defaults():
    for dt in ("u8", "u16"):
        for k in (3, 9, 11, 13, 15):
            assert irfilter.get_tuning(dt, k) == (128, irfilter.IRF_SELECT_NETWORK)
        for k in (5, 7):
            assert irfilter.get_tuning(dt, k) == (256, irfilter.IRF_SELECT_NETWORK)
        for k in range(17, 32, 2):
            assert irfilter.get_tuning(dt, k) == (256, irfilter.IRF_SELECT_GROUP)
        for k in range(33, 64, 2):
            assert irfilter.get_tuning(dt, k) == (128, irfilter.IRF_SELECT_GROUP)
    assert irfilter.get_batch_threads() == 128


def test_set_get_and_restore():
    irfilter.set_tuning("u16", 5, 128, irfilter.IRF_SELECT_BISECT)
    assert irfilter.get_tuning("u16", 5) == (128, irfilter.IRF_SELECT_BISECT)
    assert irfilter.get_tuning("u8", 5) == (256, irfilter.IRF_SELECT_NETWORK)  # per pixel type
    irfilter.set_tuning("u16", 5, 0, 0)
    assert irfilter.get_tuning("u16", 5) == (256, irfilter.IRF_SELECT_NETWORK)


@pytest.mark.parametrize("args,status", [
    (("u16", 13, 512, irfilter.IRF_SELECT_NETWORK), -11),
    (("u16", 5, 64, irfilter.IRF_SELECT_NETWORK), -11),
    (("u16", 5, 128, 3), -11),
    (("u16", 5, 128, 0), -11),
    (("u16", 4, 128, 1), -5),
    (("u16", 65, 128, 1), -5),
    (("u16", 33, 256, 3), -11),  # above 31x31: 128 threads only
    (("u16", 33, 128, 4), -11),  # and no radix select
    (("u16", 17, 128, 1), -11),  # no network above 15x15
    (("u16", 17, 128, 2), -11),  # nor one-lane bisection
    (("u16", 5, 128, 3), -11),   # group bisection only above 15x15
])
def test_invalid_tuning(args, status):
    dt, k, t, sel = args
    lib = irfilter.load()
    assert lib.ir_filter_set_tuning(irfilter._dtype_arg(dt), k, t, sel) == status
    assert lib.ir_filter_set_tuning(3, 5, 128, 1) == -4


def test_fusion_set_get_and_restore():
    for dt in ("u8", "u16"):
        for k in range(3, 16, 2):
            assert irfilter.get_fusion(dt, k) == irfilter.FUSION_AUTO
    irfilter.set_fusion("u16", 5, 256)
    assert irfilter.get_fusion("u16", 5) == 256
    irfilter.set_fusion("u16", 5, 0)
    assert irfilter.get_fusion("u16", 5) == 0
    u16_9 = irfilter.get_fusion("u16", 9)
    irfilter.set_fusion("u8", 9, 512 if u16_9 != 512 else 256)
    assert irfilter.get_fusion("u8", 9) != u16_9
    assert irfilter.get_fusion("u16", 9) == u16_9  # per pixel type
    irfilter.set_fusion("u16", 5, -1)
    irfilter.set_fusion("u8", 9, -1)
    assert irfilter.get_fusion("u16", 5) == irfilter.get_fusion("u8", 9) == irfilter.FUSION_AUTO
    irfilter.set_fusion("u16", 11, 0)  # separate passes are always available
    assert irfilter.get_fusion("u16", 11) == 0


def _covered(W, H, k, fused_threads, plain_threads):
    """Pixels two passes cover: plain 128 x TH tiles twice, or fused blocks of
    128 x TH whose outputs are 120 x (TH - k + 1)."""
    cdiv = lambda a, b: -(-a // b)
    if fused_threads == 0:
        th = plain_threads // 4
        return 2 * cdiv(W, 128) * cdiv(H, th) * 128 * th
    th = fused_threads // 4
    return 2 * cdiv(W, 120) * cdiv(H, th - k + 1) * 128 * th


@pytest.mark.parametrize("dt,k,W,H", [
    ("u8", 3, 320, 240), ("u8", 5, 320, 240), ("u16", 5, 640, 512), ("u16", 7, 640, 512),
    ("u16", 5, 1920, 1080), ("u8", 3, 364, 244), ("u16", 9, 100, 60), ("u8", 11, 320, 240),
    ("u16", 3, 1, 1), ("u8", 7, 4000, 3000), ("u8", 9, 120, 120), ("u16", 7, 120, 122)])
def test_automatic_fusion_is_separate_passes(dt, k, W, H):
    # the automatic choice runs separate passes: a fused tiling never covers
    # fewer pixels than two single passes (checked here for both fused sizes
    # and both single-pass workgroup sizes), and at equal coverage separate
    # passes measured faster
    assert irfilter.resolve_fusion(dt, k, W, H) == 0
    for plain in (128, 256):
        for t in (256, 512):
            assert _covered(W, H, k, t, plain) >= _covered(W, H, k, 0, plain), (plain, t)


def test_resolve_fusion_follows_the_setting():
    assert irfilter.resolve_fusion("u8", 5, 320, 240) == 0    # equal coverage: separate passes
    assert irfilter.resolve_fusion("u8", 3, 320, 240) == 0
    assert irfilter.resolve_fusion("u16", 5, 640, 512) == 0   # 6 fused tiles across vs 5 plain
    irfilter.set_fusion("u16", 5, 512)
    assert irfilter.resolve_fusion("u16", 5, 640, 512) == 512
    irfilter.set_fusion("u8", 3, 256)
    assert irfilter.resolve_fusion("u8", 3, 320, 240) == 256
    irfilter.set_fusion("u8", 5, 0)
    assert irfilter.resolve_fusion("u8", 5, 320, 240) == 0
    lib = irfilter.load()
    assert lib.ir_filter_resolve_fusion(2, 5, 0, 10, None) == -1
    import ctypes
    t = ctypes.c_int()
    assert lib.ir_filter_resolve_fusion(2, 5, 0, 10, ctypes.byref(t)) == -2
    assert lib.ir_filter_resolve_fusion(2, 6, 10, 10, ctypes.byref(t)) == -5


@pytest.mark.parametrize("dt,k,threads,status", [
    ("u16", 11, 256, -11), ("u16", 15, 512, -11), ("u16", 5, 128, -11), ("u16", 5, 1, -11),
    ("u16", 5, -2, -11), ("u16", 4, 256, -5), ("u16", 65, 0, -5), ("u16", 17, 256, -11),
])
def test_invalid_fusion(dt, k, threads, status):
    lib = irfilter.load()
    assert lib.ir_filter_set_fusion(irfilter._dtype_arg(dt), k, threads) == status
    assert lib.ir_filter_set_fusion(3, 5, 256) == -4
    assert lib.ir_filter_get_fusion(2, 5, None) == -1


def test_get_tuning_checks_pointers():
    assert irfilter.load().ir_filter_get_tuning(2, 5, None, None) == -1


def test_batch_threads_change_tile_count():
    assert irfilter.frame_tiles(640, 512) == 5 * 16
    irfilter.set_batch_threads(256)
    assert irfilter.get_batch_threads() == 256
    assert irfilter.frame_tiles(640, 512) == 5 * 8
    assert irfilter.frame_tiles(129, 65) == 2 * 2
    assert irfilter.load().ir_filter_set_batch_threads(192) == -11
    irfilter.set_batch_threads(0)
    assert irfilter.frame_tiles(640, 512) == 5 * 16


def test_cache_round_trip_and_apply(tmp_path):
    table = {
        "key": {"arch": "gfx950", "rocm": "test"},
        "single": {"u16": {"5": {"threads": 256, "select": "bisect", "ms": {}},
                           "7": {"threads": 128, "select": "network", "ms": {}}}},
        "fusion": {"u8": {"5": {"threads": 512, "ms": {}}}},
        "batch": {"threads": 256, "ms": {}},
    }
    path = tmp_path / "t.json"
    autotune.save(table, str(path))
    back = autotune.load_file(str(path))
    assert back == json.loads(json.dumps(table))
    autotune.apply(back)
    assert irfilter.get_tuning("u16", 5) == (256, irfilter.IRF_SELECT_BISECT)
    assert irfilter.get_tuning("u16", 7) == (128, irfilter.IRF_SELECT_NETWORK)
    assert irfilter.get_fusion("u8", 5) == 512 and irfilter.get_fusion("u16", 5) == irfilter.FUSION_AUTO
    assert irfilter.get_batch_threads() == 256


def test_apply_rejects_unknown_choices():
    with pytest.raises(irfilter.IrfError):
        autotune.apply({"single": {"u16": {"13": {"threads": 512, "select": "network"}}}})


def test_candidates_cover_every_available_kernel():
    for k in (3, 9, 15):
        c = autotune.candidates(k)
        assert (128, irfilter.IRF_SELECT_NETWORK) in c and (256, irfilter.IRF_SELECT_BISECT) in c
        assert len(c) == 4
    for k in autotune.LARGE_WINDOWS:
        assert sorted(autotune.candidates(k)) == sorted(
            [(t, s) for t in (128, 256) for s in (irfilter.IRF_SELECT_GROUP, irfilter.IRF_SELECT_HIST)])
        for t, s in autotune.candidates(k):
            irfilter.set_tuning("u8", k, t, s)
            assert irfilter.get_tuning("u8", k) == (t, s)
        irfilter.set_tuning("u8", k, 0, 0)
    for k in (33, 47, 63):
        assert autotune.candidates(k) == [(128, irfilter.IRF_SELECT_GROUP)]
    for k in autotune.LARGE_WINDOWS:
        # networks and one-lane bisection do not exist above 15x15, the radix select not below
        with pytest.raises(irfilter.IrfError):
            irfilter.set_tuning("u8", k, 256, irfilter.IRF_SELECT_NETWORK)
    with pytest.raises(irfilter.IrfError):
        irfilter.set_tuning("u16", 15, 256, irfilter.IRF_SELECT_HIST)
