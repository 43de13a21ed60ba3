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
        for k in range(3, 16, 2):
            irfilter.set_tuning(dt, k, 0, 0)
    irfilter.set_batch_threads(0)


def test_defaults():
    for dt in ("u8", "u16"):
        for k in (3, 5, 9, 11, 13, 15):
            assert irfilter.get_tuning(dt, k) == (128, irfilter.IRF_SELECT_NETWORK)
        assert irfilter.get_tuning(dt, 7) == (256, irfilter.IRF_SELECT_NETWORK)
    assert irfilter.get_batch_threads() == 128


def test_set_get_and_restore():
    irfilter.set_tuning("u16", 5, 256, irfilter.IRF_SELECT_BISECT)
    assert irfilter.get_tuning("u16", 5) == (256, irfilter.IRF_SELECT_BISECT)
    assert irfilter.get_tuning("u8", 5) == (128, irfilter.IRF_SELECT_NETWORK)  # per pixel type
    irfilter.set_tuning("u16", 5, 0, 0)
    assert irfilter.get_tuning("u16", 5) == (128, irfilter.IRF_SELECT_NETWORK)


@pytest.mark.parametrize("args,status", [
    (("u16", 13, 512, irfilter.IRF_SELECT_NETWORK), -11),
    (("u16", 5, 64, irfilter.IRF_SELECT_NETWORK), -11),
    (("u16", 5, 128, 3), -11),
    (("u16", 5, 128, 0), -11),
    (("u16", 4, 128, 1), -5),
    (("u16", 17, 128, 1), -5),
])
def test_invalid_tuning(args, status):
    dt, k, t, sel = args
    lib = irfilter.load()
    assert lib.ir_filter_set_tuning(irfilter._dtype_arg(dt), k, t, sel) == status
    assert lib.ir_filter_set_tuning(3, 5, 128, 1) == -4


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
        "batch": {"threads": 256, "ms": {}},
    }
    path = tmp_path / "t.json"
    autotune.save(table, str(path))
    back = autotune.load_file(str(path))
    assert back == json.loads(json.dumps(table))
    autotune.apply(back)
    assert irfilter.get_tuning("u16", 5) == (256, irfilter.IRF_SELECT_BISECT)
    assert irfilter.get_tuning("u16", 7) == (128, irfilter.IRF_SELECT_NETWORK)
    assert irfilter.get_batch_threads() == 256


def test_apply_rejects_unknown_choices():
    with pytest.raises(irfilter.IrfError):
        autotune.apply({"single": {"u16": {"13": {"threads": 512, "select": "network"}}}})


def test_candidates_cover_every_available_kernel():
    for k in (3, 9, 15):
        c = autotune.candidates(k)
        assert (128, irfilter.IRF_SELECT_NETWORK) in c and (256, irfilter.IRF_SELECT_BISECT) in c
        assert len(c) == 4
