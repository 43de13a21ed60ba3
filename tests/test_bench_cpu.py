"""Host logic of bench.py: the counter record (HBM traffic and VALU
instructions of the 16-bit stack kernels) and its source stamp."""

import csv
import json
import os

import pytest

import bench

K7 = "void irf::fnr_persistent_kernel<unsigned short, 7, 1, 256, 1>(irf::StackArgs)"
K5 = "void irf::fnr_persistent_kernel<unsigned short, 5, 1, 128, 1>(irf::StackArgs)"


def test_kernel_names_map_to_variants():
    assert bench._fnr_u16_variant(K7) == (7, 256, 1)
    assert bench._fnr_u16_variant(K5) == (5, 128, 1)
    # detection-only mode, 8-bit kernels and other kernels carry no record
    assert bench._fnr_u16_variant(K7.replace("7, 1, 256", "7, 0, 256")) is None
    assert bench._fnr_u16_variant(K7.replace("unsigned short", "unsigned char")) is None
    assert bench._fnr_u16_variant("__amd_rocclr_copyBuffer") is None


def test_committed_record_is_read_only_on_its_own_sources():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["kernels"], "the record holds at least one kernel"
    for key, ent in rec["kernels"].items():
        assert ent["hbm_bytes_per_launch"] > bench.BYTES_PER_PX * 1024 * 640 * 512
        assert ent["valu_insts_per_launch"] > 0
        var = tuple(int(x) for x in key.split("/"))
        if rec["source_hash"] == bench.kernel_source_hash():
            assert bench.load_traffic(*var) == ent["hbm_bytes_per_launch"]
            assert bench.load_valu(*var) == ent["valu_insts_per_launch"]
        else:  # the kernels changed since the counters were taken: reported as null
            assert bench.load_traffic(*var) is None and bench.load_valu(*var) is None


def _write_csv(path, rows):
    cols = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))


def test_ingest_round_trip(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = 1 << 20
    _write_csv(tmp_path / "cf.csv", [(copy, "FETCH_SIZE", gib_kib / 2)] * 3)
    _write_csv(tmp_path / "cw.csv", [(copy, "WRITE_SIZE", gib_kib)] * 3)
    _write_csv(tmp_path / "f.csv", [(K7, "FETCH_SIZE", 1000.0), (K7, "FETCH_SIZE", 3000.0),
                                    (K5, "FETCH_SIZE", 10.0)])
    _write_csv(tmp_path / "w.csv", [(K7, "WRITE_SIZE", 500.0), (K5, "WRITE_SIZE", 20.0)])
    out = str(tmp_path / "rec.json")
    rec = bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                                str(tmp_path / "cw.csv"), out_path=out)
    cc = rec["copy_calibration"]
    assert cc["fetch_scale"] == pytest.approx(2.0) and cc["write_scale"] == pytest.approx(1.0)
    # fetch averaged over dispatches and doubled, writes taken as they are
    assert rec["kernels"]["7/256/1"]["hbm_bytes_per_launch"] == pytest.approx(2000 * 1024 * 2 + 500 * 1024)
    _write_csv(tmp_path / "sq.csv", [(K7, "SQ_INSTS_VALU", 100.0), (K7, "SQ_INSTS_VALU", 300.0),
                                     (K7, "SQ_WAVES", 7.0), (K5, "SQ_INSTS_VALU", 50.0)])
    rec = bench.ingest_sq(str(tmp_path / "sq.csv"), out_path=out)
    assert rec["kernels"]["7/256/1"]["valu_insts_per_launch"] == 200.0
    assert rec["kernels"]["5/128/1"]["valu_insts_per_launch"] == 50.0
    # a record taken on other sources is refused
    with open(out) as fh:
        stale = json.load(fh)
    stale["source_hash"] = "0" * 16
    with open(out, "w") as fh:
        json.dump(stale, fh)
    with pytest.raises(SystemExit):
        bench.ingest_sq(str(tmp_path / "sq.csv"), out_path=out)
    assert os.path.exists(out)


def test_code_text_drops_comments_only():
    src = ('int a = 1;  // trailing\n'
           '/* a block\n   over lines */\n'
           '\n'
           'const char *s = "// kept", *t = "/* kept */";\n'
           "char q = '\\'';  int b = 2 /* inline */ + 3;\n")
    text = bench.code_text(src)
    assert text == ('int a = 1;\n'
                    'const char *s = "// kept", *t = "/* kept */";\n'
                    "char q = '\\''; int b = 2 + 3;")
    # a comment edit keeps the stamp, a code edit changes it
    assert bench.code_text(src.replace("trailing", "other words")) == text
    assert bench.code_text(src.replace("= 2", "= 4")) != text


def test_valu_peak():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert bench.VALU_PEAK_T == pytest.approx(39.3216)
