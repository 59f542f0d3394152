"""Host logic of bench.py's counter records: a committed rocprofv3 record is
reported only while the kernel's source text is the one it was taken on, and,
where it names launch shapes, only for a run of one of those shapes."""
import json

import bench


def _write(tmp_path, name, rec):
    (tmp_path / name).write_text(json.dumps(rec))


def test_record_per_shape_and_stale_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_text_sha256", lambda family: "abc")
    shape_a = {"col_block": 4, "rows_per_tile": 425, "waves": 2}
    shape_b = {"col_block": 4, "rows_per_tile": 637, "waves": 4}
    _write(tmp_path, "slice_kernel_w_traffic.json", {
        "kernel_text_sha256": "abc",
        "records": [{"shape": shape_a, "hbm_bytes_per_launch": 1.5e9},
                    {"shape": shape_b, "hbm_bytes_per_launch": 1.4e9}]})
    st = dict(shape_a, kernel=5)
    assert bench._traffic("slice_kernel", "w", st) == 1.5e9
    assert bench._traffic("slice_kernel", "w", dict(shape_b)) == 1.4e9
    assert bench._traffic("slice_kernel", "w", {"col_block": 4, "rows_per_tile": 212, "waves": 2}) is None
    # no run given: the first record
    assert bench._traffic("slice_kernel", "w") == 1.5e9
    # the kernel's source changed since the counters were taken
    monkeypatch.setattr(bench, "kernel_text_sha256", lambda family: "def")
    assert bench._traffic("slice_kernel", "w", st) is None


def test_single_record_without_shape_and_missing_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_text_sha256", lambda family: "abc")
    _write(tmp_path, "tab_kernel_x_traffic.json", {"kernel_text_sha256": "abc", "hbm_bytes_per_launch": 5e10})
    assert bench._traffic("tab_kernel", "x", {"col_block": 16, "rows_per_tile": 441, "waves": 1}) == 5e10
    assert bench._traffic("tab_kernel", "missing") is None
    (tmp_path / "tab_kernel_bad_traffic.json").write_text("{not json")
    assert bench._traffic("tab_kernel", "bad") is None


def test_shape_keys_are_run_stats_fields():
    st = {"col_block": 4, "rows_per_tile": 425, "waves": 2, "kernel": 5, "recursion_ms": 1.0}
    assert bench._shape(st) == {"col_block": 4, "rows_per_tile": 425, "waves": 2}


def test_committed_records_name_their_shape_keys():
    """Every committed record list names the same shape keys the run
    statistics carry (so that a record can match a run)."""
    import glob
    import os
    for path in glob.glob(os.path.join(bench.PROFILES, "*_traffic.json")):
        d = json.load(open(path))
        for rec in d.get("records", [d]):
            shape = rec.get("shape")
            if shape is not None:
                assert set(shape) == {"col_block", "rows_per_tile", "waves"}, path
            assert rec.get("hbm_bytes_per_launch", 0) > 0, path
