"""CPU tests of the measurement-record tooling: the copy calibration of the
HBM counters and the source gate on recorded traffic."""
import sqlite3

import pytest

from paper_2104_00794_amd import profiling


def _counters_db(path, rows):
    con = sqlite3.connect(str(path))
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()
    return str(path)


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path, monkeypatch):
    gib = 1 << 30
    # the copy of 1 GiB reads as half its bytes (128-byte requests counted as 64) and writes in full
    cf = _counters_db(tmp_path / "cf.db", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib / 2048.0)] * 3)
    cw = _counters_db(tmp_path / "cw.db", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib / 1024.0)] * 3)
    kf = _counters_db(tmp_path / "kf.db", [("void tpx::k_step<4>(...)", "FETCH_SIZE", 1000.0),
                                           ("void tpx::k_step<4>(...)", "FETCH_SIZE", 3000.0),
                                           ("void tpx::k_other(...)", "FETCH_SIZE", 9e9)])
    kw = _counters_db(tmp_path / "kw.db", [("void tpx::k_step<4>(...)", "WRITE_SIZE", 500.0)])
    monkeypatch.setattr(profiling, "PROFILES", str(tmp_path))
    out = profiling.traffic_path("wl", "k_step")
    text = profiling.write_traffic_summary(out, "k_step<4>", "wl", kf, kw, cf, cw, gib, 4096.0 * 1024, ["cmd"])
    # fetch: mean 2000 KiB x 2 = 4000 KiB; write: 500 KiB x 1
    total = (2000.0 * 2 + 500.0) * 1024
    assert "traffic_bytes_per_launch = %.0f" % total in text
    assert profiling.read_traffic("wl", "k_step") == total
    assert "| traffic / algorithmic | %.3f |" % (total / (4096.0 * 1024)) in text


def test_recorded_traffic_is_dropped_once_the_kernel_source_changes(tmp_path, monkeypatch):
    monkeypatch.setattr(profiling, "PROFILES", str(tmp_path))
    path = profiling.traffic_path("wl", "k_step")
    with open(path, "w") as f:
        f.write("traffic_bytes_per_launch = 1234\nkernel_source_sha256 = %s\n" % ("0" * 64))
    assert profiling.read_traffic("wl", "k_step") is None
    with open(path, "w") as f:
        f.write("traffic_bytes_per_launch = 1234\nkernel_source_sha256 = %s\n" % profiling.kernel_source_sha256())
    assert profiling.read_traffic("wl", "k_step") == 1234.0
    assert profiling.read_traffic("wl", "absent") is None


def test_counter_mean_needs_a_matching_kernel(tmp_path):
    db = _counters_db(tmp_path / "x.db", [("void tpx::k_a(...)", "FETCH_SIZE", 1.0)])
    with pytest.raises(ValueError):
        profiling.counter_mean(db, "FETCH_SIZE", "k_b")
