"""The rocprofv3 summary tool on small hand-made result databases."""
import sqlite3

from paper_2406_13881_amd import rocprof_summary as rs


def _db(path, rows):
    db = sqlite3.connect(str(path))
    db.execute("create table counters_collection (kernel_name text, dispatch_id int, counter_name text, value real)")
    db.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    db.commit()
    db.close()
    return str(path)


def test_counters_sum_instances_and_average_dispatches(tmp_path):
    a = _db(tmp_path / "a.db", [("ompd_k_nu(int)", 1, "SQ_WAVES", 2.0), ("ompd_k_nu(int)", 1, "SQ_WAVES", 3.0),
                                ("ompd_k_nu(int)", 2, "SQ_WAVES", 7.0), ("copy_kernel", 1, "SQ_WAVES", 9.0)])
    b = _db(tmp_path / "b.db", [("ompd_k_nu(int)", 3, "SQ_INSTS_VALU", 10.0), ("ompd_k_ave(int)", 4, "SQ_INSTS_VALU", 4.0)])
    per = rs.counters([a, b])
    assert per == {"ompd_k_nu": {"SQ_WAVES": 6.0, "SQ_INSTS_VALU": 10.0}, "ompd_k_ave": {"SQ_INSTS_VALU": 4.0}}


def test_traffic_scales_by_the_copy_calibration(tmp_path):
    f = _db(tmp_path / "f.db", [("ompd_k_later(x)", 1, "FETCH_SIZE", 100.0), ("ompd_k_later(x)", 1, "FETCH_SIZE", 100.0)])
    w = _db(tmp_path / "w.db", [("ompd_k_later(x)", 1, "WRITE_SIZE", 50.0)])
    cf = _db(tmp_path / "cf.db", [("copy", 1, "FETCH_SIZE", 2048.0)])
    cw = _db(tmp_path / "cw.db", [("copy", 1, "WRITE_SIZE", 1024.0)])
    rec = rs.traffic(f, w, cf, cw, 1 << 20)
    k = rec["per_launch"]["ompd_k_later(x)"]
    # a 1 MiB copy reads 2048 KiB by the counter: factor 0.5; writes 1024 KiB: factor 1
    assert k["read_bytes"] == 100 * 1024 and k["written_bytes"] == 50 * 1024
