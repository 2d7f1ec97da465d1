"""The rocprofv3 summariser on small synthetic result databases: kernel-trace statistics and the
calibrated traffic record (a copy of N bytes reads FETCH_SIZE = N / 2048 KiB, as gfx950 counts its
128-byte read requests as 64 bytes)."""
import json
import sqlite3

from paper_1805_03560_amd import profsum


def _trace_db(path, launches):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer, vgpr_count integer, "
                "accum_vgpr_count integer, lds_size integer)")
    t = 0
    for name, us, *lds in launches:
        con.execute("insert into kernels values (?, ?, ?, 96, 0, ?)", (name, t, t + int(us * 1000), lds[0] if lds else 0))
        t += int(us * 1000) + 500
    con.commit()
    con.close()


def _pmc_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real, lds_block_size integer)")
    for r in rows:
        con.execute("insert into counters_collection values (?, ?, ?, ?, ?)", tuple(r) + (0,) * (5 - len(r)))
    con.commit()
    con.close()


def test_trace_table_statistics(tmp_path):
    db = str(tmp_path / "t.db")
    _trace_db(db, [("k_hop<0>", 280.0), ("k_hop<0>", 290.0), ("k_fill", 2.0)])
    text = profsum.trace_table(db)
    assert "vgpr_count" in text.splitlines()[-1]
    rows = [r for r in text.splitlines() if r.startswith("| `")]
    assert rows[0].startswith("| `k_hop<0>` | 0 | 2 | 285.0 | 280.0 | 290.0 | 0.57 |")
    assert "| `k_fill` | 0 | 1 | 2.0 |" in rows[1]


def test_traffic_record_scales_by_the_copy(tmp_path):
    n = 1 << 31
    cf, cw, f, w, t = (str(tmp_path / f"{k}.db") for k in ("cf", "cw", "f", "w", "t"))
    # instances of one counter are summed per dispatch; the copy reads half its bytes in FETCH_SIZE
    _pmc_db(cf, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", n / 2048 / 2)] * 2)
    _pmc_db(cw, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", n / 1024)])
    _pmc_db(f, [(5, "k_hop<0>", "FETCH_SIZE", 1000.0), (6, "k_hop<0>", "FETCH_SIZE", 1200.0), (7, "k_other", "FETCH_SIZE", 9.0)])
    _pmc_db(w, [(5, "k_hop<0>", "WRITE_SIZE", 300.0)])
    _trace_db(t, [("k_hop<0>", 100.0), ("k_hop<0>", 300.0), ("k_hop<0>", 900.0, 512)])

    class A:
        kernel, fetch, write, copy_fetch, copy_write, copy_bytes = "k_hop", f, w, cf, cw, float(n)
        trace, algorithmic, workload, json, lds, last, trace_last = t, 1.5e6, "test", str(tmp_path / "r.json"), 0, None, None
    text = profsum.traffic(A)
    rec = json.load(open(A.json))
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert rec["bytes_per_launch"] == int(round(1100 * 1024 * 2 + 300 * 1024))
    assert rec["avg_launch_us"] == 200.0
    assert rec["source_digest"] == profsum.source_digest()
    assert "measured / algorithmic" in text


def test_traffic_uses_the_last_dispatches(tmp_path):
    n = 1 << 31
    cf, cw, f, w = (str(tmp_path / f"{k}.db") for k in ("cf", "cw", "f", "w"))
    _pmc_db(cf, [(1, "copyBuffer", "FETCH_SIZE", n / 2048)])
    _pmc_db(cw, [(1, "copyBuffer", "WRITE_SIZE", n / 1024)])
    # tuning launches first (dispatches 1, 2), the timed ones last (3, 4)
    _pmc_db(f, [(1, "k_hop<0>", "FETCH_SIZE", 9000.0), (2, "k_hop<0>", "FETCH_SIZE", 9000.0),
                (3, "k_hop<0>", "FETCH_SIZE", 1000.0), (4, "k_hop<0>", "FETCH_SIZE", 1000.0)])
    _pmc_db(w, [(3, "k_hop<0>", "WRITE_SIZE", 10.0), (4, "k_hop<0>", "WRITE_SIZE", 30.0)])

    class A:
        kernel, fetch, write, copy_fetch, copy_write, copy_bytes = "k_hop", f, w, cf, cw, float(n)
        trace, algorithmic, workload, json, lds, last, trace_last = None, None, "", None, None, 2, None
    profsum.traffic(A)
    assert profsum._one(f, "FETCH_SIZE", "k_hop", last=2) == (1000.0, 2)
    assert profsum._one(f, "FETCH_SIZE", "k_hop") == (5000.0, 4)
